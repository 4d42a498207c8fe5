// pf_adjoint.h -- adjoint (reverse mode) of one explicit step, 1D runs and 2D.
//
// For step n -> n+1, u^{n+1} = W(u^n + dt R(u^n; theta)) where W is the window
// shift (or identity) and R the right-hand sides of Eqs. cs_nonvar, cl_nonvar
// and phasefield_nonvar as discretised in pf_device.h.  Given the cotangent
// lam^{n+1} this computes lam^n = (d u^{n+1}/d u^n)^T lam^{n+1} and the
// parameter cotangents (A, alpha, lambda, W^2).  The transpose is taken stage
// by stage, in reverse order of the forward: update -> face fluxes -> cell rates
// (phi_t) -> mu_bar, each with its hand-derived local vector-Jacobian product.
//
// Tiling: a workgroup owns a tile T of cells and works on the box T + 3 held in
// LDS: u (T+3), the forward phi_t and mu_bar (T+2), and accumulators for the
// cotangents of u, mu_bar and phi_t.  It processes every face inside T+2 and
// every cell rate inside T+1 -- a superset of the computations whose stencil
// reaches T -- scattering into the accumulators with LDS atomics, and keeps the
// result on T.  Mirror ghosts are folded onto their image cells (scatter by
// canonical position); only real faces and cells are processed.  Parameter
// cotangents count each face and cell once (owned by the tile holding its
// lower cell).
#pragma once

#include <string>
#include <type_traits>

#include "pf_kernels.h"

namespace pfadj {

using pfk::Const;

constexpr int H = 3;  // box halo
constexpr int NTH = 5;  // per-block parameter cotangents: A, alpha, lambda, W^2, b

// p, 1-p, p', p'' of the interpolation function (APZ: a_p known to be zero).
template <bool APZ>
__device__ __forceinline__ void interp2(const Const& c, double phi, double& p, double& q, double& dp, double& d2p) {
  pfk::interp<APZ>(c, phi, p, q, dp);
  const double w = phi * (1.0 - phi), t = 1.0 - 2.0 * phi;
  const double d2h = c.quintic ? 60.0 * w * t : 6.0 * t;
  if constexpr (APZ) d2p = d2h;
  else d2p = d2h + c.ap * (6.0 * w * t - t * t * t);
}

// Tile geometry: DIM = 1 (growth axis only) or 2 (x transverse, z growth).
// 1D: threads per workgroup = cells of the box (tile + halo 3 on each side)
constexpr int ADJ1_NT = 256;

template <int DIM>
struct Geo {
  static constexpr int TX = (DIM == 2) ? 16 : 1;
  static constexpr int TZ = (DIM == 2) ? 16 : ADJ1_NT - 2 * H;  // 1D: one box cell per thread
  static constexpr int BX = (DIM == 2) ? TX + 2 * H : 1;
  static constexpr int BZ = TZ + 2 * H;
  static constexpr int NB = BX * BZ;
  static constexpr int HX = (DIM == 2) ? H : 0;
  static constexpr int NT = (DIM == 2) ? 256 : ADJ1_NT;
  // box index of local coordinates (lx, lz) relative to the tile origin
  __device__ static __forceinline__ int idx(int lx, int lz) { return (lx + HX) + BX * (lz + H); }
  // unit offset along axis a (0 = x in 2D, DIM-1 = z)
  __device__ static __forceinline__ int off(int a) { return (DIM == 2 && a == 0) ? 1 : BX; }
};

// Per-block description of the domain the tile belongs to.
struct Dom {
  int nx, nz;           // extents (nx = 1 in 1D)
  int px;               // periodic x
  long long base;       // first cell of the run / domain
  int x0, z0;           // tile origin
  double V, dt, zfront; // run constants
};

__device__ __forceinline__ int reflect(int g, int n) {
  while (g < 0 || g >= n) {
    if (g < 0) g = -g - 1;
    if (g >= n) g = 2 * n - g - 1;
  }
  return g;
}

template <int DIM>
struct Acc {
  double* au[3];
  double* amu;
  double* apt;
};

// Canonical box position of the box cell at local coordinates (lx, lz): mirror
// ghosts folded onto their images (z always; x when not periodic), or -1 when
// the image lies outside the box.  Tabulated once per block.
template <int DIM>
__device__ __forceinline__ int canonical(const Dom& d, int lx, int lz) {
  using G = Geo<DIM>;
  int gz = d.z0 + lz;
  if (gz < 0 || gz >= d.nz) lz = reflect(gz, d.nz) - d.z0;
  if (DIM == 2 && !d.px) {
    int gx = d.x0 + lx;
    if (gx < 0 || gx >= d.nx) lx = reflect(gx, d.nx) - d.x0;
  }
  if (lz < -H || lz >= G::TZ + H) return -1;
  if (DIM == 2 && (lx < -H || lx >= G::TX + H)) return -1;
  return G::idx(lx, lz);
}

// Scatter helper: adds v at the canonical position of box cell i (every
// scatter target of the face and cell stages lies inside the box).  2D reads
// the block's table and scatters unconditionally (zeros included; images
// outside the box go to the spare slot NB): straight-line LDS atomics, 9 %
// faster than testing each value.  1D folds its one axis inline and skips
// zeros and images outside the box.
template <int DIM>
__device__ __forceinline__ void scat(double* a, const Dom& d, const int* canon, int i, double v) {
  if constexpr (DIM == 2) {
    atomicAdd(&a[canon[i]], v);
  } else {
    if (v == 0.0) return;
    const int j = canonical<1>(d, 0, i - H);
    if (j >= 0) atomicAdd(&a[j], v);
  }
}

template <int DIM, bool APZ>
__device__ void adjoint_tile(const Const& c, const Dom& d, long long n, int shift, const double* const* u,
                             const double* const* lam1, double* const* lam0, double* theta_out, int accum) {
  using G = Geo<DIM>;
  __shared__ double su[3][G::NB], sl[3][G::NB], spt[G::NB], smu[G::NB];
  __shared__ double au[3][G::NB + 1], amu[G::NB + 1], apt[G::NB + 1];  // slot NB: discarded scatters
  // 1D: (mu_s - mu_l)/Omega of the box, computed once (2D: recomputed; no LDS room)
  __shared__ double sdm[(DIM == 1) ? G::NB : 1];
  __shared__ double red[NTH][G::NT / 64];
  __shared__ int canon[(DIM == 2) ? G::NB : 1];
  const int tid = threadIdx.x;
  const double tn = (double)n * d.dt;
  const double sn = floor(d.V * tn / c.dx);

  // ---- load u and the (shift-adjusted) cotangent on the box
  for (int i = tid; i < G::NB; i += G::NT) {
    const int lx = i % G::BX - G::HX, lz = i / G::BX - H;
    int gx = d.x0 + lx, gz = d.z0 + lz;
    if (DIM == 2) gx = pfk::map_axis(gx, d.nx, d.px);
    else gx = 0;
    gz = reflect(gz, d.nz);
    const long long o = d.base + gx + (long long)d.nx * gz;
    for (int f = 0; f < 3; ++f) su[f][i] = u[f][o];
    for (int f = 0; f < 3; ++f) {
      double v;
      if (shift) v = (gz >= 1) ? lam1[f][o - d.nx] : 0.0;
      else v = lam1[f][o];
      sl[f][i] = v;
      au[f][i] = 0.0;
    }
    amu[i] = 0.0;
    apt[i] = 0.0;
    spt[i] = 0.0;
    if (DIM == 2) {
      const int j = canonical<DIM>(d, lx, lz);
      canon[i] = (j < 0) ? G::NB : j;
    }
    {  // mu_bar, pointwise: whole box
      double p, q;
      pfk::interp_pq<APZ>(c, su[0][i], p, q);
      const double ll = pfk::flog(su[2][i]);
      const double dm = pfk::flog(su[1][i]) - ll - c.log_ke;
      smu[i] = ll + p * dm;
      if constexpr (DIM == 1) sdm[i] = dm;
    }
  }
  __syncthreads();

  auto cleq_of_lz = [&](int lz) {
    const int gz = d.z0 + lz;
    const double zlab = ((double)gz + sn + 0.5) * c.dx;
    return pfk::cleq_at(c, zlab, tn, d.V, d.zfront);
  };
  auto in_box = [&](int lx, int lz, int h) {
    return lz >= -h && lz < G::TZ + h && (DIM == 1 || (lx >= -h && lx < G::TX + h));
  };
  auto real_cell = [&](int lx, int lz) {
    const int gz = d.z0 + lz;
    if (gz < 0 || gz >= d.nz) return false;
    if (DIM == 2 && !d.px) {
      const int gx = d.x0 + lx;
      if (gx < 0 || gx >= d.nx) return false;
    }
    return true;
  };
  auto owned = [&](int lx, int lz) {  // canonical cell inside the tile and the domain
    if (!real_cell(lx, lz)) return false;
    if (lz < 0 || lz >= G::TZ || d.z0 + lz >= d.nz) return false;
    if (DIM == 2) {
      if (lx < 0 || lx >= G::TX || d.x0 + lx >= d.nx) return false;
    }
    return true;
  };

  // Central differences and Laplacian of the cell at box index i.
  auto cell_inputs = [&](int i, double* gph, double* gcs, double* gcl, double& lap) {
    lap = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int o = G::off(a);
      gph[a] = (su[0][i + o] - su[0][i - o]) * c.inv_2dx;
      gcs[a] = (su[1][i + o] - su[1][i - o]) * c.inv_2dx;
      gcl[a] = (su[2][i + o] - su[2][i - o]) * c.inv_2dx;
      lap += (su[0][i + o] - 2.0 * su[0][i] + su[0][i - o]);
    }
    lap *= c.inv_dx2;
  };

  // ---- forward cell stage on T+2
  for (int i = tid; i < G::NB; i += G::NT) {
    const int lx = i % G::BX - G::HX, lz = i / G::BX - H;
    if (!in_box(lx, lz, 2)) continue;
    double gph[DIM], gcs[DIM], gcl[DIM], lap;
    cell_inputs(i, gph, gcs, gcl, lap);
    double pt;
    if constexpr (DIM == 1) {
      double p, q, dp;
      pfk::interp<APZ>(c, su[0][i], p, q, dp);
      const double G = gph[0] * gph[0], dot = (c.Ds * gcs[0] - c.b * gcl[0]) * gph[0];
      const double kcl = (c.ke - 1.0) * cleq_of_lz(lz);
      pt = pfk::cell_rate(c, kcl, su[0][i], su[1][i], su[2][i], sdm[i], p, q, dp, G, dot, c.W2 * lap, c.eps2, c.onemA);
    } else {
      double mu;
      const double kcl = (c.ke - 1.0) * cleq_of_lz(lz);
      pfk::cell_stage<DIM, APZ>(c, kcl, su[0][i], su[1][i], su[2][i], gph, gcs, gcl, lap, pt, mu);
    }
    spt[i] = pt;
  }
  __syncthreads();

  double thA = 0.0, thAl = 0.0, thLa = 0.0, thW2 = 0.0, thB = 0.0;  // cotangents of A, alpha, lambda, W^2, b

  // ---- faces inside T+2: forward flux inputs, then their VJP
  auto do_faces = [&](auto axis) {
    constexpr int K = decltype(axis)::value;
    constexpr int J = (DIM == 2) ? 1 - K : 0;  // transverse axis (2D)
    const int oK = G::off(K);
    const int oJ = G::off(J);
    for (int i = tid; i < G::NB; i += G::NT) {
      const int lx = i % G::BX - G::HX, lz = i / G::BX - H;
      const int bx = lx + ((DIM == 2 && K == 0) ? 1 : 0), bz = lz + ((K == DIM - 1) ? 1 : 0);
      if (!in_box(lx, lz, 2) || !in_box(bx, bz, 2)) continue;
      // a real face joins two real cells (a mirror boundary face carries no flux)
      if (!real_cell(lx, lz) || !real_cell(bx, bz)) continue;
      const int ia = i, ib = i + oK;
      // forward
      double gph[DIM], gmu[DIM], gcs[DIM], gcl[DIM];
      gph[K] = (su[0][ib] - su[0][ia]) * c.inv_dx;
      gmu[K] = (smu[ib] - smu[ia]) * c.inv_dx;
      gcs[K] = (su[1][ib] - su[1][ia]) * c.inv_dx;
      gcl[K] = (su[2][ib] - su[2][ia]) * c.inv_dx;
      if (DIM == 2) {
        gph[J] = ((su[0][ia + oJ] - su[0][ia - oJ]) + (su[0][ib + oJ] - su[0][ib - oJ])) * c.inv_4dx;
        gmu[J] = ((smu[ia + oJ] - smu[ia - oJ]) + (smu[ib + oJ] - smu[ib - oJ])) * c.inv_4dx;
        gcs[J] = ((su[1][ia + oJ] - su[1][ia - oJ]) + (su[1][ib + oJ] - su[1][ib - oJ])) * c.inv_4dx;
        gcl[J] = ((su[2][ia + oJ] - su[2][ia - oJ]) + (su[2][ib + oJ] - su[2][ib - oJ])) * c.inv_4dx;
      }
      const double phf = 0.5 * (su[0][ia] + su[0][ib]);
      const double csf = 0.5 * (su[1][ia] + su[1][ib]);
      const double clf = 0.5 * (su[2][ia] + su[2][ib]);
      const double ptf = 0.5 * (spt[ia] + spt[ib]);
      // cotangents of the fluxes: cell a gains +F/dx, cell b loses it
      const double Fsb = c.dt * c.inv_dx * (sl[1][ia] - sl[1][ib]);
      const double Flb = c.dt * c.inv_dx * (sl[2][ia] - sl[2][ib]);
      // recompute the face intermediates
      double p, q, dp;
      pfk::interp<APZ>(c, phf, p, q, dp);
      double Gs = 0.0, dmu = 0.0, dcs = 0.0, dcl = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        Gs += gph[j] * gph[j];
        dmu += gph[j] * gmu[j];
        dcs += gph[j] * gcs[j];
        dcl += gph[j] * gcl[j];
      }
      const double Ms = c.Ds * csf, Ml = clf;
      const double ms = Ms * q, ml = c.b * Ml * p, Mb = ms + ml;
      const double Sg = Gs * Gs + c.eps2;
      const double iMS = pfk::frcp(Mb * Sg);  // also 1/Mb = Sg iMS and 1/S = Mb iMS
      const double R = gph[K] * Gs * iMS;  // (grad phi)_K gam / Mbar, gam = G / (G^2 + eps^2)
      const double bq = c.b * p + q;
      const double dcf = csf - clf;
      const double at = c.onemA * dcf * ptf * R;
      // reverse
      double gph_b[DIM] = {}, gmu_b[DIM] = {}, gcs_b[DIM] = {}, gcl_b[DIM] = {};
      double Mb_b = 0.0, R_b = 0.0, ms_b = 0.0, ml_b = 0.0, Ms_b = 0.0, Ml_b = 0.0, p_b = 0.0, q_b = 0.0;
      double csf_b = 0.0, clf_b = 0.0, ptf_b = 0.0;
      const double nrm_b = Fsb + Flb;
      gcs_b[K] += Fsb * c.Ds;
      const double dcs_b = -Fsb * c.Ds * Mb * R;
      Mb_b += -Fsb * c.Ds * dcs * R;
      R_b += -Fsb * c.Ds * dcs * Mb;
      const double at_b = Fsb * ms - Flb * ml;
      ms_b += Fsb * at;
      ml_b += -Flb * at;
      gcl_b[K] += Flb;
      const double dcl_b = -Flb * Mb * R;
      Mb_b += -Flb * dcl * R;
      R_b += -Flb * dcl * Mb;
      // at = (1-A) dcf ptf R
      if (owned(lx, lz)) thA += -at_b * dcf * ptf * R;
      const double dcf_b = at_b * c.onemA * ptf * R;
      ptf_b += at_b * c.onemA * dcf * R;
      R_b += at_b * c.onemA * dcf * ptf;
      csf_b += dcf_b;
      clf_b -= dcf_b;
      // nrm = Ms Ml bq dmu R
      Ms_b += nrm_b * Ml * bq * dmu * R;
      Ml_b += nrm_b * Ms * bq * dmu * R;
      const double bq_b = nrm_b * Ms * Ml * dmu * R;
      const double dmu_b = nrm_b * Ms * Ml * bq * R;
      R_b += nrm_b * Ms * Ml * bq * dmu;
      p_b += bq_b * c.b;
      q_b += bq_b;
      if (owned(lx, lz)) thB += bq_b * p;  // bq = b p + q
      // R = gph[K] G / (Mb S), S = G^2 + eps^2
      double Gs_b = R_b * gph[K] * iMS - R_b * R * 2.0 * Gs * (Mb * iMS);
      gph_b[K] += R_b * Gs * iMS;
      Mb_b += -R_b * R * (Sg * iMS);
      ms_b += Mb_b;
      ml_b += Mb_b;
      Ms_b += ms_b * q;
      q_b += ms_b * Ms;
      Ml_b += ml_b * c.b * p;
      p_b += ml_b * c.b * Ml;
      if (owned(lx, lz)) thB += ml_b * Ml * p;  // ml = b M_l p
      csf_b += Ms_b * c.Ds;
      clf_b += Ml_b;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        gph_b[j] += dmu_b * gmu[j] + dcs_b * gcs[j] + dcl_b * gcl[j] + Gs_b * 2.0 * gph[j];
        gmu_b[j] += dmu_b * gph[j];
        gcs_b[j] += dcs_b * gph[j];
        gcl_b[j] += dcl_b * gph[j];
      }
      const double phf_b = (p_b - q_b) * dp;
      // distribute to the cells of the stencil
      scat<DIM>(au[0], d, canon, ia, 0.5 * phf_b - gph_b[K] * c.inv_dx);
      scat<DIM>(au[0], d, canon, ib, 0.5 * phf_b + gph_b[K] * c.inv_dx);
      scat<DIM>(au[1], d, canon, ia, 0.5 * csf_b - gcs_b[K] * c.inv_dx);
      scat<DIM>(au[1], d, canon, ib, 0.5 * csf_b + gcs_b[K] * c.inv_dx);
      scat<DIM>(au[2], d, canon, ia, 0.5 * clf_b - gcl_b[K] * c.inv_dx);
      scat<DIM>(au[2], d, canon, ib, 0.5 * clf_b + gcl_b[K] * c.inv_dx);
      scat<DIM>(amu, d, canon, ia, -gmu_b[K] * c.inv_dx);
      scat<DIM>(amu, d, canon, ib, gmu_b[K] * c.inv_dx);
      scat<DIM>(apt, d, canon, ia, 0.5 * ptf_b);
      scat<DIM>(apt, d, canon, ib, 0.5 * ptf_b);
      if (DIM == 2) {  // transverse neighbours of both cells: box offsets +-oJ
        const double* gb[3] = {&gph_b[J], &gcs_b[J], &gcl_b[J]};
        for (int f = 0; f < 3; ++f) {
          const double v = *gb[f] * c.inv_4dx;
          scat<DIM>(au[f], d, canon, ia + oJ, v);
          scat<DIM>(au[f], d, canon, ia - oJ, -v);
          scat<DIM>(au[f], d, canon, ib + oJ, v);
          scat<DIM>(au[f], d, canon, ib - oJ, -v);
        }
        const double v = gmu_b[J] * c.inv_4dx;
        scat<DIM>(amu, d, canon, ia + oJ, v);
        scat<DIM>(amu, d, canon, ia - oJ, -v);
        scat<DIM>(amu, d, canon, ib + oJ, v);
        scat<DIM>(amu, d, canon, ib - oJ, -v);
      }
    }
  };
  do_faces(std::integral_constant<int, DIM - 1>{});
  if constexpr (DIM == 2) do_faces(std::integral_constant<int, 0>{});
  __syncthreads();

  // ---- cell rates on T+1: update/source cotangents, then the phi_t VJP
  for (int i = tid; i < G::NB; i += G::NT) {
    const int lx = i % G::BX - G::HX, lz = i / G::BX - H;
    if (!in_box(lx, lz, 1) || !real_cell(lx, lz)) continue;
    const bool own = owned(lx, lz);
    const double ph = su[0][i], cs = su[1][i], cl = su[2][i];
    const double pt = spt[i];
    double p, q, dp, d2p;
    interp2<APZ>(c, ph, p, q, dp, d2p);
    const double dc = cs - cl;
    // u' = u + dt (div F + src) (c_s, c_l), phi' = phi + dt phi_t; src = -A dc p' phi_t
    const double sb = c.dt * (sl[1][i] + sl[2][i]);
    double pt_b = apt[i] + c.dt * sl[0][i] + sb * (-c.A * dc * dp);
    if (own) thA += sb * (-dc * dp * pt);
    // source partials w.r.t. the cell's own fields
    double ph_b = sb * (-c.A * dc * d2p * pt);
    double cs_b = sb * (-c.A * dp * pt);
    double cl_b = sb * (c.A * dp * pt);
    // phi_t VJP: recompute the forward intermediates
    double gph[DIM], gcs[DIM], gcl[DIM], lap;
    cell_inputs(i, gph, gcs, gcl, lap);
    const double cleq = cleq_of_lz(lz);
    double dmu;
    if constexpr (DIM == 1) dmu = sdm[i];
    else dmu = pfk::flog(cs) - pfk::flog(cl) - c.log_ke;
    const double dGc = cs * dmu + (c.ke - 1.0) * cleq - dc;
    const double ms = c.Ds * cs * q, ml = c.b * cl * p, Mb = ms + ml;
    const double Dn = ms * (1.0 - c.A * q) + c.A * ml * p;
    double Gs = 0.0, dot = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      Gs += gph[k] * gph[k];
      dot += (c.Ds * gcs[k] - c.b * gcl[k]) * gph[k];
    }
    const double Sg = Gs * Gs + c.eps2;
    const double bq = c.b * p + q;
    const double Q = Mb * bq * Sg;
    const double pq = p * q;
    const double oA = c.onemA;
    const double fdw = 2.0 * ph * (1.0 - ph) * (1.0 - 2.0 * ph);
    const double base = c.W2 * lap - fdw - c.lambda * dGc * dp;
    const double X2 = Dn * dc * dmu * dp * bq * Sg;
    const double X3 = oA * dc * pq * dot * Gs * bq;
    const double Kd = oA * oA * c.b * dc * dc * pq * Gs;
    const double num = base * Q + c.lambda * X2 + c.lambda * X3;
    const double den = c.alpha * Q + c.lambda * Kd;
    const double iden = pfk::frcp(den);
    const double num_b = pt_b * iden;
    const double den_b = -pt_b * num * iden * iden;
    double Q_b = den_b * c.alpha + num_b * base;
    if (own) {
      thAl += den_b * Q;
      thLa += den_b * Kd + num_b * (X2 + X3);
    }
    double dc_b = 0.0, pq_b = 0.0, dot_b = 0.0, bq_b = 0.0, p_b = 0.0, q_b = 0.0, Gs_b = 0.0, Sg_b = 0.0;
    double dmu_b = 0.0, dp_b = 0.0, Dn_b = 0.0, Mb_b = 0.0, ms_b = 0.0, ml_b = 0.0, lap_b = 0.0;
    {  // Kd = (1-A)^2 b dc^2 pq G
      const double Kd_b = den_b * c.lambda;
      if (own) {
        thA += Kd_b * (-2.0 * oA * c.b * dc * dc * pq * Gs);
        thB += Kd_b * oA * oA * dc * dc * pq * Gs;
      }
      dc_b += Kd_b * 2.0 * oA * oA * c.b * dc * pq * Gs;
      pq_b += Kd_b * oA * oA * c.b * dc * dc * Gs;
      Gs_b += Kd_b * oA * oA * c.b * dc * dc * pq;
    }
    {  // X3 = (1-A) dc pq dot G bq
      const double X3_b = num_b * c.lambda;
      if (own) thA += X3_b * (-dc * pq * dot * Gs * bq);
      dc_b += X3_b * oA * pq * dot * Gs * bq;
      pq_b += X3_b * oA * dc * dot * Gs * bq;
      dot_b += X3_b * oA * dc * pq * Gs * bq;
      Gs_b += X3_b * oA * dc * pq * dot * bq;
      bq_b += X3_b * oA * dc * pq * dot * Gs;
    }
    {  // X2 = Dn dc dmu dp bq S
      const double X2_b = num_b * c.lambda;
      Dn_b += X2_b * dc * dmu * dp * bq * Sg;
      dc_b += X2_b * Dn * dmu * dp * bq * Sg;
      dmu_b += X2_b * Dn * dc * dp * bq * Sg;
      dp_b += X2_b * Dn * dc * dmu * bq * Sg;
      bq_b += X2_b * Dn * dc * dmu * dp * Sg;
      Sg_b += X2_b * Dn * dc * dmu * dp * bq;
    }
    {  // base = W2 lap - fdw - lambda dGc dp
      const double base_b = num_b * Q;
      if (own) {
        thW2 += base_b * lap;
        thLa += -base_b * dGc * dp;
      }
      lap_b += base_b * c.W2;
      ph_b += -base_b * 2.0 * (1.0 - 6.0 * ph + 6.0 * ph * ph);
      const double dGc_b = -base_b * c.lambda * dp;
      dp_b += -base_b * c.lambda * dGc;
      cs_b += dGc_b * dmu;
      dmu_b += dGc_b * cs;
      dc_b += -dGc_b;
    }
    // Q = Mb bq S, S = G^2 + eps^2
    Mb_b += Q_b * bq * Sg;
    bq_b += Q_b * Mb * Sg;
    Sg_b += Q_b * Mb * bq;
    Gs_b += Sg_b * 2.0 * Gs;
    p_b += pq_b * q + bq_b * c.b;
    q_b += pq_b * p + bq_b;
    if (own) thB += bq_b * p;  // bq = b p + q
    // Dn = ms (1 - A q) + A ml p
    ms_b += Dn_b * (1.0 - c.A * q);
    if (own) thA += Dn_b * (-ms * q + ml * p);
    q_b += Dn_b * (-c.A * ms);
    ml_b += Dn_b * c.A * p;
    p_b += Dn_b * c.A * ml;
    ms_b += Mb_b;
    ml_b += Mb_b;
    cs_b += ms_b * c.Ds * q;
    q_b += ms_b * c.Ds * cs;
    cl_b += ml_b * c.b * p;
    p_b += ml_b * c.b * cl;
    if (own) {
      thB += ml_b * cl * p;  // ml = b c_l p
      double gg = 0.0;       // dot = (Ds grad c_s - b grad c_l) . grad phi
#pragma unroll
      for (int k = 0; k < DIM; ++k) gg += gcl[k] * gph[k];
      thB += -dot_b * gg;
    }
    cs_b += dc_b;
    cl_b -= dc_b;
    const double icscl = pfk::frcp(cs * cl);
    cs_b += dmu_b * (cl * icscl);
    cl_b -= dmu_b * (cs * icscl);
    ph_b += (p_b - q_b) * dp + dp_b * d2p;
    // stencil: central differences and Laplacian
    double gph_b[DIM], gcs_b[DIM], gcl_b[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      gph_b[k] = dot_b * (c.Ds * gcs[k] - c.b * gcl[k]) + Gs_b * 2.0 * gph[k];
      gcs_b[k] = dot_b * c.Ds * gph[k];
      gcl_b[k] = -dot_b * c.b * gph[k];
    }
    scat<DIM>(au[0], d, canon, i, ph_b - 2.0 * DIM * lap_b * c.inv_dx2);
    scat<DIM>(au[1], d, canon, i, cs_b);
    scat<DIM>(au[2], d, canon, i, cl_b);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int o = G::off(k);
      scat<DIM>(au[0], d, canon, i + o, gph_b[k] * c.inv_2dx + lap_b * c.inv_dx2);
      scat<DIM>(au[0], d, canon, i - o, -gph_b[k] * c.inv_2dx + lap_b * c.inv_dx2);
      scat<DIM>(au[1], d, canon, i + o, gcs_b[k] * c.inv_2dx);
      scat<DIM>(au[1], d, canon, i - o, -gcs_b[k] * c.inv_2dx);
      scat<DIM>(au[2], d, canon, i + o, gcl_b[k] * c.inv_2dx);
      scat<DIM>(au[2], d, canon, i - o, -gcl_b[k] * c.inv_2dx);
    }
  }
  __syncthreads();

  // ---- result on T: identity + accumulated + mu_bar VJP (pointwise)
  for (int i = tid; i < G::NB; i += G::NT) {
    const int lx = i % G::BX - G::HX, lz = i / G::BX - H;
    if (!owned(lx, lz)) continue;
    const double ph = su[0][i], cs = su[1][i], cl = su[2][i];
    double p, q, dp;
    pfk::interp<APZ>(c, ph, p, q, dp);
    const double mb = amu[i];
    double dmu;
    if constexpr (DIM == 1) dmu = sdm[i];
    else dmu = pfk::flog(cs) - pfk::flog(cl) - c.log_ke;
    // mu_bar = ln cl + p dmu
    const double icscl = pfk::frcp(cs * cl);
    const double r0 = sl[0][i] + au[0][i] + mb * dmu * dp;
    const double r1 = sl[1][i] + au[1][i] + mb * p * (cl * icscl);
    const double r2 = sl[2][i] + au[2][i] + mb * q * (cs * icscl);
    const long long o = d.base + (long long)(d.x0 + lx) + (long long)d.nx * (d.z0 + lz);
    lam0[0][o] = r0;
    lam0[1][o] = r1;
    lam0[2][o] = r2;
  }
  // ---- parameter cotangents of this block: a fixed butterfly within each
  // wave, then the wave sums in wave order (deterministic)
  double th[NTH] = {thA, thAl, thLa, thW2, thB};
#pragma unroll
  for (int k = 0; k < NTH; ++k)
    for (int m = 32; m > 0; m >>= 1) th[k] += __shfl_xor(th[k], m, 64);
  if ((tid & 63) == 0)
    for (int k = 0; k < NTH; ++k) red[k][tid >> 6] = th[k];
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < NTH; ++k) {
      double t = 0.0;
      for (int w = 0; w < G::NT / 64; ++w) t += red[k][w];
      theta_out[k] = accum ? theta_out[k] + t : t;  // accum: sum over the steps of a segment
    }
}

// 1D runs (single domain = run 0): block -> (run, tile) from a table.
struct Tile1 {
  int run, z0;
};

template <bool APZ>
__global__ __launch_bounds__(ADJ1_NT) void k_adj1d(Const c, pfk::RunTab rt, const Tile1* __restrict__ tiles, long long n,
                                               int do_shift, const double* u0, const double* u1, const double* u2,
                                               const double* l0, const double* l1, const double* l2, double* o0,
                                               double* o1, double* o2, double* __restrict__ part, int accum) {
  const Tile1 t = tiles[blockIdx.x];
  Dom d;
  d.nx = 1;
  d.nz = rt.n[t.run];
  d.px = 0;
  d.base = rt.off[t.run];
  d.x0 = 0;
  d.z0 = t.z0;
  d.V = rt.V[t.run];
  d.dt = rt.dt[t.run];
  d.zfront = rt.z0[t.run];
  Const cc = c;
  cc.dt = d.dt;
  const double tn1 = (double)(n + 1) * d.dt, tn = (double)n * d.dt;
  const int shift = do_shift && (floor(d.V * tn1 / c.dx) > floor(d.V * tn / c.dx));
  const double* u[3] = {u0, u1, u2};
  const double* l[3] = {l0, l1, l2};
  double* o[3] = {o0, o1, o2};
  adjoint_tile<1, APZ>(cc, d, n, shift, u, l, o, part + NTH * blockIdx.x, accum);
}

template <bool APZ>
__global__ __launch_bounds__(256) void k_adj2d(Const c, long long n, int shift, const double* u0, const double* u1,
                                               const double* u2, const double* l0, const double* l1,
                                               const double* l2, double* o0, double* o1, double* o2,
                                               double* __restrict__ part, int accum) {
  Dom d;
  d.nx = c.nx;
  d.nz = c.nz;
  d.px = c.px;
  d.base = 0;
  d.x0 = blockIdx.x * Geo<2>::TX;
  d.z0 = blockIdx.y * Geo<2>::TZ;
  d.V = c.V;
  d.dt = c.dt;
  d.zfront = c.z0;
  const double* u[3] = {u0, u1, u2};
  const double* l[3] = {l0, l1, l2};
  double* o[3] = {o0, o1, o2};
  adjoint_tile<2, APZ>(c, d, n, shift, u, l, o, part + NTH * (blockIdx.x + gridDim.x * blockIdx.y), accum);
}

// Sum the block partials in block order and add the cotangents of
// theta = (A, M_phi, W, b): alpha = W / M_phi, lambda = lambda0 W, W^2.
__global__ void k_theta_final(Const c, const double* __restrict__ part, int nblk, double* __restrict__ dtheta) {
  __shared__ double red[NTH][256];
  double s[NTH] = {};
  for (int b = threadIdx.x; b < nblk; b += 256)
    for (int k = 0; k < NTH; ++k) s[k] += part[NTH * b + k];
  for (int k = 0; k < NTH; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < NTH; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double gA = red[0][0], gal = red[1][0], gla = red[2][0], gW2 = red[3][0], gb = red[4][0];
    dtheta[0] += gA;
    dtheta[1] += gal * (-c.W / (c.Mphi * c.Mphi));
    dtheta[2] += gal / c.Mphi + gla * c.lambda0 + gW2 * 2.0 * c.W;
    dtheta[3] += gb;
  }
}

}  // namespace pfadj
