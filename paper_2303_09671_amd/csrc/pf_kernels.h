// pf_kernels.h -- forward kernels: fused z-streaming step (2D/3D), persistent
// register-chunk kernel for single and batched 1D runs, deterministic
// reductions (energy, solute, c_max) and the k_v adjoint seed.
#pragma once

#include <type_traits>

#include "pf_device.h"

namespace pfk {

// ---------------------------------------------------------------------------
// Index helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int mirror_idx(int g, int n) {
  // reflect about the outer faces: -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2
  if (g >= 0 && g < n) return g;
  while (g < 0 || g >= n) {
    if (g < 0) g = -g - 1;
    if (g >= n) g = 2 * n - g - 1;
  }
  return g;
}
__device__ __forceinline__ int map_axis(int g, int n, int periodic) {
  if (g >= 0 && g < n) return g;
  if (periodic) {
    if (g < 0 && g + n >= 0) return g + n;
    if (g >= n && g - n < n) return g - n;
    g %= n;
    return g < 0 ? g + n : g;
  }
  return mirror_idx(g, n);
}

// ---------------------------------------------------------------------------
// Fused step for 2D and 3D: each workgroup owns a TX x TY column tile of the
// transverse plane(s) and streams through a range of z planes.  A 3-plane ring
// (z-1, z, z+1) of (phi, c_s, c_l) with an in-plane halo of 2 lives in LDS;
// phi_t and mu_bar of each plane are computed once on the tile plus an in-plane
// halo of 1 (the plane z+2 they need above comes straight from global memory)
// and kept in 2- and 3-plane rings; x/y face fluxes go through LDS and the
// z-face flux below a cell stays in a register for the next plane.  One HBM read
// and one HBM write of the three fields per cell and step, plus halo re-reads
// (mostly L2 hits); the ring planes are loaded by LDS DMA.  With a window
// shift the updated plane z is stored at z-1 and the fresh liquid layer at the
// top.
// ---------------------------------------------------------------------------
// 3D: one thread per tile column (TX * TY threads).  2D: one wave covers the
// tile (TX = 62 columns) plus its two halo columns, so the cell stage of the
// tile and halo and the TX + 1 x faces each take a single pass of the wave.
template <int DIM, int TX, int TY>
struct StreamGeom {
  static constexpr int NT = (DIM == 2) ? TX + 2 : TX * TY;
  static constexpr int BX2 = TX + 4;
  static constexpr int BY2 = (DIM == 3) ? TY + 4 : 1;
  static constexpr int BX1 = TX + 2;
  static constexpr int BY1 = (DIM == 3) ? TY + 2 : 1;
  static constexpr int P2 = BX2 * BY2;
  static constexpr int P1 = BX1 * BY1;
  static constexpr int OY2 = (DIM == 3) ? 2 : 0;
  static constexpr int OY1 = (DIM == 3) ? 1 : 0;
  static constexpr int NFX = (TX + 1) * TY;
  static constexpr int NFY = (DIM == 3) ? TX * (TY + 1) : 0;
  __device__ static __forceinline__ int i2(int lx, int ly) { return (lx + 2) + BX2 * (ly + OY2); }
  __device__ static __forceinline__ int i1(int lx, int ly) { return (lx + 1) + BX1 * (ly + OY1); }
};

template <int DIM, int TX, int TY, bool APZ, bool EQ>
__global__ __launch_bounds__((DIM == 2) ? TX + 2 : TX * TY, (DIM == 3) ? 3 : 1) void k_stream(Const c, const double* __restrict__ iph,
                                                    const double* __restrict__ ics,
                                                    const double* __restrict__ icl,
                                                    double* __restrict__ oph, double* __restrict__ ocs,
                                                    double* __restrict__ ocl, int zchunk, double t_n,
                                                    double s_n, int do_shift, int* __restrict__ err) {
  using G = StreamGeom<DIM, TX, TY>;
  // ring of three planes (z-1, z, z+1) of (phi, c_s, c_l) with in-plane halo 2
  __shared__ double su[3][3][G::P2];
  __shared__ double spt[2][G::P1];
  __shared__ double smu[3][G::P1];
  __shared__ double sfx[2][G::NFX];
  __shared__ double sfy[2][(G::NFY > 0) ? G::NFY : 1];
  // c_s at ring slot sl, position i.  The equal-potential model reads no c_s:
  // its c_s is k_e c_l exactly, the value its update stores.
  auto CS = [&](int sl, int i) -> double {
    if constexpr (EQ) return c.ke * su[sl][2][i];
    else return su[sl][1][i];
  };

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX;
  const int y0 = blockIdx.y * TY;
  const int zb = blockIdx.z * zchunk;
  const int ze = min(zb + zchunk, c.nz);
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const long long plane = (long long)nx * ny;
  // own column (2D: threads 1..TX; threads 0 and TX+1 take the halo columns)
  const int ox = (DIM == 2) ? tid - 1 : tid % TX, oy = (DIM == 2) ? 0 : tid / TX;
  const bool own = (DIM == 3) || (tid >= 1 && tid <= TX);
  const int gxo = x0 + ox, gyo = y0 + oy;
  const bool own_valid = own && (gxo < nx) && (gyo < ny);
  auto slot3 = [](int gz) { return (gz + 9) % 3; };

  // Cell-stage positions of this thread on the tile plus in-plane halo 1:
  // item 0 is the own column (so a 16-lane group reads one LDS row, free of
  // bank conflicts), item 1 one of the NP1 - NT halo cells (the rows below and
  // above the tile, then the columns left and right), taken by the first
  // threads.
  constexpr int NCS = 2;
  constexpr int NHALO = G::P1 - G::NT;
  static_assert(DIM == 2 ? NHALO == 0 : (NHALO > 0 && NHALO <= G::NT),
                "tile shape: halo cells must fit one item per thread");
  auto cs_pos = [&](int r, int& lx, int& ly) {
    if (r == 0) {
      lx = ox;
      ly = oy;
      return true;
    }
    if constexpr (DIM == 2) {
      lx = ox;
      ly = 0;
      return false;
    }
    constexpr int NROW = (DIM == 3) ? 2 * G::BX1 : 0;
    const int h = min(tid, NHALO - 1);
    if (h < NROW) {
      ly = (h < G::BX1) ? -1 : TY;
      lx = h % G::BX1 - 1;
    } else {
      const int k = h - NROW;
      lx = (k & 1) ? TX : -1;
      ly = k >> 1;
    }
    return tid < NHALO;
  };

  // In-plane global offsets of this thread's cell-stage positions (the same
  // for every plane), computed once.
  int cs_off[NCS];  // x + nx y (a plane holds fewer than 2^31 cells)
#pragma unroll
  for (int r = 0; r < NCS; ++r) {
    int lx, ly;
    cs_pos(r, lx, ly);
    const int gx = map_axis(x0 + lx, nx, c.px);
    const int gy = (DIM == 3) ? map_axis(y0 + ly, ny, c.py) : 0;
    cs_off[r] = gx + nx * gy;
  }
  // Global addressing: a plane's base pointer is uniform across the
  // workgroup; the in-plane byte offset fits 32 bits (planes hold fewer than
  // 2^28 cells), so the loads take a scalar base and a 32-bit vector offset.
  auto at = [](const double* base, unsigned cell) -> double {
    return *(const double*)((const char*)base + cell * 8u);
  };
  // Ring loads go from global memory straight into LDS (global_load_lds, 16
  // bytes a lane, no registers on the way): thread k moves ring positions 2k
  // and 2k+1 of each field when they are adjacent and 16-byte aligned in
  // global memory; the other pairs (mirror images at a non-periodic x edge,
  // periodic wraps inside a pair, odd plane sizes, unaligned bases) go through
  // registers.  The hardware writes lane l of a wave at the wave's LDS base +
  // 16 l, so the base passed is the ring position of the wave's first pair.
  // Issued after the face stage, the loads land while the update runs; each
  // wave waits for its own with dma_wait before the barrier that publishes the
  // plane.
  constexpr int NCH = G::P2 / 2;
  static_assert(G::P2 % 2 == 0 && NCH <= G::NT, "tile shape: ring pairs must fit one per thread");
  int pr_off[2];  // in-plane cell indices of ring positions 2k, 2k+1
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = 2 * min(tid, NCH - 1) + q;
    const int lx = i % G::BX2 - 2;
    const int ly = i / G::BX2 - G::OY2;
    const int gx = map_axis(x0 + lx, nx, c.px);
    const int gy = (DIM == 3) ? map_axis(y0 + ly, ny, c.py) : 0;
    pr_off[q] = gx + nx * gy;
  }
  const bool al16 =
      (((unsigned long long)iph | (unsigned long long)icl | (EQ ? 0ull : (unsigned long long)ics)) & 15ull) == 0;
  const int podd = (int)(plane & 1);
  const int wch = __builtin_amdgcn_readfirstlane(tid & ~63);  // first pair of this wave
  auto load_plane = [&](int gz) {
    if (tid >= NCH) return;
    const int slot = slot3(gz);
    const int gm = mirror_idx(gz, nz);
    const long long zo = plane * gm;
    const bool nice = al16 && pr_off[1] == pr_off[0] + 1 && (((podd & gm) + pr_off[0]) & 1) == 0;
    auto one = [&](const double* in, double* ring) {
      const double* b = in + zo;
      if (nice) {
        __builtin_amdgcn_global_load_lds((const void*)((const char*)b + (unsigned)pr_off[0] * 8u),
                                         (__attribute__((address_space(3))) void*)(ring + 2 * wch), 16, 0, 0);
      } else {
        ring[2 * tid] = at(b, (unsigned)pr_off[0]);
        ring[2 * tid + 1] = at(b, (unsigned)pr_off[1]);
      }
    };
    one(iph, su[slot][0]);
    if constexpr (!EQ) one(ics, su[slot][1]);
    one(icl, su[slot][2]);
  };
  // vmcnt(0): every global_load_lds of this wave has written LDS
  auto dma_wait = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };

  // phi_t and mu_bar of plane gz on the tile plus in-plane halo 1.  Planes gz
  // and gz-1 are in the ring; the plane above comes from the ring when
  // up_in_ring, else from global memory (it is loaded into the ring later).
  // Likewise the plane below comes from global memory when dn_global.
  // (k_e - 1) c_l^eq of plane gz is affine in gz (frozen temperature, Eq. ds1):
  // kq0 + kq1 gz, two scalars instead of the constants of the profile.
  const double kq0 = (c.ke - 1.0) * cleq_at(c, (s_n + 0.5) * c.dx, t_n, c.V, c.z0);
  const double kq1 = (1.0 - c.ke) * (1.0 - c.ke) * c.dx * c.inv_lT * c.inv_ke;
  auto cell_plane = [&](int gz, bool up_in_ring, bool dn_global) {
    const int s0 = slot3(gz), sm = slot3(gz - 1), sp = slot3(gz + 1);
    const int pt = (gz + 8) & 1, mu = (gz + 9) % 3;
    const double kcl = __builtin_fma(kq1, (double)gz, kq0);
    const long long zup = plane * mirror_idx(gz + 1, nz);
    const long long zdn = plane * mirror_idx(gz - 1, nz);
#pragma unroll
    for (int r = 0; r < NCS; ++r) {
      int lx, ly;
      if (!cs_pos(r, lx, ly)) continue;
      const int i = G::i1(lx, ly);
      const int ic = G::i2(lx, ly);
      double upP, upS, upL, dnP, dnS, dnL;
      if (up_in_ring) {
        upP = su[sp][0][ic];
        upS = CS(sp, ic);
        upL = su[sp][2][ic];
      } else {
        const unsigned o = (unsigned)cs_off[r];
        upP = at(iph + zup, o);
        upL = at(icl + zup, o);
        upS = EQ ? c.ke * upL : at(ics + zup, o);
      }
      if (dn_global) {
        const unsigned o = (unsigned)cs_off[r];
        dnP = at(iph + zdn, o);
        dnL = at(icl + zdn, o);
        dnS = EQ ? c.ke * dnL : at(ics + zdn, o);
      } else {
        dnP = su[sm][0][ic];
        dnS = CS(sm, ic);
        dnL = su[sm][2][ic];
      }
      double gph[DIM], gcs[DIM], gcl[DIM];
      const double* U0 = su[s0][0];
      const double* L0 = su[s0][2];
      const double ph = U0[ic], cs = CS(s0, ic), cl = L0[ic];
      gph[0] = U0[ic + 1] - U0[ic - 1];  // plain differences (cell_stage_raw)
      gcs[0] = CS(s0, ic + 1) - CS(s0, ic - 1);
      gcl[0] = L0[ic + 1] - L0[ic - 1];
      double lap = (U0[ic + 1] - 2.0 * ph + U0[ic - 1]);
      if (DIM == 3) {
        gph[1] = U0[ic + G::BX2] - U0[ic - G::BX2];
        gcs[1] = CS(s0, ic + G::BX2) - CS(s0, ic - G::BX2);
        gcl[1] = L0[ic + G::BX2] - L0[ic - G::BX2];
        lap += (U0[ic + G::BX2] - 2.0 * ph + U0[ic - G::BX2]);
      }
      gph[DIM - 1] = upP - dnP;
      gcs[DIM - 1] = upS - dnS;
      gcl[DIM - 1] = upL - dnL;
      lap += (upP - 2.0 * ph + dnP);
      double phit, mubar;
      cell_stage_raw<DIM, APZ, EQ>(c, kcl, ph, cs, cl, gph, gcs, gcl, lap, phit, mubar);
      spt[pt][i] = phit;
      smu[mu][i] = mubar;
    }
  };

  // Flux through the z-face between planes gz and gz+1 of the own column.
  auto zface = [&](int gz, double& Fs, double& Fl) {
    if (gz < 0 || gz + 1 >= nz) {
      Fs = 0.0;
      Fl = 0.0;
      return;
    }
    const int sa = slot3(gz), sb = slot3(gz + 1);
    const int pa = (gz + 8) & 1, pb = (gz + 9) & 1;
    const int ma = (gz + 9) % 3, mb = (gz + 10) % 3;
    const int ic = G::i2(ox, oy), i1 = G::i1(ox, oy);
    double gph[DIM], gmu[DIM], gcs[DIM], gcl[DIM];
    const double pa_ = su[sa][0][ic], pb_ = su[sb][0][ic];
    const double ca = CS(sa, ic), cb = CS(sb, ic);
    const double la = su[sa][2][ic], lb = su[sb][2][ic];
    const int k = DIM - 1;
    gph[k] = pb_ - pa_;  // dx-scaled face stage: plain differences and sums of them
    gmu[k] = smu[mb][i1] - smu[ma][i1];
    gcs[k] = cb - ca;
    gcl[k] = lb - la;
    {  // x
      gph[0] = (su[sa][0][ic + 1] - su[sa][0][ic - 1]) + (su[sb][0][ic + 1] - su[sb][0][ic - 1]);
      gmu[0] = (smu[ma][i1 + 1] - smu[ma][i1 - 1]) + (smu[mb][i1 + 1] - smu[mb][i1 - 1]);
      gcs[0] = (CS(sa, ic + 1) - CS(sa, ic - 1)) + (CS(sb, ic + 1) - CS(sb, ic - 1));
      gcl[0] = (su[sa][2][ic + 1] - su[sa][2][ic - 1]) + (su[sb][2][ic + 1] - su[sb][2][ic - 1]);
    }
    if (DIM == 3) {
      const int d2 = G::BX2, d1 = G::BX1;
      gph[1] = (su[sa][0][ic + d2] - su[sa][0][ic - d2]) + (su[sb][0][ic + d2] - su[sb][0][ic - d2]);
      gmu[1] = (smu[ma][i1 + d1] - smu[ma][i1 - d1]) + (smu[mb][i1 + d1] - smu[mb][i1 - d1]);
      gcs[1] = (CS(sa, ic + d2) - CS(sa, ic - d2)) + (CS(sb, ic + d2) - CS(sb, ic - d2));
      gcl[1] = (su[sa][2][ic + d2] - su[sa][2][ic - d2]) + (su[sb][2][ic + d2] - su[sb][2][ic - d2]);
    }
    const double ptf = 0.5 * (spt[pa][i1] + spt[pb][i1]);
    face_flux<DIM, DIM - 1, APZ, EQ>(c, 0.5 * (pa_ + pb_), 0.5 * (ca + cb), 0.5 * (la + lb), ptf, gph, gmu, gcs,
                                     gcl, Fs, Fl);
  };

  // The face normal to in-plane axis K (0 = x, 1 = y) of plane gz on the low
  // side of cell (fa, fb) of the tile, into LDS.
  auto face_item = [&](auto axis, int gz, int fa, int fb) {
    constexpr int K = decltype(axis)::value;
    constexpr int RW = (K == 0) ? TX + 1 : TX;  // faces per row
    const int s0 = slot3(gz), sm = slot3(gz - 1), sp = slot3(gz + 1);
    const int pt = (gz + 8) & 1;
    const int m0 = (gz + 9) % 3, mm = (gz + 8) % 3, mp = (gz + 10) % 3;
    double* F0 = (K == 0) ? sfx[0] : sfy[0];
    double* F1 = (K == 0) ? sfx[1] : sfy[1];
    const int f = fb * RW + fa;
    // cell a = (ax, ay), cell b = a + e_K
    const int ax = (K == 0) ? fa - 1 : fa, ay = (K == 0) ? fb : fb - 1;
    const int bx = fa, by = fb;
    const int gface = (K == 0) ? x0 + fa : y0 + fb;
    const int nk = (K == 0) ? nx : ny;
    const int pk = (K == 0) ? c.px : c.py;
    if ((!pk && (gface == 0 || gface >= nk)) || gface > nk) {
      F0[f] = 0.0;
      if constexpr (!EQ) F1[f] = 0.0;
      return;
    }
    const int ia = G::i2(ax, ay), ib = G::i2(bx, by);
    const int ja = G::i1(ax, ay), jb = G::i1(bx, by);
    double gph[DIM], gmu[DIM], gcs[DIM], gcl[DIM];
    const double pa = su[s0][0][ia], pb = su[s0][0][ib];
    const double ca = CS(s0, ia), cb = CS(s0, ib);
    const double la_ = su[s0][2][ia], lb_ = su[s0][2][ib];
    gph[K] = pb - pa;  // dx-scaled face stage: plain differences and sums of them
    gmu[K] = smu[m0][jb] - smu[m0][ja];
    gcs[K] = cb - ca;
    gcl[K] = lb_ - la_;
    if (DIM == 3) {  // the other in-plane axis
      constexpr int J = 1 - K;
      constexpr int d2 = (J == 0) ? 1 : G::BX2;
      constexpr int d1 = (J == 0) ? 1 : G::BX1;
      gph[J] = (su[s0][0][ia + d2] - su[s0][0][ia - d2]) + (su[s0][0][ib + d2] - su[s0][0][ib - d2]);
      gmu[J] = (smu[m0][ja + d1] - smu[m0][ja - d1]) + (smu[m0][jb + d1] - smu[m0][jb - d1]);
      gcs[J] = (CS(s0, ia + d2) - CS(s0, ia - d2)) + (CS(s0, ib + d2) - CS(s0, ib - d2));
      gcl[J] = (su[s0][2][ia + d2] - su[s0][2][ia - d2]) + (su[s0][2][ib + d2] - su[s0][2][ib - d2]);
    }
    constexpr int kz = DIM - 1;  // transverse z
    gph[kz] = (su[sp][0][ia] - su[sm][0][ia]) + (su[sp][0][ib] - su[sm][0][ib]);
    gmu[kz] = (smu[mp][ja] - smu[mm][ja]) + (smu[mp][jb] - smu[mm][jb]);
    gcs[kz] = (CS(sp, ia) - CS(sm, ia)) + (CS(sp, ib) - CS(sm, ib));
    gcl[kz] = (su[sp][2][ia] - su[sm][2][ia]) + (su[sp][2][ib] - su[sm][2][ib]);
    const double ptf = 0.5 * (spt[pt][ja] + spt[pt][jb]);
    double Fs, Fl;
    face_flux<DIM, K, APZ, EQ>(c, 0.5 * (pa + pb), 0.5 * (ca + cb), 0.5 * (la_ + lb_), ptf, gph, gmu, gcs, gcl, Fs,
                               Fl);
    F0[f] = Fs;
    if constexpr (!EQ) F1[f] = Fl;
  };
  // 3D only: the face normal to in-plane axis K (runtime: 0 = x, 1 = y) on the
  // low side of cell (fa, fb), with the gradient components ordered (normal,
  // other in-plane, z) so that one code path serves both axes.
  auto face_item_rt = [&](int K, int gz, int fa, int fb) {
    const int RW = (K == 0) ? TX + 1 : TX;
    const int s0 = slot3(gz), sm = slot3(gz - 1), sp = slot3(gz + 1);
    const int pt = (gz + 8) & 1;
    const int m0 = (gz + 9) % 3, mm = (gz + 8) % 3, mp = (gz + 10) % 3;
    double* F0 = (K == 0) ? sfx[0] : sfy[0];
    double* F1 = (K == 0) ? sfx[1] : sfy[1];
    const int f = fb * RW + fa;
    const int ax = (K == 0) ? fa - 1 : fa, ay = (K == 0) ? fb : fb - 1;
    const int gface = (K == 0) ? x0 + fa : y0 + fb;
    const int nk = (K == 0) ? nx : ny;
    const int pk = (K == 0) ? c.px : c.py;
    if ((!pk && (gface == 0 || gface >= nk)) || gface > nk) {
      F0[f] = 0.0;
      if constexpr (!EQ) F1[f] = 0.0;
      return;
    }
    const int ia = G::i2(ax, ay), ib = G::i2(fa, fb);
    const int ja = G::i1(ax, ay), jb = G::i1(fa, fb);
    const int d2 = (K == 0) ? G::BX2 : 1, d1 = (K == 0) ? G::BX1 : 1;  // the other in-plane axis
    double gph[3], gmu[3], gcs[3], gcl[3];
    const double pa = su[s0][0][ia], pb = su[s0][0][ib];
    const double ca = CS(s0, ia), cb = CS(s0, ib);
    const double la_ = su[s0][2][ia], lb_ = su[s0][2][ib];
    gph[0] = pb - pa;
    gmu[0] = smu[m0][jb] - smu[m0][ja];
    gcs[0] = cb - ca;
    gcl[0] = lb_ - la_;
    gph[1] = (su[s0][0][ia + d2] - su[s0][0][ia - d2]) + (su[s0][0][ib + d2] - su[s0][0][ib - d2]);
    gmu[1] = (smu[m0][ja + d1] - smu[m0][ja - d1]) + (smu[m0][jb + d1] - smu[m0][jb - d1]);
    gcs[1] = (CS(s0, ia + d2) - CS(s0, ia - d2)) + (CS(s0, ib + d2) - CS(s0, ib - d2));
    gcl[1] = (su[s0][2][ia + d2] - su[s0][2][ia - d2]) + (su[s0][2][ib + d2] - su[s0][2][ib - d2]);
    gph[2] = (su[sp][0][ia] - su[sm][0][ia]) + (su[sp][0][ib] - su[sm][0][ib]);
    gmu[2] = (smu[mp][ja] - smu[mm][ja]) + (smu[mp][jb] - smu[mm][jb]);
    gcs[2] = (CS(sp, ia) - CS(sm, ia)) + (CS(sp, ib) - CS(sm, ib));
    gcl[2] = (su[sp][2][ia] - su[sm][2][ia]) + (su[sp][2][ib] - su[sm][2][ib]);
    const double ptf = 0.5 * (spt[pt][ja] + spt[pt][jb]);
    double Fs, Fl;
    face_flux<3, 0, APZ, EQ>(c, 0.5 * (pa + pb), 0.5 * (ca + cb), 0.5 * (la_ + lb_), ptf, gph, gmu, gcs, gcl, Fs, Fl);
    F0[f] = Fs;
    if constexpr (!EQ) F1[f] = Fl;
  };
  // 3D: the x and y faces on the low side of the own cell and the z face above
  // it, from one gather of what they share: the own cell's values (phi, c_s,
  // c_l, mu_bar) and its central differences along each axis are read from LDS
  // once and enter two faces each.  Same arithmetic, in the same order, as
  // face_item and zface.
  struct F4 {
    double p, s, l, m;
  };
  auto own_faces3 = [&](int gz, double& FsU, double& FlU, F4& own, double& ptown) {
    const int s0 = slot3(gz), sm = slot3(gz - 1), sp = slot3(gz + 1);
    const int m0 = (gz + 9) % 3, mm = (gz + 8) % 3, mp = (gz + 10) % 3;
    const int ic = G::i2(ox, oy), jc = G::i1(ox, oy);
    constexpr int DY2 = G::BX2, DY1 = G::BX1;
    auto cen = [&](int sl, int ml, int i, int j) { return F4{su[sl][0][i], CS(sl, i), su[sl][2][i], smu[ml][j]}; };
    // central difference along an in-plane axis (ring offsets d2, d1)
    auto dif = [&](int sl, int ml, int i, int j, int d2, int d1) {
      return F4{su[sl][0][i + d2] - su[sl][0][i - d2], CS(sl, i + d2) - CS(sl, i - d2),
                su[sl][2][i + d2] - su[sl][2][i - d2], smu[ml][j + d1] - smu[ml][j - d1]};
    };
    // central difference along z about plane gz
    auto difz = [&](int i, int j) {
      return F4{su[sp][0][i] - su[sm][0][i], CS(sp, i) - CS(sm, i), su[sp][2][i] - su[sm][2][i],
                smu[mp][j] - smu[mm][j]};
    };
    auto add = [](const F4& u, const F4& v) { return F4{u.p + v.p, u.s + v.s, u.l + v.l, u.m + v.m}; };
    // face normal to K between cells a and b = a + e_K; t1, t2 the transverse
    // sums along the other two axes in axis order
    auto face = [&](auto axis, const F4& a, const F4& b, const F4& t1, const F4& t2, double pta, double ptb,
                    double& Fs, double& Fl) {
      constexpr int K = decltype(axis)::value;
      constexpr int J1 = (K == 0) ? 1 : 0, J2 = (K == 2) ? 1 : 2;
      double gph[3], gmu[3], gcs[3], gcl[3];
      gph[K] = b.p - a.p;
      gmu[K] = b.m - a.m;
      gcs[K] = b.s - a.s;
      gcl[K] = b.l - a.l;
      gph[J1] = t1.p;
      gmu[J1] = t1.m;
      gcs[J1] = t1.s;
      gcl[J1] = t1.l;
      gph[J2] = t2.p;
      gmu[J2] = t2.m;
      gcs[J2] = t2.s;
      gcl[J2] = t2.l;
      face_flux<3, K, APZ, EQ>(c, 0.5 * (a.p + b.p), 0.5 * (a.s + b.s), 0.5 * (a.l + b.l), 0.5 * (pta + ptb), gph,
                               gmu, gcs, gcl, Fs, Fl);
    };
    auto closed = [&](int g, int n, int per) { return (!per && (g == 0 || g >= n)) || g > n; };
    const F4 cc = cen(s0, m0, ic, jc);
    const F4 dzc = difz(ic, jc);
    const double ptc = spt[(gz + 8) & 1][jc];
    const F4 dyc = dif(s0, m0, ic, jc, DY2, DY1);
    {  // x face (a = own cell - e_x)
      double Fs = 0.0, Fl = 0.0;
      if (!closed(x0 + ox, nx, c.px)) {
        const int ia = ic - 1, ja = jc - 1;
        face(std::integral_constant<int, 0>{}, cen(s0, m0, ia, ja), cc, add(dif(s0, m0, ia, ja, DY2, DY1), dyc),
             add(difz(ia, ja), dzc), spt[(gz + 8) & 1][ja], ptc, Fs, Fl);
      }
      const int f = oy * (TX + 1) + ox;
      sfx[0][f] = Fs;
      if constexpr (!EQ) sfx[1][f] = Fl;
    }
    const F4 dxc = dif(s0, m0, ic, jc, 1, 1);
    {  // y face (a = own cell - e_y)
      double Fs = 0.0, Fl = 0.0;
      if (!closed(y0 + oy, ny, c.py)) {
        const int ia = ic - DY2, ja = jc - DY1;
        face(std::integral_constant<int, 1>{}, cen(s0, m0, ia, ja), cc, add(dif(s0, m0, ia, ja, 1, 1), dxc),
             add(difz(ia, ja), dzc), spt[(gz + 8) & 1][ja], ptc, Fs, Fl);
      }
      const int f = oy * TX + ox;
      sfy[0][f] = Fs;
      if constexpr (!EQ) sfy[1][f] = Fl;
    }
    own = cc;  // for the update
    ptown = ptc;
    FsU = 0.0;
    FlU = 0.0;
    if (gz >= 0 && gz + 1 < nz) {  // z face (b = own cell in plane gz + 1)
      const F4 cu = cen(sp, mp, ic, jc);
      face(std::integral_constant<int, 2>{}, cc, cu, add(dxc, dif(sp, mp, ic, jc, 1, 1)),
           add(dyc, dif(sp, mp, ic, jc, DY2, DY1)), ptc, spt[(gz + 9) & 1][jc], FsU, FlU);
    }
  };
  // Face items: every thread takes the x and y faces on the low side of its own
  // cell; the faces on the high side of the tile (TY of them in x, TX in y) go
  // to wave 2 (x) and wave 3 (y), as the extra cells of the cell stage go to
  // waves 0 and 1, so the four waves carry equal work per plane.
  constexpr int NW = G::NT / 64;
  constexpr int EX = (DIM == 2) ? 0 : G::NFX - G::NT, EY = G::NFY - G::NT;
  static_assert(EX >= 0 && EX <= 64 && (DIM == 2 || (EY >= 0 && EY <= 64)),
                "tile shape: leftover faces must fit one wave");
  // 3D: the TY + TX leftover faces go to one wave in a single pass (runtime axis).
  static_assert(DIM == 2 || EX + EY <= 64, "tile shape: leftover faces must fit one wave");
  constexpr int WE = NW - 1;
  const int le = tid - 64 * WE;
  const bool extra_f = (DIM == 3) && le >= 0 && le < EX + EY;

  // ---- prologue: ring = planes zb-1, zb, zb+1; rates of planes zb-1 and zb
  for (int g = zb - 1; g <= zb + 1; ++g) load_plane(g);
  dma_wait();
  __syncthreads();
  cell_plane(zb - 1, true, true);
  cell_plane(zb, true, false);
  __syncthreads();
  double FsD = 0.0, FlD = 0.0;  // flux through the face below the current plane
  if (own) zface(zb - 1, FsD, FlD);

  int errbits = 0;
  for (int z = zb; z < ze; ++z) {
    cell_plane(z + 1, false, false);  // plane z+2 read from global memory
    __syncthreads();
    double FsU = 0.0, FlU = 0.0;
    F4 ownv{};  // 3D: the own cell's (phi, c_s, c_l) and phi_t, kept for the update
    double ptv = 0.0;
    if constexpr (DIM == 3) {
      if (extra_f) {  // one call: lanes 0..EX-1 take x faces, the rest y faces
        const int K = (le < EX) ? 0 : 1;
        face_item_rt(K, z, (K == 0) ? TX : le - EX, (K == 0) ? le : TY);
      }
      own_faces3(z, FsU, FlU, ownv, ptv);
    } else {
      if (tid <= TX) face_item(std::integral_constant<int, 0>{}, z, tid, 0);  // the TX + 1 x faces in one pass
      if (own) zface(z, FsU, FlU);
    }
    __syncthreads();
    load_plane(z + 2);  // into the slot of plane z-1 (no longer read); lands during the update
    if (own_valid) {
      const int s0 = slot3(z);
      const int ic = G::i2(ox, oy), i1 = G::i1(ox, oy);
      const double ph = (DIM == 3) ? ownv.p : su[s0][0][ic];
      const double cs = (DIM == 3) ? ownv.s : CS(s0, ic);
      const double cl = (DIM == 3) ? ownv.l : su[s0][2][ic];
      const double pt = (DIM == 3) ? ptv : spt[(z + 8) & 1][i1];
      double divs = sfx[0][oy * (TX + 1) + ox + 1] - sfx[0][oy * (TX + 1) + ox];
      if (DIM == 3) divs += sfy[0][(oy + 1) * TX + ox] - sfy[0][oy * TX + ox];
      divs += FsU - FsD;
      const double nph = ph + c.dt * pt;
      double ncs, ncl;
      if constexpr (EQ) {  // conserved mixture, then the equal-potential split at the new phi
        double p, q;
        interp_pq<APZ>(c, ph, p, q);
        eq_split<APZ>(c, nph, p * cs + q * cl + c.dt * divs * c.inv_dx2, ncs, ncl);
      } else {
        double divl = sfx[1][oy * (TX + 1) + ox + 1] - sfx[1][oy * (TX + 1) + ox];
        if (DIM == 3) divl += sfy[1][(oy + 1) * TX + ox] - sfy[1][oy * TX + ox];
        divl += FlU - FlD;
        double p, q, dp;
        interp<APZ>(c, ph, p, q, dp);
        const double src = -c.A * (cs - cl) * dp * pt;
        ncs = cs + c.dt * (divs * c.inv_dx2 + src);
        ncl = cl + c.dt * (divl * c.inv_dx2 + src);
      }
      errbits |= check_bits(nph, ncs, ncl);
      const unsigned col = (unsigned)(gxo + nx * gyo) * 8u;  // byte offset in the plane
      auto put = [col](double* base, double v) { *(double*)((char*)base + col) = v; };
      if (!do_shift) {
        put(oph + plane * z, nph);
        put(ocs + plane * z, ncs);
        put(ocl + plane * z, ncl);
      } else {
        if (z >= 1) {
          put(oph + plane * (z - 1), nph);
          put(ocs + plane * (z - 1), ncs);
          put(ocl + plane * (z - 1), ncl);
        }
        if (z == nz - 1) {
          put(oph + plane * z, 0.0);
          put(ocs + plane * z, c.ke);
          put(ocl + plane * z, 1.0);
        }
      }
    }
    FsD = FsU;
    FlD = FlU;
    dma_wait();
    __syncthreads();
  }
  if (errbits) atomicOr(err, errbits);
}

// ---------------------------------------------------------------------------
// Persistent 1D kernel: one workgroup per run (single domain = one run),
// runs taken longest first.  The whole run stays in registers for all steps:
// thread t owns C = ceil(N / 1024) <= 8 consecutive cells; neighbour values are
// exchanged through LDS (cells, then phi_t and mu_bar of the chunk edges), so
// nothing is recomputed.  The window shift moves each chunk down by one cell
// with one more exchange.  Optionally stores every state to a trajectory.
// ---------------------------------------------------------------------------
constexpr int R1_THREADS = 1024;
constexpr int R1_CMAX = 8;

struct RunTab {
  const int* n;
  const long long* off;
  const double* V;
  const double* dt;
  const double* z0;
  const int* order;  // launch order (longest first)
};

// One run (the block's) for nsteps steps; CM >= ceil(N / R1_THREADS) cells per
// thread are held in registers.  xe/xd are the block's exchange buffers.
template <int CM, bool APZ, bool EQ>
__device__ __forceinline__ void run1d_body(const Const& c, const RunTab& rt, int r, double* __restrict__ gph,
                                           double* __restrict__ gcs, double* __restrict__ gcl, long long n0,
                                           long long nsteps, int do_shift, int* __restrict__ err,
                                           double* __restrict__ tph, double* __restrict__ tcs,
                                           double* __restrict__ tcl, long long tstride,
                                           double (*xe)[3][R1_THREADS], double (*xd)[2][R1_THREADS]) {
  const int N = rt.n[r];
  const long long off = rt.off[r];
  const double V = rt.V[r], dt = rt.dt[r], z0 = rt.z0[r];
  const int C = (N + R1_THREADS - 1) / R1_THREADS;
  const int t = threadIdx.x;
  const int i0 = t * C;
  const int cnt = max(0, min(C, N - i0));
  const bool at_lo = (i0 == 0);
  const bool at_hi = (cnt > 0) && (i0 + cnt == N);
  const bool has_right = (cnt > 0) && !at_hi;  // thread t+1 owns cell i0 + cnt

  double P[CM], S[CM], L[CM];
  // value of register array a at runtime position idx (static selects, no scratch)
  auto pick = [](const double (&a)[CM], int idx) {
    double v = a[0];
#pragma unroll
    for (int k = 1; k < CM; ++k) v = (k == idx) ? a[k] : v;
    return v;
  };
#pragma unroll
  for (int k = 0; k < CM; ++k) {
    if (k < cnt) {
      P[k] = gph[off + i0 + k];
      L[k] = gcl[off + i0 + k];
      S[k] = EQ ? c.ke * L[k] : gcs[off + i0 + k];  // equal potentials: c_s = k_e c_l
    } else {
      P[k] = 0.0;
      S[k] = 1.0;
      L[k] = 1.0;
    }
  }
  int errbits = 0;
  for (long long st = 0; st <= nsteps; ++st) {
    const long long n = n0 + st;
    if (tph) {
#pragma unroll
      for (int k = 0; k < CM; ++k)
        if (k < cnt) {
          const long long o = st * tstride + off + i0 + k;
          tph[o] = P[k];
          tcs[o] = S[k];
          tcl[o] = L[k];
        }
    }
    if (st == nsteps) break;
    const double tn = (double)n * dt;
    const double sn = floor(V * tn / c.dx);
    const bool shift = do_shift && (floor(V * ((double)(n + 1) * dt) / c.dx) > sn);
    // exchange 1: chunk edge cells
    if (cnt > 0) {
      xe[0][0][t] = P[0];
      xe[0][1][t] = S[0];
      xe[0][2][t] = L[0];
      xe[1][0][t] = pick(P, cnt - 1);
      xe[1][1][t] = pick(S, cnt - 1);
      xe[1][2][t] = pick(L, cnt - 1);
    }
    __syncthreads();
    double lP, lS, lL, rP, rS, rL;  // left of first cell, right of last cell (mirror at the ends)
    if (at_lo) {
      lP = P[0];
      lS = S[0];
      lL = L[0];
    } else {
      lP = xe[1][0][t - 1];
      lS = xe[1][1][t - 1];
      lL = xe[1][2][t - 1];
    }
    if (has_right) {
      rP = xe[0][0][t + 1];
      rS = xe[0][1][t + 1];
      rL = xe[0][2][t + 1];
    } else {
      rP = pick(P, cnt - 1);
      rS = pick(S, cnt - 1);
      rL = pick(L, cnt - 1);
    }
    // Cell stage of local cell k (a constant once the loops are unrolled) from
    // the old values of the cell and its neighbours; the chunk ends take their
    // outer neighbours from exchange 1.
    auto cell = [&](int k, double& pt, double& mu) {
      const double pm = (k == 0) ? lP : P[(k > 0) ? k - 1 : 0], pp = (k == cnt - 1) ? rP : P[(k + 1 < CM) ? k + 1 : k];
      const double sm = (k == 0) ? lS : S[(k > 0) ? k - 1 : 0], sp = (k == cnt - 1) ? rS : S[(k + 1 < CM) ? k + 1 : k];
      const double lm = (k == 0) ? lL : L[(k > 0) ? k - 1 : 0], lp = (k == cnt - 1) ? rL : L[(k + 1 < CM) ? k + 1 : k];
      double gph1[1] = {pp - pm};  // plain differences (cell_stage_raw)
      double gcs1[1] = {sp - sm};
      double gcl1[1] = {lp - lm};
      const double lap = pp - 2.0 * P[k] + pm;
      const double zlab = ((double)(i0 + k) + sn + 0.5) * c.dx;
      const double kcl = (c.ke - 1.0) * cleq_at(c, zlab, tn, V, z0);
      cell_stage_raw<1, APZ, EQ>(c, kcl, P[k], S[k], L[k], gph1, gcs1, gcl1, lap, pt, mu);
    };
    // phi_t and mu_bar of the chunk's first and last cells first: they go to the
    // neighbours; the others are computed as the face loop reaches them, so only
    // a few of them are live at a time
    double PT0 = 0.0, MU0 = 0.0, PTl = 0.0, MUl = 0.0;
    if (cnt > 0) cell(0, PT0, MU0);
#pragma unroll
    for (int k = 1; k < CM; ++k)
      if (k == cnt - 1) cell(k, PTl, MUl);
    if (cnt == 1) {
      PTl = PT0;
      MUl = MU0;
    }
    // exchange 2: phi_t and mu_bar of the chunk edges
    if (cnt > 0) {
      xd[0][0][t] = PT0;
      xd[0][1][t] = MU0;
      xd[1][0][t] = PTl;
      xd[1][1][t] = MUl;
    }
    __syncthreads();
    const double lPT = at_lo ? 0.0 : xd[1][0][t - 1];
    const double lMU = at_lo ? 0.0 : xd[1][1][t - 1];
    const double rPT = has_right ? xd[0][0][t + 1] : 0.0;
    const double rMU = has_right ? xd[0][1][t + 1] : 0.0;
    // Faces j = 0..cnt lie between local cells j-1 and j (mirror ends have zero
    // flux).  Rolling over the cells: face k+1 is computed before cell k is
    // updated, so no face array is kept.
    auto face = [&](bool none, double pa, double sa, double la, double ta, double ma, double pb, double sb,
                    double lb, double tb, double mb, double& Fs, double& Fl) {
      Fs = 0.0;
      Fl = 0.0;
      if (none) return;
      double g0[1] = {pb - pa};  // dx-scaled face stage: plain differences
      double g1[1] = {mb - ma};
      double g2[1] = {sb - sa};
      double g3[1] = {lb - la};
      face_flux<1, 0, APZ, EQ>(c, 0.5 * (pa + pb), 0.5 * (sa + sb), 0.5 * (la + lb), 0.5 * (ta + tb), g0, g1, g2, g3,
                               Fs, Fl);
    };
    double FsL, FlL;
    face(cnt <= 0 || at_lo, lP, lS, lL, lPT, lMU, P[0], S[0], L[0], PT0, MU0, FsL, FlL);
    double ptc = PT0, muc = MU0;  // phi_t and mu_bar of the current cell
#pragma unroll
    for (int k = 0; k < CM; ++k) {
      if (k < cnt) {
        const int k1 = (k + 1 < CM) ? k + 1 : k;  // in range; used only when k + 1 < cnt
        double ptn, mun, pn, sn1, ln;  // the cell right of face k+1
        if (k + 1 < cnt) {
          if (k + 1 == cnt - 1) {
            ptn = PTl;
            mun = MUl;
          } else {
            cell(k1, ptn, mun);
          }
          pn = P[k1];
          sn1 = S[k1];
          ln = L[k1];
        } else {
          ptn = rPT;
          mun = rMU;
          pn = rP;
          sn1 = rS;
          ln = rL;
        }
        double FsR, FlR;
        face(k == cnt - 1 && at_hi, P[k], S[k], L[k], ptc, muc, pn, sn1, ln, ptn, mun, FsR, FlR);
        double ns, nl;
        const double np_ = P[k] + dt * ptc;
        if constexpr (EQ) {  // conserved mixture, then the equal-potential split at the new phi
          double p, q;
          interp_pq<APZ>(c, P[k], p, q);
          eq_split<APZ>(c, np_, p * S[k] + q * L[k] + dt * (FsR - FsL) * c.inv_dx2, ns, nl);
        } else {
          double p, q, dp;
          interp<APZ>(c, P[k], p, q, dp);
          const double src = -c.A * (S[k] - L[k]) * dp * ptc;
          ns = S[k] + dt * ((FsR - FsL) * c.inv_dx2 + src);
          nl = L[k] + dt * ((FlR - FlL) * c.inv_dx2 + src);
        }
        P[k] = np_;
        S[k] = ns;
        L[k] = nl;
        errbits |= check_bits(P[k], S[k], L[k]);
        FsL = FsR;
        FlL = FlR;
        ptc = ptn;
        muc = mun;
      }
    }
    if (shift) {  // uniform across the workgroup
      // every thread's first cell moves to its left neighbour's last slot
      __syncthreads();  // all reads of xe from exchange 1 are done (barrier 2 passed too)
      if (cnt > 0) {
        xe[0][0][t] = P[0];
        xe[0][1][t] = S[0];
        xe[0][2][t] = L[0];
      }
      __syncthreads();
      double nP, nS, nL;
      if (has_right) {
        nP = xe[0][0][t + 1];
        nS = xe[0][1][t + 1];
        nL = xe[0][2][t + 1];
      } else {
        nP = 0.0;
        nS = c.ke;
        nL = 1.0;
      }
#pragma unroll
      for (int k = 0; k < CM; ++k) {
        if (k < cnt) {
          const bool last = (k == cnt - 1);
          P[k] = last ? nP : P[(k + 1 < CM) ? k + 1 : k];
          S[k] = last ? nS : S[(k + 1 < CM) ? k + 1 : k];
          L[k] = last ? nL : L[(k + 1 < CM) ? k + 1 : k];
        }
      }
    }
    __syncthreads();  // exchange buffers are rewritten by the next step
  }
#pragma unroll
  for (int k = 0; k < CM; ++k)
    if (k < cnt) {
      gph[off + i0 + k] = P[k];
      gcs[off + i0 + k] = S[k];
      gcl[off + i0 + k] = L[k];
    }
  if (errbits) atomicOr(err, errbits);
}

template <bool APZ, bool EQ>
__global__ __launch_bounds__(R1_THREADS) void k_run1d(Const c, RunTab rt, double* __restrict__ gph,
                                                      double* __restrict__ gcs, double* __restrict__ gcl,
                                                      long long n0, long long nsteps, int do_shift,
                                                      int* __restrict__ err, double* __restrict__ tph,
                                                      double* __restrict__ tcs, double* __restrict__ tcl,
                                                      long long tstride) {
  __shared__ double xe[2][3][R1_THREADS];  // [first|last][phi, cs, cl][thread]
  __shared__ double xd[2][2][R1_THREADS];  // [first|last][phi_t, mu_bar][thread]
  const int r = rt.order[blockIdx.x];
  const int C = (rt.n[r] + R1_THREADS - 1) / R1_THREADS;
  // register arrays sized to the run: short runs get short unrolled loops
  if (C <= 1)
    run1d_body<1, APZ, EQ>(c, rt, r, gph, gcs, gcl, n0, nsteps, do_shift, err, tph, tcs, tcl, tstride, xe, xd);
  else if (C <= 2)
    run1d_body<2, APZ, EQ>(c, rt, r, gph, gcs, gcl, n0, nsteps, do_shift, err, tph, tcs, tcl, tstride, xe, xd);
  else if (C <= 4)
    run1d_body<4, APZ, EQ>(c, rt, r, gph, gcs, gcl, n0, nsteps, do_shift, err, tph, tcs, tcl, tstride, xe, xd);
  else
    run1d_body<R1_CMAX, APZ, EQ>(c, rt, r, gph, gcs, gcl, n0, nsteps, do_shift, err, tph, tcs, tcl, tstride, xe, xd);
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Cells of each "run" (a batched 1D run, or the
// single domain as run 0) are cut into chunks of RED_CHUNK cells; one
// workgroup per chunk writes partials, then one workgroup per run reduces its
// chunks in index order.  Fixed trees, so results do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
constexpr int RED_CHUNK = 4096;

struct RedTab {
  const int* chunk_run;        // run of chunk (null: one domain, chunk k starts at cell k RED_CHUNK)
  const long long* chunk_beg;  // first cell (relative to the run) of chunk
  const int* run_chunk0;       // first chunk of run (nrun + 1 entries; null with chunk_run)
  int nchunk;                  // number of chunks of the one domain when the tables are null
};

struct Partial {
  double energy, solute, cmax;
  long long arg;
};

__device__ __forceinline__ void better(double& v, long long& a, double v2, long long a2) {
  if (v2 > v || (v2 == v && a2 < a)) {
    v = v2;
    a = a2;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_chunks(Const c, RunTab rt, RedTab red,
                                                               const double* __restrict__ ph,
                                                               const double* __restrict__ cs,
                                                               const double* __restrict__ cl, long long n,
                                                               int batched, Partial* __restrict__ out) {
  __shared__ double se[RED_THREADS], ss[RED_THREADS], sm[RED_THREADS];
  __shared__ long long sa[RED_THREADS];
  const int ch = blockIdx.x;
  const int r = red.chunk_run ? red.chunk_run[ch] : 0;
  const long long beg = red.chunk_run ? red.chunk_beg[ch] : (long long)ch * RED_CHUNK;
  const long long N = batched ? (long long)rt.n[r] : c.ncell;
  const long long off = batched ? rt.off[r] : 0;
  const double V = batched ? rt.V[r] : c.V;
  const double dt = batched ? rt.dt[r] : c.dt;
  const double z0 = batched ? rt.z0[r] : c.z0;
  const double tn = (double)n * dt;
  const double sn = floor(V * tn / c.dx);
  const long long end = min(beg + (long long)RED_CHUNK, N);
  const int nx = batched ? 1 : c.nx, ny = batched ? 1 : c.ny, nz = batched ? (int)N : c.nz;
  const long long plane = (long long)nx * ny;
  double e = 0.0, s = 0.0, mx = -INFINITY;
  long long am = -1;
  for (long long i = beg + threadIdx.x; i < end; i += RED_THREADS) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / plane);
    const double f = ph[off + i], a = cs[off + i], b = cl[off + i];
    double p, q;
    interp_pq(c, f, p, q);
    const double zlab = ((double)z + sn + 0.5) * c.dx;
    const double cleq = cleq_at(c, zlab, tn, V, z0);
    const double fs = a * flog(a) - a - a * c.log_ke + (c.ke - 1.0) * cleq;
    const double fl = b * flog(b) - b;
    const double w = f * (1.0 - f);
    double en = w * w + c.lambda * (p * fs + q * fl);
    // gradient energy on the faces above the cell (each face once)
    double gsum = 0.0;
    if (batched || c.dim == 1) {
      if (z + 1 < nz) {
        const double d = (ph[off + i + plane] - f) * c.inv_dx;
        gsum += d * d;
      }
    } else {
      if (c.px || x + 1 < nx) {
        const long long j = (long long)((x + 1) % nx) + (long long)nx * y + plane * z;
        const double d = (ph[j] - f) * c.inv_dx;
        gsum += d * d;
      }
      if (c.dim == 3 && (c.py || y + 1 < ny)) {
        const long long j = (long long)x + (long long)nx * ((y + 1) % ny) + plane * z;
        const double d = (ph[j] - f) * c.inv_dx;
        gsum += d * d;
      }
      if (z + 1 < nz) {
        const double d = (ph[i + plane] - f) * c.inv_dx;
        gsum += d * d;
      }
    }
    en += 0.5 * c.W2 * gsum;
    e += en;
    const double cc = p * a + q * b;
    s += cc;
    better(mx, am, cc, i);
  }
  se[threadIdx.x] = e;
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  sa[threadIdx.x] = am;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      se[threadIdx.x] += se[threadIdx.x + w];
      ss[threadIdx.x] += ss[threadIdx.x + w];
      double v = sm[threadIdx.x];
      long long a = sa[threadIdx.x];
      better(v, a, sm[threadIdx.x + w], sa[threadIdx.x + w]);
      sm[threadIdx.x] = v;
      sa[threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[ch].energy = se[0];
    out[ch].solute = ss[0];
    out[ch].cmax = sm[0];
    out[ch].arg = sa[0];
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_runs(Const c, RedTab red, const Partial* __restrict__ in,
                                                             Partial* __restrict__ out) {
  __shared__ double se[RED_THREADS], ss[RED_THREADS], sm[RED_THREADS];
  __shared__ long long sa[RED_THREADS];
  const int r = blockIdx.x;
  const int c0 = red.run_chunk0 ? red.run_chunk0[r] : 0;
  const int c1 = red.run_chunk0 ? red.run_chunk0[r + 1] : red.nchunk;
  double e = 0.0, s = 0.0, mx = -INFINITY;
  long long am = -1;
  for (int k = c0 + threadIdx.x; k < c1; k += RED_THREADS) {
    e += in[k].energy;
    s += in[k].solute;
    better(mx, am, in[k].cmax, in[k].arg);
  }
  se[threadIdx.x] = e;
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  sa[threadIdx.x] = am;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      se[threadIdx.x] += se[threadIdx.x + w];
      ss[threadIdx.x] += ss[threadIdx.x + w];
      double v = sm[threadIdx.x];
      long long a = sa[threadIdx.x];
      better(v, a, sm[threadIdx.x + w], sa[threadIdx.x + w]);
      sm[threadIdx.x] = v;
      sa[threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double vol = 1.0;
    for (int k = 0; k < c.dim; ++k) vol *= c.dx;
    out[r].energy = se[0] * vol;
    out[r].solute = ss[0] * vol;
    out[r].cmax = sm[0];
    out[r].arg = sa[0];
  }
}

// Copy one reduced Partial into separate device outputs (any may be null).
__global__ void k_partial_emit(const Partial* __restrict__ in, double* energy, double* total, double* cmax,
                               long long* argmax) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (energy) *energy = in->energy;
    if (total) *total = in->solute;
    if (cmax) *cmax = in->cmax;
    if (argmax) *argmax = in->arg;
  }
}

// Seed of the k_v loss: lam = sum_r dL/dk_r dk_r/du at each run's argmax cell.
__global__ void k_kv_seed(Const c, RunTab rt, int batched, const Partial* __restrict__ red,
                          const double* __restrict__ dLdk, int nrun, double* __restrict__ lph,
                          double* __restrict__ lcs, double* __restrict__ lcl, const double* __restrict__ ph,
                          const double* __restrict__ cs, const double* __restrict__ cl) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrun) return;
  const long long off = batched ? rt.off[r] : 0;
  const long long j = off + red[r].arg;
  if (red[r].arg < 0) return;
  const double cm = red[r].cmax;
  const double g = dLdk[r] / (cm * cm);
  double p, q, dp;
  interp(c, ph[j], p, q, dp);
  lph[j] = -g * dp * (cs[j] - cl[j]);
  lcs[j] = -g * p;
  lcl[j] = -g * q;
}

__global__ void k_fill(double* __restrict__ a, double v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------
// Solidification front (the interface diagnostic of Sec. V.C, where the
// interface temperature is read at phi = 1/2): in every growth-axis column the
// topmost crossing -- the largest i with phi_i >= 1/2 > phi_{i+1} -- placed by
// linear interpolation between the two cell centres, in lab coordinates
// z = (i + s + 1/2) dx + dx (phi_i - 1/2) / (phi_i - phi_{i+1}), s the window
// shift count.  Results per run (1D) or per domain (2D/3D, over the columns that
// cross): [mean z, min z, max z, (mean z - z0 - V t) / l_T, columns].
// ---------------------------------------------------------------------------
__device__ __forceinline__ double front_z(int i, double a, double b, double s, double dx) {
  return ((double)i + s + 0.5) * dx + dx * (a - 0.5) / (a - b);
}

// 2D/3D: one thread per column scans down from the top; NaN if no crossing.
__global__ void k_front_cols(const double* __restrict__ phi, long long ncol, int nz, double s, double dx,
                             double* __restrict__ zcol) {
  const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double z = __builtin_nan("");
  double b = phi[col + ncol * (long long)(nz - 1)];
  for (int i = nz - 2; i >= 0; --i) {
    const double a = phi[col + ncol * (long long)i];
    if (a >= 0.5 && b < 0.5) {
      z = front_z(i, a, b, s, dx);
      break;
    }
    b = a;
  }
  zcol[col] = z;
}

// One block: sums, extremes and count over the columns in a fixed order.
constexpr int FRONT_THREADS = 256;
__global__ void k_front_reduce(const double* __restrict__ zcol, long long ncol, double z_iso, double inv_lT,
                               double* __restrict__ out) {
  __shared__ double ssum[FRONT_THREADS], smin[FRONT_THREADS], smax[FRONT_THREADS], scnt[FRONT_THREADS];
  const int t = threadIdx.x;
  double sum = 0.0, mn = __builtin_inf(), mx = -__builtin_inf(), cnt = 0.0;
  for (long long c = t; c < ncol; c += FRONT_THREADS) {
    const double z = zcol[c];
    if (z == z) {  // not NaN
      sum += z;
      mn = fmin(mn, z);
      mx = fmax(mx, z);
      cnt += 1.0;
    }
  }
  ssum[t] = sum;
  smin[t] = mn;
  smax[t] = mx;
  scnt[t] = cnt;
  __syncthreads();
  for (int w = FRONT_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      ssum[t] += ssum[t + w];
      smin[t] = fmin(smin[t], smin[t + w]);
      smax[t] = fmax(smax[t], smax[t + w]);
      scnt[t] += scnt[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double nan = __builtin_nan("");
    const double zm = (scnt[0] > 0.0) ? ssum[0] / scnt[0] : nan;
    out[0] = zm;
    out[1] = (scnt[0] > 0.0) ? smin[0] : nan;
    out[2] = (scnt[0] > 0.0) ? smax[0] : nan;
    out[3] = (zm - z_iso) * inv_lT;
    out[4] = scnt[0];
  }
}

// 1D runs: one block per run; the largest crossing index by a block maximum.
__global__ void k_front_runs(Const c, RunTab rt, const double* __restrict__ phi, long long n,
                             double* __restrict__ out) {
  __shared__ int sbest[FRONT_THREADS];
  const int r = blockIdx.x, t = threadIdx.x;
  const int N = rt.n[r];
  const long long off = rt.off[r];
  int best = -1;
  for (int i = t; i + 1 < N; i += FRONT_THREADS)
    if (phi[off + i] >= 0.5 && phi[off + i + 1] < 0.5) best = i;  // increasing i: the last hit is the largest
  sbest[t] = best;
  __syncthreads();
  for (int w = FRONT_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) sbest[t] = max(sbest[t], sbest[t + w]);
    __syncthreads();
  }
  if (t == 0) {
    double* o = out + 5 * r;
    const int i = sbest[0];
    if (i < 0) {
      const double nan = __builtin_nan("");
      o[0] = o[1] = o[2] = o[3] = nan;
      o[4] = 0.0;
    } else {
      const double V = rt.V[r], dt = rt.dt[r];
      const double tn = (double)n * dt;
      const double s = floor(V * tn / c.dx);
      const double z = front_z(i, phi[off + i], phi[off + i + 1], s, c.dx);
      o[0] = o[1] = o[2] = z;
      o[3] = (z - rt.z0[r] - V * tn) * c.inv_lT;
      o[4] = 1.0;
    }
  }
}

}  // namespace pfk
