// pf_device.h -- device-side arithmetic of one explicit step (gfx950, FP64).
//
// The per-cell and per-face formulas of the staggered scheme for the set-2
// equations of motion (Sec. II: Eqs. cs_nonvar, cl_nonvar, phasefield_nonvar,
// and, for the variant with mu_s = mu_l imposed, Eq. solute_nonvar,
// drive of Eq. model18 reduced to dG_c - D (c_s - c_l)(mu_s - mu_l); Sec. III:
// dilute ideal alloy, Eqs. dil5.2, ds3; Sec. V.A: central gradients at cells,
// compact normal differences at faces, face-mean mobilities and anti-trapping).
// Shared by the forward kernels, the persistent 1D kernel and the adjoint.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// Derived constants of a handle, passed by value to every kernel.
struct Const {
  // grid: growth axis = z (last axis); x fastest; unused axes have extent 1
  int dim, nx, ny, nz;
  int px, py;      // periodic flags of x and y
  int quintic, pad_;
  long long ncell;
  // model
  double dx, inv_dx, inv_2dx, inv_4dx, inv_dx2, dt;
  double W, W2, alpha, lambda, lambda0, Mphi;
  double Ds, ke, log_ke, A, onemA, b, ap, inv_lT, V, z0, eps_grad, eps2;
  double eps2s, onemA_dx2;  // eps^2 dx^4 and (1-A) dx^2 of the dx-scaled face stage
  double inv_ke;
  double W2_dx2, eps2r, onemA_4dx2;  // W^2/dx^2, 16 eps^2 dx^4, 4 (1-A) dx^2: plain-difference cell stage
};

// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson steps
// (each step squares the relative error); x is positive and normal here.
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Natural logarithm for positive normal x, within 2 ulp: x = 2^e m with
// m in [1/sqrt 2, sqrt 2), ln x = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1),
// 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23) (|s| <= 0.1716, the
// series tail is below 1e-17).  NaN for x <= 0 or NaN.
__device__ __forceinline__ double flog(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double s = (m - 1.0) * frcp(m + 1.0);
  const double s2 = s * s;
  double t = 1.0 / 23.0;
  t = __builtin_fma(t, s2, 1.0 / 21.0);
  t = __builtin_fma(t, s2, 1.0 / 19.0);
  t = __builtin_fma(t, s2, 1.0 / 17.0);
  t = __builtin_fma(t, s2, 1.0 / 15.0);
  t = __builtin_fma(t, s2, 1.0 / 13.0);
  t = __builtin_fma(t, s2, 1.0 / 11.0);
  t = __builtin_fma(t, s2, 1.0 / 9.0);
  t = __builtin_fma(t, s2, 1.0 / 7.0);
  t = __builtin_fma(t, s2, 1.0 / 5.0);
  t = __builtin_fma(t, s2, 1.0 / 3.0);
  const double s_2 = s + s;
  const double lm = __builtin_fma(s_2 * s2, t, s_2);
  const double ed = (double)e;
  const double ln2_hi = 6.93147180369123816490e-01;  // ln 2 truncated to 32 significant bits (e ln2_hi exact)
  const double ln2_lo = 1.90821492927058770002e-10;  // ln 2 - ln2_hi (from 2 atanh(1/3))
  const double r = __builtin_fma(ed, ln2_hi, __builtin_fma(ed, ln2_lo, lm));
  return (x > 0.0) ? r : __builtin_nan("");
}

// Interpolation p(phi) = h + a_p (phi - 1/2) phi^2 (1-phi)^2 (Eq. interpolation2),
// its complement q = 1 - p evaluated as p(1 - phi) (antisymmetry of p; avoids the
// cancellation of 1 - p near phi = 1), and p'(phi).
// APZ: a_p is known to be zero at compile time (p = h); the launch picks the
// instantiation from the handle's a_p.
template <bool APZ = false>
__device__ __forceinline__ void interp(const Const& c, double phi, double& p, double& q, double& dp) {
  const double om = 1.0 - phi;
  const double w = phi * om;
  double h, hq, dh;
  if (c.quintic) {
    h = phi * phi * phi * (phi * (6.0 * phi - 15.0) + 10.0);
    hq = om * om * om * (om * (6.0 * om - 15.0) + 10.0);
    dh = 30.0 * w * w;
  } else {
    h = phi * phi * (3.0 - 2.0 * phi);
    hq = om * om * (3.0 - 2.0 * om);
    dh = 6.0 * w;
  }
  if constexpr (APZ) {
    p = h;
    q = hq;
    dp = dh;
  } else {
    const double a = c.ap * (phi - 0.5) * w * w;
    p = h + a;
    q = hq - a;
    const double tt = 1.0 - 2.0 * phi;
    dp = dh + c.ap * w * (w - tt * tt);
  }
}

template <bool APZ = false>
__device__ __forceinline__ void interp_pq(const Const& c, double phi, double& p, double& q) {
  const double om = 1.0 - phi;
  double h, hq;
  if (c.quintic) {
    h = phi * phi * phi * (phi * (6.0 * phi - 15.0) + 10.0);
    hq = om * om * om * (om * (6.0 * om - 15.0) + 10.0);
  } else {
    h = phi * phi * (3.0 - 2.0 * phi);
    hq = om * om * (3.0 - 2.0 * om);
  }
  if constexpr (APZ) {
    p = h;
    q = hq;
  } else {
    const double w = phi * om;
    const double a = c.ap * (phi - 0.5) * w * w;
    p = h + a;
    q = hq - a;
  }
}

// Equilibrium liquid concentration of the frozen temperature field at lab
// height zlab and time t (Eqs. dil7, ds1, reference (c_inf, T_s) at z0).
__device__ __forceinline__ double cleq_at(const Const& c, double zlab, double t, double V, double z0) {
  return (1.0 - (1.0 - c.ke) * (zlab - z0 - V * t) * c.inv_lT) * c.inv_ke;
}

// mu_bar = p mu_s + (1-p) mu_l (units of Omega, up to a constant) of one cell.
__device__ __forceinline__ double mubar_of(const Const& c, double phi, double cs, double cl) {
  double p, q;
  interp_pq(c, phi, p, q);
  const double ll = flog(cl);
  return ll + p * (flog(cs) - ll - c.log_ke);
}

// Cell stage: phi_t (Eq. phasefield_nonvar divided by H) and mu_bar.
// With Mbar = M_s(1-p) + b M_l p, G = |grad phi|^2, the regularised inverse
// gam = G / S, S = G^2 + eps^2, and the drag numerator
// Dn = M_s(1-p)(1 - A(1-p)) + A b M_l p^2 (drag D = Dn / Mbar), the rate
//   phi_t = [W^2 lap - f' - lambda (dG_c - D dc dmu) p' + X] / tau,
//   X   = lambda (1-A) dc p(1-p) (Ds grad c_s - b grad c_l).grad phi gam / Mbar,
//   tau = alpha + lambda (1-A)^2 dc^2 b p(1-p) gam / (Mbar (b p + 1 - p)),
// is evaluated with numerator and prefactor multiplied by Q = Mbar (b p + 1 - p) S:
// one reciprocal.  cell_core takes G and dot = (Ds grad c_s - b grad c_l).grad phi
// in units where the true values are k G and k dot, with eps2x = eps^2 / k^2 and
// onemAx = (1 - A) / k (the common factor k^2 of numerator and prefactor cancels);
// Wlap is W^2 lap.
// phi_t from the interpolation values p, q = 1-p, p', dmu = (mu_s - mu_l)/Omega
// and the scaled G, dot (see cell_core).
__device__ __forceinline__ double cell_rate(const Const& c, double kcl, double phi, double cs, double cl, double dmu,
                                           double p, double q, double dp, double G, double dot, double Wlap,
                                           double eps2x, double onemAx) {
  const double dc = cs - cl;
  const double dGc = cs * dmu + kcl - dc;  // Eq. dil5.2 with Eq. ds3, kcl = (k_e - 1) c_l^eq
  const double ms = c.Ds * cs * q;                          // M_s (1 - p)
  const double ml = c.b * cl * p;                           // b M_l p
  const double Mb = ms + ml;
  const double Dn = ms * (1.0 - c.A * q) + c.A * ml * p;
  const double S = G * G + eps2x;
  const double bq = c.b * p + q;
  const double Q = Mb * bq * S;
  const double pq = p * q;
  const double lAdc = c.lambda * c.onemA * dc;
  const double fdw = 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi);
  const double base = Wlap - fdw - c.lambda * dGc * dp;
  const double num = base * Q + c.lambda * Dn * dc * dmu * dp * bq * S + lAdc * pq * dot * G * bq;
  const double den = c.alpha * Q + lAdc * onemAx * dc * c.b * pq * G;
  return num * frcp(den);
}

// EQ: the equal-potential model (mu_s = mu_l = ln c_l imposed): dmu = 0.
template <bool APZ, bool EQ = false>
__device__ __forceinline__ void cell_core(const Const& c, double kcl, double phi, double cs, double cl, double G,
                                          double dot, double Wlap, double eps2x, double onemAx, double& phit,
                                          double& mubar) {
  double p, q, dp;
  interp<APZ>(c, phi, p, q, dp);
  const double ll = flog(cl);
  const double dmu = EQ ? 0.0 : flog(cs) - ll - c.log_ke;  // (mu_s - mu_l) / Omega
  mubar = ll + p * dmu;
  phit = cell_rate(c, kcl, phi, cs, cl, dmu, p, q, dp, G, dot, Wlap, eps2x, onemAx);
}

// g*[k] are the central differences (u_{+k} - u_{-k}) / (2 dx), lap the
// compact Laplacian of phi.
template <int DIM, bool APZ = false, bool EQ = false>
__device__ __forceinline__ void cell_stage(const Const& c, double kcl, double phi, double cs, double cl,
                                           const double* gph, const double* gcs, const double* gcl,
                                           double lap, double& phit, double& mubar) {
  double G = 0.0, dot = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    G += gph[k] * gph[k];
    dot += (c.Ds * gcs[k] - c.b * gcl[k]) * gph[k];
  }
  cell_core<APZ, EQ>(c, kcl, phi, cs, cl, G, dot, c.W2 * lap, c.eps2, c.onemA, phit, mubar);
}

// The same from plain differences: d*[k] = u_{+k} - u_{-k} and lsum the sum over
// axes of u_{+k} - 2 u + u_{-k} (k = 1 / (4 dx^2)).
template <int DIM, bool APZ = false, bool EQ = false>
__device__ __forceinline__ void cell_stage_raw(const Const& c, double kcl, double phi, double cs, double cl,
                                               const double* dph, const double* dcs, const double* dcl,
                                               double lsum, double& phit, double& mubar) {
  double G = 0.0, dot = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    G += dph[k] * dph[k];
    dot += (c.Ds * dcs[k] - c.b * dcl[k]) * dph[k];
  }
  cell_core<APZ, EQ>(c, kcl, phi, cs, cl, G, dot, c.W2_dx2 * lsum, c.eps2r, c.onemA_4dx2, phit, mubar);
}

// Face stage: solid and liquid fluxes (brackets of Eqs. cs_nonvar, cl_nonvar)
// through a face normal to axis K, in dx-scaled form.  phf, csf, clf, ptf are
// the face means; g*[K] is the plain difference u_b - u_a across the face and
// g*[j], j != K, the sum of the central differences (u_{+j} - u_{-j}) of the two
// cells beside it, so the face gradient is (g[K], g[j]/4) / dx.  With
// gam = G/(G^2 + eps^2) (regularised 1/|grad phi|^2) and R = (grad phi)_K gam / Mbar:
//   q_n (n n^T grad mu_bar)_K = M_s M_l (b p + 1 - p) (grad phi . grad mu_bar) R,
//   ((1 - n n^T) grad c)_K    = (grad c)_K - (grad phi . grad c) Mbar R,
//   anti-trapping_s / _l      = +/- (1-A)(c_s - c_l) phi_t R M_s(1-p) / b M_l p.
// Returned: dx times the fluxes (divergence = sum of differences / dx^2).  In
// scaled units G' = dx^2 G, eps'^2 = dx^4 eps^2 and R' = R / dx, which leaves
// every term but the anti-trapping one (factor dx^2) unchanged in form.
// EQ (equal-potential model): Fs returns the mixture flux p F_s + (1-p) F_l,
// the bracket of Eq. solute_nonvar (its anti-trapping part is
// (1-A)(c_s - c_l) a(phi) phi_t n / |grad phi| with a of Eq. shape_function);
// Fl is zero.
template <int DIM, int K, bool APZ = false, bool EQ = false>
__device__ __forceinline__ void face_flux(const Const& c, double phf, double csf, double clf, double ptf,
                                          const double* gph, const double* gmu, const double* gcs,
                                          const double* gcl, double& Fs, double& Fl) {
  double p, q;
  interp_pq<APZ>(c, phf, p, q);
  double G = gph[K] * gph[K], dmu = gph[K] * gmu[K], dcs = gph[K] * gcs[K], dcl = gph[K] * gcl[K];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    if (j == K) continue;
    const double t = 0.0625 * gph[j];
    G = __builtin_fma(t, gph[j], G);
    dmu = __builtin_fma(t, gmu[j], dmu);
    dcs = __builtin_fma(t, gcs[j], dcs);
    dcl = __builtin_fma(t, gcl[j], dcl);
  }
  const double Ms = c.Ds * csf;
  const double Ml = clf;
  const double ms = Ms * q, ml = c.b * Ml * p;
  const double Mb = ms + ml;
  const double R = gph[K] * G * frcp(Mb * (G * G + c.eps2s));
  const double nrm = Ms * Ml * (c.b * p + q) * dmu * R;
  const double at = c.onemA_dx2 * (csf - clf) * ptf * R;
  const double MbR = Mb * R;
  Fs = nrm + c.Ds * (gcs[K] - dcs * MbR) + at * ms;
  Fl = nrm + (gcl[K] - dcl * MbR) - at * ml;
  if constexpr (EQ) {
    Fs = p * Fs + q * Fl;
    Fl = 0.0;
  }
}

// Equal-potential split of the mixture concentration at phase field phi
// (dilute ideal alloy, mu_s = mu_l): c_l = c / (k_e p + 1 - p), c_s = k_e c_l.
template <bool APZ>
__device__ __forceinline__ void eq_split(const Const& c, double phi, double cmix, double& cs, double& cl) {
  double p, q;
  interp_pq<APZ>(c, phi, p, q);
  cl = cmix * frcp(__builtin_fma(c.ke, p, q));
  cs = c.ke * cl;
}

// Error word bits.
enum : int { ERR_NONFINITE = 1, ERR_NEGCONC = 2 };

__device__ __forceinline__ int check_bits(double phi, double cs, double cl) {
  int e = 0;
  if (!__builtin_isfinite(phi) || !__builtin_isfinite(cs) || !__builtin_isfinite(cl)) e |= ERR_NONFINITE;
  else if (!(cs > 0.0) || !(cl > 0.0)) e |= ERR_NEGCONC;
  return e;
}

}  // namespace pfk
