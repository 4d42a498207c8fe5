// pf_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
//
// A plain, slow, FP64 CPU oracle for one explicit time step of the variational
// phase-field model of Mukherjee, Warren & Voorhees (arXiv 2303.09671).  Only the
// tests, the smoke check and the CPU-baseline leg of the benchmark may load it.
// It shares no source with the HIP library: it is written directly from the
// paper's equations, in the paper's order, with no blocking or fusion.
//
// What one step computes (Sec. II "Alternative choice of interpolation
// functions", Eqs. cs_nonvar, cl_nonvar, phasefield_nonvar; Sec. III dilute
// alloy, Eqs. dil5.1, dil5.2, ds2, ds3; Sec. V.A numerical technique):
//   * fields phi (1 = solid), c_s, c_l at cell centres of a uniform grid,
//     concentrations in units of c_inf, lengths in the reference width W0,
//     time in W0^2/D_l, energies in H (supplement Sec. S-II);
//   * interpolation set 2: p = h + a_p (phi-1/2) phi^2 (1-phi)^2, g = p,
//     M^n from h_n = b p/(b p + 1 - p), M^t = M/p and M/(1-p)  (Eqs. normal2,
//     interpolation1, interpolation2);
//   * dilute ideal alloy with local mobilities M_i = D_i c_i / Omega, so that
//     M_i grad(mu_i) = D_i grad(c_i)  (Sec. III, Eq. dil1; supplement S-II);
//   * sources S_s = S_l = -A (c_s - c_l)  (Sec. II.B);
//   * the phi-equation driving force is taken from the general equation of
//     motion (Eq. model18) with the sources and set-2 mobilities substituted;
//     its reduced printed form (Eqs. drivingforce_nonvar, drag_coefficient)
//     carries a sign slip and drops b, see the ambiguity register;
//   * frozen temperature of directional solidification (Eq. ds1) referenced to
//     the solidus T_s of c_inf at the initial front position z0;
//   * second-order central gradients at cells, compact Laplacian, staggered
//     fluxes with mobilities / anti-trapping evaluated at the face centre from
//     face means, forward Euler (Sec. V.A);
//   * 1/|grad phi|^2 (normal projection, anti-trapping, the phi prefactor) is
//     regularised as G / (G^2 + eps^2), G = |grad phi|^2: 1/G wherever G >> eps,
//     a smooth decay to 0 where the gradient vanishes (the paper is silent);
//   * the moving window: when floor(V t_{n+1}/dx) exceeds the shift count the
//     cold-end layer is dropped and a fresh liquid layer (phi=0, c_l=1,
//     c_s=k_e) is appended at the hot end (Sec. V.A, shifting algorithm);
//   * no-flux (mirror) boundaries on the growth axis, mirror or periodic on
//     the transverse axes.
//
// model = 1 steps instead the variant with pointwise equal diffusion potentials,
// mu_s = mu_l, which is the model of the paper's asymptotic analysis (Sec. II.C;
// with A = 1 and b = k_e D_s/D_l it is the KKS model of Sec. IV, Eqs. KKS1,
// KKS2).  The phase-field rate is Eq. phasefield_nonvar with mu_s = mu_l.  A
// single conserved mixture c = p c_s + (1 - p) c_l follows the bracket of
// Eq. solute_nonvar.  After each step the phase concentrations are recovered from
// c and the new phi by the equal-potential condition of the dilute ideal alloy
// (Eq. dil1: ln(c_s/k_e) = ln c_l), i.e. c_s = k_e c_l and
// c_l = c / (k_e p + 1 - p).  The state of this model is (phi, c_l): c_s on input
// is replaced by k_e c_l.
//
// The step is templated on the scalar type so that the same code also runs on
// dual numbers, which gives exact forward-mode directional derivatives (JVPs)
// used to check the hand-written adjoint of the GPU library.
//
// Build: g++ -O2 -std=c++17 -fno-fast-math -ffp-contract=off -shared -fPIC.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Dual numbers: value + one tangent.  Exact first derivatives for +,-,*,/,log.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: constants promote implicitly
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual dlog(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline double dlog(double a) { return std::log(a); }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }

// ---------------------------------------------------------------------------
// Parameters (nondimensional; see header comment).  Mirrored field by field by
// the ctypes structure in oracle.py.
// ---------------------------------------------------------------------------
struct OrcParams {
  int32_t dim;          // 1, 2 or 3; the growth axis is the last one
  int32_t n[3];         // cells per axis (axis 0 fastest in memory)
  int32_t periodic[3];  // transverse axes: 1 periodic, 0 mirror; growth axis ignored (mirror)
  int32_t quintic;      // 1: h = phi^3(6phi^2-15phi+10); 0: h = phi^2(3-2phi)
  int32_t drag_variant; // 0: drive from Eq. model18 (used); 1: printed reduced form (mutation tests only)
  int32_t model;        // 0: separate kinetics of c_s and c_l; 1: mu_s = mu_l imposed pointwise
  int32_t mutate;       // 0 (used); > 0 plants one known mistake, for the pin tests only (see Mutation)
  int32_t pad_;
  double dx, dt;
  double W;        // interface width / W0
  double Mphi;     // phi mobility in units of 1/alpha at W = W0; alpha = W / Mphi
  double lambda0;  // coupling Omega c_inf / H at W = W0; lambda = lambda0 * W
  double Ds;       // D_s / D_l
  double ke;       // equilibrium partition coefficient
  double A;        // source (trapping) coefficient
  double b, ap;    // set-2 interpolation constants
  double inv_lT;   // 1 / thermal length (0 = isothermal at T_s)
  double V;        // pulling speed
  double z0;       // initial interface position (lab frame)
  double eps_grad; // scale of the smooth |grad phi|^2 gate
};

// Planted mistakes, selected by OrcParams::mutate.  They exist only so that
// the tests can show that each of their pins fails when the corresponding term
// of the equations is wrong; the oracle proper runs with mutate = 0.
enum Mutation : int32_t {
  MUT_NONE = 0,
  MUT_SWAP_AT_WEIGHTS = 1,     // anti-trapping weights M_s(1-p)/Mbar and b M_l p/Mbar exchanged
  MUT_FLIP_AT_SIGN = 2,        // anti-trapping terms of both fluxes with the opposite sign
  MUT_DROP_CROSS = 3,          // cross term X of the phi equation left out
  MUT_DROP_PREFACTOR = 4,      // (1-A)^2 term of the phi prefactor left out
  MUT_COMPACT_TRANSVERSE = 5,  // transverse face gradients from the low-side cell only
  MUT_ISOTHERM_BACKWARDS = 6,  // frozen temperature pulled with the opposite sign of V t
  MUT_LAB_NO_SHIFT = 7,        // lab height of a cell without the window shift count
};

// Parameters promoted to the working scalar type; theta = (A, Mphi, W, b) may carry tangents.
template <class T>
struct WP {
  T A, Mphi, W, alpha, lambda, W2, b;
};

// Double-well and interpolation functions (Sec. II; Eqs. interpolation2).
template <class T>
inline T h_of(T phi, int quintic) {
  if (quintic) return phi * phi * phi * (phi * (6.0 * phi - 15.0) + 10.0);
  return phi * phi * (3.0 - 2.0 * phi);
}
template <class T>
inline T dh_of(T phi, int quintic) {
  T w = phi * (1.0 - phi);
  if (quintic) return 30.0 * w * w;
  return 6.0 * w;
}
template <class T>
inline T p_of(T phi, int quintic, double ap) {
  T w = phi * (1.0 - phi);
  return h_of(phi, quintic) + ap * (phi - 0.5) * w * w;
}
template <class T>
inline T dp_of(T phi, int quintic, double ap) {
  // d/dphi [ (phi-1/2) w^2 ] = w^2 + (phi-1/2) * 2 w (1 - 2 phi),  w = phi(1-phi)
  T w = phi * (1.0 - phi);
  return dh_of(phi, quintic) + ap * (w * w + (phi - 0.5) * 2.0 * w * (1.0 - 2.0 * phi));
}
template <class T>
inline T dfdw_of(T phi) {  // d/dphi [phi^2 (1-phi)^2]
  return 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi);
}

struct Grid {
  int dim, n[3], per[3];
  long ncell;
  long lin(const int c[3]) const { return (long)c[0] + (long)n[0] * ((long)c[1] + (long)n[1] * c[2]); }
  // Map a possibly out-of-range coordinate to a cell (mirror or periodic).
  int map(int c, int k) const {
    int m = n[k];
    if (per[k] && k != dim - 1) {
      c %= m;
      if (c < 0) c += m;
      return c;
    }
    while (c < 0 || c >= m) {  // mirror about the outer faces: -1 -> 0, -2 -> 1, m -> m-1
      if (c < 0) c = -c - 1;
      if (c >= m) c = 2 * m - c - 1;
    }
    return c;
  }
  long at(const int c[3], int k1, int o1, int k2 = -1, int o2 = 0) const {
    int q[3] = {c[0], c[1], c[2]};
    q[k1] += o1;
    if (k2 >= 0) q[k2] += o2;
    for (int k = 0; k < dim; ++k) q[k] = map(q[k], k);
    return lin(q);
  }
};

Grid make_grid(const OrcParams& P) {
  Grid g;
  g.dim = P.dim;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = (k < P.dim) ? P.n[k] : 1;
    g.per[k] = (k < P.dim - 1) ? P.periodic[k] : 0;
  }
  g.ncell = (long)g.n[0] * g.n[1] * g.n[2];
  return g;
}

// Equilibrium liquid concentration of the frozen temperature field at the
// lab-frame height z and time t (Eqs. dil7, ds1; reference (c_inf, T_s) at z0).
inline double cleq_of(const OrcParams& P, double zlab, double t) {
  if (P.mutate == MUT_ISOTHERM_BACKWARDS) t = -t;
  return (1.0 - (1.0 - P.ke) * (zlab - P.z0 - P.V * t) * P.inv_lT) / P.ke;
}

// Pointwise thermodynamic quantities at one cell.
template <class T>
struct Pointwise {
  T p, q, dp, dmu, mubar, dc, Ms, Ml, Mbar, dG;  // q = 1 - p
};

template <class T>
Pointwise<T> pointwise(const OrcParams& P, const WP<T>& w, T phi, T cs, T cl, double cleq) {
  Pointwise<T> r;
  r.p = p_of(phi, P.quintic, P.ap);
  // 1 - p evaluated as p(1 - phi): equal by the antisymmetry of p, and free of
  // the cancellation that 1 - p suffers near phi = 1 (where it is multiplied by
  // 1/|grad phi|^2 in the interface terms).
  r.q = p_of(1.0 - phi, P.quintic, P.ap);
  r.dp = dp_of(phi, P.quintic, P.ap);
  // Diffusion potentials of the dilute ideal alloy (Eq. dil1), in units of Omega:
  // mu_s - mu_l = ln(c_s/(k_e c_l)); mu_bar = p mu_s + (1-p) mu_l up to a constant.
  T ls = dlog(cs), ll = dlog(cl);
  r.dmu = ls - ll - std::log(P.ke);
  r.mubar = r.p * (ls - std::log(P.ke)) + r.q * ll;
  if (P.model == 1) {  // mu_s = mu_l = mu = ln c_l imposed
    r.dmu = 0.0;
    r.mubar = ll;
  }
  r.dc = cs - cl;
  // Local mobilities M_i = D_i c_i / Omega in units of c_inf D_l / Omega.
  r.Ms = P.Ds * cs;
  r.Ml = cl;
  // Mbar of the numerical equations: M_s (1-p) + b M_l p.
  r.Mbar = r.Ms * r.q + w.b * r.Ml * r.p;
  // Driving forces of Eqs. dil5.1 (with mu_s) and dil5.2 (with mu_l).
  T G_mus = cl * r.dmu + (P.ke - 1.0) * cleq - r.dc;  // f_s - f_l - (c_s-c_l) mu_s
  T G_mul = cs * r.dmu + (P.ke - 1.0) * cleq - r.dc;  // f_s - f_l - (c_s-c_l) mu_l
  T S = -w.A * r.dc;                                  // S_s = S_l
  if (P.drag_variant == 0) {
    // Eq. model18 with M_s^n/Mbar_n = M_s(1-p)/Mbar and M_l^n/Mbar_n = b M_l p/Mbar:
    T ws = r.Ms * r.q / r.Mbar;
    T wl = w.b * r.Ml * r.p / r.Mbar;
    T brack_s = G_mus - S * r.q * r.dmu;           // ... - S_l (1-g)(mu_s - mu_l)
    T brack_l = G_mul - S * r.p * (-r.dmu);        // ... - S_s g (mu_l - mu_s)
    r.dG = ws * brack_s + wl * brack_l;
  } else {
    // Printed reduced form (drivingforce_nonvar), kept only so that a test can
    // show that it violates the free-energy decrease.
    T br = (r.Ms * r.q * (w.A * r.q - 1.0) - r.Ml * r.p * w.A * r.p) / r.Mbar;
    r.dG = G_mul - r.dc * r.dmu * br;
  }
  return r;
}

template <class T>
struct StepWork {
  std::vector<T> phit, mubar;
  std::vector<Pointwise<T>> pw;
};

// Central difference of a field at cell c along axis k, divided by 2 dx.
template <class T>
inline T cdiff(const Grid& g, const T* u, const int c[3], int k, double dx) {
  return (u[g.at(c, k, +1)] - u[g.at(c, k, -1)]) / (2.0 * dx);
}

// phi_t at one cell from Eq. phasefield_nonvar (nondimensional, divided by H).
template <class T>
T phi_t_at(const OrcParams& P, const WP<T>& w, const Grid& g, const T* phi, const T* cs, const T* cl,
           const Pointwise<T>& q, const int c[3]) {
  const double dx = P.dx;
  long i = g.lin(c);
  T gphi[3], gcs[3], gcl[3];
  T lap = 0.0;
  for (int k = 0; k < P.dim; ++k) {
    gphi[k] = cdiff(g, phi, c, k, dx);
    gcs[k] = cdiff(g, cs, c, k, dx);
    gcl[k] = cdiff(g, cl, c, k, dx);
    lap = lap + (phi[g.at(c, k, +1)] - 2.0 * phi[i] + phi[g.at(c, k, -1)]) / (dx * dx);
  }
  T G = 0.0;
  for (int k = 0; k < P.dim; ++k) G = G + gphi[k] * gphi[k];
  T gam = G / (G * G + P.eps_grad * P.eps_grad);  // 1/|grad phi|^2, smoothly gated below eps_grad
  T pq = q.p * q.q;
  T onemA = 1.0 - w.A;
  // Prefactor: 1/M_phi + (c_s-c_l)^2 (1-A)^2 b p(1-p) / (Mbar (b p + 1 - p)) / |grad phi|^2
  T pref = w.alpha + w.lambda * q.dc * q.dc * onemA * onemA * w.b * pq /
                         (q.Mbar * (w.b * q.p + q.q)) * gam;
  if (P.mutate == MUT_DROP_PREFACTOR) pref = w.alpha;
  // Cross term: (c_s-c_l)(1-A) p(1-p)/Mbar (M_s grad mu_s - b M_l grad mu_l) . grad phi / |grad phi|^2
  T dot = 0.0;
  for (int k = 0; k < P.dim; ++k) dot = dot + (P.Ds * gcs[k] - w.b * gcl[k]) * gphi[k];
  T cross = w.lambda * q.dc * onemA * pq / q.Mbar * dot * gam;
  if (P.mutate == MUT_DROP_CROSS) cross = 0.0;
  T rhs = w.W2 * lap - dfdw_of(phi[i]) - w.lambda * q.dG * q.dp + cross;
  return rhs / pref;
}

// Solid and liquid fluxes (the brackets of Eqs. cs_nonvar, cl_nonvar) through
// the face between cell c and c + e_k.  Returns false for a boundary face.
template <class T>
bool face_flux(const OrcParams& P, const WP<T>& w, const Grid& g, const T* phi, const T* cs,
               const T* cl, const StepWork<T>& S, const int c[3], int k, T& Js, T& Jl) {
  const double dx = P.dx;
  bool periodic_axis = g.per[k] && k != g.dim - 1;
  if (!periodic_axis && c[k] == g.n[k] - 1) {
    Js = 0.0;
    Jl = 0.0;
    return false;  // no-flux face on the boundary
  }
  long a = g.lin(c);
  long bidx = g.at(c, k, +1);
  int cb[3] = {c[0], c[1], c[2]};
  cb[k] = g.map(c[k] + 1, k);
  // Face means (mobility and anti-trapping evaluated at the face centre).
  T phif = 0.5 * (phi[a] + phi[bidx]);
  T csf = 0.5 * (cs[a] + cs[bidx]);
  T clf = 0.5 * (cl[a] + cl[bidx]);
  T phitf = 0.5 * (S.phit[a] + S.phit[bidx]);
  T pf = p_of(phif, P.quintic, P.ap);
  T qf = p_of(1.0 - phif, P.quintic, P.ap);  // 1 - p at the face, see pointwise()
  T dcf = csf - clf;
  // Face gradients: compact difference normal to the face, mean of the two
  // cells' central differences along the other axes.
  const T* fld[4] = {phi, S.mubar.data(), cs, cl};
  T grad[4][3];
  for (int f = 0; f < 4; ++f) {
    for (int j = 0; j < P.dim; ++j) {
      if (j == k) {
        grad[f][j] = (fld[f][bidx] - fld[f][a]) / dx;
      } else if (P.mutate == MUT_COMPACT_TRANSVERSE) {
        grad[f][j] = cdiff(g, fld[f], c, j, dx);
      } else {
        grad[f][j] = 0.5 * (cdiff(g, fld[f], c, j, dx) + cdiff(g, fld[f], cb, j, dx));
      }
    }
  }
  T G = 0.0, dmu = 0.0, dcs = 0.0, dcl = 0.0;
  for (int j = 0; j < P.dim; ++j) {
    G = G + grad[0][j] * grad[0][j];
    dmu = dmu + grad[0][j] * grad[1][j];
    dcs = dcs + grad[0][j] * grad[2][j];
    dcl = dcl + grad[0][j] * grad[3][j];
  }
  T gam = G / (G * G + P.eps_grad * P.eps_grad);  // smooth gate, as at cells
  // Normal projection n n^T grad u = gam (grad phi . grad u) grad phi; k-components:
  T n_mubar = gam * dmu * grad[0][k];
  T t_cs = grad[2][k] - gam * dcs * grad[0][k];
  T t_cl = grad[3][k] - gam * dcl * grad[0][k];
  T Ms = P.Ds * csf, Ml = clf;
  T Mbar = Ms * qf + w.b * Ml * pf;
  T qn = Ms * Ml * (w.b * pf + qf) / Mbar;  // Eq. normal2 reduced: M_s M_l (b p + 1 - p)/Mbar
  T at = (1.0 - w.A) * dcf * grad[0][k] * gam * phitf;
  T ws = Ms * qf / Mbar, wl = w.b * Ml * pf / Mbar;  // anti-trapping weights of Eqs. cs_nonvar, cl_nonvar
  if (P.mutate == MUT_SWAP_AT_WEIGHTS) std::swap(ws, wl);
  if (P.mutate == MUT_FLIP_AT_SIGN) at = -at;
  Js = qn * n_mubar + P.Ds * t_cs + at * ws;
  Jl = qn * n_mubar + t_cl - at * wl;
  return true;
}

// Solute flux of the equal-potential model (the bracket of Eq. solute_nonvar
// with mu_s = mu_l = mu) through the face between cell c and c + e_k, with the
// local mobilities (M_s grad mu = D_s grad c_s, M_l grad mu = grad c_l):
//   J_k = q_n (n n^T grad mu)_k + p D_s ((1 - n n^T) grad c_s)_k + (1 - p) ((1 - n n^T) grad c_l)_k
//       + (1 - A)(c_s - c_l) a(phi) phi_t (grad phi)_k / |grad phi|^2,
// a(phi) = (M_s - b M_l) p (1 - p) / Mbar (Eq. shape_function), face means and
// face gradients as in face_flux.  Returns false for a boundary face.
template <class T>
bool mixture_flux(const OrcParams& P, const WP<T>& w, const Grid& g, const T* phi, const T* cs, const T* cl,
                  const StepWork<T>& S, const int c[3], int k, T& J) {
  const double dx = P.dx;
  bool periodic_axis = g.per[k] && k != g.dim - 1;
  if (!periodic_axis && c[k] == g.n[k] - 1) {
    J = 0.0;
    return false;
  }
  long a = g.lin(c);
  long bidx = g.at(c, k, +1);
  int cb[3] = {c[0], c[1], c[2]};
  cb[k] = g.map(c[k] + 1, k);
  T phif = 0.5 * (phi[a] + phi[bidx]);
  T csf = 0.5 * (cs[a] + cs[bidx]);
  T clf = 0.5 * (cl[a] + cl[bidx]);
  T phitf = 0.5 * (S.phit[a] + S.phit[bidx]);
  T pf = p_of(phif, P.quintic, P.ap);
  T qf = p_of(1.0 - phif, P.quintic, P.ap);
  const T* fld[4] = {phi, S.mubar.data(), cs, cl};
  T grad[4][3];
  for (int f = 0; f < 4; ++f)
    for (int j = 0; j < P.dim; ++j)
      grad[f][j] = (j == k) ? (fld[f][bidx] - fld[f][a]) / dx
                            : 0.5 * (cdiff(g, fld[f], c, j, dx) + cdiff(g, fld[f], cb, j, dx));
  T G = 0.0, dmu = 0.0, dcs = 0.0, dcl = 0.0;
  for (int j = 0; j < P.dim; ++j) {
    G = G + grad[0][j] * grad[0][j];
    dmu = dmu + grad[0][j] * grad[1][j];
    dcs = dcs + grad[0][j] * grad[2][j];
    dcl = dcl + grad[0][j] * grad[3][j];
  }
  T gam = G / (G * G + P.eps_grad * P.eps_grad);
  T Ms = P.Ds * csf, Ml = clf;
  T Mbar = Ms * qf + w.b * Ml * pf;
  T qn = Ms * Ml * (w.b * pf + qf) / Mbar;       // Eq. normal2 with h_n of Eq. interpolation1
  T a_shape = (Ms - w.b * Ml) * pf * qf / Mbar;  // Eq. shape_function
  T normal = qn * gam * dmu * grad[0][k];
  T tang = pf * P.Ds * (grad[2][k] - gam * dcs * grad[0][k]) + qf * (grad[3][k] - gam * dcl * grad[0][k]);
  T anti = (1.0 - w.A) * (csf - clf) * a_shape * phitf * grad[0][k] * gam;
  J = normal + tang + anti;
  return true;
}

// Pointwise quantities, mu_bar and phi_t of every cell at time t (shift count s).
template <class T>
void cell_stage(const OrcParams& P, const WP<T>& w, const Grid& g, const T* phi, const T* cs, const T* cl,
                double t, int64_t s, StepWork<T>& S) {
  const long N = g.ncell;
  const int gz = P.dim - 1;
  S.phit.assign(N, T(0.0));
  S.mubar.assign(N, T(0.0));
  S.pw.resize(N);
  // The cell loops carry OpenMP pragmas for the all-cores timing build: every
  // cell is independent, so the result does not depend on the thread count.
#pragma omp parallel for collapse(2) schedule(static)
  for (int c2 = 0; c2 < g.n[2]; ++c2)
    for (int c1 = 0; c1 < g.n[1]; ++c1)
      for (int c0 = 0; c0 < g.n[0]; ++c0) {
        const int c[3] = {c0, c1, c2};
        long i = g.lin(c);
        double zlab = ((double)c[gz] + (P.mutate == MUT_LAB_NO_SHIFT ? 0.0 : (double)s) + 0.5) * P.dx;
        S.pw[i] = pointwise(P, w, phi[i], cs[i], cl[i], cleq_of(P, zlab, t));
        S.mubar[i] = S.pw[i].mubar;
      }
#pragma omp parallel for collapse(2) schedule(static)
  for (int c2 = 0; c2 < g.n[2]; ++c2)
    for (int c1 = 0; c1 < g.n[1]; ++c1)
      for (int c0 = 0; c0 < g.n[0]; ++c0) {
        const int c[3] = {c0, c1, c2};
        long i = g.lin(c);
        S.phit[i] = phi_t_at(P, w, g, phi, cs, cl, S.pw[i], c);
      }
}

// One forward-Euler step n -> n+1 in place.  s_shift is the number of window
// shifts done so far (lab height of cell iz is (iz + s + 1/2) dx).
template <class T>
void step_once(const OrcParams& P, const WP<T>& w, T* phi, T* cs, T* cl, long n, int64_t* s_shift) {
  Grid g = make_grid(P);
  const long N = g.ncell;
  const int gz = P.dim - 1;
  const double t = (double)n * P.dt;
  if (P.model == 1)  // c_s is not a state variable of this model: it follows c_l
    for (long i = 0; i < N; ++i) cs[i] = P.ke * cl[i];
  StepWork<T> S;
  cell_stage(P, w, g, phi, cs, cl, t, *s_shift, S);
  std::vector<T> nphi(N), ncs(N), ncl(N);
#pragma omp parallel for collapse(2) schedule(static)
  for (int c2 = 0; c2 < g.n[2]; ++c2)
    for (int c1 = 0; c1 < g.n[1]; ++c1)
      for (int c0 = 0; c0 < g.n[0]; ++c0) {
        const int c[3] = {c0, c1, c2};
        long i = g.lin(c);
        T divs = 0.0, divl = 0.0;
        for (int k = 0; k < P.dim && P.model == 0; ++k) {
          T jsp, jlp, jsm, jlm;
          face_flux(P, w, g, phi, cs, cl, S, c, k, jsp, jlp);
          bool periodic_axis = g.per[k] && k != g.dim - 1;
          if (!periodic_axis && c[k] == 0) {
            jsm = 0.0;
            jlm = 0.0;
          } else {
            int cm[3] = {c[0], c[1], c[2]};
            cm[k] = g.map(c[k] - 1, k);
            face_flux(P, w, g, phi, cs, cl, S, cm, k, jsm, jlm);
          }
          divs = divs + (jsp - jsm) / P.dx;
          divl = divl + (jlp - jlm) / P.dx;
        }
        const Pointwise<T>& q = S.pw[i];
        nphi[i] = phi[i] + P.dt * S.phit[i];
        if (P.model == 1) {
          // conserved mixture c, then the equal-potential split at the new phi
          T divc = 0.0;
          for (int k = 0; k < P.dim; ++k) {
            T jp, jm;
            mixture_flux(P, w, g, phi, cs, cl, S, c, k, jp);
            bool periodic_axis = g.per[k] && k != g.dim - 1;
            if (!periodic_axis && c[k] == 0) {
              jm = 0.0;
            } else {
              int cm[3] = {c[0], c[1], c[2]};
              cm[k] = g.map(c[k] - 1, k);
              mixture_flux(P, w, g, phi, cs, cl, S, cm, k, jm);
            }
            divc = divc + (jp - jm) / P.dx;
          }
          T cmix = q.p * cs[i] + q.q * cl[i] + P.dt * divc;
          T pn = p_of(nphi[i], P.quintic, P.ap), qn = p_of(1.0 - nphi[i], P.quintic, P.ap);
          ncl[i] = cmix / (P.ke * pn + qn);
          ncs[i] = P.ke * ncl[i];
          continue;
        }
        T src = -w.A * q.dc * q.dp * S.phit[i];  // S g'(phi) phi_t with S = -A(c_s - c_l)
        ncs[i] = cs[i] + P.dt * (divs + src);
        ncl[i] = cl[i] + P.dt * (divl + src);
      }
  // Moving window.
  const double tn1 = (double)(n + 1) * P.dt;
  bool shift = std::floor(P.V * tn1 / P.dx) > (double)(*s_shift);
  if (shift) {
    int c[3];
    for (c[2] = 0; c[2] < g.n[2]; ++c[2])
      for (c[1] = 0; c[1] < g.n[1]; ++c[1])
        for (c[0] = 0; c[0] < g.n[0]; ++c[0]) {
          long i = g.lin(c);
          if (c[gz] == g.n[gz] - 1) {
            phi[i] = 0.0;
            cs[i] = P.ke;
            cl[i] = 1.0;
          } else {
            int cu[3] = {c[0], c[1], c[2]};
            cu[gz] += 1;
            long j = g.lin(cu);
            phi[i] = nphi[j];
            cs[i] = ncs[j];
            cl[i] = ncl[j];
          }
        }
    *s_shift += 1;
  } else {
    for (long i = 0; i < N; ++i) {
      phi[i] = nphi[i];
      cs[i] = ncs[i];
      cl[i] = ncl[i];
    }
  }
}

template <class T>
WP<T> make_wp(const OrcParams& P, T A, T Mphi, T W, T b) {
  WP<T> w;
  w.A = A;
  w.Mphi = Mphi;
  w.W = W;
  w.b = b;
  w.alpha = W / Mphi;     // tau D_l / W0^2 scales with W at fixed gamma and M_phi
  w.lambda = P.lambda0 * W;  // Omega c_inf / H scales with W at fixed gamma
  w.W2 = W * W;
  return w;
}

}  // namespace

extern "C" {

// Size of the parameter structure, so the Python side can check its layout.
int orc_params_size(void) { return (int)sizeof(OrcParams); }

// Advance the fields by nsteps steps starting at step index n0.  *s_shift is
// the window shift count (in/out).  Returns 0, or -1 on bad arguments.
int orc_step(const OrcParams* P, double* phi, double* cs, double* cl, long n0, long nsteps,
             int64_t* s_shift) {
  if (!P || !phi || !cs || !cl || !s_shift || P->dim < 1 || P->dim > 3) return -1;
  WP<double> w = make_wp<double>(*P, P->A, P->Mphi, P->W, P->b);
  for (long s = 0; s < nsteps; ++s) step_once(*P, w, phi, cs, cl, n0 + s, s_shift);
  return 0;
}

// Forward-mode directional derivative of nsteps steps.  (du_phi, du_cs, du_cl)
// is the input tangent (overwritten by the output tangent) and dtheta[4] the
// tangent of (A, Mphi, W, b).  The fields are advanced as in orc_step.
int orc_jvp(const OrcParams* P, double* phi, double* cs, double* cl, double* dphi, double* dcs,
            double* dcl, const double* dtheta, long n0, long nsteps, int64_t* s_shift) {
  if (!P || !phi || !cs || !cl || !dphi || !dcs || !dcl || !dtheta || !s_shift) return -1;
  Grid g = make_grid(*P);
  long N = g.ncell;
  std::vector<Dual> uphi(N), ucs(N), ucl(N);
  for (long i = 0; i < N; ++i) {
    uphi[i] = Dual(phi[i], dphi[i]);
    ucs[i] = Dual(cs[i], dcs[i]);
    ucl[i] = Dual(cl[i], dcl[i]);
  }
  WP<Dual> w = make_wp<Dual>(*P, Dual(P->A, dtheta[0]), Dual(P->Mphi, dtheta[1]), Dual(P->W, dtheta[2]),
                             Dual(P->b, dtheta[3]));
  for (long s = 0; s < nsteps; ++s) step_once(*P, w, uphi.data(), ucs.data(), ucl.data(), n0 + s, s_shift);
  for (long i = 0; i < N; ++i) {
    phi[i] = uphi[i].v;
    dphi[i] = uphi[i].d;
    cs[i] = ucs[i].v;
    dcs[i] = ucs[i].d;
    cl[i] = ucl[i].v;
    dcl[i] = ucl[i].d;
  }
  return 0;
}

// Discrete free energy F / (H W0^d) (Eqs. model1.1 and dil_linear; the term
// linear in the total solute and the pure-solvent reference are dropped):
//   dx^d sum_cells [ f_dw + lambda (p fs + (1-p) fl) ] + dx^d sum_faces W^2/2 ((phi_b - phi_a)/dx)^2
//   fs = c_s ln c_s - c_s - c_s ln k_e + (k_e - 1) c_l^eq(z, t),  fl = c_l ln c_l - c_l.
double orc_energy(const OrcParams* P, const double* phi, const double* cs, const double* cl, long n,
                  int64_t s_shift) {
  Grid g = make_grid(*P);
  const int gz = P->dim - 1;
  const double t = (double)n * P->dt;
  const double lam = P->lambda0 * P->W;
  double vol = 1.0;
  for (int k = 0; k < P->dim; ++k) vol *= P->dx;
  double bulk = 0.0, grad = 0.0;
  int c[3];
  for (c[2] = 0; c[2] < g.n[2]; ++c[2])
    for (c[1] = 0; c[1] < g.n[1]; ++c[1])
      for (c[0] = 0; c[0] < g.n[0]; ++c[0]) {
        long i = g.lin(c);
        double zlab = ((double)c[gz] + (double)s_shift + 0.5) * P->dx;
        double p = p_of(phi[i], P->quintic, P->ap);
        double fs = cs[i] * std::log(cs[i]) - cs[i] - cs[i] * std::log(P->ke) +
                    (P->ke - 1.0) * cleq_of(*P, zlab, t);
        double fl = cl[i] * std::log(cl[i]) - cl[i];
        double fdw = phi[i] * phi[i] * (1.0 - phi[i]) * (1.0 - phi[i]);
        bulk += fdw + lam * (p * fs + (1.0 - p) * fl);
        for (int k = 0; k < P->dim; ++k) {
          bool periodic_axis = g.per[k] && k != g.dim - 1;
          if (!periodic_axis && c[k] == g.n[k] - 1) continue;
          double d = (phi[g.at(c, k, +1)] - phi[i]) / P->dx;
          grad += 0.5 * P->W * P->W * d * d;
        }
      }
  return vol * (bulk + grad);
}

// Total solute dx^d sum c with c = p c_s + (1-p) c_l (Eq. model1 with g = p),
// its maximum and the first index attaining it.
int orc_solute(const OrcParams* P, const double* phi, const double* cs, const double* cl, double* total,
               double* cmax, long* argmax) {
  Grid g = make_grid(*P);
  double vol = 1.0;
  for (int k = 0; k < P->dim; ++k) vol *= P->dx;
  double sum = 0.0, mx = -INFINITY;
  long am = -1;
  for (long i = 0; i < g.ncell; ++i) {
    double p = p_of(phi[i], P->quintic, P->ap);
    double c = p * cs[i] + (1.0 - p) * cl[i];
    sum += c;
    if (c > mx) {
      mx = c;
      am = i;
    }
  }
  if (total) *total = vol * sum;
  if (cmax) *cmax = mx;
  if (argmax) *argmax = am;
  return 0;
}

// Solidification front (the phi = 1/2 level set) and its temperature, the
// interface diagnostics of Sec. V.C (interface temperature T_I, read where
// phi crosses one half).  In every growth-axis column (solid below, liquid
// above) the front is the topmost crossing: the largest i with
// phi_i >= 1/2 > phi_{i+1}, placed by linear interpolation between the two
// cell centres, in lab coordinates z = (i + s + 1/2) dx + dx (phi_i - 1/2) /
// (phi_i - phi_{i+1}) with s the window shift count.  Over the columns that
// have a crossing: out = [mean z, min z, max z, (mean z - z0 - V t_n) / l_T,
// number of such columns]; the fourth entry is (T_I - T_s) / dT0 of the
// frozen temperature (Eq. ds1 with dT0 = G l_T, T_s the solidus of c_inf).
// NaN for the first four when no column has a crossing.
int orc_front(const OrcParams* P, const double* phi, long n, int64_t s_shift, double* out) {
  Grid g = make_grid(*P);
  const int gz = P->dim - 1;
  const int nz = g.n[gz];
  long ncol = 1;
  for (int k = 0; k < gz; ++k) ncol *= g.n[k];
  double sum = 0.0, zmin = INFINITY, zmax = -INFINITY;
  long cnt = 0;
  for (long col = 0; col < ncol; ++col) {
    for (int i = nz - 2; i >= 0; --i) {
      const double a = phi[col + ncol * (long)i], b = phi[col + ncol * (long)(i + 1)];
      if (a >= 0.5 && b < 0.5) {
        const double z = ((double)i + (double)s_shift + 0.5) * P->dx + P->dx * (a - 0.5) / (a - b);
        sum += z;
        zmin = std::min(zmin, z);
        zmax = std::max(zmax, z);
        ++cnt;
        break;
      }
    }
  }
  if (cnt == 0) {
    out[0] = out[1] = out[2] = out[3] = NAN;
  } else {
    out[0] = sum / (double)cnt;
    out[1] = zmin;
    out[2] = zmax;
    out[3] = (out[0] - P->z0 - P->V * ((double)n * P->dt)) * P->inv_lT;
  }
  out[4] = (double)cnt;
  return 0;
}

// Face fluxes for tests: for every cell c, the solid and liquid fluxes
// (the brackets of Eqs. cs_nonvar, cl_nonvar, in the sign convention
// d c / dt = div J + sources) and the mixture flux of Eq. solute_nonvar
// (mixture_flux, the equal-potential model's flux) through the face between c
// and c + e_k, and p at that face.  Boundary faces of non-periodic axes give
// zero.  Computed from the state at step n (shift count s) with the cell-stage
// quantities of that step.
int orc_face_fluxes(const OrcParams* P, const double* phi, const double* cs, const double* cl, long n,
                    int64_t s_shift, int k, double* js, double* jl, double* jmix, double* pface) {
  if (!P || k < 0 || k >= P->dim) return -1;
  Grid g = make_grid(*P);
  WP<double> w = make_wp<double>(*P, P->A, P->Mphi, P->W, P->b);
  StepWork<double> S;
  cell_stage(*P, w, g, phi, cs, cl, (double)n * P->dt, s_shift, S);
  int c[3];
  for (c[2] = 0; c[2] < g.n[2]; ++c[2])
    for (c[1] = 0; c[1] < g.n[1]; ++c[1])
      for (c[0] = 0; c[0] < g.n[0]; ++c[0]) {
        long i = g.lin(c);
        double a = 0.0, b = 0.0, m = 0.0;
        bool inner = face_flux(*P, w, g, phi, cs, cl, S, c, k, a, b);
        mixture_flux(*P, w, g, phi, cs, cl, S, c, k, m);
        if (js) js[i] = a;
        if (jl) jl[i] = b;
        if (jmix) jmix[i] = m;
        if (pface) pface[i] = inner ? p_of(0.5 * (phi[i] + phi[g.at(c, k, +1)]), P->quintic, P->ap) : 0.0;
      }
  return 0;
}

// Pointwise quantities for tests: out = [h, p, p', f_dw', dmu, mubar, dG].
int orc_pointwise(const OrcParams* P, double phi, double cs, double cl, double cleq, double* out) {
  WP<double> w = make_wp<double>(*P, P->A, P->Mphi, P->W, P->b);
  Pointwise<double> q = pointwise(*P, w, phi, cs, cl, cleq);
  out[0] = h_of(phi, P->quintic);
  out[1] = q.p;
  out[2] = q.dp;
  out[3] = dfdw_of(phi);
  out[4] = q.dmu;
  out[5] = q.mubar;
  out[6] = q.dG;
  return 0;
}

// phi_t on the whole grid (no update), for tests.
int orc_phi_t(const OrcParams* P, const double* phi, const double* cs, const double* cl, long n,
              int64_t s_shift, double* phit) {
  Grid g = make_grid(*P);
  WP<double> w = make_wp<double>(*P, P->A, P->Mphi, P->W, P->b);
  StepWork<double> S;
  cell_stage(*P, w, g, phi, cs, cl, (double)n * P->dt, s_shift, S);
  for (long i = 0; i < g.ncell; ++i) phit[i] = S.phit[i];
  return 0;
}

}  // extern "C"
