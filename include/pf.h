/*
 * pf.h -- C ABI of the MI355X (gfx950) library for the explicit time stepping
 * of the variational phase-field model of rapid alloy solidification of
 * Mukherjee, Warren & Voorhees (arXiv 2303.09671).
 *
 * The library advances the phase field phi (1 = solid, 0 = liquid) and the
 * separate solid and liquid concentrations c_s, c_l of a dilute binary alloy on
 * a uniform 1D/2D/3D grid under directional solidification.  One step is the
 * forward-Euler update of the set-2 equations of motion (Sec. II, Eqs.
 * cs_nonvar, cl_nonvar and phasefield_nonvar, with the drive of Eq. model18),
 * discretised on a staggered grid with face-centred mobilities and
 * anti-trapping terms (Sec. V.A), for the dilute ideal alloy of Sec. III
 * (Eqs. dil1, dil5.1, dil5.2) in the frozen temperature field of Eq. ds1, with
 * the moving-window shift of Sec. V.A.
 *
 * Units (supplement Sec. S-II): lengths in the reference width W0, time in
 * W0^2/D_l, concentrations in c_inf, energies in H.
 *
 * Memory: every field pointer is DEVICE memory owned by the caller: contiguous
 * float64 arrays, structure of arrays, x fastest.  The growth axis is always the
 * last axis: 1D [N]; 2D [nz][nx]; 3D [nz][ny][nx].  Batched mode (dim = 1,
 * nbatch > 0) concatenates nbatch independent 1D runs; run r occupies
 * [run_off[r], run_off[r] + run_n[r]).  The library owns its scratch (a twin of
 * the fields for ping-pong, reduction partials, an error word).
 *
 * Streams: all device work of a handle is enqueued on the hipStream_t given to
 * pf_create.  Calls returning host values synchronise that stream.  A handle is
 * not thread-safe: use it from one host thread at a time.
 *
 * Errors: every call returns PF_OK (0) or a negative code; no exception crosses
 * the ABI.  pf_strerror gives a message; pf_last_error_detail the most recent
 * detail text of this thread.
 */
#ifndef PF_H
#define PF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PF_OK = 0,
  PF_EINVAL = -1,        /* bad argument or parameter set (incl. q_n < 0)     */
  PF_EUNSTABLE_DT = -2,  /* dt above the explicit stability bound             */
  PF_ENONFINITE = -3,    /* a NaN/Inf appeared in the fields                   */
  PF_ENEGCONC = -4,      /* c_s or c_l became <= 0 (log undefined)             */
  PF_EDEVICE = -5,       /* a HIP runtime call failed                          */
  PF_ENOMEM = -6         /* device allocation failed                           */
};

/* Model and grid parameters (nondimensional).  Field order is ABI. */
typedef struct pf_params {
  int32_t dim;          /* 1, 2 or 3; the growth axis is the last axis            */
  int32_t n[3];         /* cells per axis, axis 0 fastest (1D: n[0] = N)           */
  int32_t periodic[3];  /* transverse axes only: 1 periodic, 0 no-flux (mirror)    */
  int32_t quintic;      /* 1: h = phi^3(6 phi^2 - 15 phi + 10); 0: phi^2 (3 - 2 phi) */
  int32_t shift;        /* 1: moving window (Sec. V.A); 0: fixed frame              */
  int32_t check_every;  /* >0: pf_step syncs every check_every steps and reports  */
                        /*     PF_ENONFINITE / PF_ENEGCONC; 0: fully asynchronous   */
  double dx, dt;        /* grid spacing, time step                                  */
  double W;             /* interface width / W0                  (theta[2])         */
  double Mphi;          /* phi mobility, alpha = W / Mphi        (theta[1])         */
  double lambda0;       /* Omega c_inf / H at W = W0; lambda = lambda0 * W          */
  double Ds;            /* D_s / D_l                                               */
  double ke;            /* equilibrium partition coefficient, 0 < k_e < 1           */
  double A;             /* source coefficient S = -A (c_s - c_l)  (theta[0])        */
  double b, ap;         /* set-2 interpolation constants (Eqs. interpolation1, 2)   */
  double inv_lT;        /* 1 / thermal length l_T = dT0 / G (0: isothermal at T_s)  */
  double V;             /* pulling speed (single domain)                            */
  double z0;            /* initial front height (lab frame)                         */
  double eps_grad;      /* eps of 1/|grad phi|^2 ~ G / (G^2 + eps^2), G = |grad phi|^2 */
  /* batched 1D runs: nbatch > 0 and dim == 1.  Host arrays, copied by pf_create. */
  int32_t nbatch;
  int32_t model;        /* 0: set-2 equations, separate kinetics of c_s and c_l (above);
                         * 1: equal diffusion potentials imposed pointwise, mu_s = mu_l
                         *    (the model of the asymptotic analysis, Sec. II.C; with A = 1
                         *    and b = k_e D_s/D_l the KKS model, Sec. IV, Eqs. KKS1, KKS2):
                         *    phi_t from Eq. phasefield_nonvar with mu_s = mu_l, the mixture
                         *    c = p c_s + (1-p) c_l conserved with the flux of Eq.
                         *    solute_nonvar, and after every step c_l = c / (k_e p + 1 - p),
                         *    c_s = k_e c_l (Eq. dil1).  The fields keep the (phi, c_s, c_l)
                         *    layout, but the state is (phi, c_l): c_s on input is not read
                         *    (taken as k_e c_l) and is written after every step.  The
                         *    adjoint entry points return PF_EINVAL for model 1.           */
  const int32_t* run_n;    /* cells of run r (3 <= run_n[r] <= 8192)               */
  const int64_t* run_off;  /* first cell of run r in the field arrays              */
  const double* run_V;     /* pulling speed of run r                               */
  const double* run_dt;    /* time step of run r                                   */
  const double* run_z0;    /* initial front height of run r                        */
} pf_params;

typedef struct pf_handle pf_handle;

/* Create a handle over caller-owned device fields phi, cs, cl (see layout
 * above) and the HIP stream `stream` (NULL = default stream) for the problem
 * of Secs. II-III: the set-2 equations of motion (Eqs. cs_nonvar, cl_nonvar,
 * phasefield_nonvar) of a dilute alloy (Eq. dil1) in the frozen temperature
 * field of Eq. ds1, discretised as in Sec. V.A.  Validates the parameters:
 * PF_EINVAL for a bad grid or model constants (0 < k_e < 1, D_s, W, M_phi,
 * lambda0, dx, dt > 0, b > 0, b p + 1 - p > 0 and q_n >= 0 over phi in [0, 1],
 * transverse planes of at most 2^28 cells); PF_EUNSTABLE_DT if dt exceeds
 * 0.9 min(dx^2/(2 d max(1, D_s)), alpha dx^2/(2 d W^2), 0.2 dx/V) per run.
 * The step counter starts at 0.  On success *out receives the handle.
 *
 * Regime (measured, not checked here): the bound above covers diffusion, phi
 * relaxation and window advection only.  Where the phase field flattens inside
 * an interface, the (1-A)^2 term of the phi prefactor and the anti-trapping
 * flux grow as 1/|grad phi|^2 and phi_t/|grad phi|; with |1 - A| of order one
 * (the paper's A = 2) and a gate scale eps_grad well below 1e-3 this diverges
 * from an undercooled start within tens of steps at any dt (the error word
 * then reports PF_ENEGCONC or PF_ENONFINITE).  eps_grad = 3e-3 steps A = 2 on
 * the 1D, 2D, 3D, k(V) and band workloads; slow steady fronts (V ~ 0.005) at
 * A = 2 can still fail after ~1e4 steps through a ghost-concentration
 * oscillation. */
int pf_create(const pf_params* p, double* phi, double* cs, double* cl, void* stream, pf_handle** out);

/* Advance the fields by nsteps explicit forward-Euler steps of the staggered
 * scheme (Sec. V.A), with the moving-window shift of Sec. V.A (asynchronous on
 * the stream unless check_every > 0).  After the stream is synchronised the caller's
 * buffers hold the state at step n + nsteps.  1D single runs and batches run
 * as one persistent launch per call; 2D/3D as one fused launch per step. */
int pf_step(pf_handle* h, int64_t nsteps);

/* Same as pf_step but also records the state before every step:
 * traj[f] + k * stride (f = phi, c_s, c_l; k = 0..nsteps) receives the state at
 * step n + k (device buffers of (nsteps + 1) * stride doubles, stride >= the
 * field length).  Used to replay a checkpoint segment for the adjoint. */
int pf_step_traj(pf_handle* h, int64_t nsteps, double* traj_phi, double* traj_cs, double* traj_cl,
                 int64_t stride);

/* Step counter n (the window shift count is floor(V n dt / dx) per run). */
int pf_get_step(const pf_handle* h, int64_t* n);
int pf_set_step(pf_handle* h, int64_t n);

/* Discrete free energy F / (H W0^d) at the current step (Eqs. model1.1,
 * dil_linear; terms linear in the total solute dropped): one value, or one per
 * run in batched mode, written to the HOST array out.  Synchronous. */
int pf_energy(pf_handle* h, double* out);

/* Total solute dx^d sum (p c_s + (1-p) c_l), its maximum c_max and the first
 * linear index attaining it (per run in batched mode; the index is relative to
 * the run's first cell).  HOST outputs; any pointer may be NULL.  The
 * partition coefficient of Sec. V.C is k = 1 / c_max.  Synchronous. */
int pf_solute(pf_handle* h, double* total, double* cmax, int64_t* argmax);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of pf_solute and pf_energy for one domain (nbatch = 0), without
 * a handle and without any allocation.  p describes the grid and model as for
 * pf_create; phi, cs, cl are the caller's device fields in that layout,
 * holding the state of step n (which sets t_n and the shift count of the
 * frozen temperature in the energy).  Outputs are DEVICE scalars written
 * asynchronously on `stream` (NULL = default stream); any of them may be NULL:
 * total solute dx^d sum (p c_s + (1-p) c_l), c_max and its first linear index,
 * and the free energy F / (H W0^d).  The reduction partials live in a static
 * device array of the library (2 MiB per GPU, held until the process ends):
 * grids of more than 2^28 cells are rejected with PF_EINVAL.  Every call on a
 * GPU uses that GPU's one array, so calls that overlap in time on one GPU
 * (other streams or host threads) race; calls ordered on one stream do not.
 * Errors: PF_EINVAL for bad parameters (as pf_create), PF_EDEVICE for a HIP
 * error. */
int pf_solute_noalloc(const pf_params* p, const double* phi, const double* cs, const double* cl, int64_t n,
                      void* stream, double* total, double* cmax, int64_t* argmax, double* energy);

/* Solidification front and interface temperature (Sec. V.C reads the
 * interface temperature where phi = 1/2): in every growth-axis column the
 * topmost crossing -- the largest i with phi_i >= 1/2 > phi_{i+1} -- placed by
 * linear interpolation between the two cell centres, in lab coordinates
 * z = (i + s + 1/2) dx + dx (phi_i - 1/2) / (phi_i - phi_{i+1}) (s = window
 * shift count of the current step).  Per run in batched mode (one column), else
 * over the columns of the domain that cross: z_mean, z_min, z_max, the
 * temperature T_front = (z_mean - z0 - V t_n) / l_T = (T_I - T_s) / dT0 of the
 * frozen temperature field, and the number of crossing columns (0, with NaN
 * heights and temperature, when nothing crosses).  HOST outputs (nbatch values,
 * or 1); any pointer may be NULL.  Synchronous. */
int pf_front(pf_handle* h, double* z_mean, double* z_min, double* z_max, double* T_front, int64_t* ncol);

/* Error word of the fields since creation (or the last call of this
 * function): PF_OK, PF_ENONFINITE or PF_ENEGCONC.  Synchronous; clears it. */
int pf_check(pf_handle* h);

/* Adjoint of one step (transpose of the Jacobian of step n -> n + 1) of model 0
 * (Eqs. cs_nonvar, cl_nonvar, phasefield_nonvar as discretised by pf_step):
 *   lam_n = (d u^{n+1} / d u^n)^T lam_np1,
 *   dtheta += (d u^{n+1} / d theta)^T lam_np1,  theta = (A, M_phi, W, b),
 * with alpha = W / M_phi and lambda = lambda0 W (gamma, Omega, D and the grid
 * fixed) and b the mobility-interpolation constant of Eq. interpolation1 (the
 * three fitting constants of Sec. V.D are A, b and W).  u_n[f], lam_np1[f],
 * lam_n[f] (f = phi, c_s, c_l) are device arrays in the field layout; lam_n
 * may not alias lam_np1.  dtheta is a device double[4], accumulated.  The
 * window shift of step n is held fixed (it is
 * piecewise constant in theta).  Built for 1D runs and 2D grids (3D:
 * PF_EINVAL).  Asynchronous on the stream. */
int pf_adjoint_step(pf_handle* h, int64_t n, const double* const u_n[3], const double* const lam_np1[3],
                    double* const lam_n[3], double* dtheta);

/* The adjoint over a checkpoint segment: m steps of pf_adjoint_step taken
 * backwards, n = n0 + m - 1 down to n0, in one call.  Row j (j = 0..m-1) of the
 * device trajectory traj_*[j * stride + i] holds the state at step n0 + j (as
 * written by pf_step_traj; stride >= the field size).  On entry lam[f] holds
 * lam^{n0+m}, on return lam^{n0}; work[f] are caller-owned device arrays of the
 * field size used for the ping-pong (contents undefined afterwards; they may
 * not alias lam).  dtheta (device double[4]) is accumulated once for the whole
 * segment: the per-block sums are carried over the m steps and reduced at the
 * end, so the result equals the sum of m pf_adjoint_step calls up to rounding
 * order.  Asynchronous on the stream. */
int pf_adjoint_segment(pf_handle* h, int64_t n0, int64_t m, const double* traj_phi, const double* traj_cs,
                       const double* traj_cl, int64_t stride, double* const lam[3], double* const work[3],
                       double* dtheta);

/* Adjoint seed of the partition-coefficient loss: for every run r (or the
 * single domain) with k_r = 1 / c_max, writes lam[f] = sum_r dL_dk[r] dk_r/du[f]
 * at the first cell attaining c_max and zero elsewhere (dk/dc_s = -p/c_max^2,
 * dk/dc_l = -(1-p)/c_max^2, dk/dphi = -p' (c_s - c_l)/c_max^2).  dL_dk is a
 * HOST array (nbatch values, or 1); lam[3] are device arrays.  Synchronous. */
int pf_kv_seed(pf_handle* h, const double* dL_dk, double* const lam[3]);

void pf_destroy(pf_handle* h);
const char* pf_strerror(int code);
const char* pf_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
