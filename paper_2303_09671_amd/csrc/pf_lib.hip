// pf_lib.hip -- host side of the C ABI declared in include/pf.h (gfx950).
//
// Parameter validation and stability checks, device scratch, launch
// geometry, the window-shift schedule and the deterministic reductions.  All
// arithmetic of the method runs in the kernels of pf_kernels.h / pf_adjoint.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "pf.h"
#include "pf_kernels.h"
#include "pf_adjoint.h"

namespace {

thread_local std::string g_detail;

int fail(int code, const std::string& msg) {
  g_detail = msg;
  return code;
}

#define PF_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(PF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

// Launch geometry of the streaming kernel: in-plane tiles; the z range of a
// grid column is cut into chunks so that the launch holds about `target`
// workgroups (prologue cost: two extra planes of cell rates per chunk).
constexpr int S3_TX = 32, S3_TY = 8;  // 3D: 256 threads (4 waves), 3 workgroups per CU
constexpr int S2_TX = 62;             // 2D: 62 columns + 2 halo columns = 64 threads (1 wave)

int zchunk_for(int nz, long long tiles, long long target, int zmin) {
  long long split = std::max<long long>(1, (target + tiles - 1) / tiles);
  int zc = (int)((nz + split - 1) / split);
  return std::max(std::min(zc, nz), std::min(zmin, nz));
}

}  // namespace

struct pf_handle {
  pf_params p{};
  pfk::Const c{};
  hipStream_t stream = nullptr;
  double* f[3] = {nullptr, nullptr, nullptr};   // caller's fields
  double* tw[3] = {nullptr, nullptr, nullptr};  // twin (ping-pong), 2D/3D only
  long long ntot = 0;                           // doubles per field
  int batched = 0;                              // 1D (single or batched): persistent kernel
  int nrun = 1;
  std::vector<int> h_n;
  std::vector<long long> h_off;
  std::vector<double> h_V, h_dt, h_z0;
  int* d_n = nullptr;
  long long* d_off = nullptr;
  double *d_V = nullptr, *d_dt = nullptr, *d_z0 = nullptr;
  int* d_order = nullptr;
  // reductions
  int nchunk = 0;
  int* d_chunk_run = nullptr;
  long long* d_chunk_beg = nullptr;
  int* d_run_chunk0 = nullptr;
  pfk::Partial* d_part = nullptr;
  pfk::Partial* d_runred = nullptr;
  double* d_dldk = nullptr;
  double* d_theta_part = nullptr;  // adjoint: per-block parameter cotangents
  int ntheta_part = 0;
  pfadj::Tile1* d_tiles = nullptr;   // adjoint: (run, tile) table of 1D runs
  int ntiles = 0;
  int* d_err = nullptr;
  double* d_front = nullptr;      // front diagnostic: 5 values per run
  double* d_front_col = nullptr;  // 2D/3D: crossing height per column
  int zchunk = 32;  // z planes per workgroup of the streaming kernel
  long long n = 0;  // step counter

  pfk::RunTab runtab() const {
    pfk::RunTab t;
    t.n = d_n;
    t.off = d_off;
    t.V = d_V;
    t.dt = d_dt;
    t.z0 = d_z0;
    t.order = d_order;
    return t;
  }
  pfk::RedTab redtab() const {
    pfk::RedTab t;
    t.chunk_run = d_chunk_run;
    t.chunk_beg = d_chunk_beg;
    t.run_chunk0 = d_run_chunk0;
    t.nchunk = nchunk;
    return t;
  }
};

namespace {

template <class T>
int dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(PF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return PF_OK;
}

template <class T>
int upload(T** d, const std::vector<T>& h, hipStream_t s) {
  int rc = dalloc(d, h.size());
  if (rc) return rc;
  PF_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return PF_OK;
}

double dt_bound(const pf_params& p, double V) {
  const double alpha = p.W / p.Mphi;
  const double d = (double)p.dim;
  double b = std::min(p.dx * p.dx / (2.0 * d * std::max(1.0, p.Ds)), alpha * p.dx * p.dx / (2.0 * d * p.W * p.W));
  if (p.shift && V > 0.0) b = std::min(b, 0.2 * p.dx / V);
  return 0.9 * b;
}

// q_n >= 0 and b p + 1 - p > 0 on phi in [0, 1] (Eqs. normal2, interpolation1).
bool interp_admissible(const pf_params& p) {
  for (int i = 0; i <= 2000; ++i) {
    const double phi = i / 2000.0;
    const double om = 1.0 - phi, w = phi * om;
    double h, hq;
    if (p.quintic) {
      h = phi * phi * phi * (phi * (6.0 * phi - 15.0) + 10.0);
      hq = om * om * om * (om * (6.0 * om - 15.0) + 10.0);
    } else {
      h = phi * phi * (3.0 - 2.0 * phi);
      hq = om * om * (3.0 - 2.0 * om);
    }
    const double a = p.ap * (phi - 0.5) * w * w;
    const double pp = h + a, qq = hq - a;
    if (!(p.b * pp + qq > 0.0)) return false;
    // Mbar = D_s c_s q + b c_l p must stay positive for positive concentrations
    if (pp < -1e-12 || qq < -1e-12) return false;
  }
  return true;
}

int validate(const pf_params& p) {
  if (p.dim < 1 || p.dim > 3) return fail(PF_EINVAL, "dim must be 1, 2 or 3");
  if (p.nbatch == 0) {  // batched runs carry their own lengths
    for (int k = 0; k < p.dim; ++k)
      if (p.n[k] < 1) return fail(PF_EINVAL, "n[k] must be >= 1");
    if (p.n[p.dim - 1] < 3) return fail(PF_EINVAL, "the growth axis needs at least 3 cells");
    long long tr = 1;  // cells of one transverse plane: indexed with 32-bit offsets
    for (int k = 0; k + 1 < p.dim; ++k) tr *= p.n[k];
    if (tr > (1LL << 28)) return fail(PF_EINVAL, "a transverse plane must hold at most 2^28 cells");
  }
  if (!(p.dx > 0) || !(p.dt > 0) || !(p.W > 0) || !(p.Mphi > 0) || !(p.lambda0 > 0) || !(p.Ds > 0) ||
      !(p.b > 0))
    return fail(PF_EINVAL, "dx, dt, W, Mphi, lambda0, Ds and b must be > 0");
  if (!(p.ke > 0 && p.ke < 1)) return fail(PF_EINVAL, "k_e must lie in (0, 1)");
  if (!(p.eps_grad >= 0) || !std::isfinite(p.inv_lT) || !std::isfinite(p.V) || !std::isfinite(p.z0) ||
      !std::isfinite(p.A) || !std::isfinite(p.ap))
    return fail(PF_EINVAL, "non-finite parameter");
  if (!interp_admissible(p)) return fail(PF_EINVAL, "b and a_p give q_n < 0 or p outside [0, 1]");
  if (p.model != 0 && p.model != 1) return fail(PF_EINVAL, "model must be 0 or 1");
  if (p.nbatch < 0) return fail(PF_EINVAL, "nbatch < 0");
  if (p.nbatch > 0) {
    if (p.dim != 1) return fail(PF_EINVAL, "batched mode needs dim == 1");
    if (!p.run_n || !p.run_off || !p.run_V || !p.run_dt || !p.run_z0)
      return fail(PF_EINVAL, "batched mode needs run_n, run_off, run_V, run_dt and run_z0");
  }
  return PF_OK;
}

pfk::Const make_const(const pf_params& p) {
  pfk::Const c{};
  c.dim = p.dim;
  c.nz = p.n[p.dim - 1];
  c.nx = (p.dim >= 2) ? p.n[0] : 1;
  c.ny = (p.dim == 3) ? p.n[1] : 1;
  c.px = (p.dim >= 2) ? (p.periodic[0] != 0) : 0;
  c.py = (p.dim == 3) ? (p.periodic[1] != 0) : 0;
  c.quintic = p.quintic ? 1 : 0;
  c.ncell = (long long)c.nx * c.ny * c.nz;
  c.dx = p.dx;
  c.inv_dx = 1.0 / p.dx;
  c.inv_2dx = 1.0 / (2.0 * p.dx);
  c.inv_4dx = 1.0 / (4.0 * p.dx);
  c.inv_dx2 = 1.0 / (p.dx * p.dx);
  c.dt = p.dt;
  c.W = p.W;
  c.W2 = p.W * p.W;
  c.Mphi = p.Mphi;
  c.alpha = p.W / p.Mphi;
  c.lambda0 = p.lambda0;
  c.lambda = p.lambda0 * p.W;
  c.Ds = p.Ds;
  c.ke = p.ke;
  c.log_ke = std::log(p.ke);
  c.A = p.A;
  c.onemA = 1.0 - p.A;
  c.b = p.b;
  c.ap = p.ap;
  c.inv_lT = p.inv_lT;
  c.V = p.V;
  c.z0 = p.z0;
  c.eps_grad = p.eps_grad;
  c.eps2 = p.eps_grad * p.eps_grad;
  c.eps2s = c.eps2 * (p.dx * p.dx) * (p.dx * p.dx);
  c.onemA_dx2 = (1.0 - p.A) * p.dx * p.dx;
  c.inv_ke = 1.0 / p.ke;
  c.W2_dx2 = c.W2 / (p.dx * p.dx);
  c.eps2r = 16.0 * c.eps2s;
  c.onemA_4dx2 = 4.0 * c.onemA_dx2;
  return c;
}

int read_err(pf_handle* h, bool clear) {
  int e = 0;
  PF_HIP(hipMemcpyAsync(&e, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  PF_HIP(hipStreamSynchronize(h->stream));
  if (clear && e) {
    int z = 0;
    PF_HIP(hipMemcpyAsync(h->d_err, &z, sizeof(int), hipMemcpyHostToDevice, h->stream));
    PF_HIP(hipStreamSynchronize(h->stream));
  }
  if (e & pfk::ERR_NONFINITE) return fail(PF_ENONFINITE, "a NaN or Inf appeared in the fields");
  if (e & pfk::ERR_NEGCONC) return fail(PF_ENEGCONC, "c_s or c_l became <= 0");
  return PF_OK;
}

// Launch the 2D/3D fused step n -> n+1 from src to dst.
int launch_stream(pf_handle* h, double* const src[3], double* const dst[3], long long n) {
  const pfk::Const& c = h->c;
  const double tn = (double)n * c.dt;
  const double sn = std::floor(c.V * tn / c.dx);
  const int sh = (h->p.shift && std::floor(c.V * ((double)(n + 1) * c.dt) / c.dx) > sn) ? 1 : 0;
  const bool apz = (c.ap == 0.0), eq = (h->p.model == 1);
  if (c.dim == 3) {
    const int zc = h->zchunk;
    dim3 grid((c.nx + S3_TX - 1) / S3_TX, (c.ny + S3_TY - 1) / S3_TY, (c.nz + zc - 1) / zc);
    auto k = eq ? (apz ? pfk::k_stream<3, S3_TX, S3_TY, true, true> : pfk::k_stream<3, S3_TX, S3_TY, false, true>)
                : (apz ? pfk::k_stream<3, S3_TX, S3_TY, true, false> : pfk::k_stream<3, S3_TX, S3_TY, false, false>);
    hipLaunchKernelGGL(k, grid, dim3(S3_TX * S3_TY), 0, h->stream, c, src[0], src[1], src[2], dst[0], dst[1],
                       dst[2], zc, tn, sn, sh, h->d_err);
  } else {
    const int zc = h->zchunk;
    dim3 grid((c.nx + S2_TX - 1) / S2_TX, 1, (c.nz + zc - 1) / zc);
    auto k = eq ? (apz ? pfk::k_stream<2, S2_TX, 1, true, true> : pfk::k_stream<2, S2_TX, 1, false, true>)
                : (apz ? pfk::k_stream<2, S2_TX, 1, true, false> : pfk::k_stream<2, S2_TX, 1, false, false>);
    hipLaunchKernelGGL(k, grid, dim3(S2_TX + 2), 0, h->stream, c, src[0], src[1], src[2], dst[0], dst[1], dst[2],
                       zc, tn, sn, sh, h->d_err);
  }
  PF_HIP(hipGetLastError());
  return PF_OK;
}

int reduce(pf_handle* h) {
  hipLaunchKernelGGL(pfk::k_reduce_chunks, dim3(h->nchunk), dim3(pfk::RED_THREADS), 0, h->stream, h->c,
                     h->runtab(), h->redtab(), h->f[0], h->f[1], h->f[2], h->n, h->batched, h->d_part);
  PF_HIP(hipGetLastError());
  hipLaunchKernelGGL(pfk::k_reduce_runs, dim3(h->nrun), dim3(pfk::RED_THREADS), 0, h->stream, h->c, h->redtab(),
                     h->d_part, h->d_runred);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

int fill(pf_handle* h, double* a, double v, long long n) {
  long long blocks = std::min<long long>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(pfk::k_fill, dim3((unsigned)blocks), dim3(256), 0, h->stream, a, v, n);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

// Reduction partials of pf_solute_noalloc: one Partial per chunk of RED_CHUNK
// cells plus the reduced result, in a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  Host code uses
// only the address hipGetSymbolAddress returns for the current device, never
// the array's name.
constexpr long long NOALLOC_MAX_CHUNKS = 65536;  // up to 2^28 cells (2 MiB)
__device__ __align__(256) pfk::Partial scratch[NOALLOC_MAX_CHUNKS + 1];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[NOALLOC_MAX_DEVICES];

// Address of the current device's scratch array, looked up once per device.
int scratch_ptr(pfk::Partial** out) {
  int dev = 0;
  PF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(PF_EDEVICE, "device index beyond the scratch table");
  ScratchSlot& s = g_scratch[dev];
  std::call_once(s.once, [&s] { s.err = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch)); });
  if (s.err != hipSuccess || !s.ptr)
    return fail(PF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(s.err));
  *out = (pfk::Partial*)s.ptr;
  return PF_OK;
}

}  // namespace

extern "C" {

int pf_create(const pf_params* p, double* phi, double* cs, double* cl, void* stream, pf_handle** out) {
  if (!p || !phi || !cs || !cl || !out) return fail(PF_EINVAL, "null argument");
  *out = nullptr;
  int rc = validate(*p);
  if (rc) return rc;
  pf_handle* h = new pf_handle();
  h->p = *p;
  h->c = make_const(*p);
  h->stream = (hipStream_t)stream;
  h->f[0] = phi;
  h->f[1] = cs;
  h->f[2] = cl;
  h->batched = (p->dim == 1) ? 1 : 0;
  if (p->dim == 1) {
    if (p->nbatch > 0) {
      h->nrun = p->nbatch;
      for (int r = 0; r < p->nbatch; ++r) {
        h->h_n.push_back(p->run_n[r]);
        h->h_off.push_back(p->run_off[r]);
        h->h_V.push_back(p->run_V[r]);
        h->h_dt.push_back(p->run_dt[r]);
        h->h_z0.push_back(p->run_z0[r]);
      }
    } else {
      h->nrun = 1;
      h->h_n.push_back(p->n[0]);
      h->h_off.push_back(0);
      h->h_V.push_back(p->V);
      h->h_dt.push_back(p->dt);
      h->h_z0.push_back(p->z0);
    }
    long long tot = 0;
    for (int r = 0; r < h->nrun; ++r) {
      if (h->h_n[r] < 3 || h->h_n[r] > pfk::R1_THREADS * pfk::R1_CMAX) {
        delete h;
        return fail(PF_EINVAL, "1D runs need 3 <= N <= 8192 cells");
      }
      if (h->h_off[r] < 0 || !(h->h_dt[r] > 0) || !std::isfinite(h->h_V[r])) {
        delete h;
        return fail(PF_EINVAL, "bad run table entry");
      }
      const double bound = dt_bound(*p, h->h_V[r]);
      if (h->h_dt[r] > bound) {
        delete h;
        char buf[160];
        snprintf(buf, sizeof buf, "run %d: dt = %g exceeds the stability bound %g", r, h->h_dt[r], bound);
        return fail(PF_EUNSTABLE_DT, buf);
      }
      tot = std::max(tot, h->h_off[r] + (long long)h->h_n[r]);
    }
    h->ntot = tot;
  } else {
    if (p->nbatch > 0) {
      delete h;
      return fail(PF_EINVAL, "batched mode needs dim == 1");
    }
    const double bound = dt_bound(*p, p->V);
    if (p->dt > bound) {
      delete h;
      char buf[160];
      snprintf(buf, sizeof buf, "dt = %g exceeds the stability bound %g", p->dt, bound);
      return fail(PF_EUNSTABLE_DT, buf);
    }
    h->ntot = h->c.ncell;
    h->h_n.push_back(0);
    h->h_off.push_back(0);
    h->h_V.push_back(p->V);
    h->h_dt.push_back(p->dt);
    h->h_z0.push_back(p->z0);
  }
  // run order: longest first (ties by index)
  std::vector<int> order(h->nrun);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->h_n[a] > h->h_n[b]; });
  // reduction chunks
  std::vector<int> chunk_run, run_chunk0;
  std::vector<long long> chunk_beg;
  for (int r = 0; r < h->nrun; ++r) {
    run_chunk0.push_back((int)chunk_run.size());
    const long long N = h->batched ? (long long)h->h_n[r] : h->c.ncell;
    for (long long b = 0; b < N; b += pfk::RED_CHUNK) {
      chunk_run.push_back(r);
      chunk_beg.push_back(b);
    }
  }
  run_chunk0.push_back((int)chunk_run.size());
  h->nchunk = (int)chunk_run.size();
  auto cleanup_fail = [&](int code) {
    pf_destroy(h);
    return code;
  };
  if ((rc = upload(&h->d_n, h->h_n, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_off, h->h_off, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_V, h->h_V, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_dt, h->h_dt, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_z0, h->h_z0, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_order, order, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_chunk_run, chunk_run, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_chunk_beg, chunk_beg, h->stream))) return cleanup_fail(rc);
  if ((rc = upload(&h->d_run_chunk0, run_chunk0, h->stream))) return cleanup_fail(rc);
  if ((rc = dalloc(&h->d_part, h->nchunk))) return cleanup_fail(rc);
  if ((rc = dalloc(&h->d_runred, h->nrun))) return cleanup_fail(rc);
  if ((rc = dalloc(&h->d_dldk, h->nrun))) return cleanup_fail(rc);
  if ((rc = dalloc(&h->d_err, 1))) return cleanup_fail(rc);
  {
    int z = 0;
    hipError_t e = hipMemcpyAsync(h->d_err, &z, sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return cleanup_fail(fail(PF_EDEVICE, hipGetErrorString(e)));
  }
  if (!h->batched) {
    for (int k = 0; k < 3; ++k)
      if ((rc = dalloc(&h->tw[k], (size_t)h->ntot))) return cleanup_fail(rc);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const pfk::Const& c = h->c;
    if (c.dim == 3) {
      const long long tiles = (long long)((c.nx + S3_TX - 1) / S3_TX) * ((c.ny + S3_TY - 1) / S3_TY);
      // ~3.7 rounds of 3 workgroups per CU; chunks of at most 96 planes on large grids
      // (measured at 1024 x 1024 x 512: 96 planes 20.4 ms per step, one 512-plane chunk 21.3 ms)
      h->zchunk = std::min(zchunk_for(c.nz, tiles, 11LL * ncu, 16), 96);
    } else {
      const long long tiles = (c.nx + S2_TX - 1) / S2_TX;
      // about 13 one-wave workgroups per CU: chunks of 6 planes at 1024^2 (measured: 6 planes
      // 30.1 us per step, 4: 33.4, 5: 31.1, 7: 31.7, 8: 35.0)
      h->zchunk = zchunk_for(c.nz, tiles, 13LL * ncu, 4);
    }
    if (const char* e = std::getenv("PF_ZCHUNK")) {  // tuning override
      const int v = std::atoi(e);
      if (v > 0) h->zchunk = v;
    }
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return cleanup_fail(fail(PF_EDEVICE, hipGetErrorString(e)));
  *out = h;
  return PF_OK;
}

static int step_impl(pf_handle* h, int64_t nsteps, double* const traj[3], int64_t stride) {
  if (!h || nsteps < 0) return fail(PF_EINVAL, "bad handle or nsteps");
  if (nsteps == 0 && !traj[0]) return PF_OK;
  if (h->batched) {
    const int ce = h->p.check_every;
    long long done = 0;
    while (done < nsteps || (nsteps == 0 && done == 0)) {
      long long chunk = nsteps - done;
      if (ce > 0) chunk = std::min<long long>(chunk, ce);
      double* t0 = traj[0] ? traj[0] + done * stride : nullptr;
      double* t1 = traj[1] ? traj[1] + done * stride : nullptr;
      double* t2 = traj[2] ? traj[2] + done * stride : nullptr;
      const bool apz = (h->c.ap == 0.0), eq = (h->p.model == 1);
      auto k = eq ? (apz ? pfk::k_run1d<true, true> : pfk::k_run1d<false, true>)
                  : (apz ? pfk::k_run1d<true, false> : pfk::k_run1d<false, false>);
      hipLaunchKernelGGL(k, dim3(h->nrun), dim3(pfk::R1_THREADS), 0, h->stream, h->c, h->runtab(),
                         h->f[0], h->f[1], h->f[2], (long long)(h->n + done), chunk, h->p.shift, h->d_err, t0, t1,
                         t2, (long long)stride);
      PF_HIP(hipGetLastError());
      done += chunk;
      if (ce > 0) {
        int rc = read_err(h, false);
        if (rc) {
          h->n += done;
          return rc;
        }
      }
      if (nsteps == 0) break;
    }
    h->n += nsteps;
    return PF_OK;
  }
  // 2D / 3D: one fused launch per step.  Without a trajectory: ping-pong
  // between the caller's fields and the twin.  With one: each step reads
  // trajectory row s and writes row s + 1, and the caller's fields receive the
  // newest row at the end (or when a check fails).
  const size_t bytes = (size_t)h->ntot * sizeof(double);
  if (traj[0]) {
    for (int k = 0; k < 3; ++k)
      PF_HIP(hipMemcpyAsync(traj[k], h->f[k], bytes, hipMemcpyDeviceToDevice, h->stream));
    long long s = 0;
    int rc = PF_OK;
    for (; s < nsteps; ++s) {
      double* src[3] = {traj[0] + s * stride, traj[1] + s * stride, traj[2] + s * stride};
      double* dst[3] = {traj[0] + (s + 1) * stride, traj[1] + (s + 1) * stride, traj[2] + (s + 1) * stride};
      rc = launch_stream(h, src, dst, h->n + s);
      if (rc) return rc;
      if (h->p.check_every > 0 && ((s + 1) % h->p.check_every == 0)) {
        rc = read_err(h, false);
        if (rc) {
          ++s;
          break;
        }
      }
    }
    for (int k = 0; k < 3; ++k)
      PF_HIP(hipMemcpyAsync(h->f[k], traj[k] + s * stride, bytes, hipMemcpyDeviceToDevice, h->stream));
    h->n += s;
    return rc;
  }
  double* cur[3] = {h->f[0], h->f[1], h->f[2]};
  double* nxt[3] = {h->tw[0], h->tw[1], h->tw[2]};
  for (long long s = 0; s < nsteps; ++s) {
    int rc = launch_stream(h, cur, nxt, h->n + s);
    if (rc) return rc;
    for (int k = 0; k < 3; ++k) std::swap(cur[k], nxt[k]);
    if (h->p.check_every > 0 && ((s + 1) % h->p.check_every == 0)) {
      rc = read_err(h, false);
      if (rc) {
        // leave the caller's buffers holding the newest state
        if (cur[0] != h->f[0])
          for (int k = 0; k < 3; ++k)
            PF_HIP(hipMemcpyAsync(h->f[k], cur[k], bytes, hipMemcpyDeviceToDevice, h->stream));
        h->n += s + 1;
        return rc;
      }
    }
  }
  if (cur[0] != h->f[0]) {
    for (int k = 0; k < 3; ++k) PF_HIP(hipMemcpyAsync(h->f[k], cur[k], bytes, hipMemcpyDeviceToDevice, h->stream));
  }
  h->n += nsteps;
  return PF_OK;
}

int pf_step(pf_handle* h, int64_t nsteps) {
  double* none[3] = {nullptr, nullptr, nullptr};
  return step_impl(h, nsteps, none, 0);
}

int pf_step_traj(pf_handle* h, int64_t nsteps, double* traj_phi, double* traj_cs, double* traj_cl, int64_t stride) {
  if (!traj_phi || !traj_cs || !traj_cl || !h || stride < h->ntot) return fail(PF_EINVAL, "bad trajectory buffers");
  double* t[3] = {traj_phi, traj_cs, traj_cl};
  return step_impl(h, nsteps, t, stride);
}

int pf_get_step(const pf_handle* h, int64_t* n) {
  if (!h || !n) return fail(PF_EINVAL, "null argument");
  *n = h->n;
  return PF_OK;
}

int pf_set_step(pf_handle* h, int64_t n) {
  if (!h || n < 0) return fail(PF_EINVAL, "bad argument");
  h->n = n;
  return PF_OK;
}

int pf_energy(pf_handle* h, double* out) {
  if (!h || !out) return fail(PF_EINVAL, "null argument");
  int rc = reduce(h);
  if (rc) return rc;
  std::vector<pfk::Partial> r(h->nrun);
  PF_HIP(hipMemcpyAsync(r.data(), h->d_runred, sizeof(pfk::Partial) * h->nrun, hipMemcpyDeviceToHost, h->stream));
  PF_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < h->nrun; ++i) out[i] = r[i].energy;
  return PF_OK;
}

int pf_solute(pf_handle* h, double* total, double* cmax, int64_t* argmax) {
  if (!h) return fail(PF_EINVAL, "null handle");
  int rc = reduce(h);
  if (rc) return rc;
  std::vector<pfk::Partial> r(h->nrun);
  PF_HIP(hipMemcpyAsync(r.data(), h->d_runred, sizeof(pfk::Partial) * h->nrun, hipMemcpyDeviceToHost, h->stream));
  PF_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < h->nrun; ++i) {
    if (total) total[i] = r[i].solute;
    if (cmax) cmax[i] = r[i].cmax;
    if (argmax) argmax[i] = r[i].arg;
  }
  return PF_OK;
}

int pf_solute_noalloc(const pf_params* p, const double* phi, const double* cs, const double* cl, int64_t n,
                      void* stream, double* total, double* cmax, int64_t* argmax, double* energy) {
  if (!p || !phi || !cs || !cl) return fail(PF_EINVAL, "null argument");
  if (n < 0) return fail(PF_EINVAL, "n must be >= 0");
  int rc = validate(*p);
  if (rc) return rc;
  if (p->nbatch != 0) return fail(PF_EINVAL, "pf_solute_noalloc takes one domain (nbatch = 0)");
  const pfk::Const c = make_const(*p);
  const long long nchunk = (c.ncell + pfk::RED_CHUNK - 1) / pfk::RED_CHUNK;
  if (nchunk > NOALLOC_MAX_CHUNKS) {
    char buf[160];
    snprintf(buf, sizeof buf, "%lld cells exceed the scratch of pf_solute_noalloc (at most %lld)", c.ncell,
             NOALLOC_MAX_CHUNKS * (long long)pfk::RED_CHUNK);
    return fail(PF_EINVAL, buf);
  }
  pfk::Partial* part = nullptr;
  if ((rc = scratch_ptr(&part))) return rc;
  hipStream_t s = (hipStream_t)stream;
  pfk::RunTab rt{};  // one domain: the run table is not read
  pfk::RedTab red{};
  red.nchunk = (int)nchunk;
  // every chunk slot is written before it is read, so nothing needs clearing
  hipLaunchKernelGGL(pfk::k_reduce_chunks, dim3((unsigned)nchunk), dim3(pfk::RED_THREADS), 0, s, c, rt, red, phi,
                     cs, cl, (long long)n, 0, part);
  PF_HIP(hipGetLastError());
  hipLaunchKernelGGL(pfk::k_reduce_runs, dim3(1), dim3(pfk::RED_THREADS), 0, s, c, red, part,
                     part + NOALLOC_MAX_CHUNKS);
  PF_HIP(hipGetLastError());
  hipLaunchKernelGGL(pfk::k_partial_emit, dim3(1), dim3(64), 0, s, part + NOALLOC_MAX_CHUNKS, energy, total, cmax,
                     (long long*)argmax);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

int pf_front(pf_handle* h, double* z_mean, double* z_min, double* z_max, double* T_front, int64_t* ncol) {
  if (!h) return fail(PF_EINVAL, "null handle");
  int rc;
  if (!h->d_front && (rc = dalloc(&h->d_front, (size_t)5 * h->nrun))) return rc;
  const pfk::Const& c = h->c;
  if (h->batched) {
    hipLaunchKernelGGL(pfk::k_front_runs, dim3(h->nrun), dim3(pfk::FRONT_THREADS), 0, h->stream, c, h->runtab(),
                       h->f[0], (long long)h->n, h->d_front);
    PF_HIP(hipGetLastError());
  } else {
    const int nz = c.nz;  // 2D and 3D (1D runs take the batched path)
    const long long cols = h->ntot / nz;
    if (!h->d_front_col && (rc = dalloc(&h->d_front_col, (size_t)cols))) return rc;
    const double tn = (double)h->n * c.dt;
    const double s = std::floor(c.V * tn / c.dx);
    hipLaunchKernelGGL(pfk::k_front_cols, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, h->stream, h->f[0],
                       cols, nz, s, c.dx, h->d_front_col);
    PF_HIP(hipGetLastError());
    hipLaunchKernelGGL(pfk::k_front_reduce, dim3(1), dim3(pfk::FRONT_THREADS), 0, h->stream, h->d_front_col, cols,
                       c.z0 + c.V * tn, c.inv_lT, h->d_front);
    PF_HIP(hipGetLastError());
  }
  std::vector<double> r((size_t)5 * h->nrun);
  PF_HIP(hipMemcpyAsync(r.data(), h->d_front, sizeof(double) * r.size(), hipMemcpyDeviceToHost, h->stream));
  PF_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < h->nrun; ++i) {
    if (z_mean) z_mean[i] = r[5 * i];
    if (z_min) z_min[i] = r[5 * i + 1];
    if (z_max) z_max[i] = r[5 * i + 2];
    if (T_front) T_front[i] = r[5 * i + 3];
    if (ncol) ncol[i] = (int64_t)r[5 * i + 4];
  }
  return PF_OK;
}

int pf_check(pf_handle* h) {
  if (!h) return fail(PF_EINVAL, "null handle");
  return read_err(h, true);
}

int pf_kv_seed(pf_handle* h, const double* dL_dk, double* const lam[3]) {
  if (!h || !dL_dk || !lam || !lam[0] || !lam[1] || !lam[2]) return fail(PF_EINVAL, "null argument");
  int rc = reduce(h);
  if (rc) return rc;
  PF_HIP(hipMemcpyAsync(h->d_dldk, dL_dk, sizeof(double) * h->nrun, hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < 3; ++k)
    if ((rc = fill(h, lam[k], 0.0, h->ntot))) return rc;
  hipLaunchKernelGGL(pfk::k_kv_seed, dim3((h->nrun + 63) / 64), dim3(64), 0, h->stream, h->c, h->runtab(),
                     h->batched, h->d_runred, h->d_dldk, h->nrun, lam[0], lam[1], lam[2], h->f[0], h->f[1], h->f[2]);
  PF_HIP(hipGetLastError());
  PF_HIP(hipStreamSynchronize(h->stream));
  return PF_OK;
}

// Tiles and partial-sum buffer of the adjoint launches; returns the block count.
static int adj_prepare(pf_handle* h, int* nblk_out) {
  const pfk::Const& c = h->c;
  int nblk = 0;
  if (h->p.model != 0) return fail(PF_EINVAL, "the adjoint step is built for model 0");
  if (h->batched) {
    if (!h->d_tiles) {
      std::vector<pfadj::Tile1> tiles;
      for (int r = 0; r < h->nrun; ++r)
        for (int z = 0; z < h->h_n[r]; z += pfadj::Geo<1>::TZ) tiles.push_back(pfadj::Tile1{r, z});
      int rc = upload(&h->d_tiles, tiles, h->stream);
      if (rc) return rc;
      h->ntiles = (int)tiles.size();
    }
    nblk = h->ntiles;
  } else if (c.dim == 2) {
    if (c.px && c.nx < pfadj::Geo<2>::TX + 2 * pfadj::H)
      return fail(PF_EINVAL, "adjoint: a periodic x axis needs nx >= 22");
    nblk = ((c.nx + pfadj::Geo<2>::TX - 1) / pfadj::Geo<2>::TX) * ((c.nz + pfadj::Geo<2>::TZ - 1) / pfadj::Geo<2>::TZ);
  } else {
    return fail(PF_EINVAL, "adjoint step is built for 1D runs and 2D grids");
  }
  if (nblk > h->ntheta_part) {
    if (h->d_theta_part) (void)hipFree(h->d_theta_part);
    h->d_theta_part = nullptr;
    int rc = dalloc(&h->d_theta_part, (size_t)nblk * pfadj::NTH);
    if (rc) return rc;
    h->ntheta_part = nblk;
  }
  *nblk_out = nblk;
  return PF_OK;
}

// One adjoint-step launch; block partials of the parameter cotangents are
// written (accum = 0) or added (accum = 1) to the partial-sum buffer.
static int adj_launch(pf_handle* h, int64_t n, const double* const u_n[3], const double* const lam_np1[3],
                      double* const lam_n[3], int nblk, int accum) {
  const pfk::Const& c = h->c;
  const bool apz = (c.ap == 0.0);
  if (h->batched) {
    auto k = apz ? pfadj::k_adj1d<true> : pfadj::k_adj1d<false>;
    hipLaunchKernelGGL(k, dim3(nblk), dim3(pfadj::ADJ1_NT), 0, h->stream, c, h->runtab(), h->d_tiles, (long long)n, h->p.shift,
                       u_n[0], u_n[1], u_n[2], lam_np1[0], lam_np1[1], lam_np1[2], lam_n[0], lam_n[1], lam_n[2],
                       h->d_theta_part, accum);
  } else {
    const double tn = (double)n * c.dt;
    const int sh = (h->p.shift && std::floor(c.V * ((double)(n + 1) * c.dt) / c.dx) > std::floor(c.V * tn / c.dx));
    dim3 grid((c.nx + pfadj::Geo<2>::TX - 1) / pfadj::Geo<2>::TX, (c.nz + pfadj::Geo<2>::TZ - 1) / pfadj::Geo<2>::TZ);
    auto k = apz ? pfadj::k_adj2d<true> : pfadj::k_adj2d<false>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, h->stream, c, (long long)n, sh, u_n[0], u_n[1], u_n[2], lam_np1[0],
                       lam_np1[1], lam_np1[2], lam_n[0], lam_n[1], lam_n[2], h->d_theta_part, accum);
  }
  PF_HIP(hipGetLastError());
  return PF_OK;
}

static bool any_alias(const double* const a[3], const double* const b[3]) {
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      if (a[k] == b[j]) return true;
  return false;
}

int pf_adjoint_step(pf_handle* h, int64_t n, const double* const u_n[3], const double* const lam_np1[3],
                    double* const lam_n[3], double* dtheta) {
  if (!h || !u_n || !lam_np1 || !lam_n || !dtheta || n < 0) return fail(PF_EINVAL, "null argument");
  for (int k = 0; k < 3; ++k)
    if (!u_n[k] || !lam_np1[k] || !lam_n[k]) return fail(PF_EINVAL, "null field pointer");
  const double* const l0c[3] = {lam_n[0], lam_n[1], lam_n[2]};
  if (any_alias(l0c, lam_np1)) return fail(PF_EINVAL, "lam_n may not alias lam_np1");
  int nblk = 0;
  int rc = adj_prepare(h, &nblk);
  if (rc) return rc;
  if ((rc = adj_launch(h, n, u_n, lam_np1, lam_n, nblk, 0))) return rc;
  hipLaunchKernelGGL(pfadj::k_theta_final, dim3(1), dim3(256), 0, h->stream, h->c, h->d_theta_part, nblk, dtheta);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

int pf_adjoint_segment(pf_handle* h, int64_t n0, int64_t m, const double* traj_phi, const double* traj_cs,
                       const double* traj_cl, int64_t stride, double* const lam[3], double* const work[3],
                       double* dtheta) {
  if (!h || !traj_phi || !traj_cs || !traj_cl || !lam || !work || !dtheta || n0 < 0 || m < 0)
    return fail(PF_EINVAL, "null argument");
  if (stride < h->ntot) return fail(PF_EINVAL, "trajectory stride below the field size");
  for (int k = 0; k < 3; ++k)
    if (!lam[k] || !work[k]) return fail(PF_EINVAL, "null field pointer");
  const double* const lc[3] = {lam[0], lam[1], lam[2]};
  const double* const wc[3] = {work[0], work[1], work[2]};
  if (any_alias(lc, wc)) return fail(PF_EINVAL, "work may not alias lam");
  if (m == 0) return PF_OK;
  int nblk = 0;
  int rc = adj_prepare(h, &nblk);
  if (rc) return rc;
  double* a[3] = {lam[0], lam[1], lam[2]};  // holds lam^{n0 + j + 1}
  double* b[3] = {work[0], work[1], work[2]};
  for (int64_t j = m - 1; j >= 0; --j) {
    const double* u[3] = {traj_phi + j * stride, traj_cs + j * stride, traj_cl + j * stride};
    const double* ac[3] = {a[0], a[1], a[2]};
    if ((rc = adj_launch(h, n0 + j, u, ac, b, nblk, j < m - 1 ? 1 : 0))) return rc;
    for (int k = 0; k < 3; ++k) std::swap(a[k], b[k]);
  }
  if (a[0] != lam[0]) {
    const size_t bytes = (size_t)h->ntot * sizeof(double);
    for (int k = 0; k < 3; ++k) PF_HIP(hipMemcpyAsync(lam[k], a[k], bytes, hipMemcpyDeviceToDevice, h->stream));
  }
  hipLaunchKernelGGL(pfadj::k_theta_final, dim3(1), dim3(256), 0, h->stream, h->c, h->d_theta_part, nblk, dtheta);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

void pf_destroy(pf_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (int k = 0; k < 3; ++k)
    if (h->tw[k]) (void)hipFree(h->tw[k]);
  (void)hipFree(h->d_n);
  (void)hipFree(h->d_off);
  (void)hipFree(h->d_V);
  (void)hipFree(h->d_dt);
  (void)hipFree(h->d_z0);
  (void)hipFree(h->d_order);
  (void)hipFree(h->d_chunk_run);
  (void)hipFree(h->d_chunk_beg);
  (void)hipFree(h->d_run_chunk0);
  (void)hipFree(h->d_part);
  (void)hipFree(h->d_runred);
  (void)hipFree(h->d_dldk);
  (void)hipFree(h->d_theta_part);
  (void)hipFree(h->d_tiles);
  (void)hipFree(h->d_err);
  (void)hipFree(h->d_front);
  (void)hipFree(h->d_front_col);
  delete h;
}

const char* pf_strerror(int code) {
  switch (code) {
    case PF_OK: return "ok";
    case PF_EINVAL: return "invalid argument";
    case PF_EUNSTABLE_DT: return "time step above the explicit stability bound";
    case PF_ENONFINITE: return "non-finite value in the fields";
    case PF_ENEGCONC: return "non-positive phase concentration";
    case PF_EDEVICE: return "HIP runtime error";
    case PF_ENOMEM: return "device allocation failed";
    default: return "unknown error";
  }
}

const char* pf_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
