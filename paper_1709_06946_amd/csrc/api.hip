// C ABI of the PSE library and the orchestration of its stages.
//
//  mobility: real part (cell list + pair sum) and wave part
//    (spread -> FFT -> k-space kernel -> inverse FFT -> interpolate),
//    Eq. pairsums with M = M_r + M_w (Sec. II.B-C).
//  sampler:  Eq. split; Lanczos for M_r^(1/2), Eq. FFTsqrt for M_w^(1/2).
//  step:     the four-step mid-point scheme of Sec. III.D / Appendix B, with
//            GMRES on the stresslet constraint (Eq. rigidconstraint).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pse_internal.h"

struct pse_handle {
  pse::Handle h;
};

struct pse_step_graph {
  pse_handle *hd;
  hipGraphExec_t exec;
  int steps;
};

namespace pse {

static thread_local std::string g_create_error = "no error";

template <typename T> GridSet<T> &grids(Handle &h);
template <> GridSet<double> &grids<double>(Handle &h) { return h.g64; }
template <> GridSet<float> &grids<float>(Handle &h) { return h.g32; }

// ------------------------------------------------------- small kernels --

// out = wrap(x + c v) for wrapped positions x and velocities v (rows of
// stride vstride).  Deformed lattices: x in lattice coordinates, the step
// c A^-1 v taken there and wrapped; out in lattice coordinates (cartesian =
// 0, the library's mid-point) or mapped back by A (cartesian = 1, the
// caller's positions).
__global__ void advance_kernel(const double *__restrict__ x, const double *__restrict__ v,
                               int vstride, double c, int64_t n, double L,
                               double *__restrict__ out, Deform df, int cartesian) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double dv[3] = {v[i * vstride], v[i * vstride + 1], v[i * vstride + 2]};
  if (df.on) {
    const double e[3] = {dv[0], dv[1], dv[2]};
    for (int r = 0; r < 3; ++r)
      dv[r] = df.Ai[3 * r] * e[0] + df.Ai[3 * r + 1] * e[1] + df.Ai[3 * r + 2] * e[2];
  }
  double y[3];
  for (int d = 0; d < 3; ++d) {
    double t = x[3 * i + d] + c * dv[d];
    t -= L * floor(t / L);
    if (t >= L) t -= L;
    if (t < 0) t = 0;
    y[d] = t;
  }
  for (int d = 0; d < 3; ++d)
    out[3 * i + d] = (df.on && cartesian)
                         ? df.A[3 * d] * y[0] + df.A[3 * d + 1] * y[1] + df.A[3 * d + 2] * y[2]
                         : y[d];
}

// slip = c (y1 + y2) on U and E components, Omega from y1 alone is not
// formed (positions do not need it): those entries are set to 0.
__global__ void slip_kernel(const double *__restrict__ y1, const double *__restrict__ y2,
                            double c, int64_t n, double *__restrict__ slip) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < NC; ++k) {
    const bool om = k >= 3 && k < 6;
    slip[i * NC + k] = om ? 0.0 : c * (y1[i * NC + k] + y2[i * NC + k]);
  }
}

// b = -(slip_E + m_E) (N x 5); m may be NULL
__global__ void rhs_kernel(const double *__restrict__ slip, const double *__restrict__ m,
                           int64_t n, double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 5; ++k)
    b[i * 5 + k] = -(slip[i * NC + 6 + k] + (m ? m[i * NC + 6 + k] : 0.0));
}

// moments (N x 11) = [FL | S]
__global__ void moments_kernel(const double *__restrict__ FL, const double *__restrict__ S,
                               int64_t n, double *__restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 6; ++k) q[i * NC + k] = FL ? FL[i * 6 + k] : 0.0;
  for (int k = 0; k < 5; ++k) q[i * NC + 6 + k] = S ? S[i * 5 + k] : 0.0;
}

// RPY step: slip = c (y1 + y2), U = slip + m (all N x 3, flat; m may be NULL)
__global__ void rpy_velocity_kernel(const double *__restrict__ y1, const double *__restrict__ y2,
                                    const double *__restrict__ m, double c, int64_t n3,
                                    double *__restrict__ slip, double *__restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double s = c * (y1[i] + y2[i]);
  slip[i] = s;
  U[i] = s + (m ? m[i] : 0.0);
}

// U = slip_U + m_U (N x 3)
__global__ void velocity_kernel(const double *__restrict__ slip, const double *__restrict__ m,
                                int64_t n, double *__restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) U[i * 3 + k] = slip[i * NC + k] + m[i * NC + k];
}

// step counter of PSE_STEP_DEVICE: set (add = 0) or advanced by one (add = 1)
__global__ void step_counter_kernel(uint64_t *c, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = add ? c[0] + 1 : 0;
}

__global__ void step_counter_set_kernel(uint64_t *c, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = v;
}

// statistics of an asynchronous call: cleared at its start ...
__global__ void stats_init_kernel(pse_stats *st, int *status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->lanczos_iters = 0;
  st->gmres_iters = 0;
  st->refine_passes = 0;
  st->converged = 1;
  st->lanczos_change = 0.0;
  st->gmres_residual = 0.0;
  st->fp64_residual = -1.0;
  st->status = 0;
  st->reserved = 0;
  status[0] = 0;
}

// ... the FP64 relative residual of a refinement pass (the last pass also
// decides convergence) ...
__global__ void refine_stats_kernel(const double *bnorm2, const double *rnorm2, int pass,
                                    int last, double tol, pse_stats *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double r = bnorm2[0] > 0.0 ? sqrt(fmax(rnorm2[0], 0.0) / bnorm2[0]) : 0.0;
  st->fp64_residual = r;
  st->refine_passes = pass + 1;
  if (last && !(r < tol)) st->converged = 0;
}

// ... the FP64 GMRES residual is the FP64 residual ...
__global__ void gmres_as_fp64_kernel(pse_stats *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->fp64_residual = st->gmres_residual;
}

// ... and copied out at its end with the status bits (out: device or pinned
// host memory, may be NULL)
__global__ void stats_finish_kernel(pse_stats *st, const int *status, pse_stats *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->status = status[0];
  if (out) *out = *st;
}

__global__ void twiddle_kernel64(double2 *tw, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincospi(-2.0 * i / n, &s, &c);
  tw[i] = double2{c, s};
}

__global__ void twiddle_kernel32(float2 *tw, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincospi(-2.0 * i / n, &s, &c);
  tw[i] = float2{(float)c, (float)s};
}

__global__ void d2f_kernel(const double2 *src, float2 *dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float2{(float)src[i].x, (float)src[i].y};
}

__global__ void f2d_kernel(const float2 *src, double2 *dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = double2{src[i].x, src[i].y};
}

// ------------------------------------------------------------ operators --

template <typename T>
static void wave_apply(Handle &h, const double *xw, const double *in, Layout lin,
                       const CompSet &cin, double *out, Layout lout, const CompSet &cout,
                       bool accumulate, bool reuse_ft) {
  GridSet<T> &G = grids<T>(h);
  T *gin = reinterpret_cast<T *>(G.gin), *gout = reinterpret_cast<T *>(G.gout);
  if (h.def.on) {
    // deformed lattice: full 3D transforms around a k-space kernel that
    // forms each mode's wave vector and radial factors itself
    spread<T>(h, xw, in, lin, cin, gin);
    rfft3d<T>(h, gin, G.twiddle, cin.n, -1);
    kspace_deformed<T>(h, G.gin, cin, G.gout, cout);
    rfft3d<T>(h, gout, G.twiddle, cout.n, +1);
    interpolate<T>(h, xw, gout, cout, out, lout, accumulate, 1.0);
    return;
  }
  // Where the set holds a grid per component, a contiguous run of input
  // components takes the slots of their codes (forces and torques 0-5,
  // stresslets 6-10), so a product without forces and torques leaves their
  // slots as they were; with reuse_ft (same positions, same forces and
  // torques, nothing written to those slots since) the x-y transformed
  // grids of an earlier product there serve again, and only the stresslets
  // are spread and transformed.
  const int slots = (sizeof(T) == 8 && h.mixed) ? 2 * MIXED_FP64_PACK : 2 * MAX_PACK;
  bool run = cin.n > 0;
  for (int k = 1; k < cin.n; ++k) run = run && cin.idx[k] == cin.idx[0] + k;
  const int s0 = (slots >= NC && run) ? cin.idx[0] : 0;
  if (reuse_ft && s0 == 0 && slots >= NC && run && cin.n == NC) {
    const CompSet st = comps_range(6, NC);
    spread<T>(h, xw, in, lin, st, gin + 6 * h.ngrid);
    rfft_xy<T>(h, gin + 6 * h.ngrid, G.twiddle, st.n, -1);
  } else {
    spread<T>(h, xw, in, lin, cin, gin + (size_t)s0 * h.ngrid);
    rfft_xy<T>(h, gin + (size_t)s0 * h.ngrid, G.twiddle, cin.n, -1);
  }
  kspace_fused<T>(h, G.gin + (size_t)s0 * (h.ngrid / 2), cin, G.gout, cout, G.twiddle);
  rfft_xy<T>(h, gout, G.twiddle, cout.n, +1);
  interpolate<T>(h, xw, gout, cout, out, lout, accumulate, 1.0);
}

// Derivative gridding of a wave-space product (handles that use it): the
// forces go onto three grids as their moments, the couplets (torques and
// stresslets) onto three grids with the Gaussian's gradient; the velocity
// comes from three grids by plain interpolation, rotation and strain from
// the gradient of three more -- at most six grids each way instead of eleven.
// It applies when the product involves a couplet on either side and every
// input group (forces, torques, stresslets) is complete or absent.
struct DGPlan {
  bool ok = false, hf = false, hL = false, hS = false, hu = false, hv = false;
  CompSet gin{}, gout{};   // grid codes (see kspace_fused)
};

static DGPlan dg_plan(const Handle &h, const CompSet &cin, const CompSet &cout) {
  DGPlan d;
  if (!h.deriv || h.def.on) return d;
  int cnt[3] = {0, 0, 0}, last = -1;
  for (int k = 0; k < cin.n; ++k) {
    const int c = cin.idx[k];
    if (c <= last) return d;
    last = c;
    ++cnt[c < 3 ? 0 : (c < 6 ? 1 : 2)];
  }
  if ((cnt[0] && cnt[0] != 3) || (cnt[1] && cnt[1] != 3) || (cnt[2] && cnt[2] != 5)) return d;
  d.hf = cnt[0] > 0;
  d.hL = cnt[1] > 0;
  d.hS = cnt[2] > 0;
  for (int k = 0; k < cout.n; ++k) (cout.idx[k] < 3 ? d.hu : d.hv) = true;
  if (!(d.hL || d.hS || d.hv)) return d;   // forces to velocities: the moment product
  // velocities alone are interpolated from their grids in order
  if (!d.hv && !(cout.n == 3 && cout.idx[0] == 0 && cout.idx[1] == 1 && cout.idx[2] == 2))
    return d;
  if (d.hf) for (int k = 0; k < 3; ++k) d.gin.idx[d.gin.n++] = k;
  if (d.hL || d.hS) for (int k = 3; k < 6; ++k) d.gin.idx[d.gin.n++] = k;
  if (d.hu) for (int k = 0; k < 3; ++k) d.gout.idx[d.gout.n++] = k;
  if (d.hv) for (int k = 3; k < 6; ++k) d.gout.idx[d.gout.n++] = k;
  d.ok = d.gin.n > 0;
  return d;
}

template <typename T>
static void wave_apply_dg(Handle &h, const DGPlan &d, const double *xw, const double *in,
                          Layout lin, const CompSet &cin, double *out, Layout lout,
                          const CompSet &cout, bool accumulate, bool reuse_forces) {
  GridSet<T> &G = grids<T>(h);
  T *gin = reinterpret_cast<T *>(G.gin), *gout = reinterpret_cast<T *>(G.gout);
  // the forces' three moment grids live in slots 0-2 and the couplets' in
  // slots 3-5, also without forces, so a product without forces leaves the
  // slots 0-2 of an earlier one as they were: with reuse_forces the forces'
  // x-y transformed grids there (same positions, same forces, same
  // precision, nothing since writing those slots) serve again
  T *gc = gin + 3 * h.ngrid;
  const bool hc = d.hL || d.hS;
  if (d.hf && !reuse_forces)
    spread<T>(h, xw, in, lin, comps_range(0, 3), gin);   // forces: moment grids
  if (hc) {
    // couplets onto the next three grids (measured faster than spreading
    // forces and couplets in one launch: 1.4 + 1.4 against 3.9 ms at 512^3)
    CompSet cc{};
    for (int k = 0; k < cin.n; ++k)
      if (cin.idx[k] >= 3) cc.idx[cc.n++] = cin.idx[k];
    spread_deriv<T>(h, in, lin, cc, false, d.hL, d.hS, gc);
  }
  if (d.hf && !reuse_forces) rfft_xy<T>(h, gin, G.twiddle, d.gin.n, -1);
  else if (hc) rfft_xy<T>(h, gc, G.twiddle, 3, -1);
  const cplx<T> *gk = d.hf ? G.gin : G.gin + 3 * (h.ngrid / 2);
  kspace_fused<T>(h, gk, d.gin, G.gout, d.gout, G.twiddle, true);
  rfft_xy<T>(h, gout, G.twiddle, d.gout.n, +1);
  if (d.hv) interp_deriv<T>(h, xw, gout, d.hu, cout, out, lout, accumulate, 1.0);
  else interpolate<T>(h, xw, gout, cout, out, lout, accumulate, 1.0);
}

// out[cout] = M(cin -> cout) in[cin] at wrapped positions xw whose cell list
// is current; in and out are particle vectors in layouts lin and lout.  fp64
// forces the FP64 kernels in a mixed handle.
static void mobility(Handle &h, const double *xw, bool want_real, bool want_wave,
                     const double *in, Layout lin, const CompSet &cin, double *out,
                     Layout lout, const CompSet &cout, bool fp64, bool reuse_forces = false) {
  const bool f32 = h.mixed && !fp64;
  bool acc = false;
  if (want_real) {
    if (f32) real_apply<float>(h, xw, in, lin, cin, out, lout, cout, false);
    else real_apply<double>(h, xw, in, lin, cin, out, lout, cout, false);
    acc = true;
  }
  if (want_wave) {
    const DGPlan d = dg_plan(h, cin, cout);
    if (d.ok) {
      if (f32) wave_apply_dg<float>(h, d, xw, in, lin, cin, out, lout, cout, acc, reuse_forces);
      else wave_apply_dg<double>(h, d, xw, in, lin, cin, out, lout, cout, acc, reuse_forces);
    } else {
      if (f32) wave_apply<float>(h, xw, in, lin, cin, out, lout, cout, acc, reuse_forces);
      else wave_apply<double>(h, xw, in, lin, cin, out, lout, cout, acc, reuse_forces);
    }
  }
}

// out[E] = M_ES in[S] (layouts lin, lout), the operator of the stresslet
// constraint (derivative gridding for the wave part when the handle uses it).
static void es_apply(Handle &h, const double *xw, bool want_real, bool want_wave,
                     const double *in, Layout lin, double *out, Layout lout, bool fp64) {
  const CompSet es = comps_range(6, 11);
  mobility(h, xw, want_real, want_wave, in, lin, es, out, lout, es, fp64);
}

template <typename T>
static void wave_sqrt_t(Handle &h, const double *xw, const double *psi, uint64_t seed,
                        uint64_t counter, double *out, const CompSet &cout, Layout lout) {
  GridSet<T> &G = grids<T>(h);
  T *gout = reinterpret_cast<T *>(G.gout);
  const DGPlan d = dg_plan(h, CompSet{}, cout);
  if (d.hv) {
    // derivative gridding of the rotation and strain outputs
    if (kspace_noise_z<T>(h, psi, seed, counter, G.gout, d.gout, G.twiddle)) {
      rfft_xy<T>(h, gout, G.twiddle, d.gout.n, +1);
    } else {
      kspace_noise<T>(h, psi, seed, counter, G.gout, d.gout, true);
      rfft3d<T>(h, gout, G.twiddle, d.gout.n, +1);
    }
    interp_deriv<T>(h, xw, gout, d.hu, cout, out, lout, false, 1.0);
    return;
  }
  kspace_noise<T>(h, psi, seed, counter, G.gout, cout);
  rfft3d<T>(h, gout, G.twiddle, cout.n, +1);
  interpolate<T>(h, xw, gout, cout, out, lout, false, 1.0);
}

static void wave_sqrt(Handle &h, const double *xw, const double *psi, uint64_t seed,
                      uint64_t counter, double *out, const CompSet &cout,
                      Layout lout = FULL_LAYOUT) {
  if (h.mixed) wave_sqrt_t<float>(h, xw, psi, seed, counter, out, cout, lout);
  else wave_sqrt_t<double>(h, xw, psi, seed, counter, out, cout, lout);
}

static KrylovResult real_sqrt(Handle &h, const double *xw, const double *psi, double *out) {
  const CompSet all = comps_range(0, NC);
  Op A = [&](const double *in, double *o) {
    if (h.mixed) real_apply<float>(h, xw, in, FULL_LAYOUT, all, o, FULL_LAYOUT, all, false);
    else real_apply<double>(h, xw, in, FULL_LAYOUT, all, o, FULL_LAYOUT, all, false);
  };
  if (h.async) {
    lanczos_sqrt_dev(h, A, psi, (size_t)h.n * NC, out, h.lz_cap, h.d.lanczos_tol);
    return KrylovResult{0, 0.0, true};
  }
  return lanczos_sqrt(h, A, psi, (size_t)h.n * NC, out, h.d.lanczos_maxit, h.d.lanczos_tol,
                      &h.lz_prev);
}

static void prepare_positions(Handle &h, const double *x, double *xw) {
  wrap_positions(h, x, xw);
  build_cells(h, xw);
}

void clear_graphs(Handle &h) {
  if (h.graphs.empty()) return;
  std::unique_lock<std::shared_mutex> lk(capture_gate());
  for (auto &kv : h.graphs) (void)hipGraphExecDestroy(kv.second);
  h.graphs.clear();
}

// Runs fn, an operator application on the handle's stream, from a captured
// graph: on the first call for (in, out, kind) the launches are captured
// (thread-local capture mode, so other threads' handles are unaffected) and
// instantiated, and every call replays the graph.  The launches read all
// per-step data (positions, lists, moments) from device memory at fixed
// addresses, so one capture serves every later step.  Eager when graphs are
// off, while the stage profiler runs, on the legacy null stream, and for the
// handle's very first application (lazy kernel attributes are set then).
// A capture that fails (begin, a launch into it, end or instantiation) is
// discarded, graphs are switched off for the handle (graph_error keeps the
// reason) and the application runs eagerly; a launch error that is not a
// capture error then reappears in the eager run and is reported as usual.
template <typename F>
static void run_graphed(Handle &h, const void *in, const void *out, int kind, F &&fn) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (h.stream) (void)hipStreamIsCapturing(h.stream, &cap);
  if (!h.use_graphs || h.prof.on || h.stream == nullptr || !h.graph_warm ||
      cap != hipStreamCaptureStatusNone) {
    // (the caller capturing this stream records the launches themselves)
    fn();
    h.graph_warm = true;
    return;
  }
  const auto key = std::make_tuple(in, (const void *)out, kind);
  auto it = h.graphs.find(key);
  if (it == h.graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::string why;
    std::shared_lock<std::shared_mutex> gate(capture_gate());
    hipError_t e = hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      why = std::string("hipStreamBeginCapture: ") + hipGetErrorString(e);
    } else {
      try {
        fn();
      } catch (const Error &err) {
        why = "launch during capture: " + err.msg;
      } catch (...) {
        why = "exception during capture";
      }
      e = hipStreamEndCapture(h.stream, &g);
      if (why.empty() && e != hipSuccess)
        why = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
      if (why.empty()) {
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          why = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
          ex = nullptr;
        }
      }
      if (g) (void)hipGraphDestroy(g);
    }
    gate.unlock();
    if (!why.empty()) {
      (void)hipGetLastError();
      h.use_graphs = false;
      h.graph_error = why;
      fn();
      return;
    }
    it = h.graphs.emplace(key, ex).first;
  }
  PSE_HIP(hipGraphLaunch(it->second, h.stream));
}

// Solve M_ES S = b at xh (cell list current).  Mixed handles run FP32 GMRES
// inside FP64 residual refinement: r = b - M_ES^(64) S, correction from the
// FP32 operator, until the FP64 relative residual meets gmres_tol.
// Right preconditioner of the constraint solve: out = P v with
// P = (1 + d/a0)/a0 - M_r,ES / a0^2, the first-order Neumann approximation of
// the inverse of M_ES's real-space part around its diagonal (d: the
// real-space self term, a0: the whole operator's; the neighbours' near-field
// coupling is what the approximation removes).  GMRES solves M_ES P y = b and
// S = P y, so its residual is the residual of M_ES S = b itself.  One
// real-space pair sum per application, in the precision of the operator.
static void es_precond(Handle &h, const double *xh, const double *v, double *out, bool fp64) {
  const size_t n5 = (size_t)h.n * 5;
  const Layout l5{5, 6};
  const CompSet es = comps_range(6, 11);
  if (h.mixed && !fp64) real_apply<float>(h, xh, v, l5, es, out, l5, es, false);
  else real_apply<double>(h, xh, v, l5, es, out, l5, es, false);
  const double a0 = h.es_self_total;
  vaxpby(h, (1.0 + h.es_self_real / a0) / a0, v, -1.0 / (a0 * a0), out, n5);
}

static void stresslet_solve(Handle &h, const double *xh, const double *b, double *S,
                            pse_stats &st, bool &converged) {
  const size_t n5 = (size_t)h.n * 5;
  // the operator reads and writes the 5-component vectors directly
  const Layout l5{5, 6};
  // the preconditioned operator M_ES P (graph kinds 3 and 4) and M_ES itself
  // (1 and 2, for the FP64 residual)
  auto make_op = [&, l5](bool fp64, bool precond) {
    return Op([&, fp64, precond, l5](const double *in, double *o) {
      run_graphed(h, in, o, (fp64 ? 1 : 2) + (precond ? 2 : 0), [&] {
        const double *x = in;
        if (precond) {
          es_precond(h, xh, in, h.es_p, fp64);
          x = h.es_p;
        }
        es_apply(h, xh, true, true, x, l5, o, l5, fp64);
      });
    });
  };
  // S = P y in place (y in v, tmp a scratch vector)
  auto unprecondition = [&](double *v) {
    es_precond(h, xh, v, h.es_p, !h.mixed);
    vcopy(h, v, h.es_p, n5);
  };
  if (h.async) {
    // device-checked: GMRES of exactly gmres_maxit iterations; mixed handles
    // run refine_passes passes, each an FP32 solve for the correction and an
    // FP64 residual (statistics on the device)
    const int K = h.gm_cap;
    if (!h.mixed) {
      gmres_dev(h, make_op(true, true), b, n5, S, K, h.d.gmres_tol);
      unprecondition(S);
      hipLaunchKernelGGL(gmres_as_fp64_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats);
      PSE_LAUNCH_CHECK();
      return;
    }
    Op A32 = make_op(false, true), A64 = make_op(true, false);
    double *b2 = h.small + h.small_len - 4, *r2 = b2 + 1;
    vzero(h, S, n5);
    vcopy(h, h.es_r, b, n5);
    multi_dot(h, b, n5, 1, b, n5, b2);
    for (int pass = 0; pass < h.ref_cap; ++pass) {
      gmres_dev(h, A32, h.es_r, n5, h.es_d, K, h.d.gmres_tol);
      unprecondition(h.es_d);
      vaxpby(h, 1.0, h.es_d, 1.0, S, n5);
      A64(S, h.es_r);
      vaxpby(h, 1.0, b, -1.0, h.es_r, n5);
      multi_dot(h, h.es_r, n5, 1, h.es_r, n5, r2);
      hipLaunchKernelGGL(refine_stats_kernel, dim3(1), dim3(1), 0, h.stream,
                         (const double *)b2, (const double *)r2, pass,
                         pass + 1 == h.ref_cap ? 1 : 0, h.d.gmres_tol, h.dstats);
      PSE_LAUNCH_CHECK();
    }
    return;
  }
  if (!h.mixed) {
    KrylovResult r = gmres(h, make_op(true, true), b, n5, S, h.d.gmres_restart,
                           h.d.gmres_maxit, h.d.gmres_tol, &h.gm_prev[0]);
    unprecondition(S);
    st.gmres_iters += r.iters;
    st.gmres_residual = r.resid;
    st.fp64_residual = r.resid;
    converged = converged && r.converged;
    return;
  }
  Op A32 = make_op(false, true), A64 = make_op(true, false);
  vzero(h, S, n5);
  vcopy(h, h.es_r, b, n5);
  double bnorm2 = 0.0;
  {
    double *tmp = h.small + h.small_len - 4;
    multi_dot(h, b, n5, 1, b, n5, tmp);
    PSE_HIP(hipMemcpyAsync(&bnorm2, tmp, sizeof(double), hipMemcpyDeviceToHost, h.stream));
    PSE_HIP(hipStreamSynchronize(h.stream));
  }
  const double bnorm = std::sqrt(bnorm2);
  if (!(bnorm > 0)) {
    st.fp64_residual = 0.0;
    return;
  }
  bool ok = false;
  for (int pass = 0; pass < h.d.refine_passes; ++pass) {
    KrylovResult r = gmres(h, A32, h.es_r, n5, h.es_d, h.d.gmres_restart, h.d.gmres_maxit,
                           h.d.gmres_tol, pass == 0 ? &h.gm_prev[1] : nullptr);
    st.gmres_iters += r.iters;
    st.gmres_residual = r.resid;
    st.refine_passes = pass + 1;
    unprecondition(h.es_d);
    vaxpby(h, 1.0, h.es_d, 1.0, S, n5);
    A64(S, h.es_r);
    vaxpby(h, 1.0, b, -1.0, h.es_r, n5);
    double rn2 = 0.0;
    double *tmp = h.small + h.small_len - 4;
    multi_dot(h, h.es_r, n5, 1, h.es_r, n5, tmp);
    PSE_HIP(hipMemcpyAsync(&rn2, tmp, sizeof(double), hipMemcpyDeviceToHost, h.stream));
    PSE_HIP(hipStreamSynchronize(h.stream));
    st.fp64_residual = std::sqrt(rn2) / bnorm;
    if (st.fp64_residual < h.d.gmres_tol) {
      ok = true;
      break;
    }
  }
  converged = converged && ok;
}

static const char *kPkNames[PK_COUNT] = {"spread", "fft", "kspace", "interp", "zero",
                                          "real", "cells", "krylov", "noise", "misc"};

__global__ void noop_kernel() {}

// Median event times of an empty bracket (two records back to back) and of
// a bracket around an empty one-thread kernel.
static void bracket_overhead(Handle &h, double &empty_ms, double &noop_ms) {
  constexpr int REPS = 16;
  hipEvent_t a, b;
  PSE_HIP(hipEventCreate(&a));
  PSE_HIP(hipEventCreate(&b));
  std::vector<double> t[2];
  for (int i = 0; i < 2 * REPS; ++i) {
    const bool with_kernel = i & 1;
    PSE_HIP(hipEventRecord(a, h.stream));
    if (with_kernel) {
      hipLaunchKernelGGL(noop_kernel, dim3(1), dim3(1), 0, h.stream);
      PSE_LAUNCH_CHECK();
    }
    PSE_HIP(hipEventRecord(b, h.stream));
    PSE_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    PSE_HIP(hipEventElapsedTime(&ms, a, b));
    t[with_kernel].push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  for (auto &v : t) std::sort(v.begin(), v.end());
  empty_ms = t[0][REPS / 2];
  noop_ms = t[1][REPS / 2];
}

void prof_resolve(Handle &h) {
  Profiler &P = h.prof;
  for (const ProfRecord &r : P.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      P.ms[r.kind] += std::max(0.0, (double)ms - P.bracket_ms);
      P.launches[r.kind] += 1;
      P.bytes[r.kind] += r.bytes;
    }
  }
  P.pending.clear();
  P.used = 0;
}

std::shared_mutex &capture_gate() {
  static std::shared_mutex m;
  return m;
}

void dev_alloc(void **p, size_t bytes) {
  std::unique_lock<std::shared_mutex> lk(capture_gate());
  PSE_HIP(hipMalloc(p, bytes));
}

void dev_free(void *p) {
  if (!p) return;
  std::unique_lock<std::shared_mutex> lk(capture_gate());
  (void)hipFree(p);
}

hipError_t dev_copy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  std::unique_lock<std::shared_mutex> lk(capture_gate());
  return hipMemcpy(dst, src, bytes, kind);
}

void handle_alloc(Handle &h, void **p, size_t bytes) {
  if (!h.arena) {
    dev_alloc(p, bytes);
    return;
  }
  const size_t off = (h.arena_used + 255) & ~(size_t)255;
  if (off > h.arena_size || bytes > h.arena_size - off)
    throw Error{PSE_ERR_NOMEM, "the allocation-free product needs more than its " +
                                   std::to_string(h.arena_size >> 20) +
                                   " MiB of static scratch (fewer particles or a smaller grid)"};
  *p = h.arena + off;
  h.arena_used = off + bytes;
}

static void create(const pse_params &p, Handle &h) {
  derive(p, h.d);
  h.p = p;
  h.n = p.n;
  h.mixed = p.precision == PSE_MIXED;
  h.use_graphs = p.graphs >= 0;
  h.async = p.async_calls != 0;
  deformation(p, h.def);
  h.lz_cap = h.d.lanczos_maxit;
  h.gm_cap = h.d.gmres_maxit;
  h.ref_cap = h.d.refine_passes;
  h.ngrid = (size_t)h.d.grid * h.d.grid * h.d.grid;
  h.cells.nc = h.d.cells;
  // spreading tiles of stile^3 grid points gather from the 27 neighbouring
  // tiles, so a stencil (P points) must not reach beyond one tile.
  // (deformed lattices spread with atomics: the Gaussian does not factorise
  // over the lattice axes, which the tile records rely on)
  h.stile = h.def.on ? 0 : spread_tile(h.d.grid, h.d.support);
  h.sbins.nc = h.stile ? h.d.grid / h.stile : 0;
  h.deriv = h.d.deriv_gridding == 2;
  if (p.stream || h.arena) {
    // the caller's stream (an allocation-free handle creates none: NULL is
    // the null stream there)
    h.stream = (hipStream_t)p.stream;
    h.own_stream = false;
  } else {
    std::unique_lock<std::shared_mutex> lk(capture_gate());
    PSE_HIP(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
    h.own_stream = true;
  }
  {
    int dev = 0, lds = 0;
    PSE_HIP(hipGetDevice(&dev));
    PSE_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    h.max_lds = lds;
    int cus = 0;
    PSE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    h.num_cu = cus > 0 ? cus : 1;
  }
  const size_t n = (size_t)h.n;
  const int ng = h.d.grid;
  const size_t packs64 = h.mixed ? MIXED_FP64_PACK : MAX_PACK;
  handle_alloc(h, (void **)&h.g64.gin, packs64 * h.ngrid * sizeof(double2));
  handle_alloc(h, (void **)&h.g64.gout, packs64 * h.ngrid * sizeof(double2));
  handle_alloc(h, (void **)&h.g64.twiddle, ng * sizeof(double2));
  hipLaunchKernelGGL(twiddle_kernel64, dim3(nblocks(ng, 256)), dim3(256), 0, h.stream,
                     h.g64.twiddle, ng);
  PSE_LAUNCH_CHECK();
  if (h.mixed) {
    handle_alloc(h, (void **)&h.g32.gin, MAX_PACK * h.ngrid * sizeof(float2));
    handle_alloc(h, (void **)&h.g32.gout, MAX_PACK * h.ngrid * sizeof(float2));
    handle_alloc(h, (void **)&h.g32.twiddle, ng * sizeof(float2));
    hipLaunchKernelGGL(twiddle_kernel32, dim3(nblocks(ng, 256)), dim3(256), 0, h.stream,
                       h.g32.twiddle, ng);
    PSE_LAUNCH_CHECK();
  }
  build_tables(h);
  handle_alloc(h, (void **)&h.ktab, (size_t)ktable_len(ng) * 4 * sizeof(double));
  if (h.mixed) handle_alloc(h, (void **)&h.ktab32, (size_t)ktable_len(ng) * 4 * sizeof(float));
  if (h.deriv) {
    handle_alloc(h, (void **)&h.kdg, (size_t)ktable_len(ng) * sizeof(double));
    if (h.mixed) handle_alloc(h, (void **)&h.kdg32, (size_t)ktable_len(ng) * sizeof(float));
  }
  handle_alloc(h, (void **)&h.bad_pos, 64);
  build_ktable(h);
  if (h.stile) {
    const size_t ntile = (size_t)h.sbins.nc * h.sbins.nc * h.sbins.nc;
    handle_alloc(h, (void **)&h.tl_cnt, ntile * sizeof(int));
    handle_alloc(h, (void **)&h.tl_start, (ntile + 1) * sizeof(int));
    handle_alloc(h, (void **)&h.tl_scan, ((ntile + 1023) / 1024 + 8) * sizeof(int));
    h.tl_cap = n * tiles_per_particle(h.d.support, h.stile);
    handle_alloc(h, (void **)&h.tl_rec, h.tl_cap * tile_record_bytes(h.stile) + 256);
  }
  handle_alloc(h, (void **)&h.pl_cnt, n * sizeof(int));
  handle_alloc(h, (void **)&h.pl_start, (n + 1) * sizeof(int));
  handle_alloc(h, (void **)&h.pl_scan, ((n + 1023) / 1024 + 8) * sizeof(int));
  // the list of an asynchronous handle cannot grow (no host read of its
  // length): twice the capacity up front
  h.pl_cap = (h.async ? 2 : 1) * pair_capacity(h.p, h.d);
  pair_storage(h, h.pl_cap, true);
  if (h.deriv) handle_alloc(h, (void **)&h.dg_mu, 6 * n * sizeof(double));
  handle_alloc(h, (void **)&h.mpack, 12 * n * sizeof(double));
  for (Bins *b : {&h.cells, &h.sbins}) {
    if (b->nc == 0) continue;
    const size_t ncells = (size_t)b->nc * b->nc * b->nc;
    handle_alloc(h, (void **)&b->start, (ncells + 1) * sizeof(int));
    handle_alloc(h, (void **)&b->count, ncells * sizeof(int));
    handle_alloc(h, (void **)&b->scan_tmp, ((ncells + 1023) / 1024 + 8) * sizeof(int));
    handle_alloc(h, (void **)&b->of, n * sizeof(int));
    handle_alloc(h, (void **)&b->slot, n * sizeof(int));
    handle_alloc(h, (void **)&b->scat, n * sizeof(int));
    handle_alloc(h, (void **)&b->perm, n * sizeof(int));
  }
  // block-order traversal of the real-space cells (interpolation order)
  handle_alloc(h, (void **)&h.cells.trav, n * sizeof(int));
  handle_alloc(h, (void **)&h.cells.bcount, (size_t)h.cells.nc * h.cells.nc * h.cells.nc * sizeof(int));
  handle_alloc(h, (void **)&h.cells.bstart,
               ((size_t)h.cells.nc * h.cells.nc * h.cells.nc + 1) * sizeof(int));
  handle_alloc(h, (void **)&h.xw, 3 * n * sizeof(double));
  handle_alloc(h, (void **)&h.xh, 3 * n * sizeof(double));
  double **vs[6] = {&h.v0, &h.v1, &h.v2, &h.v3, &h.v4, &h.v5};
  for (double **v : vs) handle_alloc(h, (void **)v, NC * n * sizeof(double));
  double **es[5] = {&h.es_b, &h.es_x, &h.es_r, &h.es_d, &h.es_p};
  for (double **v : es) handle_alloc(h, (void **)v, 5 * n * sizeof(double));
  handle_alloc(h, (void **)&h.lz_V, (size_t)(h.d.lanczos_maxit + 1) * NC * n * sizeof(double));
  handle_alloc(h, (void **)&h.gm_V, (size_t)(h.d.gmres_restart + 1) * 5 * n * sizeof(double));
  const size_t M = h.d.lanczos_maxit, R = h.d.gmres_restart;
  h.small_len = std::max((M + 1) * 10 + (M + 3) * (M + 1), (R + 1) * (R + 1) + 8 * (R + 2)) + 64;
  handle_alloc(h, (void **)&h.small, h.small_len * sizeof(double));
  h.dots_len = 1024 * (std::max(M, R) + 2);
  handle_alloc(h, (void **)&h.dots, h.dots_len * sizeof(double));
  handle_alloc(h, (void **)&h.dctl, CTL_WORDS * sizeof(int));
  handle_alloc(h, (void **)&h.dstats, sizeof(pse_stats));
  handle_alloc(h, (void **)&h.dstep, sizeof(uint64_t));
  fill_int(h, h.dctl, CTL_WORDS, 0);
  hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(1), 0, h.stream, h.dstep, 0);
  PSE_LAUNCH_CHECK();
  // self terms of M_ES for the constraint solve's preconditioner: the
  // real-space part from the coefficient table's r = 0 row (the pair block at
  // zero separation acting on a stresslet gives 9 (3 d2 + d3) S), the whole
  // operator's from the isolated sphere, 3 / (20 pi eta a^3)
  double co0[NCOEF];
  PSE_HIP(hipMemcpyAsync(co0, h.g64.table, sizeof(co0), hipMemcpyDeviceToHost, h.stream));
  PSE_HIP(hipStreamSynchronize(h.stream));
  h.es_self_real = 9.0 * (3.0 * co0[4] + co0[5]);
  h.es_self_total = 3.0 / (20.0 * M_PI * h.p.viscosity * std::pow(h.p.radius, 3));
}

static void release(Handle &h) {
  void *ptrs[] = {h.g64.gin, h.g64.gout, h.g64.twiddle, h.g64.table, h.g32.gin, h.g32.gout,
                  h.g32.twiddle, h.g32.table, h.cells.start, h.cells.count,
                  h.cells.scan_tmp, h.cells.of, h.cells.slot, h.cells.scat, h.cells.perm,
                  h.sbins.start, h.sbins.count, h.sbins.scan_tmp, h.sbins.of, h.sbins.slot,
                  h.sbins.scat, h.sbins.perm, h.cells.trav, h.cells.bcount, h.cells.bstart,
                  h.xw, h.xh, h.v0, h.v1, h.v2, h.v3, h.v4, h.v5, h.es_b, h.es_x, h.es_r,
                  h.es_d, h.es_p, h.lz_V, h.gm_V, h.small, h.dots, h.ktab, h.pl_cnt,
                  h.pl_start, h.pl_scan, h.pl_nbr, h.pl_rec64, h.pl_rec32, h.tl_cnt, h.tl_start,
                  h.tl_scan, h.tl_rec, h.bad_pos, h.ktab32, h.dctl, h.dstats, h.dstep,
                  h.dg_mu, h.mpack, h.kdg, h.kdg32};
  if (!h.arena)
    for (void *p : ptrs) dev_free(p);
  clear_graphs(h);
  for (hipEvent_t e : h.prof.pool) (void)hipEventDestroy(e);
  h.prof.pool.clear();
  if (h.own_stream && h.stream) {
    std::unique_lock<std::shared_mutex> lk(capture_gate());
    (void)hipStreamDestroy(h.stream);
  }
}

template <typename F> static int guarded(pse_handle *hd, F &&f) {
  RelaxedCaptureScope relaxed;
  // an error left by the caller's own runtime calls is not this call's
  (void)hipGetLastError();
  try {
    f();
    if (hd && !hd->h.prof.pending.empty()) {
      PSE_HIP(hipStreamSynchronize(hd->h.stream));
      prof_resolve(hd->h);
    }
    return PSE_OK;
  } catch (const Error &e) {
    if (hd) hd->h.err = e.msg;
    else g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (hd) hd->h.err = "host allocation failed";
    else g_create_error = "host allocation failed";
    return PSE_ERR_NOMEM;
  } catch (...) {
    if (hd) hd->h.err = "unexpected exception";
    else g_create_error = "unexpected exception";
    return PSE_ERR_HIP;
  }
}

// ---- static scratch of the allocation-free product

// Device scratch of pse_mobility_apply_noalloc: every buffer of its
// transient handle (grids, tables, bins, lists) is carved from it.  Each
// device holds its own copy from the time the library's code object is
// loaded on it until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of the current device's copy of `scratch`, looked up once
// per device (the array's name is a host-side stand-in in host code).
static unsigned char *scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static unsigned char *addr[kMaxDevices] = {};
  int dev = 0;
  PSE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error{PSE_ERR_INVALID, "device index above 63"};
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    PSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = static_cast<unsigned char *>(p);
  }
  return addr[dev];
}

}  // namespace pse

using namespace pse;

extern "C" {

int pse_derive(const pse_params *p, pse_derived *out) {
  if (!p || !out) return PSE_ERR_INVALID;
  return guarded(nullptr, [&] { derive(*p, *out); });
}

int pse_footprint_bytes(const pse_params *p, size_t *bytes) {
  if (!p || !bytes) return PSE_ERR_INVALID;
  return guarded(nullptr, [&] {
    pse_derived d;
    derive(*p, d);
    *bytes = footprint(*p, d);
  });
}

int pse_create(const pse_params *p, pse_handle **out) {
  if (!p || !out) {
    g_create_error = "null argument";
    return PSE_ERR_INVALID;
  }
  *out = nullptr;
  pse_handle *hd = new (std::nothrow) pse_handle();
  if (!hd) return PSE_ERR_NOMEM;
  const int rc = guarded(nullptr, [&] { create(*p, hd->h); });
  if (rc != PSE_OK) {
    release(hd->h);
    delete hd;
    return rc;
  }
  *out = hd;
  return PSE_OK;
}

int pse_destroy(pse_handle *hd) {
  if (!hd) return PSE_OK;
  RelaxedCaptureScope relaxed;
  (void)hipStreamSynchronize(hd->h.stream);
  release(hd->h);
  delete hd;
  return PSE_OK;
}

int pse_get_derived(const pse_handle *hd, pse_derived *out) {
  if (!hd || !out) return PSE_ERR_INVALID;
  *out = hd->h.d;
  return PSE_OK;
}

const char *pse_last_error(const pse_handle *hd) {
  return hd ? hd->h.err.c_str() : g_create_error.c_str();
}

int pse_mobility_apply(pse_handle *hd, const double *x, const double *in, double *out,
                       unsigned parts) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !in || !out || (parts & 3u) == 0 || (parts & ~7u)) {
    hd->h.err = "pse_mobility_apply: null pointer or bad parts";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    const CompSet all = comps_range(0, NC);
    prepare_positions(h, x, h.xw);
    if (parts & PSE_ES_BLOCK)
      es_apply(h, h.xw, parts & PSE_REAL, parts & PSE_WAVE, in, FULL_LAYOUT, out, FULL_LAYOUT,
               false);
    else
      mobility(h, h.xw, parts & PSE_REAL, parts & PSE_WAVE, in, FULL_LAYOUT, all, out,
               FULL_LAYOUT, all, false);
    if (!h.async && check_finite(h, out, (size_t)h.n * NC))
      throw Error{PSE_ERR_NONFINITE, "non-finite mobility product (non-finite input?)"};
  });
}

int pse_mobility_apply_noalloc(const pse_params *p, const double *x, const double *in,
                               double *out, unsigned parts) {
  if (!p || !x || !in || !out || (parts & 3u) == 0 || (parts & ~7u)) {
    g_create_error = "pse_mobility_apply_noalloc: null pointer or bad parts";
    return PSE_ERR_INVALID;
  }
  Handle h;
  const int rc = guarded(nullptr, [&] {
    // a product needs no Krylov bases and no captured graphs
    pse_params q = *p;
    q.lanczos_maxit = 1;
    q.gmres_restart = 1;
    q.graphs = -1;
    h.arena = scratch_address();
    h.arena_size = kScratchBytes;
    create(q, h);
    const CompSet all = comps_range(0, NC);
    prepare_positions(h, x, h.xw);
    if (parts & PSE_ES_BLOCK)
      es_apply(h, h.xw, parts & PSE_REAL, parts & PSE_WAVE, in, FULL_LAYOUT, out, FULL_LAYOUT,
               false);
    else
      mobility(h, h.xw, parts & PSE_REAL, parts & PSE_WAVE, in, FULL_LAYOUT, all, out,
               FULL_LAYOUT, all, false);
    if (check_finite(h, out, (size_t)h.n * NC))
      throw Error{PSE_ERR_NONFINITE, "non-finite mobility product (non-finite input?)"};
  });
  RelaxedCaptureScope relaxed;
  (void)hipStreamSynchronize(h.stream);
  release(h);
  return rc;
}

int pse_set_krylov(pse_handle *hd, int async_calls, int lanczos_iters, int gmres_iters,
                   int refine_passes, uint64_t next_step) {
  if (!hd) return PSE_ERR_INVALID;
  Handle &h = hd->h;
  if (async_calls &&
      (lanczos_iters < 1 || lanczos_iters > h.d.lanczos_maxit || gmres_iters < 1 ||
       gmres_iters > h.d.gmres_restart || refine_passes < 1)) {
    h.err = "pse_set_krylov: iterations beyond the handle's Krylov bases (lanczos_maxit, "
            "gmres_restart) or below 1";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    PSE_HIP(hipStreamSynchronize(h.stream));
    if (async_calls) {
      // the pair list cannot grow without a host read: headroom over the
      // last count
      const size_t want = h.pl_pairs + h.pl_pairs / 2 + 1024;
      if (h.pl_cap < want && !h.arena) {
        clear_graphs(h);
        pair_storage(h, want, false);
      }
      h.lz_cap = lanczos_iters;
      h.gm_cap = gmres_iters;
      h.ref_cap = refine_passes;
    }
    h.async = async_calls != 0;
    hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(1), 0, h.stream, h.dstep, 0);
    PSE_LAUNCH_CHECK();
    if (next_step) {
      hipLaunchKernelGGL(step_counter_set_kernel, dim3(1), dim3(1), 0, h.stream, h.dstep,
                         next_step);
      PSE_LAUNCH_CHECK();
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
  });
}

int pse_synchronize(pse_handle *hd) {
  if (!hd) return PSE_ERR_INVALID;
  return guarded(hd, [&] { PSE_HIP(hipStreamSynchronize(hd->h.stream)); });
}

int pse_step_graph_create(pse_handle *hd, double *x, const double *FL, double dt,
                          uint64_t seed, int steps, pse_stats *stats, pse_step_graph **out) {
  if (!hd || !out || !x || steps < 1 || !(dt > 0)) return PSE_ERR_INVALID;
  *out = nullptr;
  Handle &h = hd->h;
  if (!h.async || !h.own_stream) {
    h.err = "pse_step_graph_create: needs an asynchronous handle on its own stream";
    return PSE_ERR_INVALID;
  }
  hipGraphExec_t exec = nullptr;
  const int rc = guarded(hd, [&] {
    PSE_HIP(hipStreamSynchronize(h.stream));
    hipGraph_t g = nullptr;
    std::string why;
    {
      std::shared_lock<std::shared_mutex> gate(capture_gate());
      PSE_HIP(hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal));
      int src = PSE_OK;
      for (int k = 0; k < steps && src == PSE_OK; ++k)
        src = pse_constrained_step(hd, x, FL, dt, seed, PSE_STEP_DEVICE, nullptr, stats);
      if (src != PSE_OK) why = h.err;
      const hipError_t e = hipStreamEndCapture(h.stream, &g);
      if (why.empty() && e != hipSuccess)
        why = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
      if (why.empty()) {
        const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) why = std::string("hipGraphInstantiate: ") + hipGetErrorString(ie);
      }
      if (g) (void)hipGraphDestroy(g);
    }
    if (!why.empty()) {
      (void)hipGetLastError();
      throw Error{PSE_ERR_HIP, "step capture failed: " + why};
    }
  });
  if (rc != PSE_OK) return rc;
  pse_step_graph *sg = new (std::nothrow) pse_step_graph{hd, exec, steps};
  if (!sg) {
    (void)hipGraphExecDestroy(exec);
    return PSE_ERR_NOMEM;
  }
  *out = sg;
  return PSE_OK;
}

int pse_step_graph_launch(pse_step_graph *sg) {
  if (!sg) return PSE_ERR_INVALID;
  return guarded(sg->hd, [&] { PSE_HIP(hipGraphLaunch(sg->exec, sg->hd->h.stream)); });
}

int pse_step_graph_destroy(pse_step_graph *sg) {
  if (!sg) return PSE_OK;
  (void)hipStreamSynchronize(sg->hd->h.stream);
  (void)hipGraphExecDestroy(sg->exec);
  delete sg;
  return PSE_OK;
}

int pse_brownian_sample(pse_handle *hd, const double *x, const double *psi_real,
                        const double *psi_wave, uint64_t seed, uint64_t counter,
                        double *out_real, double *out_wave, pse_stats *stats) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x) {
    hd->h.err = "pse_brownian_sample: null positions";
    return PSE_ERR_INVALID;
  }
  int warn = PSE_OK;
  const int rc = guarded(hd, [&] {
    Handle &h = hd->h;
    pse_stats st{};
    st.converged = 1;
    st.fp64_residual = -1;
    if (h.async) {
      hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         h.dctl + CTL_STATUS);
      PSE_LAUNCH_CHECK();
    }
    // pair sums and interpolation only: no spreading tile lists
    wrap_positions(h, x, h.xw);
    build_cells(h, h.xw, false);
    if (out_real) {
      const double *psi = psi_real;
      if (!psi) {
        real_noise(h, seed, counter, h.v2);
        psi = h.v2;
      }
      KrylovResult r = real_sqrt(h, h.xw, psi, out_real);
      st.lanczos_iters = r.iters;
      st.lanczos_change = r.resid;
      if (!r.converged) {
        st.converged = 0;
        warn = PSE_WARN_NOT_CONVERGED;
      }
    }
    if (out_wave) wave_sqrt(h, h.xw, psi_wave, seed, counter, out_wave, comps_range(0, NC));
    if (h.async) {
      hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         (const int *)(h.dctl + CTL_STATUS), stats);
      PSE_LAUNCH_CHECK();
      return;
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
    if (stats) *stats = st;
  });
  return rc != PSE_OK ? rc : warn;
}

int pse_constrained_step(pse_handle *hd, double *x, const double *FL, double dt,
                         uint64_t seed, uint64_t step, const pse_step_io *io,
                         pse_stats *stats) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !(dt > 0)) {
    hd->h.err = "pse_constrained_step: null positions or dt <= 0";
    return PSE_ERR_INVALID;
  }
  int warn = PSE_OK;
  const int rc = guarded(hd, [&] {
    Handle &h = hd->h;
    const int64_t n = h.n;
    pse_stats st{};
    st.fp64_residual = -1;
    bool converged = true;
    const bool dev_step = h.async && step == PSE_STEP_DEVICE;
    h.counter_dev = dev_step ? h.dstep : nullptr;
    if (h.async) {
      hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         h.dctl + CTL_STATUS);
      PSE_LAUNCH_CHECK();
    }
    // 1. slip velocities at x_k: pair sums and the wave noise's
    // interpolation only (every spreading of the step runs at the mid-point),
    // so no spreading tile lists here
    wrap_positions(h, x, h.xw);
    build_cells(h, h.xw, false);
    const double *psi = io ? io->psi_real : nullptr;
    if (!psi) {
      real_noise(h, seed, step, h.v2);
      psi = h.v2;
    }
    KrylovResult lr = real_sqrt(h, h.xw, psi, h.v0);
    st.lanczos_iters = lr.iters;
    st.lanczos_change = lr.resid;
    converged = converged && lr.converged;
    CompSet ue{};
    ue.n = 8;
    for (int k = 0; k < 3; ++k) ue.idx[k] = k;
    for (int k = 0; k < 5; ++k) ue.idx[3 + k] = 6 + k;
    wave_sqrt(h, h.xw, io ? io->psi_wave : nullptr, seed, step, h.v1, ue);
    double *slip = h.v3;
    hipLaunchKernelGGL(slip_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, h.v0,
                       h.v1, std::sqrt(2.0 * h.p.kT / dt), n, slip);
    PSE_LAUNCH_CHECK();
    // 2. mid-point
    hipLaunchKernelGGL(advance_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, h.xw,
                       slip, NC, 0.5 * dt, n, h.p.box, h.xh, h.def, 0);
    PSE_LAUNCH_CHECK();
    build_cells(h, h.xh);
    // 3. constraint at the mid-point: M_ES S = -E^B - M_EF F^P
    const CompSet fl = comps_range(0, 6), es = comps_range(6, 11);
    if (FL) {
      hipLaunchKernelGGL(moments_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, FL,
                         (const double *)nullptr, n, h.v4);
      PSE_LAUNCH_CHECK();
      mobility(h, h.xh, true, true, h.v4, FULL_LAYOUT, fl, h.v5, FULL_LAYOUT, es, false);
    }
    hipLaunchKernelGGL(rhs_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, slip,
                       FL ? (const double *)h.v5 : nullptr, n, h.es_b);
    PSE_LAUNCH_CHECK();
    stresslet_solve(h, h.xh, h.es_b, h.es_x, st, converged);
    // U = U^B + M_UF F^P + M_US S
    hipLaunchKernelGGL(moments_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, FL,
                       (const double *)h.es_x, n, h.v4);
    PSE_LAUNCH_CHECK();
    const CompSet u3 = comps_range(0, 3);
    // the right-hand side's product left the forces' (with moment gridding
    // also the torques') transformed grids in the first input slots (same
    // positions, same forces and torques; the constraint solve in between
    // uses other slots), so the final product spreads and transforms the rest
    mobility(h, h.xh, true, true, h.v4, FULL_LAYOUT, FL ? comps_range(0, 11) : es, h.v5,
             FULL_LAYOUT, u3, false, FL != nullptr);
    double *U = h.v2;   // N x 3
    hipLaunchKernelGGL(velocity_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, slip,
                       h.v5, n, U);
    PSE_LAUNCH_CHECK();
    // 4. x_{k+1} = x_k + dt U
    hipLaunchKernelGGL(advance_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, h.xw,
                       U, 3, dt, n, h.p.box, x, h.def, 1);
    PSE_LAUNCH_CHECK();
    if (io) {
      if (io->slip) PSE_HIP(hipMemcpyAsync(io->slip, slip, NC * n * sizeof(double),
                                           hipMemcpyDeviceToDevice, h.stream));
      if (io->stresslet) PSE_HIP(hipMemcpyAsync(io->stresslet, h.es_x, 5 * n * sizeof(double),
                                                hipMemcpyDeviceToDevice, h.stream));
      if (io->velocity) PSE_HIP(hipMemcpyAsync(io->velocity, U, 3 * n * sizeof(double),
                                               hipMemcpyDeviceToDevice, h.stream));
    }
    if (h.async) {
      if (dev_step) {
        hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(1), 0, h.stream, h.dstep, 1);
        PSE_LAUNCH_CHECK();
      }
      h.counter_dev = nullptr;
      hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         (const int *)(h.dctl + CTL_STATUS), stats);
      PSE_LAUNCH_CHECK();
      return;
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
    st.converged = converged ? 1 : 0;
    if (!converged) warn = PSE_WARN_NOT_CONVERGED;
    if (stats) *stats = st;
  });
  if (hd) hd->h.counter_dev = nullptr;
  return rc != PSE_OK ? rc : warn;
}

// ---- RPY-level (unconstrained) PSE ----

// Particle vectors of the force-velocity block: N x 3, components 0..2.
static const Layout RPY_LAYOUT{3, 0};

int pse_rpy_apply(pse_handle *hd, const double *x, const double *F, double *U,
                  unsigned parts) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !F || !U || parts == 0 || (parts & ~3u)) {
    hd->h.err = "pse_rpy_apply: null pointer or bad parts";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    const CompSet u3 = comps_range(0, 3);
    prepare_positions(h, x, h.xw);
    mobility(h, h.xw, parts & PSE_REAL, parts & PSE_WAVE, F, RPY_LAYOUT, u3, U, RPY_LAYOUT, u3,
             false);
    if (!h.async && check_finite(h, U, (size_t)h.n * 3))
      throw Error{PSE_ERR_NONFINITE, "non-finite mobility product (non-finite input?)"};
  });
}

int pse_rpy_step(pse_handle *hd, double *x, const double *F, double dt, uint64_t seed,
                 uint64_t step, const pse_step_io *io, pse_stats *stats) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !(dt > 0)) {
    hd->h.err = "pse_rpy_step: null positions or dt <= 0";
    return PSE_ERR_INVALID;
  }
  int warn = PSE_OK;
  const int rc = guarded(hd, [&] {
    Handle &h = hd->h;
    const int64_t n = h.n;
    const CompSet u3 = comps_range(0, 3);
    pse_stats st{};
    st.fp64_residual = -1;
    const bool dev_step = h.async && step == PSE_STEP_DEVICE;
    h.counter_dev = dev_step ? h.dstep : nullptr;
    if (h.async) {
      hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         h.dctl + CTL_STATUS);
      PSE_LAUNCH_CHECK();
    }
    prepare_positions(h, x, h.xw);
    // (M_r)_UF^(1/2) psi1 by Lanczos on the UF block of the pair sum
    const double *psi = io ? io->psi_real : nullptr;
    if (!psi) {
      real_noise(h, seed, step, h.v2, 3);
      psi = h.v2;
    }
    Op A = [&](const double *in, double *o) {
      if (h.mixed) real_apply<float>(h, h.xw, in, RPY_LAYOUT, u3, o, RPY_LAYOUT, u3, false);
      else real_apply<double>(h, h.xw, in, RPY_LAYOUT, u3, o, RPY_LAYOUT, u3, false);
    };
    KrylovResult lr{0, 0.0, true};
    if (h.async)
      lanczos_sqrt_dev(h, A, psi, (size_t)n * 3, h.v0, h.lz_cap, h.d.lanczos_tol);
    else
      lr = lanczos_sqrt(h, A, psi, (size_t)n * 3, h.v0, h.d.lanczos_maxit, h.d.lanczos_tol,
                        &h.lz_prev_rpy);
    st.lanczos_iters = lr.iters;
    st.lanczos_change = lr.resid;
    // (M_w)_UF^(1/2) psi2: the wave sampler's velocity rows
    wave_sqrt(h, h.xw, io ? io->psi_wave : nullptr, seed, step, h.v1, u3, RPY_LAYOUT);
    // M_UF F at x_k
    if (F) mobility(h, h.xw, true, true, F, RPY_LAYOUT, u3, h.v4, RPY_LAYOUT, u3, false);
    double *slip = h.v3, *U = h.v5;
    hipLaunchKernelGGL(rpy_velocity_kernel, dim3(nblocks(3 * n, 256)), dim3(256), 0, h.stream,
                       h.v0, h.v1, F ? (const double *)h.v4 : nullptr,
                       std::sqrt(2.0 * h.p.kT / dt), 3 * n, slip, U);
    PSE_LAUNCH_CHECK();
    hipLaunchKernelGGL(advance_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, h.xw,
                       U, 3, dt, n, h.p.box, x, h.def, 1);
    PSE_LAUNCH_CHECK();
    if (io) {
      if (io->slip) PSE_HIP(hipMemcpyAsync(io->slip, slip, 3 * n * sizeof(double),
                                           hipMemcpyDeviceToDevice, h.stream));
      if (io->velocity) PSE_HIP(hipMemcpyAsync(io->velocity, U, 3 * n * sizeof(double),
                                               hipMemcpyDeviceToDevice, h.stream));
    }
    if (h.async) {
      if (dev_step) {
        hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(1), 0, h.stream, h.dstep, 1);
        PSE_LAUNCH_CHECK();
      }
      h.counter_dev = nullptr;
      hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(1), 0, h.stream, h.dstats,
                         (const int *)(h.dctl + CTL_STATUS), stats);
      PSE_LAUNCH_CHECK();
      return;
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
    st.converged = lr.converged ? 1 : 0;
    if (!lr.converged) warn = PSE_WARN_NOT_CONVERGED;
    if (stats) *stats = st;
  });
  if (hd) hd->h.counter_dev = nullptr;
  return rc != PSE_OK ? rc : warn;
}

int pse_fft3d(pse_handle *hd, double *data, int ncomp, int direction) {
  if (!hd) return PSE_ERR_INVALID;
  if (!data || ncomp < 1 || ncomp > MAX_PACK || (direction != 1 && direction != -1)) {
    hd->h.err = "pse_fft3d: bad arguments";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    if (!h.mixed) {
      fft3d<double>(h, (double2 *)data, h.g64.twiddle, ncomp, direction);
    } else {
      const size_t cnt = (size_t)ncomp * h.ngrid;
      hipLaunchKernelGGL(d2f_kernel, dim3(nblocks(cnt, 256)), dim3(256), 0, h.stream,
                         (const double2 *)data, h.g32.gin, cnt);
      PSE_LAUNCH_CHECK();
      fft3d<float>(h, h.g32.gin, h.g32.twiddle, ncomp, direction);
      hipLaunchKernelGGL(f2d_kernel, dim3(nblocks(cnt, 256)), dim3(256), 0, h.stream,
                         (const float2 *)h.g32.gin, (double2 *)data, cnt);
      PSE_LAUNCH_CHECK();
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
  });
}

int pse_rfft3d(pse_handle *hd, double *data, int ncomp, int direction) {
  if (!hd) return PSE_ERR_INVALID;
  if (!data || ncomp < 1 || ncomp > NC || (direction != 1 && direction != -1)) {
    hd->h.err = "pse_rfft3d: bad arguments";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    const size_t cnt = (size_t)ncomp * h.ngrid;   // reals = 2 x the half-spectrum complex
    if (h.mixed) {
      float *g = reinterpret_cast<float *>(h.g32.gin);
      from_double<float>(h, data, cnt, g);
      rfft3d<float>(h, g, h.g32.twiddle, ncomp, direction);
      to_double<float>(h, g, cnt, data);
    } else {
      double *g = reinterpret_cast<double *>(h.g64.gin);
      from_double<double>(h, data, cnt, g);
      rfft3d<double>(h, g, h.g64.twiddle, ncomp, direction);
      to_double<double>(h, g, cnt, data);
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
  });
}

int pse_spread(pse_handle *hd, const double *x, const double *q, int ncomp, double *out) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !q || !out || ncomp < 1 || ncomp > NC) {
    hd->h.err = "pse_spread: bad arguments";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    prepare_positions(h, x, h.xw);
    const CompSet cs = comps_range(0, ncomp);
    const size_t cnt = (size_t)ncomp * h.ngrid;
    if (h.mixed) {
      float *g = reinterpret_cast<float *>(h.g32.gin);
      spread<float>(h, h.xw, q, Layout{ncomp, 0}, cs, g);
      to_double<float>(h, g, cnt, out);
    } else {
      double *g = reinterpret_cast<double *>(h.g64.gin);
      spread<double>(h, h.xw, q, Layout{ncomp, 0}, cs, g);
      to_double<double>(h, g, cnt, out);
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
  });
}

int pse_interpolate(pse_handle *hd, const double *x, const double *g, int ncomp,
                    double *out) {
  if (!hd) return PSE_ERR_INVALID;
  if (!x || !g || !out || ncomp < 1 || ncomp > NC) {
    hd->h.err = "pse_interpolate: bad arguments";
    return PSE_ERR_INVALID;
  }
  return guarded(hd, [&] {
    Handle &h = hd->h;
    prepare_positions(h, x, h.xw);
    const CompSet cs = comps_range(0, ncomp);
    const size_t cnt = (size_t)ncomp * h.ngrid;
    if (h.mixed) {
      float *gg = reinterpret_cast<float *>(h.g32.gout);
      from_double<float>(h, g, cnt, gg);
      interpolate<float>(h, h.xw, gg, cs, out, Layout{ncomp, 0}, false, 1.0);
    } else {
      double *gg = reinterpret_cast<double *>(h.g64.gout);
      from_double<double>(h, g, cnt, gg);
      interpolate<double>(h, h.xw, gg, cs, out, Layout{ncomp, 0}, false, 1.0);
    }
    PSE_HIP(hipStreamSynchronize(h.stream));
  });
}

int pse_profile(pse_handle *hd, int enable) {
  if (!hd) return PSE_ERR_INVALID;
  Profiler &P = hd->h.prof;
  if (enable) {
    for (int k = 0; k < PK_COUNT; ++k) {
      P.launches[k] = 0;
      P.ms[k] = 0;
      P.bytes[k] = 0;
    }
    P.pending.clear();
    P.used = 0;
    const int rc = guarded(hd, [&] { bracket_overhead(hd->h, P.bracket_ms, P.noop_ms); });
    if (rc != PSE_OK) return rc;
  }
  P.on = enable != 0;
  return PSE_OK;
}

int pse_profile_read(pse_handle *hd, pse_kernel_stat *out, int max, int *count) {
  if (!hd || !out || !count || max < 0) return PSE_ERR_INVALID;
  Profiler &P = hd->h.prof;
  int c = 0;
  for (int k = 0; k < PK_COUNT && c < max; ++k) {
    if (P.launches[k] == 0) continue;
    out[c++] = pse_kernel_stat{kPkNames[k], P.launches[k], P.ms[k], P.bytes[k]};
  }
  if (c < max) out[c++] = pse_kernel_stat{"bracket", 1, P.bracket_ms, 0.0};
  if (c < max) out[c++] = pse_kernel_stat{"bracket_noop", 1, P.noop_ms, 0.0};
  *count = c;
  return PSE_OK;
}

}  // extern "C"
