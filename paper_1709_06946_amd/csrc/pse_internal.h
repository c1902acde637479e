// Internal declarations of the PSE library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <shared_mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pse.h"

namespace pse {

constexpr int NC = 11;           // generalized force/velocity components
constexpr int MAX_PACK = 6;      // packed complex grids (two real grids each)
// FP64 packed grids per set of a mixed handle: its FP64 work is the
// residual of the constraint solve, M_ES on five components at most
constexpr int MIXED_FP64_PACK = 3;
constexpr int NCOEF = 7;         // real-space coefficient functions

// Error carrying a status code; converted at the ABI boundary.
struct Error {
  int code;
  std::string msg;
};

#define PSE_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::pse::Error{e_ == hipErrorOutOfMemory ? PSE_ERR_NOMEM          \
                                                   : PSE_ERR_HIP,            \
                         std::string(#call) + " (" + __FILE__ + ":" +       \
                             std::to_string(__LINE__) + "): " +                \
                             hipGetErrorString(e_)};                           \
  } while (0)

#define PSE_LAUNCH_CHECK() PSE_HIP(hipGetLastError())

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

// Which 11-vector components an operator reads and writes.
// Where particle vector components live: component c of particle p is at
// ptr[p * stride + c - off] (the full 11-component layout is {NC, 0}; the
// 5-component stresslet / strain vectors of the constraint solve are {5, 6}).
struct Layout {
  int stride;
  int off;
};
constexpr Layout FULL_LAYOUT{NC, 0};

struct CompSet {
  int n;          // number of components
  int idx[NC];    // component indices into the 11-vector
};

// Deformation of the periodic lattice: lattice vectors are the columns of
// L A (row-major A, det 1), Ai = A^-1, G = A^T A as (xx, yy, zz, xy, xz, yz).
// Deformed handles keep positions in lattice coordinates A^-1 x, wrapped into
// [0, L)^3, so that bins, stencils and grids are those of the cube; only
// distances are mapped back by A.
struct Deform {
  int on;
  double A[9], Ai[9], G[6];
  double lambda_max;
  double width;    // thinnest width of the cell over L
};

// Squared length of A d for lattice-coordinate offsets d.
__host__ __device__ inline double qform(const double *G, double dx, double dy, double dz) {
  return G[0] * dx * dx + G[1] * dy * dy + G[2] * dz * dz +
         2.0 * (G[3] * dx * dy + G[4] * dx * dz + G[5] * dy * dz);
}

// Geometry and quadrature constants passed by value to kernels.
struct GridGeom {
  int ng;          // grid points per side
  int P;           // support
  double L, h;     // box, spacing
  double kcoef;    // Gaussian: K1d(d) = knorm exp(-kcoef d^2)
  double knorm;
  int def;         // deformed lattice: distances |A d|^2 = qform(G, d)
  double G[6];
};

// Device workspace of one precision.
template <typename T> struct GridSet {
  cplx<T> *gin = nullptr;    // MAX_PACK packed complex grids
  cplx<T> *gout = nullptr;   // MAX_PACK packed complex grids
  cplx<T> *twiddle = nullptr;  // ng entries exp(-2 pi i m / ng)
  T *table = nullptr;        // real-space coefficient table (ntab x NCOEF)
};

// Counting-sort bins of particles on a uniform nc^3 lattice of the box.
struct Bins {
  int nc = 0;                // bins per side
  int *start = nullptr;      // nc^3 + 1: first slot of each bin in perm
  int *count = nullptr;      // nc^3
  int *of = nullptr;         // N: bin of each particle
  int *slot = nullptr;       // N: arrival slot of the particle within its bin
  int *scat = nullptr;       // N: particles by bin, in arrival order
  int *perm = nullptr;       // N: particles ordered by bin, by index within a bin
  int *scan_tmp = nullptr;   // block sums of the scan
  // the same particles with the bins visited block by block (BIN_BLOCK^3
  // bins per block, blocks in lexicographic order), for the gathers whose
  // neighbouring particles share grid data (interpolation): a contiguous
  // range of it covers a compact region of the box
  int *trav = nullptr;       // N
  int *bcount = nullptr;     // nc^3: bin counts in block order
  int *bstart = nullptr;     // nc^3 + 1: their exclusive sums
};
constexpr int BIN_BLOCK = 4;

// Kernel classes timed by the optional profiler.
enum ProfKind {
  PK_SPREAD = 0, PK_FFT, PK_KSPACE, PK_INTERP, PK_ZERO, PK_REAL, PK_CELLS,
  PK_KRYLOV, PK_NOISE, PK_MISC, PK_COUNT
};

struct ProfRecord {
  int kind;
  hipEvent_t start, stop;
  double bytes;
};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRecord> pending;
  int64_t launches[PK_COUNT] = {};
  double ms[PK_COUNT] = {};
  double bytes[PK_COUNT] = {};
  // event time of an empty bracket (two records back to back; median of a
  // few, taken when profiling starts): the time the two timestamps add to
  // the kernels between them, subtracted once per bracket
  double bracket_ms = 0.0;
  // the same around an empty one-thread kernel (reported only)
  double noop_ms = 0.0;
};

struct Handle {
  pse_params p;
  pse_derived d;
  int64_t n;
  size_t ngrid;              // ng^3
  hipStream_t stream;
  bool own_stream;
  std::string err;

  GridSet<double> g64;
  GridSet<float> g32;
  bool mixed;

  // real-space table layout: uniform spacing dr, node 0 at r = 0, node
  // n2a at r = 2a; ntab nodes in total.
  int ntab, n2a;
  double dr;

  // particle bins: the real-space cell list (side >= rcut) and the
  // spreading tiles (stile^3 grid points each)
  Bins cells;
  Bins sbins;
  int stile;                 // grid points per spreading tile side (0: atomics)
  bool tiles_current = false; // tile lists built at the last cell build's positions
  int max_lds = 65536;       // dynamic LDS a workgroup may use on this device
  int num_cu = 256;          // compute units of the device

  // particle work vectors (double, N x 11 each)
  double *xw = nullptr;      // wrapped positions N x 3
  double *xh = nullptr;      // mid-point positions N x 3
  double *v0 = nullptr, *v1 = nullptr, *v2 = nullptr, *v3 = nullptr;
  double *v4 = nullptr, *v5 = nullptr;
  double *es_b = nullptr, *es_x = nullptr, *es_r = nullptr, *es_d = nullptr;  // N x 5
  double *es_p = nullptr;    // N x 5: the preconditioned vector of the constraint solve
  // self terms of M_ES (real-space part, whole operator) for its preconditioner
  double es_self_real = 0.0, es_self_total = 0.0;

  double *ktab = nullptr;    // per-|k|^2 radial factors (4 doubles per entry)
  float *ktab32 = nullptr;   // the same rounded to float (mixed handles)
  double *kdg = nullptr;     // derivative gridding: the constraint operator's k-space
  float *kdg32 = nullptr;    // factor -9 f1^2 mob per |k|^2 (FP64; FP32 in mixed handles)
  int *bad_pos = nullptr;    // set by the wrap kernel on a non-finite coordinate
  double *dg_mu = nullptr;   // derivative gridding: moment corrections, 6 per particle
  void *mpack = nullptr;     // pair sums: moments packed 12 per particle (FP64 size)
  // real-space pair list (CSR in cell order): start[N+1], neighbour index and
  // 10 numbers of pair data per entry (doubles in FP64 handles, floats in
  // mixed ones); counts and scan scratch
  int *pl_cnt = nullptr, *pl_start = nullptr, *pl_scan = nullptr, *pl_nbr = nullptr;
  double *pl_rec64 = nullptr;
  float *pl_rec32 = nullptr;
  size_t pl_cap = 0, pl_pairs = 0;
  // spreading-tile candidate lists (CSR over tiles): one record per (tile,
  // particle) pair, tl_cap records at most
  int *tl_cnt = nullptr, *tl_start = nullptr, *tl_scan = nullptr;
  void *tl_rec = nullptr;
  size_t tl_cap = 0;

  // Krylov storage
  double *lz_V = nullptr;    // (lanczos_maxit + 1) x 11N
  double *gm_V = nullptr;    // (gmres_restart + 1) x 5N
  double *small = nullptr;   // device scratch for dots / tridiagonal / Hessenberg
  size_t small_len;
  double *dots = nullptr;    // partial sums for reductions
  size_t dots_len;

  Profiler prof;

  // captured constraint-operator applications, keyed by (input, output,
  // kind); cleared when a buffer baked into them is reallocated
  bool use_graphs = true;
  bool deriv = false;        // derivative gridding in the constraint operator
  // iteration counts of the previous Lanczos and GMRES (FP64, FP32) solves
  int lz_prev = 0;
  int lz_prev_rpy = 0;       // the same for the RPY sampler's UF-block Lanczos
  int gm_prev[2] = {0, 0};
  bool graph_warm = false;   // one eager application before the first capture
  std::string graph_error;   // why graphs were switched off after a failed capture
  std::map<std::tuple<const void *, const void *, int>, hipGraphExec_t> graphs;

  // Asynchronous handles (params.async_calls): Krylov solves checked on the
  // device, no host synchronisation inside a call.  dctl: device control
  // words (CTL_*), dstats: the step statistics kept on the device, dstep:
  // the device step counter used for step = PSE_STEP_DEVICE, counter_dev:
  // that counter while a call uses it (else NULL).
  bool async = false;
  int lz_cap = 0, gm_cap = 0, ref_cap = 0;   // iterations / passes of those solves
  int *dctl = nullptr;
  pse_stats *dstats = nullptr;
  uint64_t *dstep = nullptr;
  const uint64_t *counter_dev = nullptr;

  Deform def{};              // lattice deformation (def.on = 0: the cube)

  // A handle with an arena takes every device buffer from it (bump
  // allocation, 256-byte aligned) instead of the runtime, and frees nothing.
  unsigned char *arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
};

// Device control words of a handle (ints at h.dctl): Lanczos and GMRES
// selection state (found, count, not converged), the status bits
// (PSE_STATUS_*) of asynchronous calls.
enum { CTL_LZ = 0, CTL_GM = 4, CTL_STATUS = 8, CTL_WORDS = 16 };

// Device buffer of a handle: from its arena when it has one (throws
// PSE_ERR_NOMEM when the arena is full), else from the runtime (dev_alloc).
void handle_alloc(Handle &h, void **p, size_t bytes);

// Destroys every captured graph of the handle.
void clear_graphs(Handle &h);

// The runtime refuses allocations, frees and legacy-stream copies while any
// stream of the process captures a graph (and such a call invalidates the
// capture), even when the capturing stream is non-blocking and owned by
// another thread.  The library's captures hold this gate shared; its
// allocations, frees and synchronous copies (dev_alloc, dev_free, dev_copy)
// hold it exclusively, so the two never overlap across threads.
std::shared_mutex &capture_gate();
void dev_alloc(void **p, size_t bytes);          // hipMalloc; throws on failure
void dev_free(void *p);                          // hipFree of a non-null pointer
hipError_t dev_copy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);

// Sets the calling thread's stream-capture interaction mode to relaxed for
// the scope (restoring the previous mode after).  Allocations, frees and
// synchronous copies made by this thread while another thread captures a
// graph on its own stream are then not refused; the library's captures hold
// kernel launches on the capturing handle's stream only, which such calls do
// not touch.
struct RelaxedCaptureScope {
  hipStreamCaptureMode prev = hipStreamCaptureModeRelaxed;
  RelaxedCaptureScope() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
  ~RelaxedCaptureScope() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
  RelaxedCaptureScope(const RelaxedCaptureScope &) = delete;
  RelaxedCaptureScope &operator=(const RelaxedCaptureScope &) = delete;
};

// Brackets the launches of one stage with events when profiling is on.
struct ProfScope {
  Handle &h;
  int idx = -1;
  ProfScope(Handle &hh, int kind, double bytes) : h(hh) {
    if (!h.prof.on) return;
    Profiler &P = h.prof;
    while (P.pool.size() < P.used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      P.pool.push_back(e);
    }
    ProfRecord r{kind, P.pool[P.used], P.pool[P.used + 1], bytes};
    P.used += 2;
    (void)hipEventRecord(r.start, h.stream);
    idx = (int)P.pending.size();
    P.pending.push_back(r);
  }
  ~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(h.prof.pending[idx].stop, h.stream);
  }
};

// Accumulate the pending records (the stream must be idle).
void prof_resolve(Handle &h);

// ---- params.cpp
void derive(const pse_params &p, pse_derived &d);
void deformation(const pse_params &p, Deform &df);   // throws when det A != 1
size_t footprint(const pse_params &p, const pse_derived &d);

// ---- fft.hip
// complex 3D transform of ncomp full grids [c][z][y][x] (diagnostic)
template <typename T>
void fft3d(Handle &h, cplx<T> *data, const cplx<T> *twiddle, int ncomp, int dir);
// real 3D transform of ncomp real grids [c][z][y][x] in place: dir = -1
// leaves half spectra [c][kz][ky][kx < n/2], dir = +1 inverts
template <typename T>
void rfft3d(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir);
// the x and y passes (forward: x then y; inverse: y then x) and the z pass
template <typename T>
void rfft_xy(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir);
template <typename T>
void rfft_z(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir);

// ---- grid.hip
// Real grids [c][z][y][x] (T), half spectra [c][kz][ky][kx < n/2] (cplx<T>)
// in the same storage; component stride ngrid reals = ngrid/2 complex.
template <typename T>
void spread(Handle &h, const double *x, const double *q, Layout lq, const CompSet &cs,
            T *grids);
template <typename T>
void interpolate(Handle &h, const double *x, const T *grids, const CompSet &cs, double *out,
                 Layout lo, bool accumulate, double scale);
// dg: outputs are the grid codes of derivative gridding (see kspace_fused)
template <typename T>
void kspace_noise(Handle &h, const double *psi, uint64_t seed, uint64_t counter,
                  cplx<T> *out, const CompSet &cout, bool dg = false);
// the same for derivative-gridding codes, with the inverse z transform
// fused; false (nothing launched) where that form is not built
template <typename T>
bool kspace_noise_z(Handle &h, const double *psi, uint64_t seed, uint64_t counter,
                    cplx<T> *out, const CompSet &cout, const cplx<T> *tw);
// z transform + k-space + inverse z transform in one kernel; dg: cin and
// cout are grid codes of derivative gridding, 0-2 force grids (in) or
// velocity grids j0 u (out), 3-5 couplet grids (in) or 3 f1 u grids (out)
template <typename T>
void kspace_fused(Handle &h, const cplx<T> *in, const CompSet &cin, cplx<T> *out,
                  const CompSet &cout, const cplx<T> *tw, bool dg = false);
// derivative gridding: forces (hf: all three in cs, first) onto three grids
// and couplets (torques with hasL, stresslets with hasS, complete groups in
// cs, in that order) onto three more; interpolation of velocity (hu) from
// the first three of six grids and of rotation and strain from the gradient
// of the other three (any components cs)
template <typename T>
void spread_deriv(Handle &h, const double *q, Layout lq, const CompSet &cs, bool hf, bool hasL,
                  bool hasS, T *grids);
template <typename T>
void interp_deriv(Handle &h, const double *x, const T *grids, bool hu, const CompSet &cs,
                  double *out, Layout lo, bool accumulate, double scale);
// k-space kernel of a deformed lattice on full half spectra (all three
// axes transformed)
template <typename T>
void kspace_deformed(Handle &h, const cplx<T> *in, const CompSet &cin, cplx<T> *out,
                     const CompSet &cout);
template <typename T> void zero_grids(Handle &h, T *g, int ncomp);
void build_tile_lists(Handle &h, const double *xw);
// moment corrections of the gradient weights (derivative-gridding handles)
void build_dg_mu(Handle &h, const double *xw);
size_t tile_record_bytes(int S);                  // one (tile, particle) record
int ktable_len(int grid);                         // entries of the |k|^2 table
void build_ktable(Handle &h);
template <typename T> void from_double(Handle &h, const double *src, size_t n, T *dst);
template <typename T> void to_double(Handle &h, const T *src, size_t n, double *dst);

// Initial capacity of the real-space pair list: twice the pair count of a
// uniform suspension (neighbours within rcut), plus slack.
// Pair-list storage for cap entries (neighbour indices and pair data): at
// creation from the handle's workspace, later replacing the previous storage.
void pair_storage(Handle &h, size_t cap, bool at_create);
// bytes of one pair-list entry
inline size_t pair_entry_bytes(bool mixed) {
  return sizeof(int) + 10 * (mixed ? sizeof(float) : sizeof(double));
}
inline size_t pair_capacity(const pse_params &p, const pse_derived &d) {
  const double dens = (double)p.n / (p.box * p.box * p.box);
  const double nb = 4.18879020478639098 * d.rcut * d.rcut * d.rcut * dens;
  return (size_t)(2.0 * nb * (double)p.n) + 1024;
}

// Most spreading tiles (S^3 points) one P-point stencil can meet.
inline size_t tiles_per_particle(int P, int S) {
  const size_t k = (size_t)((P - 1 + S - 1) / S + 1);
  return k * k * k;
}
// Spreading tile side: the stencil may reach one tile beyond its particle's
// bin, with one grid point of slack for rounding in the bin assignment.
inline int spread_tile(int grid, int P) {
  for (int S : {8, 4, 16}) {
    const int need = (P & 1) ? P + 1 : P + 2;
    if (grid % S == 0 && grid / S >= 3 && need <= 2 * S) return S;
  }
  return 0;
}

// Workgroups are dispatched to the 8 XCDs in turn; this maps the dispatch
// index to a logical block so that each XCD takes a contiguous range of
// logical blocks (and its L2 sees neighbouring work).  A bijection of
// [0, nb).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % 8, i = b / 8, per = nb / 8, rem = nb % 8;
  return x * per + (x < rem ? x : rem) + i;
}

// ---- neighbour-bin enumeration (device helpers shared by the list builders)

// Lanes 0..26 of a wavefront take the 27 bins around (cx, cy, cz) of a
// periodic nc^3 lattice (bin offsets in x fastest) and load their first slot
// and length (none for a lane whose skip is set); an inclusive scan over the
// wavefront gives each bin's offset `pre` in the concatenated candidate
// sequence of length `total`.
__device__ __forceinline__ void nbr27_setup(int lane, int cx, int cy, int cz, int nc,
                                            const int *__restrict__ start, int &first,
                                            int &pre, int &total, bool skip = false) {
  int len = 0;
  first = 0;
  if (lane < 27 && !skip) {
    const int bx = (cx + lane % 3 - 1 + nc) % nc;
    const int by = (cy + (lane / 3) % 3 - 1 + nc) % nc;
    const int bz = (cz + lane / 9 - 1 + nc) % nc;
    const int b = (bz * nc + by) * nc + bx;
    first = start[b];
    len = start[b + 1] - first;
  }
  int incl = len;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  pre = incl - len;
  total = __shfl(incl, 63, 64);
}

// Slot (in the bins' permutation) of candidate idx < total; every lane of
// the wavefront must call it (binary search over the lanes' offsets).
__device__ __forceinline__ int nbr27_slot(int idx, int first, int pre) {
  int lo = 0;
#pragma unroll
  for (int step = 16; step > 0; step >>= 1) {
    const int c = lo + step;
    const int pc = __shfl(pre, c < 27 ? c : 26, 64);
    if (c < 27 && pc <= idx) lo = c;
  }
  return __shfl(first, lo, 64) + idx - __shfl(pre, lo, 64);
}

// ---- real.hip
void build_tables(Handle &h);
void exclusive_scan(Handle &h, const int *in, int *out, int *tmp, int n);
// Cell list and pair list for wrapped positions xw, the spreading bins and
// tile lists too unless spreading is false (positions where only pair sums
// and interpolation run).
void build_cells(Handle &h, const double *xw, bool spreading = true);
template <typename T>
void real_apply(Handle &h, const double *x, const double *in, Layout lin,
                const CompSet &cin, double *out, Layout lout, const CompSet &cout,
                bool accumulate);
void wrap_positions(Handle &h, const double *x, double *xw);

// ---- krylov.hip / blas
void vzero(Handle &h, double *v, size_t n);
void fill_int(Handle &h, int *v, size_t n, int value);   // kernel, not a memset node
void vcopy(Handle &h, double *dst, const double *src, size_t n);
void vaxpby(Handle &h, double a, const double *x, double b, double *y, size_t n);
void multi_dot(Handle &h, const double *V, size_t ldv, int m, const double *w,
               size_t n, double *dev_out);
void vsub_multi(Handle &h, double *w, const double *V, size_t ldv, int m,
                const double *coef_dev, size_t n);
void gemv_small(Handle &h, const double *V, size_t ldv, int m,
                const double *coef_dev, double *y, size_t n, double alpha,
                bool accumulate, const int *m_dev = nullptr);
void vscale_dev(Handle &h, double *dst, const double *src, const double *s_dev,
                bool invert, size_t n);
void gather_comps(Handle &h, const double *src, int sstride, const CompSet &cs,
                  double *dst, size_t n);
void scatter_comps(Handle &h, const double *src, const CompSet &cs,
                   double *dst, int dstride, size_t n, bool accumulate,
                   double alpha);
int check_finite(Handle &h, const double *v, size_t n);

struct KrylovResult {
  int iters;
  double resid;      // Lanczos: last relative change; GMRES: relative residual
  bool converged;
};
using Op = std::function<void(const double *in, double *out)>;
// prev_iters (may be null): the previous solve's iteration count, read and
// updated; the convergence checks start two iterations before it.
KrylovResult lanczos_sqrt(Handle &h, const Op &A, const double *b, size_t n,
                          double *y, int maxit, double tol, int *prev_iters);
KrylovResult gmres(Handle &h, const Op &A, const double *b, size_t n, double *x,
                   int restart, int maxit, double tol, int *prev_iters);
// Device-checked forms for asynchronous handles: exactly K iterations, the
// result taken at the first one that met tol (no restarts); iteration
// counts, residuals and convergence go to h.dstats.
void lanczos_sqrt_dev(Handle &h, const Op &A, const double *b, size_t n, double *y, int K,
                      double tol);
void gmres_dev(Handle &h, const Op &A, const double *b, size_t n, double *x, int K,
               double tol);

// ---- grid.hip (noise)
// N x ncomp standard normals (the first ncomp of each particle's Philox
// draws, so the F components agree for every ncomp).
void real_noise(Handle &h, uint64_t seed, uint64_t counter, double *out, int ncomp = NC);

inline CompSet comps_range(int lo, int hi) {
  CompSet c{};
  c.n = hi - lo;
  for (int i = 0; i < c.n; ++i) c.idx[i] = lo + i;
  return c;
}

inline unsigned nblocks(size_t n, unsigned t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

}  // namespace pse
