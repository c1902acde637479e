// Real-space part of the Ewald sum (Sec. II.C.1, Eqs. MUFr-MDCr, pairsums).
//
// Pair functions.  Writing T_pq for the inverse transform of
// f_p f_q (I - kk) / (eta k^2) (f_0 = j0(ka), f_1 = (sin ka - ka cos ka)/(ka)^3,
// the shape factors of Eqs. MUF-MDC), with k_n <-> -i d_n:
//   M_UF = T00,  M_UC_imn = -3 d_n T01_im,  M_DF_ijm = 3 d_j T01_im,
//   M_DC_ijmn = -9 d_j d_n T11_im,   T_pq = (grad grad - I lap) phi_pq,
// phi_pq the inverse transform of f_p f_q / (eta k^4).  With
// Phi_n = ((1/r) d/dr)^n phi every block follows from seven radial
// coefficients (the count of the paper's F1 F2 / G1 G2 / K1 K2 K3):
//   a = -(r^2 Phi2 + 2 Phi1), b = r^2 Phi2                 (pq = 00)
//   c1 = r^3 Phi3, c2 = r Phi2                             (pq = 01)
//   d2 = Phi2, d3 = r^2 Phi3, d4 = r^4 Phi4                (pq = 11)
// The real-space part (factor 1 - H) is "free space" minus "H part":
//  * free space: f_0 and f_1 transform to a shell density
//    delta(r - a)/(4 pi a^2) and a ball density 1/(4 pi a^3), and 1/k^4 to
//    -r/(8 pi), so phi_pq = -(1/8 pi eta) (shell/ball autocorrelation * r).
//    Carrying out the radial integrals gives, with A = -1/(8 pi eta),
//      phi00 = A (4a/3 + r^2/3a - r^3/24a^2),              r < 2a
//            = A (r + 2a^2/3r),                             r >= 2a
//      phi01 = A (2a/5 + r^2/9a - r^4/120a^3 + r^5/720a^4), r < 2a
//            = A (r/3 + 8a^2/45r),                          r >= 2a
//      phi11 = A (4a/35 + 2r^2/45a - r^4/180a^3 + r^5/720a^4
//                 - r^7/40320a^6),                          r < 2a
//            = A (r/9 + 2a^2/45r),                          r >= 2a
//    whose Phi_n are written out in free_coefficients();
//  * H part: Phi_n^H(r) = 1/(2 pi^2 eta) int_0^inf H(k) f_p f_q (-1)^n
//    k^(2n-2) j_n(kr)/(kr)^n dk, by the trapezoidal rule, which converges
//    geometrically for this even, Gaussian-damped integrand.
// Both are tabulated once per handle on the GPU (FP64) on a uniform r grid
// with a node at r = 2a, and interpolated with 4-point Lagrange stencils that
// never straddle r = 2a.
#include "pse_internal.h"

namespace pse {

// ------------------------------------------------------------- tables --

__device__ double jn_over_xn(int n, double x) {
  // j_n(x)/x^n: power series below x = 4, upward recurrence above.
  if (x < 4.0) {
    double df = 1.0;
    for (int k = 3; k <= 2 * n + 1; k += 2) df *= k;
    double term = 1.0 / df, acc = term;
    const double t = -0.5 * x * x;
    for (int k = 1; k < 40; ++k) {
      term *= t / (k * (2 * n + 2 * k + 1));
      acc += term;
    }
    return acc;
  }
  double s, c;
  sincos(x, &s, &c);
  double jm = s / x;                   // j0
  if (n == 0) return jm;
  double j = s / (x * x) - c / x;      // j1
  for (int m = 1; m < n; ++m) {
    const double jp = (2 * m + 1) / x * j - jm;
    jm = j;
    j = jp;
  }
  double xn = x;
  for (int m = 1; m < n; ++m) xn *= x;
  return j / xn;
}

__device__ void free_coefficients(double r, double a, double eta, double *co) {
  const double A = -1.0 / (8.0 * M_PI * eta);
  double v[NCOEF];
  if (r < 2.0 * a) {
    const double a2 = a * a, a3 = a2 * a, a4 = a3 * a, a6 = a3 * a3;
    const double r2 = r * r, r3 = r2 * r;
    // phi00: Phi1 = 2/3a - r/8a^2, Phi2 = -1/(8 a^2 r)
    v[0] = -4.0 / (3.0 * a) + 3.0 * r / (8.0 * a2);
    v[1] = -r / (8.0 * a2);
    // phi01: Phi2 = -1/15a^3 + r/48a^4, Phi3 = 1/(48 a^4 r)
    v[2] = r2 / (48.0 * a4);
    v[3] = -r / (15.0 * a3) + r2 / (48.0 * a4);
    // phi11: Phi2 = -2/45a^3 + r/48a^4 - r^3/1152a^6,
    //        Phi3 = 1/(48 a^4 r) - r/384a^6, Phi4 = -1/(48 a^4 r^3) - 1/(384 a^6 r)
    v[4] = -2.0 / (45.0 * a3) + r / (48.0 * a4) - r3 / (1152.0 * a6);
    v[5] = r / (48.0 * a4) - r3 / (384.0 * a6);
    v[6] = -r / (48.0 * a4) - r3 / (384.0 * a6);
  } else {
    const double a2 = a * a, r2 = r * r, r3 = r2 * r, r4 = r2 * r2, r5 = r4 * r;
    // phi00: Phi1 = 1/r - 2a^2/3r^3, Phi2 = -1/r^3 + 2a^2/r^5
    v[0] = -(1.0 / r + 2.0 * a2 / (3.0 * r3));
    v[1] = -1.0 / r + 2.0 * a2 / r3;
    // phi01: Phi2 = -1/3r^3 + 8a^2/15r^5, Phi3 = 1/r^5 - 8a^2/3r^7
    v[2] = 1.0 / r2 - 8.0 * a2 / (3.0 * r4);
    v[3] = -1.0 / (3.0 * r2) + 8.0 * a2 / (15.0 * r4);
    // phi11: Phi2 = -1/9r^3 + 2a^2/15r^5, Phi3 = 1/3r^5 - 2a^2/3r^7,
    //        Phi4 = -5/3r^7 + 14a^2/3r^9
    v[4] = -1.0 / (9.0 * r3) + 2.0 * a2 / (15.0 * r5);
    v[5] = 1.0 / (3.0 * r3) - 2.0 * a2 / (3.0 * r5);
    v[6] = -5.0 / (3.0 * r3) + 14.0 * a2 / (3.0 * r5);
  }
  for (int i = 0; i < NCOEF; ++i) co[i] = A * v[i];
}

__global__ void table_kernel(double *__restrict__ tab, float *__restrict__ tab32,
                             int ntab, double dr, double a, double eta, double xi,
                             double dk, int nk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntab) return;
  const double r = i * dr;
  double fc[NCOEF];
  free_coefficients(r, a, eta, fc);
  // H part: Phi1_00, Phi2_00, Phi2_01, Phi3_01, Phi2_11, Phi3_11, Phi4_11
  double S[7] = {0, 0, 0, 0, 0, 0, 0};
  const double inv4xi2 = 1.0 / (4.0 * xi * xi);
  for (int m = 0; m <= nk; ++m) {
    const double k = m * dk;
    const double w = (m == 0) ? 0.5 * dk : dk;
    const double u = k * k * inv4xi2;
    const double H = (1.0 + u) * exp(-u);
    const double f0 = jn_over_xn(0, k * a), f1 = jn_over_xn(1, k * a);
    const double kr = k * r;
    const double J1 = jn_over_xn(1, kr), J2 = jn_over_xn(2, kr);
    const double J3 = jn_over_xn(3, kr), J4 = jn_over_xn(4, kr);
    const double k2 = k * k, k4 = k2 * k2, k6 = k4 * k2;
    const double wh = w * H;
    S[0] += -wh * f0 * f0 * J1;
    S[1] += wh * f0 * f0 * k2 * J2;
    S[2] += wh * f0 * f1 * k2 * J2;
    S[3] += -wh * f0 * f1 * k4 * J3;
    S[4] += wh * f1 * f1 * k2 * J2;
    S[5] += -wh * f1 * f1 * k4 * J3;
    S[6] += wh * f1 * f1 * k6 * J4;
  }
  const double c = 1.0 / (2.0 * M_PI * M_PI * eta);
  for (int j = 0; j < 7; ++j) S[j] *= c;
  const double r2 = r * r;
  double hc[NCOEF];
  hc[0] = -(r2 * S[1] + 2.0 * S[0]);
  hc[1] = r2 * S[1];
  hc[2] = r2 * r * S[3];
  hc[3] = r * S[2];
  hc[4] = S[4];
  hc[5] = r2 * S[5];
  hc[6] = r2 * r2 * S[6];
  for (int j = 0; j < NCOEF; ++j) {
    const double v = fc[j] - hc[j];
    tab[(size_t)i * NCOEF + j] = v;
    tab32[(size_t)i * NCOEF + j] = (float)v;
  }
}

void build_tables(Handle &h) {
  const double a = h.p.radius, xi = h.d.xi;
  h.n2a = 2048;
  h.dr = 2.0 * a / h.n2a;
  h.ntab = (int)std::ceil(h.d.rcut / h.dr) + 8;
  handle_alloc(h, (void **)&h.g64.table, (size_t)h.ntab * NCOEF * sizeof(double));
  handle_alloc(h, (void **)&h.g32.table, (size_t)h.ntab * NCOEF * sizeof(float));
  const double rmax = h.ntab * h.dr;
  const double dk = M_PI / (2.0 * a + rmax + 7.0 / xi);
  const double kmax = 2.0 * xi * std::sqrt(50.0);
  const int nk = (int)std::ceil(kmax / dk);
  hipLaunchKernelGGL(table_kernel, dim3(nblocks(h.ntab, 128)), dim3(128), 0,
                     h.stream, h.g64.table, h.g32.table, h.ntab, h.dr, a,
                     h.p.viscosity, xi, dk, nk);
  PSE_LAUNCH_CHECK();
}

// ---------------------------------------------------------- positions --

// Non-finite coordinates raise *bad and are replaced by 0, so that every
// later kernel stays in bounds until the host reports the error.
// Positions of a deformed lattice to lattice coordinates A^-1 x (then
// wrapped like the cube's).
__global__ void lattice_coords_kernel(const double *__restrict__ x, double *__restrict__ xl,
                                      int64_t n, Deform df) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double p[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
  for (int r = 0; r < 3; ++r)
    xl[3 * i + r] = df.Ai[3 * r] * p[0] + df.Ai[3 * r + 1] * p[1] + df.Ai[3 * r + 2] * p[2];
}

__global__ void wrap_kernel(const double *__restrict__ x, double *__restrict__ xw,
                            int64_t n3, double L, int *__restrict__ bad,
                            int *__restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = x[i];
  if (!isfinite(v)) {
    *bad = 1;
    atomicOr(status, (int)PSE_STATUS_NONFINITE_POS);
    v = 0.0;
  }
  v -= L * floor(v / L);
  if (v >= L) v -= L;
  if (v < 0) v = 0;
  xw[i] = v;
}

void wrap_positions(Handle &h, const double *x, double *xw) {
  // the flag is cleared by a kernel, not a memset node, so that the launches
  // can be captured into graphs
  fill_int(h, h.bad_pos, 1, 0);
  if (h.def.on) {
    // lattice coordinates first, then wrapped in place like the cube's
    hipLaunchKernelGGL(lattice_coords_kernel, dim3(nblocks(h.n, 256)), dim3(256), 0,
                       h.stream, x, xw, h.n, h.def);
    PSE_LAUNCH_CHECK();
    x = xw;
  }
  hipLaunchKernelGGL(wrap_kernel, dim3(nblocks(3 * h.n, 256)), dim3(256), 0,
                     h.stream, x, xw, 3 * h.n, h.p.box, h.bad_pos, h.dctl + CTL_STATUS);
  PSE_LAUNCH_CHECK();
}

// ----------------------------------------------------------- cell list --

__global__ void cell_assign_kernel(const double *__restrict__ xw, int64_t n,
                                   int nc, double inv_cs, int *__restrict__ cell_of,
                                   int *__restrict__ slot, int *__restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3];
  for (int d = 0; d < 3; ++d) {
    int v = (int)(xw[3 * i + d] * inv_cs);
    c[d] = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
  }
  const int cell = (c[2] * nc + c[1]) * nc + c[0];
  cell_of[i] = cell;
  slot[i] = atomicAdd(&count[cell], 1);
}

// Exclusive scan in chunks of 1024 (256 threads x 4).
__global__ void scan_block_kernel(const int *__restrict__ in, int *__restrict__ out,
                                  int *__restrict__ block_sums, int n) {
  __shared__ int s[256];
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  int v[4], sum = 0;
  for (int j = 0; j < 4; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    sum += v[j];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int run = s[threadIdx.x] - sum;
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 255) block_sums[blockIdx.x] = s[255];
}

__global__ void scan_sums_kernel(int *__restrict__ sums, int nb, int *__restrict__ total) {
  // single block: exclusive scan of nb block sums with a running carry
  __shared__ int s[256];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += 256) {
    const int i = b0 + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += s[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void scan_add_kernel(int *__restrict__ out, const int *__restrict__ sums, int n) {
  const int i = blockIdx.x * 1024 + threadIdx.x * 4;
  const int add = sums[blockIdx.x];
  for (int j = 0; j < 4; ++j)
    if (i + j < n) out[i + j] += add;
}

// Exclusive scan of at most 1024 x SCAN1_PER ints in one workgroup: thread
// t takes a contiguous chunk, the chunk totals are scanned within each wave
// (shuffles) and across the 16 waves (LDS), and every thread then writes its
// chunk's prefixes; out[n] = total.  One launch instead of three.
constexpr int SCAN1_PER = 16;

__global__ void __launch_bounds__(1024)
scan_single_kernel(const int *__restrict__ in, int *__restrict__ out, int n) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int per = (n + 1023) / 1024;
  const int lo = t * per, hi = min(lo + per, n);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += in[i];
  int incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    const int w = lane < 16 ? wsum[lane] : 0;
    int wi = w;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int u = __shfl_up(wi, off, 64);
      if (lane >= off) wi += u;
    }
    if (lane < 16) wsum[lane] = wi - w;
  }
  __syncthreads();
  int run = wsum[wv] + incl - sum;
  for (int i = lo; i < hi; ++i) {
    const int x = in[i];
    out[i] = run;
    run += x;
  }
  if (t == 1023) out[n] = run;
}

__global__ void cell_scatter_kernel(const int *__restrict__ cell_of,
                                    const int *__restrict__ slot,
                                    const int *__restrict__ start, int64_t n,
                                    int *__restrict__ scat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  scat[start[cell_of[i]] + slot[i]] = (int)i;
}

// The arrival order within a bin (atomic slots) varies from run to run; every
// later sum runs in bin order, so each bin's members are put in increasing
// particle index: one wavefront per bin, member p going to the position of
// its rank among the bin's indices.  Results are then reproducible bit for
// bit.
__global__ void __launch_bounds__(256)
cell_order_kernel(const int *__restrict__ start, const int *__restrict__ scat, int nbins,
                  int *__restrict__ perm) {
  const int bin = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (bin >= nbins) return;
  const int lo = start[bin], k = start[bin + 1] - lo;
  for (int p = lane; p < k; p += 64) {
    const int v = scat[lo + p];
    int rank = 0;
    for (int q = 0; q < k; ++q) rank += scat[lo + q] < v ? 1 : 0;
    perm[lo + rank] = v;
  }
}

// Bin b of an nc^3 lattice (x fastest) at its position in block order:
// blocks of BIN_BLOCK^3 bins in lexicographic order, bins lexicographic
// within a block (partial blocks at the far faces).
__device__ __forceinline__ int block_order_pos(int b, int nc) {
  const int bx = b % nc, by = (b / nc) % nc, bz = b / (nc * nc);
  const int B = BIN_BLOCK, nb = (nc + B - 1) / B;
  const int Bx = bx / B, By = by / B, Bz = bz / B;
  // bins before this block: full slabs and rows of blocks, with the widths
  // of the partial blocks at the far faces
  const auto w = [&](int blk) { return blk + 1 < nb ? B : nc - B * (nb - 1); };
  const int wx = w(Bx), wy = w(By);
  const int before = Bz * B * nc * nc + By * B * nc * w(Bz) + Bx * B * wy * w(Bz);
  const int lx = bx - Bx * B, ly = by - By * B, lz = bz - Bz * B;
  return before + (lz * wy + ly) * wx + lx;
}

// counts permuted into block order
__global__ void block_count_kernel(const int *__restrict__ count, int nc,
                                   int *__restrict__ bcount) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nc * nc * nc) return;
  bcount[block_order_pos(b, nc)] = count[b];
}

// trav: each bin's members (in perm order) at the bin's block-order offset
__global__ void block_trav_kernel(const int *__restrict__ start, const int *__restrict__ perm,
                                  const int *__restrict__ bstart, int nc,
                                  int *__restrict__ trav) {
  const int b = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (b >= nc * nc * nc) return;
  const int lo = start[b], k = start[b + 1] - lo, dst = bstart[block_order_pos(b, nc)];
  for (int p = lane; p < k; p += 64) trav[dst + p] = perm[lo + p];
}

// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total); tmp holds
// n/1024 + 8 ints.
void exclusive_scan(Handle &h, const int *in, int *out, int *tmp, int n) {
  if (n <= 1024 * SCAN1_PER) {
    hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(1024), 0, h.stream, in, out, n);
    PSE_LAUNCH_CHECK();
    return;
  }
  const int sb = (n + 1023) / 1024;
  hipLaunchKernelGGL(scan_block_kernel, dim3(sb), dim3(256), 0, h.stream, in, out, tmp, n);
  PSE_LAUNCH_CHECK();
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, h.stream, tmp, sb, out + n);
  PSE_LAUNCH_CHECK();
  hipLaunchKernelGGL(scan_add_kernel, dim3(sb), dim3(256), 0, h.stream, out, tmp, n);
  PSE_LAUNCH_CHECK();
}

static void build_bins(Handle &h, const double *xw, Bins &b) {
  const int nc = b.nc;
  const int ncells = nc * nc * nc;
  fill_int(h, b.count, ncells, 0);
  hipLaunchKernelGGL(cell_assign_kernel, dim3(nblocks(h.n, 256)), dim3(256), 0,
                     h.stream, xw, h.n, nc, nc / h.p.box, b.of, b.slot, b.count);
  PSE_LAUNCH_CHECK();
  exclusive_scan(h, b.count, b.start, b.scan_tmp, ncells);
  hipLaunchKernelGGL(cell_scatter_kernel, dim3(nblocks(h.n, 256)), dim3(256), 0,
                     h.stream, b.of, b.slot, b.start, h.n, b.scat);
  PSE_LAUNCH_CHECK();
  hipLaunchKernelGGL(cell_order_kernel, dim3((unsigned)((ncells + 3) / 4)), dim3(256), 0,
                     h.stream, b.start, b.scat, ncells, b.perm);
  PSE_LAUNCH_CHECK();
  if (b.trav) {
    hipLaunchKernelGGL(block_count_kernel, dim3(nblocks(ncells, 256)), dim3(256), 0, h.stream,
                       b.count, nc, b.bcount);
    PSE_LAUNCH_CHECK();
    exclusive_scan(h, b.bcount, b.bstart, b.scan_tmp, ncells);
    hipLaunchKernelGGL(block_trav_kernel, dim3((unsigned)((ncells + 3) / 4)), dim3(256), 0,
                       h.stream, b.start, b.perm, b.bstart, nc, b.trav);
    PSE_LAUNCH_CHECK();
  }
}

// ------------------------------------------------------------ pair sum --

template <typename T>
__device__ __forceinline__ void lookup(const T *__restrict__ tab, T r, T inv_dr,
                                       int n2a, int ntab, T *co) {
  const T f = r * inv_dr;
  int i0 = (int)f;
  int base;
  if (i0 < n2a) {
    base = i0 - 1;
    if (base < 0) base = 0;
    if (base > n2a - 3) base = n2a - 3;
  } else {
    base = i0 - 1;
    if (base < n2a) base = n2a;
    if (base > ntab - 4) base = ntab - 4;
  }
  const T t = f - (T)base;
  const T w0 = -(t - 1) * (t - 2) * (t - 3) / (T)6;
  const T w1 = t * (t - 2) * (t - 3) / (T)2;
  const T w2 = -t * (t - 1) * (t - 3) / (T)2;
  const T w3 = t * (t - 1) * (t - 2) / (T)6;
  const T *p = tab + (size_t)base * NCOEF;
#pragma unroll
  for (int j = 0; j < NCOEF; ++j)
    co[j] = w0 * p[j] + w1 * p[NCOEF + j] + w2 * p[2 * NCOEF + j] + w3 * p[3 * NCOEF + j];
}

// Acting with the pair block M(r) on (F, C) of the partner; adds to U and D.
// UF, UC: forces, couplets present; OU, OD: velocity, gradient wanted (the
// coefficients a, b serve F -> U; c1, c2 serve F -> D and C -> U; d2, d3, d4
// serve C -> D; only those of the selected couplings are read).
template <typename T, bool UF, bool UC, bool OU, bool OD>
__device__ __forceinline__ void pair_action(const T *co, const T *e, const T *F,
                                                const T (*C)[3], T *U, T (*D)[3]) {
  const T a = co[0], b = co[1], c1 = co[2], c2 = co[3];
  const T d2 = co[4], d3 = co[5], d4 = co[6];
  const T c14 = c1 + (T)4 * c2;
  if constexpr (UF) {
    const T eF = e[0] * F[0] + e[1] * F[1] + e[2] * F[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if constexpr (OU) U[i] += a * F[i] + b * e[i] * eF;
      if constexpr (OD)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          D[i][j] += (T)3 * (c1 * e[i] * e[j] * eF + c2 * ((i == j ? eF : (T)0) + F[j] * e[i])
                             - c14 * F[i] * e[j]);
    }
  }
  if constexpr (UC) {
    T Ce[3], CTe[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Ce[i] = C[i][0] * e[0] + C[i][1] * e[1] + C[i][2] * e[2];
      CTe[i] = C[0][i] * e[0] + C[1][i] * e[1] + C[2][i] * e[2];
    }
    const T eCe = e[0] * Ce[0] + e[1] * Ce[1] + e[2] * Ce[2];
    const T k7 = (T)7 * d3 + d4, k5 = (T)5 * d2 + d3;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if constexpr (OU) U[i] += (T)(-3) * (c1 * e[i] * eCe + c2 * CTe[i] - c14 * Ce[i]);
      if constexpr (OD)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const T s = d4 * e[i] * e[j] * eCe
                      + d3 * ((i == j ? eCe : (T)0) + e[j] * Ce[i] + e[j] * CTe[i]
                              + e[i] * Ce[j] + e[i] * CTe[j])
                      + d2 * (C[i][j] + C[j][i]) - k7 * e[j] * Ce[i] - k5 * C[i][j];
          D[i][j] += (T)(-9) * s;
        }
    }
  }
}

// The moments of the particles packed for the pair sums: 12 numbers per
// particle in the sum's precision, (F, L, s1..s5, 0), components absent
// from the input mask zero, so that a neighbour's moments take three
// 16-byte loads (FP32) or six (FP64) instead of one load per component.
template <typename T>
__global__ void __launch_bounds__(256)
pack_moments_kernel(const double *__restrict__ in, Layout lin, int mask, int64_t n,
                    T *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 12) return;
  const int64_t p = t / 12;
  const int c = (int)(t % 12);
  const int grp = c < 3 ? 1 : (c < 6 ? 2 : 4);
  out[t] = (c < NC && (mask & grp)) ? (T)in[p * lin.stride + c - lin.off] : (T)0;
}

template <typename T>
__device__ __forceinline__ void load_packed(const T *__restrict__ m, int mask, T *F,
                                            T (*C)[3]) {
  T v[12];
  if constexpr (sizeof(T) == 4) {
    const float4 *m4 = reinterpret_cast<const float4 *>(m);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 a = m4[k];
      v[4 * k] = a.x; v[4 * k + 1] = a.y; v[4 * k + 2] = a.z; v[4 * k + 3] = a.w;
    }
  } else {
    const double2 *m2 = reinterpret_cast<const double2 *>(m);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2 a = m2[k];
      v[2 * k] = a.x; v[2 * k + 1] = a.y;
    }
  }
  const T r2 = (T)0.70710678118654752440, r6 = (T)0.40824829046386301637;
  for (int i = 0; i < 3; ++i) {
    F[i] = v[i];
    for (int j = 0; j < 3; ++j) C[i][j] = (T)0;
  }
  if (mask & 2) {
    // C^A_mn = -1/2 eps_mnk L_k
    const T Lx = v[3], Ly = v[4], Lz = v[5];
    C[0][1] -= (T)0.5 * Lz; C[1][0] += (T)0.5 * Lz;
    C[0][2] += (T)0.5 * Ly; C[2][0] -= (T)0.5 * Ly;
    C[1][2] -= (T)0.5 * Lx; C[2][1] += (T)0.5 * Lx;
  }
  if (mask & 4) {
    const T s1 = v[6], s2 = v[7], s3 = v[8], s4 = v[9], s5 = v[10];
    C[0][1] += r2 * s1; C[1][0] += r2 * s1;
    C[0][2] += r2 * s2; C[2][0] += r2 * s2;
    C[1][2] += r2 * s3; C[2][1] += r2 * s3;
    C[0][0] += r2 * s4 + r6 * s5;
    C[1][1] += -r2 * s4 + r6 * s5;
    C[2][2] += (T)(-2) * r6 * s5;
  }
}

// A group of GROUP lanes works on one particle.  One thread per particle
// would leave most of the chip idle for N ~ 1e4.
constexpr int GROUP = 16;

template <typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = GROUP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GROUP);
  return v;
}

// ------------------------------------------------------------ pair list --
// The positions stay fixed over all the operator applications of a Krylov
// solve, so the neighbours within rcut are found once per position update
// and stored as a CSR list in cell order: row t holds the neighbours of
// particle perm[t].  Rows are filled in a fixed order (cells, then
// candidates, ranked with a ballot inside the group).  Each entry holds the
// neighbour index and the pair's data -- the seven interpolated radial
// coefficients and the unit vector -- in the precision of the handle's own
// pair sums (FP64 handles: doubles; mixed handles: floats, read by their
// FP32 sums).  A sum in the other precision (the FP64 residual of a mixed
// handle, once per step) forms the data from the positions itself.

constexpr int PAIR_REC = 10;   // co[7], e[3]

struct PairArgs {
  int64_t n;
  int nc;
  double L, rcut2;
  double inv_cs, cs2;   // cells per unit length, squared cell side
  double inv_dr;
  int n2a, ntab;
  int64_t cap;     // pair-list capacity: entries at or beyond it are not written
  int *status;     // PSE_STATUS_PAIR_OVERFLOW is or-ed in when one is dropped
  int def;         // deformed lattice: positions are lattice coordinates and
  double A[9];     // separations are mapped back by A
};

// Separation x_i - x_j of wrapped positions: nearest image, and on a
// deformed lattice mapped from lattice offsets to Cartesian ones (the cutoff
// is at most a third of the cell's thinnest width, so the image is the
// nearest one).
__device__ __forceinline__ void separation(const double *__restrict__ xw, double xi0, double xi1,
                                           double xi2, int j, double L, int def, const double *A,
                                           double *d) {
  d[0] = xi0 - xw[3 * j];
  d[1] = xi1 - xw[3 * j + 1];
  d[2] = xi2 - xw[3 * j + 2];
  // positions are wrapped into [0, L): one image shift per axis suffices
  const double hL = 0.5 * L;
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] += d[k] > hL ? -L : (d[k] < -hL ? L : 0.0);
  if (def) {
    const double e[3] = {d[0], d[1], d[2]};
#pragma unroll
    for (int r = 0; r < 3; ++r) d[r] = A[3 * r] * e[0] + A[3 * r + 1] * e[1] + A[3 * r + 2] * e[2];
  }
}

__device__ __forceinline__ bool near_pair(const double *__restrict__ xw, double xi0, double xi1,
                                          double xi2, int j, const PairArgs &pa, double *d) {
  separation(xw, xi0, xi1, xi2, j, pa.L, pa.def, pa.A, d);
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < pa.rcut2;
}

// FILL = false: count the neighbours of each row into cnt[t]; FILL = true:
// write them from start[t] on.  One wavefront per row enumerates the
// candidates of the 27 cells around the particle 64 at a time.
template <bool FILL>
__global__ void __launch_bounds__(256)
pair_list_kernel(const double *__restrict__ xw, const int *__restrict__ perm,
                 const int *__restrict__ cell_start, const int *__restrict__ cell_of,
                 PairArgs pa, int *__restrict__ cnt, const int *__restrict__ start,
                 const double *__restrict__ tab, int *__restrict__ nbr,
                 double *__restrict__ rec64, float *__restrict__ rec32) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  if (t >= pa.n) return;
  const int i = perm[t];
  const double xi0 = xw[3 * i], xi1 = xw[3 * i + 1], xi2 = xw[3 * i + 2];
  const int nc = pa.nc;
  const int ci = cell_of[i];
  const int cc[3] = {ci % nc, (ci / nc) % nc, ci / (nc * nc)};
  // a neighbouring cell whose gap to the particle exceeds the cutoff holds no
  // neighbour: it is skipped (the list is the same; on a deformed lattice,
  // where cell units are not lengths, every cell is searched)
  bool skip = false;
  if (!pa.def && lane < 27) {
    const int off[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
    const double xi[3] = {xi0, xi1, xi2};
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = xi[d] * pa.inv_cs - cc[d];   // position in the cell, cell units
      const double gap = off[d] > 0 ? 1.0 - u : (off[d] < 0 ? u : 0.0);
      if (gap > 0.0) g2 += gap * gap;
    }
    skip = g2 * pa.cs2 > pa.rcut2 * (1.0 + 1e-9);
  }
  int first, pre, total;
  nbr27_setup(lane, cc[0], cc[1], cc[2], nc, cell_start, first, pre, total, skip);
  int pos = FILL ? start[t] : 0;
  int count = 0;
  for (int base = 0; base < total; base += 64) {
    const int idx = base + lane;
    const int s = nbr27_slot(idx, first, pre);
    double d[3];
    int j = -1;
    bool ok = false;
    if (idx < total) {
      j = perm[s];
      ok = j != i && near_pair(xw, xi0, xi1, xi2, j, pa, d);
    }
    if (!FILL) {
      count += ok ? 1 : 0;
    } else {
      const unsigned long long m = __ballot(ok);
      const int slot = pos + __popcll(m & ((1ull << lane) - 1ull));
      if (ok && slot >= pa.cap) {
        atomicOr(pa.status, (int)PSE_STATUS_PAIR_OVERFLOW);
        ok = false;
      }
      if (ok) {
        nbr[slot] = j;
        if (rec64 || rec32) {
          // field-major: field k of entry s at rec[k * cap + s]; the unit
          // vector now, the distance in field 0 for pair_coef_kernel (the
          // table interpolation runs there on every lane, not on the few
          // lanes of a candidate batch that found a neighbour)
          const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          const double inv = r > 0 ? 1.0 / r : 0.0;
          const size_t cap = (size_t)pa.cap;
          if (rec64) {
            rec64[slot] = r;
#pragma unroll
            for (int k = 0; k < 3; ++k) rec64[(NCOEF + k) * cap + slot] = d[k] * inv;
          } else {
            rec32[slot] = (float)r;
#pragma unroll
            for (int k = 0; k < 3; ++k) rec32[(NCOEF + k) * cap + slot] = (float)(d[k] * inv);
          }
        }
      }
      pos += __popcll(m);
    }
  }
  if (!FILL) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
    if (lane == 0) cnt[t] = count;
  }
}

// The seven radial coefficients of every stored pair, interpolated from the
// table at the distance the fill left in field 0 (entries up to the list's
// length, read on the device, and its capacity).
// In the records' precision, from the table of that precision.
template <typename R>
__global__ void __launch_bounds__(256)
pair_coef_kernel(R *__restrict__ rec, const int *__restrict__ total, int64_t cap,
                 const R *__restrict__ tab, double inv_dr, int n2a, int ntab) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t len = min((int64_t)total[0], cap);
  if (s >= len) return;
  R co[NCOEF];
  lookup<R>(tab, rec[s], (R)inv_dr, n2a, ntab, co);
#pragma unroll
  for (int k = 0; k < NCOEF; ++k) rec[(size_t)k * cap + s] = co[k];
}

struct RealArgs {
  int64_t n;
  int in_mask;    // 1: F, 2: L, 4: S
  int out_mask;   // 1: U, 2: Omega, 4: E
  int accumulate;
  Layout lin, lout;
  int64_t cap;    // pair-list capacity (entries beyond it were never written)
  double L;       // box; deformed lattice: separations mapped by A
  int def;
  double A[9];
  double inv_dr;  // radial table: spacing, rows of the near part, rows
  int n2a, ntab;
};

// M_r applied from the pair list: the self block (r = 0: only the isotropic
// coefficients, table row 0) plus one pair block per stored neighbour.
// UF, UC: forces / couplets among the inputs; OU, OD: velocity / gradient
// outputs (from ra's masks); a stored entry's fields are read only when one
// of the selected couplings uses them.
template <typename T, bool UF, bool UC, bool OU, bool OD>
__global__ void __launch_bounds__(256)
real_pair_kernel(const double *__restrict__ xw, const T *__restrict__ in,
                 double *__restrict__ out, const int *__restrict__ perm,
                 const int *__restrict__ start, const int *__restrict__ nbr,
                 const T *__restrict__ rec, const T *__restrict__ tab, RealArgs ra) {
  const int64_t t =
      ((int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / GROUP;
  const int lane = threadIdx.x % GROUP;
  if (t >= ra.n) return;
  const int i = perm[t];
  T U[3] = {0, 0, 0};
  T D[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T F[3], C[3][3];
  if (lane == 0) {
    T co[NCOEF];
    for (int j = 0; j < NCOEF; ++j) co[j] = tab[j];
    const T e0[3] = {0, 0, 0};
    load_packed<T>(in + (size_t)i * 12, ra.in_mask, F, C);
    pair_action<T, UF, UC, OU, OD>(co, e0, F, C, U, D);
  }
  constexpr bool NEED_AB = UF && OU, NEED_C12 = (UF && OD) || (UC && OU), NEED_D = UC && OD;
  const int s1 = (int)min((int64_t)start[t + 1], ra.cap);
  const double xi0 = xw[3 * i], xi1 = xw[3 * i + 1], xi2 = xw[3 * i + 2];
  const size_t cap = (size_t)ra.cap;
  for (int s = start[t] + lane; s < s1; s += GROUP) {
    const int j = nbr[s];
    T co[NCOEF] = {}, e[3];
    if (rec) {
      if constexpr (NEED_AB) {
        co[0] = rec[s];
        co[1] = rec[cap + s];
      }
      if constexpr (NEED_C12) {
        co[2] = rec[2 * cap + s];
        co[3] = rec[3 * cap + s];
      }
      if constexpr (NEED_D) {
        co[4] = rec[4 * cap + s];
        co[5] = rec[5 * cap + s];
        co[6] = rec[6 * cap + s];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) e[k] = rec[(NCOEF + k) * cap + s];
    } else {
      double d[3];
      separation(xw, xi0, xi1, xi2, j, ra.L, ra.def, ra.A, d);
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double inv = r > 0 ? 1.0 / r : 0.0;
      lookup<T>(tab, (T)r, (T)ra.inv_dr, ra.n2a, ra.ntab, co);
#pragma unroll
      for (int k = 0; k < 3; ++k) e[k] = (T)(d[k] * inv);
    }
    load_packed<T>(in + (size_t)j * 12, ra.in_mask, F, C);
    pair_action<T, UF, UC, OU, OD>(co, e, F, C, U, D);
  }
  if constexpr (OU)
#pragma unroll
    for (int k = 0; k < 3; ++k) U[k] = group_sum(U[k]);
  if constexpr (OD)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) D[a][b] = group_sum(D[a][b]);
  if (lane != 0) return;
  // component c of the output at out[row + c - off]
  const size_t row = (size_t)i * ra.lout.stride;
  auto O = [&](int c) -> double & { return out[row + c - ra.lout.off]; };
  const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637;
  if (ra.out_mask & 1) {
    for (int k = 0; k < 3; ++k) O(k) = (ra.accumulate ? O(k) : 0.0) + (double)U[k];
  }
  if (ra.out_mask & 2) {
    // Omega = -1/2 eps : D
    const double om[3] = {-0.5 * ((double)D[1][2] - D[2][1]),
                          -0.5 * ((double)D[2][0] - D[0][2]),
                          -0.5 * ((double)D[0][1] - D[1][0])};
    for (int k = 0; k < 3; ++k) O(3 + k) = (ra.accumulate ? O(3 + k) : 0.0) + om[k];
  }
  if (ra.out_mask & 4) {
    const double e5[5] = {r2 * ((double)D[0][1] + D[1][0]), r2 * ((double)D[0][2] + D[2][0]),
                          r2 * ((double)D[1][2] + D[2][1]), r2 * ((double)D[0][0] - D[1][1]),
                          r6 * ((double)D[0][0] + D[1][1] - 2.0 * D[2][2])};
    for (int k = 0; k < 5; ++k) O(6 + k) = (ra.accumulate ? O(6 + k) : 0.0) + e5[k];
  }
}

// Second half of the pair-list fill: the coefficients of the stored pairs
// (grid over pl_pairs: the count in synchronous handles, the capacity in
// asynchronous ones, whose kernel reads the count on the device).
static void pair_coefficients(Handle &h) {
  if (h.pl_pairs == 0 || (!h.pl_rec64 && !h.pl_rec32)) return;
  const dim3 grid(nblocks(h.pl_pairs, 256)), block(256);
  const int *total = h.pl_start + h.n;
  if (h.pl_rec64)
    hipLaunchKernelGGL(pair_coef_kernel<double>, grid, block, 0, h.stream, h.pl_rec64, total,
                       (int64_t)h.pl_cap, (const double *)h.g64.table, 1.0 / h.dr, h.n2a,
                       h.ntab);
  else
    hipLaunchKernelGGL(pair_coef_kernel<float>, grid, block, 0, h.stream, h.pl_rec32, total,
                       (int64_t)h.pl_cap, (const float *)h.g32.table, 1.0 / h.dr, h.n2a,
                       h.ntab);
  PSE_LAUNCH_CHECK();
}

// Builds the pair list for the current cell list; grows its storage when
// the count exceeds the capacity (one host read of the total per update).
static void build_pair_list(Handle &h, const double *xw) {
  PairArgs pa;
  pa.n = h.n;
  pa.nc = h.cells.nc;
  pa.L = h.p.box;
  pa.rcut2 = h.d.rcut * h.d.rcut;
  // the cell assignment's own scale (cell = floor(x nc / L))
  pa.inv_cs = pa.nc / h.p.box;
  pa.cs2 = (h.p.box / pa.nc) * (h.p.box / pa.nc);
  pa.inv_dr = 1.0 / h.dr;
  pa.n2a = h.n2a;
  pa.ntab = h.ntab;
  pa.cap = (int64_t)h.pl_cap;
  pa.status = h.dctl + CTL_STATUS;
  pa.def = h.def.on;
  for (int i = 0; i < 9; ++i) pa.A[i] = h.def.A[i];
  const unsigned nb = nblocks((size_t)h.n * 64, 256);
  hipLaunchKernelGGL((pair_list_kernel<false>), dim3(nb), dim3(256), 0, h.stream, xw,
                     h.cells.perm, h.cells.start, h.cells.of, pa, h.pl_cnt, nullptr, nullptr,
                     nullptr, nullptr, nullptr);
  PSE_LAUNCH_CHECK();
  const int n = (int)h.n;
  exclusive_scan(h, h.pl_cnt, h.pl_start, h.pl_scan, n);
  if (h.async) {
    // no host read: the list keeps its capacity, pairs beyond it are dropped
    // and flagged in the device status (non-finite positions are flagged by
    // the wrap kernel)
    h.pl_pairs = h.pl_cap;
    hipLaunchKernelGGL((pair_list_kernel<true>), dim3(nb), dim3(256), 0, h.stream, xw,
                       h.cells.perm, h.cells.start, h.cells.of, pa, nullptr, h.pl_start,
                       h.g64.table, h.pl_nbr, h.pl_rec64, h.pl_rec32);
    PSE_LAUNCH_CHECK();
    pair_coefficients(h);
    return;
  }
  int total = 0, bad = 0;
  PSE_HIP(hipMemcpyAsync(&total, h.pl_start + n, sizeof(int), hipMemcpyDeviceToHost,
                         h.stream));
  PSE_HIP(hipMemcpyAsync(&bad, h.bad_pos, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  PSE_HIP(hipStreamSynchronize(h.stream));
  if (bad) throw Error{PSE_ERR_NONFINITE, "non-finite particle position"};
  if ((size_t)total > h.pl_cap) {
    if (h.arena)
      throw Error{PSE_ERR_NOMEM, "real-space pair list beyond its capacity in the "
                                 "allocation-free product (" + std::to_string(total) +
                                 " pairs)"};
    clear_graphs(h);   // captured real-space launches hold the old buffers
    const size_t cap = (size_t)total + total / 4 + 1024;
    pair_storage(h, cap, false);
    pa.cap = (int64_t)cap;
  }
  h.pl_pairs = (size_t)total;
  hipLaunchKernelGGL((pair_list_kernel<true>), dim3(nb), dim3(256), 0, h.stream, xw,
                     h.cells.perm, h.cells.start, h.cells.of, pa, nullptr, h.pl_start,
                     h.g64.table, h.pl_nbr, h.pl_rec64, h.pl_rec32);
  PSE_LAUNCH_CHECK();
  pair_coefficients(h);
}

void pair_storage(Handle &h, size_t cap, bool at_create) {
  if (!at_create) {
    dev_free(h.pl_nbr);
    dev_free(h.pl_rec64);
    dev_free(h.pl_rec32);
    h.pl_nbr = nullptr;
    h.pl_rec64 = nullptr;
    h.pl_rec32 = nullptr;
    h.pl_cap = 0;
  }
  const auto alloc = [&](void **ptr, size_t bytes) {
    if (at_create) handle_alloc(h, ptr, bytes);
    else dev_alloc(ptr, bytes);
  };
  alloc((void **)&h.pl_nbr, cap * sizeof(int));
  if (h.mixed) alloc((void **)&h.pl_rec32, cap * PAIR_REC * sizeof(float));
  else alloc((void **)&h.pl_rec64, cap * PAIR_REC * sizeof(double));
  h.pl_cap = cap;
}

// Cell list, spreading bins and pair list for wrapped positions xw.
void build_cells(Handle &h, const double *xw, bool spreading) {
  const bool tiles = h.stile && spreading;
  const double nc3 = (double)h.cells.nc * h.cells.nc * h.cells.nc
                     + (tiles ? (double)h.sbins.nc * h.sbins.nc * h.sbins.nc : 0.0);
  ProfScope ps(h, PK_CELLS, (double)h.n * (24 + 16) * (tiles ? 2 : 1) + 12.0 * nc3);
  build_bins(h, xw, h.cells);
  if (tiles) {
    build_bins(h, xw, h.sbins);
    build_tile_lists(h, xw);
  }
  if (h.stile) build_dg_mu(h, xw);
  h.tiles_current = tiles;
  build_pair_list(h, xw);
}

static int mask_of(const CompSet &cs, bool input) {
  int m = 0;
  for (int k = 0; k < cs.n; ++k) {
    const int c = cs.idx[k];
    m |= c < 3 ? 1 : (c < 6 ? 2 : 4);
  }
  (void)input;
  return m;
}

template <typename T>
void real_apply(Handle &h, const double *xw, const double *in, Layout lin, const CompSet &cin,
                double *out, Layout lout, const CompSet &cout, bool accumulate) {
  RealArgs ra;
  ra.n = h.n;
  ra.lin = lin;
  ra.lout = lout;
  ra.in_mask = mask_of(cin, true);
  ra.out_mask = mask_of(cout, false);
  ra.accumulate = accumulate ? 1 : 0;
  ra.cap = (int64_t)h.pl_cap;
  ra.L = h.p.box;
  ra.def = h.def.on;
  for (int k = 0; k < 9; ++k) ra.A[k] = h.def.A[k];
  ra.inv_dr = 1.0 / h.dr;
  ra.n2a = h.n2a;
  ra.ntab = h.ntab;
  const T *tab, *rec;
  if constexpr (sizeof(T) == 8) {
    tab = h.g64.table;
    rec = h.pl_rec64;
  } else {
    tab = h.g32.table;
    rec = h.pl_rec32;
  }
  ProfScope ps(h, PK_REAL, (double)h.pl_pairs * (4.0 + (rec ? PAIR_REC * sizeof(T) : 0)) +
                               (double)h.n * (NC * 8 * 2 + 8 + 24));
  const bool uf = ra.in_mask & 1, uc = (ra.in_mask & 6) != 0;
  const bool ou = ra.out_mask & 1, od = (ra.out_mask & 6) != 0;
  T *mp = reinterpret_cast<T *>(h.mpack);
  hipLaunchKernelGGL(pack_moments_kernel<T>, dim3(nblocks((size_t)h.n * 12, 256)), dim3(256),
                     0, h.stream, in, lin, ra.in_mask, h.n, mp);
  PSE_LAUNCH_CHECK();
  const dim3 grid(nblocks((size_t)h.n * GROUP, 256)), block(256);
  const auto launch = [&](auto UF, auto UC, auto OU, auto OD) {
    hipLaunchKernelGGL((real_pair_kernel<T, decltype(UF)::value, decltype(UC)::value,
                                         decltype(OU)::value, decltype(OD)::value>),
                       grid, block, 0, h.stream, xw, (const T *)mp, out, h.cells.perm,
                       h.pl_start, h.pl_nbr, rec, tab, ra);
  };
  using Y = std::true_type;
  using N = std::false_type;
  if (uf && uc) {
    if (ou && od) launch(Y(), Y(), Y(), Y());
    else if (ou) launch(Y(), Y(), Y(), N());
    else launch(Y(), Y(), N(), Y());
  } else if (uf) {
    if (ou && od) launch(Y(), N(), Y(), Y());
    else if (ou) launch(Y(), N(), Y(), N());
    else launch(Y(), N(), N(), Y());
  } else {
    if (ou && od) launch(N(), Y(), Y(), Y());
    else if (ou) launch(N(), Y(), Y(), N());
    else launch(N(), Y(), N(), Y());
  }
  PSE_LAUNCH_CHECK();
}

template void real_apply<double>(Handle &, const double *, const double *, Layout,
                                 const CompSet &, double *, Layout, const CompSet &, bool);
template void real_apply<float>(Handle &, const double *, const double *, Layout,
                                const CompSet &, double *, Layout, const CompSet &, bool);

}  // namespace pse
