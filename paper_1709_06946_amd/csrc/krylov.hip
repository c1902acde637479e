// FP64 vector kernels and small dense solvers of the Krylov iterations:
// the Lanczos square root of M_r (Sec. III.B, Chow & Saad) and GMRES on the
// stresslet constraint M_ES S = b (Eq. rigidconstraint).  All scalars stay
// on the device; the host only reads a few numbers back per iteration to
// decide when to stop.
#include <cmath>
#include <vector>

#include "pse_internal.h"

namespace pse {

constexpr int RED_BLOCKS = 1024;   // partial-sum blocks of a reduction
constexpr int MAX_DOTS = 128;      // dot products of one fused subtraction pass

__global__ void zero_kernel_d(double *v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0.0;
}

__global__ void fill_kernel_d(double *v, size_t n, double value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = value;
}

__global__ void fill_kernel_i(int *v, size_t n, int value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = value;
}

__global__ void copy_kernel_d(double *dst, const double *src, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void axpby_kernel(double a, const double *x, double b, double *y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

// Sum over a 256-thread block: within each wave by shuffles, then the four
// wave sums in a fixed order (valid in thread 0).
__device__ __forceinline__ double block_sum256(double v, double *s4) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// partial[j * nb + blk] = sum over the block's share of V_j . w
__global__ void __launch_bounds__(256)
multi_dot_partial(const double *__restrict__ V, size_t ldv, const double *__restrict__ w,
                  size_t n, double *__restrict__ partial) {
  __shared__ double s[4];
  const int j = blockIdx.y;
  const double *v = V + (size_t)j * ldv;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    acc += v[i] * w[i];
  acc = block_sum256(acc, s);
  if (threadIdx.x == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256)
reduce_partial(const double *__restrict__ partial, int nb, double *__restrict__ out) {
  __shared__ double s[4];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += partial[(size_t)j * nb + b];
  acc = block_sum256(acc, s);
  if (threadIdx.x == 0) out[j] = acc;
}

// The second Gram-Schmidt pass's subtraction fused with the dot products
// that follow it: w -= sum_{j<m} coef_j V_j, then partial[j nb + blk] =
// V_j . w for j <= m over the block's share (V_m is w itself, so the last
// entry is w . w).  Each thread updates and then reads back only its own
// elements, in the grid-stride order of multi_dot_partial, so the sums are
// those of a separate subtraction and multi_dot_partial bit for bit.
__global__ void __launch_bounds__(256)
sub_dot_partial(double *w, const double *V, size_t ldv, int m, const double *__restrict__ coef,
                size_t n, double *__restrict__ partial) {
  __shared__ double s[4][MAX_DOTS];
  const int nb = gridDim.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t i0 = (size_t)blockIdx.x * 256 + threadIdx.x, step = (size_t)nb * 256;
  for (size_t i = i0; i < n; i += step) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += coef[j] * V[(size_t)j * ldv + i];
    w[i] -= acc;
  }
#pragma unroll 4
  for (int j = 0; j <= m; ++j) {
    const double *v = V + (size_t)j * ldv;
    double acc = 0.0;
    for (size_t i = i0; i < n; i += step) acc += v[i] * w[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) s[wv][j] = acc;
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= m; j += 256)
    partial[(size_t)j * nb + blockIdx.x] = (s[0][j] + s[1][j]) + (s[2][j] + s[3][j]);
}

// The same in one pass over the elements when m + 1 <= SDF: a thread loads
// V_0..V_{m-1} at each of its elements once, subtracts, stores w and adds
// the products into the m + 1 sums from the loaded values, so each vector
// is read once instead of twice.  The per-thread order of every sum and the
// reduction are those of sub_dot_partial, so the results agree bit for bit.
constexpr int SDF = 8;

__global__ void __launch_bounds__(256)
sub_dot_partial1(double *w, const double *V, size_t ldv, int m, const double *__restrict__ coef,
                 size_t n, double *__restrict__ partial) {
  __shared__ double s[4][SDF];
  const int nb = gridDim.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t i0 = (size_t)blockIdx.x * 256 + threadIdx.x, step = (size_t)nb * 256;
  double cf[SDF - 1], acc[SDF];
#pragma unroll
  for (int j = 0; j < SDF - 1; ++j) cf[j] = j < m ? coef[j] : 0.0;
#pragma unroll
  for (int j = 0; j < SDF; ++j) acc[j] = 0.0;
  for (size_t i = i0; i < n; i += step) {
    double v[SDF - 1];
#pragma unroll
    for (int j = 0; j < SDF - 1; ++j) v[j] = j < m ? V[(size_t)j * ldv + i] : 0.0;
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < SDF - 1; ++j)
      if (j < m) a += cf[j] * v[j];
    const double wn = w[i] - a;
    w[i] = wn;
#pragma unroll
    for (int j = 0; j < SDF - 1; ++j)
      if (j < m) acc[j] += v[j] * wn;
#pragma unroll
    for (int j = 0; j < SDF; ++j)
      if (j == m) acc[j] += wn * wn;
  }
#pragma unroll
  for (int j = 0; j < SDF; ++j) {
    if (j > m) break;
    double a = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) s[wv][j] = a;
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= m; j += 256)
    partial[(size_t)j * nb + blockIdx.x] = (s[0][j] + s[1][j]) + (s[2][j] + s[3][j]);
}

// w -= sum_j coef_j V_j
__global__ void sub_multi_kernel(double *__restrict__ w, const double *__restrict__ V,
                                 size_t ldv, int m, const double *__restrict__ coef,
                                 size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += coef[j] * V[(size_t)j * ldv + i];
  w[i] -= acc;
}

// w = (w - sum_{j<m} coef_j V_j) / s with s a device scalar (0 if s <= 0)
__global__ void sub_scale_kernel(double *__restrict__ w, const double *__restrict__ V,
                                 size_t ldv, int m, const double *__restrict__ coef,
                                 const double *__restrict__ s, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += coef[j] * V[(size_t)j * ldv + i];
  const double f = s[0] > 0.0 ? 1.0 / s[0] : 0.0;
  w[i] = (w[i] - acc) * f;
}

// y = (acc ? y : 0) + alpha sum_j coef_j V_j (m from m_dev when given)
__global__ void gemv_small_kernel(const double *__restrict__ V, size_t ldv, int m,
                                  const double *__restrict__ coef, double *__restrict__ y,
                                  size_t n, double alpha, int accumulate,
                                  const int *__restrict__ m_dev) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (m_dev) m = *m_dev;
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += coef[j] * V[(size_t)j * ldv + i];
  y[i] = (accumulate ? y[i] : 0.0) + alpha * acc;
}

// dst = src * s or src / s with s a device scalar (dst may equal src)
__global__ void scale_dev_kernel(double *dst, const double *src, const double *s,
                                 int invert, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = invert ? (*s != 0.0 ? 1.0 / *s : 0.0) : *s;
  dst[i] = src[i] * f;
}

__global__ void gather_kernel(const double *__restrict__ src, int sstride, CompSet cs,
                              double *__restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < cs.n; ++k) dst[i * cs.n + k] = src[i * sstride + cs.idx[k]];
}

__global__ void scatter_kernel(const double *__restrict__ src, CompSet cs,
                               double *__restrict__ dst, int dstride, size_t n,
                               int accumulate, double alpha) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < cs.n; ++k) {
    double *o = dst + i * dstride + cs.idx[k];
    const double v = alpha * src[i * cs.n + k];
    *o = accumulate ? *o + v : v;
  }
}

__global__ void finite_kernel(const double *v, size_t n, int *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) atomicOr(flag, 1);
}

// ------------------------------------------------------------ host glue --

void vzero(Handle &h, double *v, size_t n) {
  hipLaunchKernelGGL(zero_kernel_d, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, v, n);
  PSE_LAUNCH_CHECK();
}
void fill_int(Handle &h, int *v, size_t n, int value) {
  hipLaunchKernelGGL(fill_kernel_i, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, v, n,
                     value);
  PSE_LAUNCH_CHECK();
}

static void fill_double(Handle &h, double *v, size_t n, double value) {
  hipLaunchKernelGGL(fill_kernel_d, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, v, n,
                     value);
  PSE_LAUNCH_CHECK();
}

void vcopy(Handle &h, double *dst, const double *src, size_t n) {
  hipLaunchKernelGGL(copy_kernel_d, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, dst,
                     src, n);
  PSE_LAUNCH_CHECK();
}
void vaxpby(Handle &h, double a, const double *x, double b, double *y, size_t n) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, a, x,
                     b, y, n);
  PSE_LAUNCH_CHECK();
}

void multi_dot(Handle &h, const double *V, size_t ldv, int m, const double *w,
               size_t n, double *dev_out) {
  int nb = (int)std::min<size_t>(RED_BLOCKS, (n + 255) / 256);
  if (nb < 1) nb = 1;
  if ((size_t)nb * m > h.dots_len) throw Error{PSE_ERR_INVALID, "reduction scratch too small"};
  ProfScope ps(h, PK_KRYLOV, (double)(m + 1) * n * 8);
  hipLaunchKernelGGL(multi_dot_partial, dim3(nb, m), dim3(256), 0, h.stream, V, ldv, w, n,
                     h.dots);
  PSE_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partial, dim3(m), dim3(256), 0, h.stream, h.dots, nb, dev_out);
  PSE_LAUNCH_CHECK();
}

void vsub_multi(Handle &h, double *w, const double *V, size_t ldv, int m,
                const double *coef_dev, size_t n) {
  ProfScope ps(h, PK_KRYLOV, (double)(m + 2) * n * 8);
  hipLaunchKernelGGL(sub_multi_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, w,
                     V, ldv, m, coef_dev, n);
  PSE_LAUNCH_CHECK();
}

void gemv_small(Handle &h, const double *V, size_t ldv, int m, const double *coef_dev,
                double *y, size_t n, double alpha, bool accumulate, const int *m_dev) {
  ProfScope ps(h, PK_KRYLOV, (double)(m + 1 + (accumulate ? 1 : 0)) * n * 8);
  hipLaunchKernelGGL(gemv_small_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, V,
                     ldv, m, coef_dev, y, n, alpha, accumulate ? 1 : 0, m_dev);
  PSE_LAUNCH_CHECK();
}

void vscale_dev(Handle &h, double *dst, const double *src, const double *s_dev,
                bool invert, size_t n) {
  hipLaunchKernelGGL(scale_dev_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream,
                     dst, src, s_dev, invert ? 1 : 0, n);
  PSE_LAUNCH_CHECK();
}

void gather_comps(Handle &h, const double *src, int sstride, const CompSet &cs,
                  double *dst, size_t n) {
  hipLaunchKernelGGL(gather_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, src,
                     sstride, cs, dst, n);
  PSE_LAUNCH_CHECK();
}

void scatter_comps(Handle &h, const double *src, const CompSet &cs, double *dst,
                   int dstride, size_t n, bool accumulate, double alpha) {
  hipLaunchKernelGGL(scatter_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, src,
                     cs, dst, dstride, n, accumulate ? 1 : 0, alpha);
  PSE_LAUNCH_CHECK();
}

int check_finite(Handle &h, const double *v, size_t n) {
  int *flag = reinterpret_cast<int *>(h.small + h.small_len - 2);
  PSE_HIP(hipMemsetAsync(flag, 0, sizeof(int), h.stream));
  hipLaunchKernelGGL(finite_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, v, n,
                     flag);
  PSE_LAUNCH_CHECK();
  int hv = 0;
  PSE_HIP(hipMemcpyAsync(&hv, flag, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  PSE_HIP(hipStreamSynchronize(h.stream));
  return hv;
}

// ----------------------------------------------------- small dense work --

// Eigen-decomposition of the symmetric tridiagonal matrix (diag d, off-diag
// e) by the implicit QL iteration with Wilkinson-type shifts; z accumulates
// the eigenvectors (column k belongs to eigenvalue d[k]).  m <= ldz.  Run by
// one wavefront: every lane computes the scalar recurrences alike (each lane
// reads back only its own writes of d and e, which are the same in all
// lanes), and each plane rotation is applied to the rows of z in parallel,
// row k by lane k mod 64 (a lane touches only its own rows).
__device__ void tridiag_ql(double *d, double *e, double *z, int m, int ldz) {
  const int lane = threadIdx.x, nt = blockDim.x;
  for (int i = lane; i < m; i += nt)
    for (int j = 0; j < m; ++j) z[i * ldz + j] = (i == j) ? 1.0 : 0.0;
  if (m == 1) return;
  e[m - 1] = 0.0;
  for (int l = 0; l < m; ++l) {
    for (int iter = 0; iter < 60; ++iter) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
        if (fabs(e[mm]) <= 1e-16 * dd) break;
      }
      if (mm == l) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = mm - 1;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = lane; k < m; k += nt) {
          const double zf = z[k * ldz + i + 1];
          z[k * ldz + i + 1] = s * z[k * ldz + i] + c * zf;
          z[k * ldz + i] = c * z[k * ldz + i] - s * zf;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
}

// coef = bnorm * f(T) e_1 with f = sqrt, T = tridiag(alpha, beta) of size m;
// also the relative change against the previous coefficient vector
// (zero-padded), written to out_change.  One wavefront (64 threads): inputs
// loaded in parallel, the eigenproblem by tridiag_ql, coefficient i by lane
// i mod 64, the change summed in index order by lane 0.
// Device-checked solves (sel != NULL): sel[0] is set once the first
// iteration that met the tolerance (or broke down: vn_hist[m-1] <= 1e-14 |b|)
// is found, sel[1] holds its size m and coef_sel its coefficients; at the
// last iteration (last != 0) without one, m is taken and sel[2] = 1 (not
// converged).
__global__ void __launch_bounds__(64)
lanczos_sqrt_kernel(const double *alpha, const double *beta, int m, const double *bnorm_dev,
                    double *work, int ldz, double *coef, double *coef_prev,
                    double *out_change, double *chg_hist, int *sel, double *coef_sel,
                    const double *vn_hist, double tol, int last) {
  // LDS: the new and previous coefficients (2m), then d, e and z when they
  // fit (ldz == m; the host sizes the dynamic shared memory), else those
  // live in the global work area
  extern __shared__ double lds_work[];
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x, nt = blockDim.x;
  const double bnorm = *bnorm_dev;
  double *cbuf = lds_work, *pbuf = lds_work + m;
  double *base = ldz == m ? lds_work + 2 * m : work;
  double *d = base, *e = base + ldz, *z = base + 2 * ldz;
  for (int i = lane; i < m; i += nt) {
    d[i] = alpha[i];
    e[i] = i + 1 < m ? beta[i] : 0.0;
    pbuf[i] = i < m - 1 ? coef_prev[i] : 0.0;
  }
  __syncthreads();
  tridiag_ql(d, e, z, m, ldz);
  __syncthreads();
  for (int i = lane; i < m; i += nt) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
      const double lam = d[k] > 0.0 ? sqrt(d[k]) : 0.0;
      acc += z[i * ldz + k] * lam * z[0 * ldz + k];
    }
    cbuf[i] = bnorm * acc;
    coef[i] = cbuf[i];
  }
  __syncthreads();
  if (lane != 0) return;
  double num = 0.0, den = 0.0;
  for (int i = 0; i < m; ++i) {
    const double c = cbuf[i], prev = pbuf[i];
    num += (c - prev) * (c - prev);
    den += c * c;
    coef_prev[i] = c;
  }
  out_change[0] = den > 0.0 ? sqrt(num / den) : 0.0;
  chg_hist[m - 1] = out_change[0];
  if (!sel || sel[0]) return;
  const bool brk = vn_hist[m - 1] <= 1e-14 * bnorm;
  const bool conv = m > 1 && out_change[0] < tol;
  if (brk || conv || last) {
    sel[0] = 1;
    sel[1] = m;
    sel[2] = (brk || conv) ? 0 : 1;
    for (int i = 0; i < m; ++i) coef_sel[i] = cbuf[i];
  }
}

// y = R^{-1} g for the k x k upper-triangular part of H (k from k_dev when
// given).
__global__ void backsub_kernel(const double *H, int ldh, int k, const double *g, double *y,
                               const int *k_dev) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (k_dev) k = *k_dev;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[(size_t)j * ldh + i] * y[j];
    y[i] = s / H[(size_t)i * ldh + i];
  }
}

// GMRES column j from the two Gram-Schmidt passes: H[i][j] = h1[i] + h2[i]
// (i <= j); h2[j+1] holds w.w after the first pass, so the norm of the
// twice-orthogonalised w is sqrt(w.w - |h2|^2) (V orthonormal).  Then the
// previous Givens rotations are applied to the column, the new one is
// formed and g updated; vnorm = H[j+1][j], resid = |g_{j+1}|.
// One wavefront: the column, its squared norm and the previous rotations
// are loaded in parallel into LDS (3j + 2 doubles, sized by the host), then
// lane 0 applies the rotations.
// Device-checked solves (sel != NULL): sel[0] is set at the first column
// whose residual met tol |b| or whose new vector vanished (vn <= 1e-15 |b|),
// sel[1] = its column count k (0 for b = 0); at the last column (last != 0)
// without one, k = j + 1 and sel[2] = 1 (not converged).
__global__ void __launch_bounds__(64)
hess_givens_kernel(double *__restrict__ H, int ldh, int j, const double *__restrict__ h1,
                   const double *__restrict__ h2, double *__restrict__ cs,
                   double *__restrict__ sn, double *__restrict__ g, double *__restrict__ vnorm,
                   double *__restrict__ resid, double *__restrict__ vn_hist,
                   double *__restrict__ res_hist, int *__restrict__ sel,
                   const double *__restrict__ bnorm_dev, double tol, int last) {
  extern __shared__ double sm[];
  if (blockIdx.x != 0) return;
  double *cl = sm, *cs_l = sm + (j + 2), *sn_l = cs_l + j;
  const int lane = threadIdx.x, nt = blockDim.x;
  double p2 = 0.0;
  for (int i = lane; i <= j; i += nt) {
    const double b2 = h2[i];
    cl[i] = h1[i] + b2;
    p2 += b2 * b2;
  }
  for (int i = lane; i < j; i += nt) {
    cs_l[i] = cs[i];
    sn_l[i] = sn[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) p2 += __shfl_xor(p2, off, 64);
  __syncthreads();
  if (lane != 0) return;
  double *col = H + (size_t)j * ldh;
  const double nn = sqrt(fmax(h2[j + 1] - p2, 0.0));
  cl[j + 1] = nn;
  vnorm[0] = nn;
  for (int i = 0; i < j; ++i) {
    const double t = cs_l[i] * cl[i] + sn_l[i] * cl[i + 1];
    cl[i + 1] = -sn_l[i] * cl[i] + cs_l[i] * cl[i + 1];
    cl[i] = t;
  }
  const double a = cl[j], b = cl[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0 ? a / r : 1.0, s = r > 0 ? b / r : 0.0;
  cs[j] = c;
  sn[j] = s;
  for (int i = 0; i < j; ++i) col[i] = cl[i];
  col[j] = r;
  col[j + 1] = 0.0;
  const double gj = g[j];
  g[j + 1] = -s * gj;
  g[j] = c * gj;
  resid[0] = fabs(g[j + 1]);
  vn_hist[j] = nn;
  res_hist[j] = resid[0];
  if (!sel || sel[0]) return;
  const double bn = *bnorm_dev;
  const bool done = resid[0] < tol * bn || nn <= 1e-15 * bn;
  if (done || last) {
    sel[0] = 1;
    sel[1] = bn > 0.0 ? j + 1 : 0;
    sel[2] = done ? 0 : 1;
  }
}

__global__ void sqrt_kernel(const double *in, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = sqrt(fmax(in[0], 0.0));
}

__global__ void set_g0_kernel(double *g, int len, const double *beta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int i = 0; i < len; ++i) g[i] = 0.0;
    g[0] = beta[0];
  }
}

// Lanczos tridiagonal entries from the two Gram-Schmidt passes:
// alpha_j = h1[j] + h2[j]; h2[j+1] holds w.w after the first pass, so
// beta_j = sqrt(w.w - |h2|^2) is the norm of the twice-orthogonalised w.
__global__ void lanczos_fill_kernel(double *alpha, double *beta, int j, const double *h1,
                                    const double *h2, double *vnorm, double *vn_hist) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  alpha[j] = h1[j] + h2[j];
  double p2 = 0.0;
  for (int i = 0; i <= j; ++i) p2 += h2[i] * h2[i];
  const double nn = sqrt(fmax(h2[j + 1] - p2, 0.0));
  beta[j] = nn;
  vnorm[0] = nn;
  vn_hist[j] = nn;
}

// ---------------------------------------------------- host algorithms --

// Reads n Krylov scalars; any non-finite one is reported as an error (a
// non-finite input vector or operator result).
static void host_read(Handle &h, const double *dev, double *host, int n) {
  PSE_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  PSE_HIP(hipStreamSynchronize(h.stream));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) throw Error{PSE_ERR_NONFINITE, "non-finite Krylov scalar"};
}

// Reads the first n values of two device histories that lie stride doubles
// apart (a and a + stride) into ha and ha + stride, with one copy and one
// synchronisation.
static void host_read2(Handle &h, const double *a, double *ha, int stride, int n) {
  PSE_HIP(hipMemcpyAsync(ha, a, (size_t)(stride + n) * sizeof(double), hipMemcpyDeviceToHost,
                         h.stream));
  PSE_HIP(hipStreamSynchronize(h.stream));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(ha[i]) || !std::isfinite(ha[stride + i]))
      throw Error{PSE_ERR_NONFINITE, "non-finite Krylov scalar"};
}

static void norm2_dev(Handle &h, const double *v, size_t n, double *dev_norm2) {
  multi_dot(h, v, n, 1, v, n, dev_norm2);
}

// Two-pass classical Gram-Schmidt of w = V[m] against V[0..m-1] (leading dim
// n): h1 = V^T w, w -= V h1; then h2[0..m] = [V, w]^T w (h2[m] = w.w).  The
// second subtraction is fused with the normalisation (sub_scale) once the
// norm is known on the device.
static void cgs2_pass(Handle &h, const double *V, size_t n, int m, double *w, double *h1,
                      double *h2) {
  multi_dot(h, V, n, m, w, n, h1);
  if (m + 1 > MAX_DOTS || w != V + (size_t)m * n) {
    vsub_multi(h, w, V, n, m, h1, n);
    multi_dot(h, V, n, m + 1, w, n, h2);
    return;
  }
  // w = V_m: the subtraction and the second pass's dot products in one launch
  int nb = (int)std::min<size_t>(RED_BLOCKS, (n + 255) / 256);
  if (nb < 1) nb = 1;
  if ((size_t)nb * (m + 1) > h.dots_len) throw Error{PSE_ERR_INVALID, "reduction scratch too small"};
  // one pass reads V_0..V_{m-1} and w and writes w; the two-loop form reads
  // them twice
  ProfScope ps(h, PK_KRYLOV, (double)(m + 1 <= SDF ? m + 2 : 2 * m + 3) * n * 8);
  if (m + 1 <= SDF)
    hipLaunchKernelGGL(sub_dot_partial1, dim3(nb), dim3(256), 0, h.stream, w, V, n, m, h1, n,
                       h.dots);
  else
    hipLaunchKernelGGL(sub_dot_partial, dim3(nb), dim3(256), 0, h.stream, w, V, n, m, h1, n,
                       h.dots);
  PSE_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partial, dim3(m + 1), dim3(256), 0, h.stream, h.dots, nb, h2);
  PSE_LAUNCH_CHECK();
}

static void sub_scale(Handle &h, double *w, const double *V, size_t n, int m,
                      const double *coef, const double *s) {
  ProfScope ps(h, PK_KRYLOV, (double)(m + 2) * n * 8);
  hipLaunchKernelGGL(sub_scale_kernel, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, w, V, n,
                     m, coef, s, n);
  PSE_LAUNCH_CHECK();
}

// Lanczos approximation of y = A^(1/2) b (Chow & Saad): full
// reorthogonalization, stop when the relative change of the iterate falls
// below tol.  The iterate is y_m = |b| V_m f(T_m) e_1; with V_m orthonormal
// its change is the change of the small coefficient vector.
// Convergence checks read per-iteration scalars on the host, each a stall of
// the stream.  The iteration counts of successive solves on a handle barely
// change, so a solve reads them from two iterations before the previous
// solve's count on (every iteration on the first solve); per-iteration
// values are kept on the device, so the first converged iteration (or a
// breakdown) is still found exactly and later iterations are discarded.

KrylovResult lanczos_sqrt(Handle &h, const Op &A, const double *b, size_t n, double *y,
                          int maxit, double tol, int *prev_iters) {
  const int M = maxit;
  const int ldz = M + 1;
  double *s = h.small;
  double *alpha = s, *beta = alpha + (M + 1), *h1 = beta + (M + 1), *h2 = h1 + (M + 1);
  double *norm2 = h2 + (M + 1), *vnorm = norm2 + 1, *bn = vnorm + 1, *change = bn + 1;
  double *coef = change + 1, *coef_prev = coef + (M + 1);
  double *vn_hist = coef_prev + (M + 1), *chg_hist = vn_hist + (M + 1);
  double *work = chg_hist + (M + 1);
  if ((size_t)(work - s) + (size_t)(2 + ldz) * ldz + 8 > h.small_len)
    throw Error{PSE_ERR_INVALID, "Lanczos scratch too small"};
  double *V = h.lz_V;
  KrylovResult res{0, 0.0, false};
  norm2_dev(h, b, n, norm2);
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, h.stream, norm2, bn);
  PSE_LAUNCH_CHECK();
  double hb[2];
  host_read(h, bn, hb, 1);
  const double bnorm = hb[0];
  if (!(bnorm > 0)) {
    vzero(h, y, n);
    res.converged = true;
    return res;
  }
  fill_double(h, coef_prev, M + 1, 0.0);
  // iterations before the first read leave their change unset: zero, so that
  // the history read back is finite
  fill_double(h, chg_hist, M + 1, 0.0);
  vscale_dev(h, V, b, bn, true, n);
  auto sqrt_coef = [&](int mm) {
    // LDS holds the two coefficient vectors, and d, e and the mm^2
    // eigenvectors when they fit in 48 KiB
    const size_t coefs = (size_t)2 * mm * sizeof(double);
    const size_t lds = coefs + (size_t)(2 * mm + mm * mm) * sizeof(double);
    const bool fits = lds <= 49152;
    hipLaunchKernelGGL(lanczos_sqrt_kernel, dim3(1), dim3(64), fits ? lds : coefs, h.stream, alpha,
                       beta, mm, (const double *)bn, work, fits ? mm : ldz, coef, coef_prev,
                       change, chg_hist, (int *)nullptr, (double *)nullptr,
                       (const double *)nullptr, 0.0, 0);
    PSE_LAUNCH_CHECK();
  };
  const int check_from = (prev_iters && *prev_iters > 3) ? *prev_iters - 2 : 0;
  std::vector<double> hist(2 * (M + 1));
  int m = 0;
  for (int j = 0; j < M; ++j) {
    double *w = V + (size_t)(j + 1) * n;
    A(V + (size_t)j * n, w);
    cgs2_pass(h, V, n, j + 1, w, h1, h2);
    hipLaunchKernelGGL(lanczos_fill_kernel, dim3(1), dim3(1), 0, h.stream, alpha, beta, j,
                       h1, h2, vnorm, vn_hist);
    PSE_LAUNCH_CHECK();
    sub_scale(h, w, V, n, j + 1, h2, vnorm);
    // f(T) e_1 is needed from one iteration before the first read on (the
    // change there is taken against it); a breakdown recomputes its own
    if (j + 2 >= check_from || j + 1 >= M) sqrt_coef(j + 1);
    m = j + 1;
    res.iters = m;
    if (m < check_from && m < M) continue;
    host_read2(h, vn_hist, hist.data(), M + 1, j + 1);  // vn_hist, then chg_hist
    const double *vh = hist.data(), *ch = vh + (M + 1);
    int brk = -1;
    for (int i = 0; i <= j; ++i)
      if (vh[i] <= 1e-14 * bnorm) {
        brk = i;
        break;
      }
    if (brk >= 0) {
      // breakdown: the Krylov space is exhausted after brk + 1 vectors
      if (brk < j) sqrt_coef(brk + 1);
      m = brk + 1;
      res.resid = ch[brk];
      res.converged = true;
      break;
    }
    res.resid = ch[j];
    if (j > 0 && ch[j] < tol) {
      res.converged = true;
      break;
    }
  }
  if (prev_iters) *prev_iters = res.iters;
  gemv_small(h, V, n, m, coef, y, n, 1.0, false, nullptr);
  return res;
}

// Restarted GMRES(restart) for A x = b from x = 0, stopping at relative
// residual tol or after maxit iterations.  Modified to classical
// Gram-Schmidt with a second pass (CGS2) so that each Arnoldi step costs two
// fused reductions; Givens rotations on the device.
KrylovResult gmres(Handle &h, const Op &A, const double *b, size_t n, double *x,
                   int restart, int maxit, double tol, int *prev_iters) {
  const int R = restart;
  const int ldh = R + 1;
  double *s = h.small;
  double *H = s, *cs = H + (size_t)ldh * R, *sn = cs + (R + 1), *g = sn + (R + 1);
  double *h1 = g + (R + 1), *h2 = h1 + (R + 1), *norm2 = h2 + (R + 1);
  double *vnorm = norm2 + 1, *bn = vnorm + 1, *resid = bn + 1, *ycoef = resid + 1;
  double *vn_hist = ycoef + (R + 1), *res_hist = vn_hist + (R + 1);
  if ((size_t)(res_hist - s) + R + 8 > h.small_len)
    throw Error{PSE_ERR_INVALID, "GMRES scratch too small"};
  double *V = h.gm_V;
  KrylovResult res{0, 0.0, false};
  vzero(h, x, n);
  norm2_dev(h, b, n, norm2);
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, h.stream, norm2, bn);
  PSE_LAUNCH_CHECK();
  double bnorm;
  host_read(h, bn, &bnorm, 1);
  if (!(bnorm > 0)) {
    res.converged = true;
    if (prev_iters) *prev_iters = 0;
    return res;
  }
  double rel = 1.0;
  int total = 0;
  bool first = true;
  // only the first cycle reads late (see above); restarts check every step
  int check_from = (prev_iters && *prev_iters > 3) ? *prev_iters - 2 : 0;
  std::vector<double> hist(2 * (R + 1));
  while (total < maxit) {
    // r = b - A x; on the first cycle x = 0, so r = b and its norm is the
    // |b| already on the device and the host
    double *r = V;
    const double *beta_dev = bn;
    double beta = bnorm;
    if (!first) {
      A(x, r);
      vaxpby(h, 1.0, b, -1.0, r, n);
      check_from = 0;
      norm2_dev(h, r, n, norm2);
      hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, h.stream, norm2, vnorm);
      PSE_LAUNCH_CHECK();
      host_read(h, vnorm, &beta, 1);
      beta_dev = vnorm;
    }
    rel = beta / bnorm;
    if (rel < tol) {
      res.converged = true;
      break;
    }
    // v_0 = r / beta
    vscale_dev(h, r, first ? b : r, beta_dev, true, n);
    first = false;
    hipLaunchKernelGGL(set_g0_kernel, dim3(1), dim3(1), 0, h.stream, g, R + 1, beta_dev);
    PSE_LAUNCH_CHECK();
    int k = 0;
    for (int j = 0; j < R && total < maxit; ++j) {
      double *w = V + (size_t)(j + 1) * n;
      A(V + (size_t)j * n, w);
      cgs2_pass(h, V, n, j + 1, w, h1, h2);
      hipLaunchKernelGGL(hess_givens_kernel, dim3(1), dim3(64),
                         (size_t)(3 * j + 2) * sizeof(double), h.stream, H, ldh, j, h1, h2,
                         cs, sn, g, vnorm, resid, vn_hist, res_hist, (int *)nullptr,
                         (const double *)nullptr, 0.0, 0);
      PSE_LAUNCH_CHECK();
      sub_scale(h, w, V, n, j + 1, h2, vnorm);
      ++total;
      k = j + 1;
      if (k < check_from && j + 1 < R && total < maxit) continue;
      host_read2(h, vn_hist, hist.data(), R + 1, j + 1);  // vn_hist, then res_hist
      const double *vh = hist.data(), *rh = vh + (R + 1);
      // first column at which the residual met tol or the space was exhausted;
      // later columns (and Givens entries) are not used by the update
      int stop = -1;
      for (int i = 0; i <= j; ++i)
        if (rh[i] / bnorm < tol || vh[i] <= 1e-15 * bnorm) {
          stop = i;
          break;
        }
      if (stop >= 0) {
        k = stop + 1;
        rel = rh[stop] / bnorm;
        break;
      }
      rel = rh[j] / bnorm;
    }
    hipLaunchKernelGGL(backsub_kernel, dim3(1), dim3(1), 0, h.stream, H, ldh, k, g, ycoef,
                       (const int *)nullptr);
    PSE_LAUNCH_CHECK();
    gemv_small(h, V, n, k, ycoef, x, n, 1.0, true, nullptr);
    if (rel < tol) {
      res.converged = true;
      break;
    }
  }
  res.iters = total;
  res.resid = rel;
  if (prev_iters) *prev_iters = total;
  return res;
}

// ------------------------------------------- device-checked solves --
//
// Used by asynchronous handles: no host reads.  A solve runs exactly K
// iterations; kernels record on the device the first iteration that met the
// tolerance (or exhausted the Krylov space), and the result is formed from
// that iteration's quantities, so that it equals the result of stopping
// there (the later iterations are computed and discarded).  With no such
// iteration within K, the K-th iterate is taken and the solve is reported
// as not converged.

// stats after a Lanczos solve: iterations, last change, convergence
__global__ void lanczos_stats_kernel(const int *sel, const double *chg_hist, pse_stats *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = sel[1];
  st->lanczos_iters = m;
  st->lanczos_change = m > 0 ? chg_hist[m - 1] : 0.0;
  if (sel[2]) st->converged = 0;
}

// stats after a GMRES solve (accumulated over refinement passes)
__global__ void gmres_stats_kernel(const int *sel, const double *res_hist, const double *bn,
                                   pse_stats *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = sel[1];
  st->gmres_iters += k;
  st->gmres_residual = (k > 0 && bn[0] > 0.0) ? res_hist[k - 1] / bn[0] : 0.0;
  if (sel[2]) st->converged = 0;
}

void lanczos_sqrt_dev(Handle &h, const Op &A, const double *b, size_t n, double *y, int K,
                      double tol) {
  const int M = K;
  const int ldz = M + 1;
  double *s = h.small;
  double *alpha = s, *beta = alpha + (M + 1), *h1 = beta + (M + 1), *h2 = h1 + (M + 1);
  double *norm2 = h2 + (M + 1), *vnorm = norm2 + 1, *bn = vnorm + 1, *change = bn + 1;
  double *coef = change + 1, *coef_prev = coef + (M + 1);
  double *vn_hist = coef_prev + (M + 1), *chg_hist = vn_hist + (M + 1);
  double *coef_sel = chg_hist + (M + 1);
  double *work = coef_sel + (M + 1);
  if ((size_t)(work - s) + (size_t)(2 + ldz) * ldz + 8 > h.small_len)
    throw Error{PSE_ERR_INVALID, "Lanczos scratch too small"};
  int *sel = h.dctl + CTL_LZ;
  double *V = h.lz_V;
  norm2_dev(h, b, n, norm2);
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, h.stream, norm2, bn);
  PSE_LAUNCH_CHECK();
  fill_double(h, coef_prev, M + 1, 0.0);
  fill_double(h, chg_hist, M + 1, 0.0);
  fill_int(h, sel, 3, 0);
  vscale_dev(h, V, b, bn, true, n);
  for (int j = 0; j < M; ++j) {
    double *w = V + (size_t)(j + 1) * n;
    A(V + (size_t)j * n, w);
    cgs2_pass(h, V, n, j + 1, w, h1, h2);
    hipLaunchKernelGGL(lanczos_fill_kernel, dim3(1), dim3(1), 0, h.stream, alpha, beta, j,
                       h1, h2, vnorm, vn_hist);
    PSE_LAUNCH_CHECK();
    sub_scale(h, w, V, n, j + 1, h2, vnorm);
    const int mm = j + 1;
    const size_t coefs = (size_t)2 * mm * sizeof(double);
    const size_t lds = coefs + (size_t)(2 * mm + mm * mm) * sizeof(double);
    const bool fits = lds <= 49152;
    hipLaunchKernelGGL(lanczos_sqrt_kernel, dim3(1), dim3(64), fits ? lds : coefs, h.stream,
                       alpha, beta, mm, (const double *)bn, work, fits ? mm : ldz, coef,
                       coef_prev, change, chg_hist, sel, coef_sel, (const double *)vn_hist,
                       tol, j + 1 == M ? 1 : 0);
    PSE_LAUNCH_CHECK();
  }
  gemv_small(h, V, n, M, coef_sel, y, n, 1.0, false, sel + 1);
  hipLaunchKernelGGL(lanczos_stats_kernel, dim3(1), dim3(1), 0, h.stream, (const int *)sel,
                     (const double *)chg_hist, h.dstats);
  PSE_LAUNCH_CHECK();
}

void gmres_dev(Handle &h, const Op &A, const double *b, size_t n, double *x, int K,
               double tol) {
  const int R = K;
  const int ldh = R + 1;
  double *s = h.small;
  double *H = s, *cs = H + (size_t)ldh * R, *sn = cs + (R + 1), *g = sn + (R + 1);
  double *h1 = g + (R + 1), *h2 = h1 + (R + 1), *norm2 = h2 + (R + 1);
  double *vnorm = norm2 + 1, *bn = vnorm + 1, *resid = bn + 1, *ycoef = resid + 1;
  double *vn_hist = ycoef + (R + 1), *res_hist = vn_hist + (R + 1);
  if ((size_t)(res_hist - s) + R + 8 > h.small_len)
    throw Error{PSE_ERR_INVALID, "GMRES scratch too small"};
  if ((size_t)R > (size_t)h.d.gmres_restart)
    throw Error{PSE_ERR_INVALID, "GMRES basis smaller than its iteration count"};
  int *sel = h.dctl + CTL_GM;
  double *V = h.gm_V;
  vzero(h, x, n);
  norm2_dev(h, b, n, norm2);
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, h.stream, norm2, bn);
  PSE_LAUNCH_CHECK();
  fill_int(h, sel, 3, 0);
  vscale_dev(h, V, b, bn, true, n);
  hipLaunchKernelGGL(set_g0_kernel, dim3(1), dim3(1), 0, h.stream, g, R + 1,
                     (const double *)bn);
  PSE_LAUNCH_CHECK();
  for (int j = 0; j < R; ++j) {
    double *w = V + (size_t)(j + 1) * n;
    A(V + (size_t)j * n, w);
    cgs2_pass(h, V, n, j + 1, w, h1, h2);
    hipLaunchKernelGGL(hess_givens_kernel, dim3(1), dim3(64),
                       (size_t)(3 * j + 2) * sizeof(double), h.stream, H, ldh, j, h1, h2, cs,
                       sn, g, vnorm, resid, vn_hist, res_hist, sel, (const double *)bn, tol,
                       j + 1 == R ? 1 : 0);
    PSE_LAUNCH_CHECK();
    sub_scale(h, w, V, n, j + 1, h2, vnorm);
  }
  hipLaunchKernelGGL(backsub_kernel, dim3(1), dim3(1), 0, h.stream, H, ldh, R, g, ycoef,
                     (const int *)(sel + 1));
  PSE_LAUNCH_CHECK();
  gemv_small(h, V, n, R, ycoef, x, n, 1.0, true, sel + 1);
  hipLaunchKernelGGL(gmres_stats_kernel, dim3(1), dim3(1), 0, h.stream, (const int *)sel,
                     (const double *)res_hist, (const double *)bn, h.dstats);
  PSE_LAUNCH_CHECK();
}

}  // namespace pse
