// Batched 3D complex FFT for the wave-space NUFFT (Sec. II.C: the F of
// Eq. WSops2).  Unnormalized: dir = -1 computes sum_n f_n exp(-2 pi i k n / N)
// along each axis, dir = +1 the conjugate sum.
//
// One kernel per axis.  A workgroup loads TL whole lines of length N into
// LDS, runs a Stockham autosort FFT (radix 4, 2, 3 stages; Govindaraju et
// al., SC'08 formulation) between two LDS buffers, and writes the lines back
// in place.  LDS is laid out [position][line] so that, along the y and z
// axes, consecutive threads touch consecutive x addresses both in HBM and in
// LDS.
#include "pse_internal.h"

namespace pse {

struct FftPlan {
  int n;        // line length
  int m;        // stored extent of the x axis (n for full complex grids,
                // n/2 for half spectra)
  int tl;       // lines per workgroup
  int nst;      // number of stages
  int r[16];    // radix per stage
};

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) {
  C c; c.x = a.x + b.x; c.y = a.y + b.y; return c;
}
template <typename C> __device__ __forceinline__ C csub(C a, C b) {
  C c; c.x = a.x - b.x; c.y = a.y - b.y; return c;
}
// multiply by -i*s (s = +1) or +i (s = -1): forward rotation for dir = -1
template <typename C> __device__ __forceinline__ C rot(C a, int dir) {
  C c;
  if (dir < 0) { c.x = a.y; c.y = -a.x; }   // -i a
  else         { c.x = -a.y; c.y = a.x; }   // +i a
  return c;
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T> *v, int dir) {
  using C = cplx<T>;
  if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]), t3 = rot(csub(v[1], v[3]), dir);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 3) {
    const T s = (T)0.86602540378443864676;  // sqrt(3)/2
    C a = v[0];
    C t1 = cadd(v[1], v[2]);
    C t2; t2.x = a.x - (T)0.5 * t1.x; t2.y = a.y - (T)0.5 * t1.y;
    C d = csub(v[1], v[2]);
    C t3 = rot(d, dir);              // -i d (forward) or +i d (inverse)
    t3.x *= s; t3.y *= s;
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
}

template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cplx<T> *__restrict__ src,
                                               cplx<T> *__restrict__ dst, int N,
                                               int TL, int Ns,
                                               const cplx<T> *__restrict__ tw,
                                               int dir) {
  using C = cplx<T>;
  const int nbf = N / R;
  const int tstep = N / (Ns * R);
  for (int w = threadIdx.x; w < nbf * TL; w += blockDim.x) {
    const int line = w % TL;
    const int j = w / TL;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nbf) * TL + line];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C t = tw[k * r * tstep];
        if (dir > 0) t.y = -t.y;
        v[r] = cmul(v[r], t);
      }
    }
    dft_small<T, R>(v, dir);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * TL + line] = v[r];
  }
}

// Runs all stages between the two LDS buffers; returns the buffer holding
// the result.
template <typename T>
__device__ cplx<T> *stockham_all(cplx<T> *src, cplx<T> *dst, const FftPlan &plan,
                                 const cplx<T> *__restrict__ tw, int dir) {
  const int N = plan.n, TL = plan.tl;
  int Ns = 1;
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.r[s];
    if (R == 4)      stockham_stage<T, 4>(src, dst, N, TL, Ns, tw, dir);
    else if (R == 2) stockham_stage<T, 2>(src, dst, N, TL, Ns, tw, dir);
    else             stockham_stage<T, 3>(src, dst, N, TL, Ns, tw, dir);
    __syncthreads();
    cplx<T> *t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// pass 0: lines along x (contiguous); 1: along y; 2: along z.
template <typename T>
__global__ void __launch_bounds__(256)
fft_pass(cplx<T> *__restrict__ data, const cplx<T> *__restrict__ tw,
         FftPlan plan, int pass, int dir) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf0 = reinterpret_cast<C *>(smem_raw);
  const int N = plan.n, M = plan.m, TL = plan.tl;
  C *buf1 = buf0 + N * TL;
  // stored array per component: [z][y][x] with extents N, N, M
  const size_t row = M, plane = (size_t)N * M, vol = plane * N;
  size_t base, ls, es;
  const size_t b = blockIdx.x;
  if (pass == 0) {
    base = b * TL * (size_t)N;
    ls = N;
    es = 1;
  } else {
    const int tiles = M / TL;
    const size_t xt = b % tiles;
    const size_t rest = b / tiles;       // (c, z) for pass 1, (c, y) for pass 2
    const size_t c = rest / N, o = rest % N;
    if (pass == 1) {
      base = c * vol + o * plane + xt * TL;
      ls = 1;
      es = row;
    } else {
      base = c * vol + o * row + xt * TL;
      ls = 1;
      es = plane;
    }
  }
  const int total = N * TL;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    int line, pos;
    if (pass == 0) { pos = w % N; line = w / N; }
    else           { line = w % TL; pos = w / TL; }
    buf0[pos * TL + line] = data[base + line * ls + pos * es];
  }
  __syncthreads();
  C *src = stockham_all<T>(buf0, buf1, plan, tw, dir);
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    int line, pos;
    if (pass == 0) { pos = w % N; line = w / N; }
    else           { line = w % TL; pos = w / TL; }
    data[base + line * ls + pos * es] = src[pos * TL + line];
  }
}

// x pass of the real transforms.  Real grids R[c][z][y][x] and half spectra
// H[c][z][y][kx], kx in [0, n/2), share the same memory (a row of n reals
// holds n/2 complex).  The Nyquist column kx = n/2 is not stored: the
// k-space kernels zero every Nyquist mode.  Rows y and y+1 travel together
// as one complex line z = a + i b; after the complex FFT the two spectra are
// A(k) = (Z(k) + conj Z(-k))/2 and B(k) = (Z(k) - conj Z(-k))/2i.
template <typename T>
__global__ void __launch_bounds__(256)
fft_x_r2c(T *__restrict__ data, const cplx<T> *__restrict__ tw, FftPlan plan) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf0 = reinterpret_cast<C *>(smem_raw);
  const int N = plan.n, TL = plan.tl, H = N / 2;
  C *buf1 = buf0 + N * TL;
  const size_t row0 = (size_t)blockIdx.x * TL * 2;   // first real row of the block
  for (int w = threadIdx.x; w < N * TL; w += blockDim.x) {
    const int pos = w % N, line = w / N;
    const T *r = data + (row0 + 2 * line) * N;
    C z;
    z.x = r[pos];
    z.y = r[N + pos];
    buf0[pos * TL + line] = z;
  }
  __syncthreads();
  C *Z = stockham_all<T>(buf0, buf1, plan, tw, -1);
  for (int w = threadIdx.x; w < H * TL; w += blockDim.x) {
    const int k = w % H, line = w / H;
    const C zp = Z[k * TL + line], zm = Z[((N - k) % N) * TL + line];
    C a, bb;
    a.x = (T)0.5 * (zp.x + zm.x);
    a.y = (T)0.5 * (zp.y - zm.y);
    bb.x = (T)0.5 * (zp.y + zm.y);
    bb.y = (T)0.5 * (zm.x - zp.x);
    C *out = reinterpret_cast<C *>(data + (row0 + 2 * line) * N);
    out[k] = a;
    out[H + k] = bb;        // the next row starts n/2 complex further on
  }
}

// Inverse: Z(k) = A(k) + i B(k) with A(-k) = conj A(k) (Nyquist zero), the
// complex inverse FFT gives rows y (real part) and y+1 (imaginary part).
template <typename T>
__global__ void __launch_bounds__(256)
fft_x_c2r(T *__restrict__ data, const cplx<T> *__restrict__ tw, FftPlan plan) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf0 = reinterpret_cast<C *>(smem_raw);
  const int N = plan.n, TL = plan.tl, H = N / 2;
  C *buf1 = buf0 + N * TL;
  const size_t row0 = (size_t)blockIdx.x * TL * 2;
  for (int w = threadIdx.x; w < N * TL; w += blockDim.x) {
    const int k = w % N, line = w / N;
    const C *in = reinterpret_cast<const C *>(data + (row0 + 2 * line) * N);
    C z;
    if (k < H) {
      const C a = in[k], bb = in[H + k];
      z.x = a.x - bb.y;
      z.y = a.y + bb.x;
    } else if (k == H) {
      z.x = (T)0;
      z.y = (T)0;
    } else {
      const C a = in[N - k], bb = in[H + N - k];   // conj A(N-k) + i conj B(N-k)
      z.x = a.x + bb.y;
      z.y = -a.y + bb.x;
    }
    buf0[k * TL + line] = z;
  }
  __syncthreads();
  C *Z = stockham_all<T>(buf0, buf1, plan, tw, +1);
  for (int w = threadIdx.x; w < N * TL; w += blockDim.x) {
    const int pos = w % N, line = w / N;
    T *r = data + (row0 + 2 * line) * N;
    const C z = Z[pos * TL + line];
    r[pos] = z.x;
    r[N + pos] = z.y;
  }
}

static FftPlan make_plan(int n, size_t elem_bytes) {
  FftPlan p{};
  p.n = n;
  int m = n;
  if (m % 3 == 0) { p.r[p.nst++] = 3; m /= 3; }
  while (m % 4 == 0) { p.r[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { p.r[p.nst++] = 2; m /= 2; }
  if (m != 1) throw Error{PSE_ERR_INVALID, "unsupported FFT length"};
  // two LDS buffers of N * TL elements within 64 KiB
  int tl = (int)(65536 / (2 * elem_bytes * n));
  if (tl > n) tl = n;
  int t = 1;
  while (t * 2 <= tl && n % (t * 2) == 0) t *= 2;
  p.tl = t;
  p.m = n;
  return p;
}

template <typename T>
void fft3d(Handle &h, cplx<T> *data, const cplx<T> *twiddle, int ncomp, int dir) {
  const int n = h.d.grid;
  FftPlan plan = make_plan(n, sizeof(cplx<T>));
  const size_t lds = 2 * (size_t)n * plan.tl * sizeof(cplx<T>);
  const unsigned nb = (unsigned)((size_t)ncomp * n * n / plan.tl);
  for (int pass = 0; pass < 3; ++pass) {
    ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(cplx<T>));
    hipLaunchKernelGGL(fft_pass<T>, dim3(nb), dim3(256), lds, h.stream, data,
                       twiddle, plan, pass, dir);
    PSE_LAUNCH_CHECK();
  }
}

// Real 3D transforms of ncomp real grids stored [c][z][y][x], in place.
// Forward leaves half spectra [c][kz][ky][kx < n/2]; inverse takes them back.
template <typename T>
static void half_passes(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  const int n = h.d.grid;
  FftPlan plan = make_plan(n, sizeof(cplx<T>));
  plan.m = n / 2;
  while (plan.tl > 1 && (n / 2) % plan.tl) plan.tl /= 2;
  const size_t lds = 2 * (size_t)n * plan.tl * sizeof(cplx<T>);
  const unsigned nb = (unsigned)((size_t)ncomp * n * (n / 2) / plan.tl);
  const int order[2] = {dir < 0 ? 1 : 2, dir < 0 ? 2 : 1};
  for (int i = 0; i < 2; ++i) {
    ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(T));
    hipLaunchKernelGGL(fft_pass<T>, dim3(nb), dim3(256), lds, h.stream,
                       reinterpret_cast<cplx<T> *>(grids), tw, plan, order[i], dir);
    PSE_LAUNCH_CHECK();
  }
}

template <typename T>
static void x_pass(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  const int n = h.d.grid;
  FftPlan plan = make_plan(n, sizeof(cplx<T>));
  // plan.tl counts row pairs here; rows per component n^2 (even)
  while (plan.tl > 1 && ((size_t)n * n / 2) % plan.tl) plan.tl /= 2;
  const size_t lds = 2 * (size_t)n * plan.tl * sizeof(cplx<T>);
  const unsigned nb = (unsigned)((size_t)ncomp * n * n / 2 / plan.tl);
  ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(T));
  if (dir < 0)
    hipLaunchKernelGGL(fft_x_r2c<T>, dim3(nb), dim3(256), lds, h.stream, grids, tw, plan);
  else
    hipLaunchKernelGGL(fft_x_c2r<T>, dim3(nb), dim3(256), lds, h.stream, grids, tw, plan);
  PSE_LAUNCH_CHECK();
}

template <typename T>
void rfft3d(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir) {
  if (dir < 0) {
    x_pass<T>(h, grids, twiddle, ncomp, dir);
    half_passes<T>(h, grids, twiddle, ncomp, dir);
  } else {
    half_passes<T>(h, grids, twiddle, ncomp, dir);
    x_pass<T>(h, grids, twiddle, ncomp, dir);
  }
}

template void rfft3d<double>(Handle &, double *, const double2 *, int, int);
template void rfft3d<float>(Handle &, float *, const float2 *, int, int);
template void fft3d<double>(Handle &, double2 *, const double2 *, int, int);
template void fft3d<float>(Handle &, float2 *, const float2 *, int, int);

}  // namespace pse
