// Batched 3D complex FFT for the wave-space NUFFT (Sec. II.C: the F of
// Eq. WSops2).  Unnormalized: dir = -1 computes sum_n f_n exp(-2 pi i k n / N)
// along each axis, dir = +1 the conjugate sum.
//
// One kernel per axis.  A workgroup loads TL whole lines of length N into
// LDS, runs the Stockham autosort FFT of stockham.h between two LDS buffers,
// and writes the lines back in place.  LDS is laid out [position][line] so that, along the y and z
// axes, consecutive threads touch consecutive x addresses both in HBM and in
// LDS.
#include "stockham.h"

namespace pse {

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
static void half_pass(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir, int pass) {
  const int n = h.d.grid;
  FftPlan plan = make_plan(n, sizeof(cplx<T>));
  plan.m = n / 2;
  while (plan.tl > 1 && (n / 2) % plan.tl) plan.tl /= 2;
  const size_t lds = 2 * (size_t)n * plan.tl * sizeof(cplx<T>);
  const unsigned nb = (unsigned)((size_t)ncomp * n * (n / 2) / plan.tl);
  ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(T));
  hipLaunchKernelGGL(fft_pass<T>, dim3(nb), dim3(256), lds, h.stream,
                     reinterpret_cast<cplx<T> *>(grids), tw, plan, pass, dir);
  PSE_LAUNCH_CHECK();
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
void rfft_xy(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir) {
  if (dir < 0) {
    x_pass<T>(h, grids, twiddle, ncomp, dir);
    half_pass<T>(h, grids, twiddle, ncomp, dir, 1);
  } else {
    half_pass<T>(h, grids, twiddle, ncomp, dir, 1);
    x_pass<T>(h, grids, twiddle, ncomp, dir);
  }
}

template <typename T>
void rfft_z(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir) {
  half_pass<T>(h, grids, twiddle, ncomp, dir, 2);
}

template <typename T>
void rfft3d(Handle &h, T *grids, const cplx<T> *twiddle, int ncomp, int dir) {
  if (dir < 0) {
    rfft_xy<T>(h, grids, twiddle, ncomp, dir);
    rfft_z<T>(h, grids, twiddle, ncomp, dir);
  } else {
    rfft_z<T>(h, grids, twiddle, ncomp, dir);
    rfft_xy<T>(h, grids, twiddle, ncomp, dir);
  }
}

#define INST(T, C)                                                  \
  template void rfft3d<T>(Handle &, T *, const C *, int, int);      \
  template void rfft_xy<T>(Handle &, T *, const C *, int, int);     \
  template void rfft_z<T>(Handle &, T *, const C *, int, int);
INST(double, double2)
INST(float, float2)
#undef INST
template void fft3d<double>(Handle &, double2 *, const double2 *, int, int);
template void fft3d<float>(Handle &, float2 *, const float2 *, int, int);

}  // namespace pse
