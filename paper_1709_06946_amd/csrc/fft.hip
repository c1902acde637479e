// Batched 3D FFTs of the wave-space NUFFT (Sec. II.C: the F of Eq. WSops2),
// unnormalised: dir = -1 computes sum_n f_n exp(-2 pi i k n / N) along each
// axis, dir = +1 the conjugate sum.
//
// One kernel per axis, built on the register-resident line FFT of fftreg.h.
// Grids of real components R[c][z][y][x] are transformed in place into half
// spectra H[c][kz][ky][kx < N/2] (a row of N reals holds N/2 complex); the
// Nyquist column kx = N/2 is not stored, and every Nyquist mode is zero in
// the spectra the k-space kernels produce.
#include <algorithm>
#include <mutex>

#include "fftreg.h"

namespace pse {

// ------------------------------------------------------------- x passes --

// Contiguous-line LDS layout of the x steps: one pad element after every PAD
// positions, PAD = the first radix of the direction (see padpos), and a line
// stride of xstride(N, PAD) elements.
template <int N, int E> constexpr int xstride_max() {
  return xstride(N, Shape<N, E>::first(false)) > xstride(N, Shape<N, E>::first(true))
             ? xstride(N, Shape<N, E>::first(false))
             : xstride(N, Shape<N, E>::first(true));
}

// Rows y and y+1 travel as one complex line z = a + i b.  After the forward
// transform the two half spectra are A(k) = (Z(k) + conj Z(-k))/2 and
// B(k) = (Z(k) - conj Z(-k))/2i, separated from LDS and written over the rows.
template <typename T, int N>
__global__ void __launch_bounds__(256)
fft_x_r2c_kernel(T *__restrict__ data, const cplx<T> *__restrict__ tw, int TL) {
  using C = cplx<T>;
  constexpr int E = line_e(N), TPL = N / E, H = N / 2;
  using S = Shape<N, E>;
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const size_t pair = (size_t)blockIdx.x * TL + line;
  T *row = data + 2 * pair * N;
  constexpr int R0 = S::first(false);
  C v[E];
#pragma unroll
  for (int b = 0; b < E / R0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int pos = reg_pos<N, E, R0>(t, b, r);
      v[b * R0 + r] = C{row[pos], row[N + pos]};
    }
  constexpr int PAD = S::first(false), LS = xstride(N, PAD);
  const int off = line * LS;
  reg_fft_forward<T, N, E, PAD>(v, t, lds, 1, off, tw);
  constexpr int RL = S::last(false);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < E / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) lds[off + padpos<PAD>(reg_pos<N, E, RL>(t, b, r))] = v[b * RL + r];
  __syncthreads();
  const C *Z = lds;
  for (int w = threadIdx.x; w < TL * H; w += blockDim.x) {
    const int ln = w / H, k = w % H;
    const C zp = Z[ln * LS + padpos<PAD>(k)], zm = Z[ln * LS + padpos<PAD>((N - k) % N)];
    C a, bb;
    a.x = (T)0.5 * (zp.x + zm.x);
    a.y = (T)0.5 * (zp.y - zm.y);
    bb.x = (T)0.5 * (zp.y + zm.y);
    bb.y = (T)0.5 * (zm.x - zp.x);
    C *out = reinterpret_cast<C *>(data + 2 * ((size_t)blockIdx.x * TL + ln) * N);
    out[k] = a;
    out[H + k] = bb;
  }
}

// Inverse: Z(k) = A(k) + i B(k), with A(-k) = conj A(k) and B likewise and
// the Nyquist term zero; the complex inverse transform returns rows y (real
// part) and y+1 (imaginary part).
template <typename T, int N>
__global__ void __launch_bounds__(256)
fft_x_c2r_kernel(T *__restrict__ data, const cplx<T> *__restrict__ tw, int TL) {
  using C = cplx<T>;
  constexpr int E = line_e(N), TPL = N / E, H = N / 2;
  using S = Shape<N, E>;
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  constexpr int PAD = S::first(true), LS = xstride(N, PAD);
  // the workgroup is TL lines of TPL threads, so every thread takes H / TPL
  // of the TL * H input pairs: all its loads are issued before the first
  // LDS store
  constexpr int IT = H / TPL;
  static_assert(IT * TPL == H, "pairs per thread");
  C a[IT], bb[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = threadIdx.x + i * blockDim.x, ln = w / H, k = w % H;
    const C *in = reinterpret_cast<const C *>(data + 2 * ((size_t)blockIdx.x * TL + ln) * N);
    a[i] = in[k];
    bb[i] = in[H + k];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = threadIdx.x + i * blockDim.x, ln = w / H, k = w % H;
    C *Z = lds + ln * LS;
    Z[padpos<PAD>(k)] = C{a[i].x - bb[i].y, a[i].y + bb[i].x};
    if (k > 0) Z[padpos<PAD>(N - k)] = C{a[i].x + bb[i].y, bb[i].x - a[i].y};
    else Z[padpos<PAD>(H)] = C{(T)0, (T)0};
  }
  __syncthreads();
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const int off = line * LS;
  constexpr int R0 = S::first(true);
  C v[E];
#pragma unroll
  for (int b = 0; b < E / R0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) v[b * R0 + r] = lds[off + padpos<PAD>(reg_pos<N, E, R0>(t, b, r))];
  reg_fft_inverse<T, N, E, PAD>(v, t, lds, 1, off, tw);
  constexpr int RL = S::last(true);
  T *row = data + 2 * ((size_t)blockIdx.x * TL + line) * N;
#pragma unroll
  for (int b = 0; b < E / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int pos = reg_pos<N, E, RL>(t, b, r);
      row[pos] = v[b * RL + r].x;
      row[N + pos] = v[b * RL + r].y;
    }
}

// Complex lines along x (contiguous), for the full complex transform.
template <typename T, int N>
__global__ void __launch_bounds__(256)
fft_xc_kernel(cplx<T> *__restrict__ data, const cplx<T> *__restrict__ tw, int dir, int TL) {
  using C = cplx<T>;
  constexpr int E = line_e(N), TPL = N / E;
  using S = Shape<N, E>;
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  C *ln = data + ((size_t)blockIdx.x * TL + line) * N;
  const int off = line * xstride_max<N, E>();
  C v[E];
  if (dir < 0) {
    constexpr int R0 = S::first(false), RL = S::last(false);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = ln[reg_pos<N, E, R0>(t, b, r)];
    reg_fft_forward<T, N, E, S::first(false)>(v, t, lds, 1, off, tw);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) ln[reg_pos<N, E, RL>(t, b, r)] = v[b * RL + r];
  } else {
    constexpr int R0 = S::first(true), RL = S::last(true);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = ln[reg_pos<N, E, R0>(t, b, r)];
    reg_fft_inverse<T, N, E, S::first(true)>(v, t, lds, 1, off, tw);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) ln[reg_pos<N, E, RL>(t, b, r)] = v[b * RL + r];
  }
}

// ------------------------------------------------- x and y in one kernel --

// Elements per thread in the plane kernel (as the line passes: fewer
// exchanges; eight per thread measured slower at 128^2).
constexpr int plane_e(int n) { return line_e(n); }

// Forward (INV = false): a workgroup transforms z-planes of the real
// components, one at a time: x transforms of the N/2 row pairs (registers +
// LDS exchanges in a padded [pair][LS] layout), separation of the two half
// spectra into a [y][kx < N/2] layout in the same LDS buffer, then y
// transforms of the N/2 columns, written to the plane's half spectrum.
// Inverse (INV = true): the same steps in reverse order.  Each plane travels
// through HBM once each way instead of twice.  The kernel is persistent: a
// workgroup takes planes blockIdx.x, blockIdx.x + gridDim.x, ... and loads
// the next plane into registers while it transforms the current one (the
// plane's LDS footprint allows one or two workgroups per CU, which leaves
// registers to spare); the inverse takes one plane per workgroup.  Thread (line, t) is (tid / TPL, tid % TPL) in the x
// steps and (tid % H, tid / H) in the y steps.
template <typename T, int N, bool INV>
__global__ void __launch_bounds__(512)
fft_xy_plane_kernel(T *__restrict__ data, const cplx<T> *__restrict__ tw, int nplanes) {
  using C = cplx<T>;
  constexpr int E = plane_e(N), TPL = N / E, H = N / 2, NT = H * TPL;
  using S = Shape<N, E>;
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  // the plane's LDS (the padded x layout or the [y][kx] layout), then the
  // twiddle table
  constexpr int LSX = xstride_max<N, E>(), AREA = H * LSX > N * H ? H * LSX : N * H;
  C *twl = lds + AREA;
  const C tw0 = tw_fetch<C, N>(tw);
  const int tid = threadIdx.x;
  const int xl = tid / TPL, xt = tid % TPL;          // x steps: pair xl, thread xt
  const int yl = tid % H, yt = tid / H;              // y steps: column yl, thread yt
  constexpr int NTASK = H * H / NT;                  // separation tasks per thread
  const int step = gridDim.x;
  int pl = blockIdx.x;
  if (pl >= nplanes) return;
  C v[E];
  if (!INV) {
    C vn[E];
    constexpr int R0 = S::first(false), RL = S::last(false);
    constexpr int PAD = R0, LS = xstride(N, PAD);
    const int xoff = xl * LS;
    {
      const T *pr = data + (size_t)pl * N * N;
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int pos = reg_pos<N, E, R0>(xt, b, r);
          vn[b * R0 + r] = C{pr[(2 * xl) * N + pos], pr[(2 * xl + 1) * N + pos]};
        }
    }
    tw_store<C, N>(twl, tw0, tw);
    for (; pl < nplanes; pl += step) {
      // the thread coordinates are made opaque in each iteration so that the
      // transforms' twiddle loads stay inside the loop instead of holding
      // registers across it
      int xt_ = xt, yt_ = yt;
      asm volatile("" : "+v"(xt_), "+v"(yt_));
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = vn[e];
      if (pl + step < nplanes) {
        const T *pr = data + (size_t)(pl + step) * N * N;
#pragma unroll
        for (int b = 0; b < E / R0; ++b)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const int pos = reg_pos<N, E, R0>(xt, b, r);
            vn[b * R0 + r] = C{pr[(2 * xl) * N + pos], pr[(2 * xl + 1) * N + pos]};
          }
      }
      reg_fft_forward<T, N, E, PAD>(v, xt_, lds, 1, xoff, twl);
      __syncthreads();
#pragma unroll
      for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r)
          lds[xoff + padpos<PAD>(reg_pos<N, E, RL>(xt_, b, r))] = v[b * RL + r];
      __syncthreads();
      // A(k) = (Z(k) + conj Z(-k))/2 (row 2p), B(k) = (Z(k) - conj Z(-k))/2i (row 2p+1)
      C A[NTASK], B[NTASK];
#pragma unroll
      for (int j = 0; j < NTASK; ++j) {
        const int w = tid + j * NT, ln = w / H, k = w % H;
        const C zp = lds[ln * LS + padpos<PAD>(k)], zm = lds[ln * LS + padpos<PAD>((N - k) % N)];
        A[j] = C{(T)0.5 * (zp.x + zm.x), (T)0.5 * (zp.y - zm.y)};
        B[j] = C{(T)0.5 * (zp.y + zm.y), (T)0.5 * (zm.x - zp.x)};
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NTASK; ++j) {
        const int w = tid + j * NT, ln = w / H, k = w % H;
        lds[(2 * ln) * H + k] = A[j];
        lds[(2 * ln + 1) * H + k] = B[j];
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) v[b * R0 + r] = lds[reg_pos<N, E, R0>(yt_, b, r) * H + yl];
      reg_fft_forward<T, N, E>(v, yt_, lds, H, yl, twl);
      C *spec = reinterpret_cast<C *>(data + (size_t)pl * N * N);
#pragma unroll
      for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) spec[reg_pos<N, E, RL>(yt_, b, r) * H + yl] = v[b * RL + r];
    }
  } else {
    // one plane per workgroup (the prefetching loop measured slower here)
    constexpr int R0 = S::first(true), RL = S::last(true);
    constexpr int PAD = R0, LS = xstride(N, PAD);
    const int xoff = xl * LS;
    const C *sp = reinterpret_cast<const C *>(data + (size_t)pl * N * N);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = sp[reg_pos<N, E, R0>(yt, b, r) * H + yl];
    tw_store<C, N>(twl, tw0, tw);
    reg_fft_inverse<T, N, E>(v, yt, lds, H, yl, twl);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) lds[reg_pos<N, E, RL>(yt, b, r) * H + yl] = v[b * RL + r];
    __syncthreads();
    // Z(k) = A(k) + i B(k); Z(N-k) = conj A(k) + i conj B(k); Z(N/2) = 0
    C Zp[NTASK], Zm[NTASK];
#pragma unroll
    for (int j = 0; j < NTASK; ++j) {
      const int w = tid + j * NT, ln = w / H, k = w % H;
      const C a = lds[(2 * ln) * H + k], bb = lds[(2 * ln + 1) * H + k];
      Zp[j] = C{a.x - bb.y, a.y + bb.x};
      Zm[j] = C{a.x + bb.y, bb.x - a.y};
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NTASK; ++j) {
      const int w = tid + j * NT, ln = w / H, k = w % H;
      lds[ln * LS + padpos<PAD>(k)] = Zp[j];
      if (k > 0) lds[ln * LS + padpos<PAD>(N - k)] = Zm[j];
      else lds[ln * LS + padpos<PAD>(H)] = C{(T)0, (T)0};
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        v[b * R0 + r] = lds[xoff + padpos<PAD>(reg_pos<N, E, R0>(xt, b, r))];
    reg_fft_inverse<T, N, E, PAD>(v, xt, lds, 1, xoff, twl);
    T *pr = data + (size_t)pl * N * N;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int pos = reg_pos<N, E, RL>(xt, b, r);
        pr[(2 * xl) * N + pos] = v[b * RL + r].x;
        pr[(2 * xl + 1) * N + pos] = v[b * RL + r].y;
      }
  }
}

// ------------------------------------------------------- y and z passes --

// Lines along y (axis 1) or z (axis 2) of complex arrays [c][z][y][x] with
// extents N, N, M.  A workgroup owns TL neighbouring x positions; thread
// (t, line) = (tid / TL, tid % TL), so every global access of a wavefront
// covers TL consecutive x addresses.
template <typename T, int N>
__global__ void __launch_bounds__(512)
fft_lines_kernel(cplx<T> *__restrict__ data, const cplx<T> *__restrict__ tw, int M, int axis,
                 int dir, int TL) {
  using C = cplx<T>;
  constexpr int E = line_e(N);
  using S = Shape<N, E>;
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  const int tiles = M / TL;
  // neighbouring x tiles share cache lines when a row segment is shorter
  // than a line: they run on one XCD (one L2)
  const size_t lb = xcd_block(blockIdx.x, gridDim.x);
  const size_t xt = lb % tiles, rest = lb / tiles;
  const size_t c = rest / N, o = rest % N;
  const size_t plane = (size_t)N * M, vol = plane * N;
  const int line = threadIdx.x % TL, t = threadIdx.x / TL;
  size_t base, es;
  if (axis == 1) {
    base = c * vol + o * plane + xt * TL + line;
    es = M;
  } else {
    base = c * vol + o * M + xt * TL + line;
    es = plane;
  }
  C v[E];
  if (dir < 0) {
    constexpr int R0 = S::first(false), RL = S::last(false);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = data[base + reg_pos<N, E, R0>(t, b, r) * es];
    reg_fft_forward<T, N, E>(v, t, lds, TL, line, tw);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) data[base + reg_pos<N, E, RL>(t, b, r) * es] = v[b * RL + r];
  } else {
    constexpr int R0 = S::first(true), RL = S::last(true);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = data[base + reg_pos<N, E, R0>(t, b, r) * es];
    reg_fft_inverse<T, N, E>(v, t, lds, TL, line, tw);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) data[base + reg_pos<N, E, RL>(t, b, r) * es] = v[b * RL + r];
  }
}

// -------------------------------------------------------------- host side --

// Lines per workgroup: a power of two dividing `count`, about 256 threads,
// LDS within 64 KiB.
int lines_per_block(int n, int tpl, size_t line_bytes, size_t count, int max_threads) {
  int tl = 1;
  while (tl * 2 * tpl <= max_threads && count % (size_t)(tl * 2) == 0 &&
         (size_t)(tl * 2) * line_bytes <= 65536)
    tl *= 2;
  return tl;
}

namespace {

template <typename T, int N>
void launch_x(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  constexpr int TPL = N / line_e(N);
  const size_t pairs = (size_t)ncomp * N * N / 2;
  constexpr int LS = xstride_max<N, line_e(N)>();
  const int tl = lines_per_block(N, TPL, LS * sizeof(cplx<T>), pairs);
  const size_t lds = (size_t)tl * LS * sizeof(cplx<T>);
  const unsigned nb = (unsigned)(pairs / tl);
  if (dir < 0)
    hipLaunchKernelGGL((fft_x_r2c_kernel<T, N>), dim3(nb), dim3(tl * TPL), lds, h.stream, grids,
                       tw, tl);
  else
    hipLaunchKernelGGL((fft_x_c2r_kernel<T, N>), dim3(nb), dim3(tl * TPL), lds, h.stream, grids,
                       tw, tl);
  PSE_LAUNCH_CHECK();
}

template <typename T, int N>
void launch_xc(Handle &h, cplx<T> *data, const cplx<T> *tw, int ncomp, int dir) {
  constexpr int TPL = N / line_e(N);
  const size_t lines = (size_t)ncomp * N * N;
  constexpr int LS = xstride_max<N, line_e(N)>();
  const int tl = lines_per_block(N, TPL, LS * sizeof(cplx<T>), lines);
  const size_t lds = (size_t)tl * LS * sizeof(cplx<T>);
  hipLaunchKernelGGL((fft_xc_kernel<T, N>), dim3((unsigned)(lines / tl)), dim3(tl * TPL), lds,
                     h.stream, data, tw, dir, tl);
  PSE_LAUNCH_CHECK();
}

template <typename T, int N>
void launch_lines(Handle &h, cplx<T> *data, const cplx<T> *tw, int ncomp, int M, int axis,
                  int dir) {
  constexpr int TPL = N / line_e(N);
  // up to 512 threads: 16 lines of 512 points in FP32 (128-byte row segments)
  const int tl = lines_per_block(N, TPL, N * sizeof(cplx<T>), (size_t)M, 512);
  const size_t lds = (size_t)tl * N * sizeof(cplx<T>);
  const unsigned nb = (unsigned)((size_t)ncomp * N * (M / tl));
  hipLaunchKernelGGL((fft_lines_kernel<T, N>), dim3(nb), dim3(tl * TPL), lds, h.stream, data,
                     tw, M, axis, dir, tl);
  PSE_LAUNCH_CHECK();
}

// Plane kernel: N/2 * TPL threads and max(H * LS, N * H) + N complex of LDS
// (the padded x layout and the [y][kx] layout, then the twiddles), when these
// fit (returns false otherwise).
template <typename T, int N>
bool launch_xy_plane(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  constexpr int TPL = N / plane_e(N), H = N / 2;
  constexpr int threads = H * TPL;
  constexpr int LS = xstride_max<N, plane_e(N)>();
  // the plane's layouts and the twiddle table
  const size_t lds = (size_t)((H * LS > N * H ? H * LS : N * H) + N) * sizeof(cplx<T>);
  if (threads > 512 || threads < 64 || lds > (size_t)h.max_lds) return false;
  static std::once_flag once[2];
  hipError_t attr = hipSuccess;
  std::call_once(once[dir < 0 ? 0 : 1], [&] {
    attr = dir < 0 ? hipFuncSetAttribute((const void *)fft_xy_plane_kernel<T, N, false>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                   : hipFuncSetAttribute((const void *)fft_xy_plane_kernel<T, N, true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  PSE_HIP(attr);
  // forward: persistent, as many workgroups as fit at once (LDS bound);
  // inverse: one workgroup per plane (measured faster without the prefetch)
  const int nplanes = ncomp * N;
  const int per_cu = std::max(1, (int)(163840 / lds));
  const unsigned nb =
      dir < 0 ? (unsigned)std::min(nplanes, h.num_cu * per_cu) : (unsigned)nplanes;
  if (dir < 0)
    hipLaunchKernelGGL((fft_xy_plane_kernel<T, N, false>), dim3(nb), dim3(threads), lds,
                       h.stream, grids, tw, nplanes);
  else
    hipLaunchKernelGGL((fft_xy_plane_kernel<T, N, true>), dim3(nb), dim3(threads), lds,
                       h.stream, grids, tw, nplanes);
  PSE_LAUNCH_CHECK();
  return true;
}

}  // namespace

#define PSE_CASE_X(NN) case NN: launch_x<T, NN>(h, grids, tw, ncomp, dir); break;
#define PSE_CASE_XC(NN) case NN: launch_xc<T, NN>(h, data, tw, ncomp, dir); break;
#define PSE_CASE_L(NN) case NN: launch_lines<T, NN>(h, data, tw, ncomp, M, axis, dir); break;

template <typename T>
static void x_pass(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(T));
  switch (h.d.grid) {
    PSE_FOR_EACH_N(PSE_CASE_X)
    default: throw Error{PSE_ERR_INVALID, "unsupported FFT length"};
  }
}

template <typename T>
static void line_pass(Handle &h, cplx<T> *data, const cplx<T> *tw, int ncomp, int M, int axis,
                      int dir) {
  ProfScope ps(h, PK_FFT, 2.0 * ncomp * (double)h.d.grid * h.d.grid * M * sizeof(cplx<T>));
  switch (h.d.grid) {
    PSE_FOR_EACH_N(PSE_CASE_L)
    default: throw Error{PSE_ERR_INVALID, "unsupported FFT length"};
  }
}

template <typename T>
void fft3d(Handle &h, cplx<T> *data, const cplx<T> *tw, int ncomp, int dir) {
  const int n = h.d.grid;
  {
    ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(cplx<T>));
    switch (n) {
      PSE_FOR_EACH_N(PSE_CASE_XC)
      default: throw Error{PSE_ERR_INVALID, "unsupported FFT length"};
    }
  }
  line_pass<T>(h, data, tw, ncomp, n, 1, dir);
  line_pass<T>(h, data, tw, ncomp, n, 2, dir);
}

#define PSE_CASE_P(NN) case NN: done = launch_xy_plane<T, NN>(h, grids, tw, ncomp, dir); break;

template <typename T>
void rfft_xy(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  const int n = h.d.grid;
  if (n <= 128) {
    bool done = false;
    {
      ProfScope ps(h, PK_FFT, 2.0 * ncomp * h.ngrid * sizeof(T));
      switch (n) {
        PSE_FOR_EACH_SMALL_N(PSE_CASE_P)
        default: break;
      }
    }
    if (done) return;
  }
  cplx<T> *spec = reinterpret_cast<cplx<T> *>(grids);
  if (dir < 0) {
    x_pass<T>(h, grids, tw, ncomp, dir);
    line_pass<T>(h, spec, tw, ncomp, n / 2, 1, dir);
  } else {
    line_pass<T>(h, spec, tw, ncomp, n / 2, 1, dir);
    x_pass<T>(h, grids, tw, ncomp, dir);
  }
}

template <typename T>
void rfft_z(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  line_pass<T>(h, reinterpret_cast<cplx<T> *>(grids), tw, ncomp, h.d.grid / 2, 2, dir);
}

template <typename T>
void rfft3d(Handle &h, T *grids, const cplx<T> *tw, int ncomp, int dir) {
  if (dir < 0) {
    rfft_xy<T>(h, grids, tw, ncomp, dir);
    rfft_z<T>(h, grids, tw, ncomp, dir);
  } else {
    rfft_z<T>(h, grids, tw, ncomp, dir);
    rfft_xy<T>(h, grids, tw, ncomp, dir);
  }
}

#define INST(T, C)                                                  \
  template void rfft3d<T>(Handle &, T *, const C *, int, int);      \
  template void rfft_xy<T>(Handle &, T *, const C *, int, int);     \
  template void rfft_z<T>(Handle &, T *, const C *, int, int);      \
  template void fft3d<T>(Handle &, C *, const C *, int, int);
INST(double, double2)
INST(float, float2)
#undef INST

}  // namespace pse
