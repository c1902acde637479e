// Register-resident mixed-radix FFT on lines of compile-time length N (the F
// of Eq. WSops2).
//
// Each line is transformed by TPL = N / E threads that hold E elements each in
// registers.  The transform is a Stockham sequence of radix-R passes (R in
// {2, 3, 4, 8, 12, 16}, every R dividing E); between passes the elements go
// through one LDS buffer (write, barrier, read), so a length-128 line needs a
// single exchange instead of one LDS round trip per radix-4 stage.
//
// Register layout.  With radix R first, thread t holds in v[b*R + r] the
// element at position t + b*TPL + r*N/R (b < E/R).  After the last pass of
// radix R', v[b*R' + r] holds the output at position t + b*TPL + r*N/R'.  The
// inverse runs the radices in reverse order, so the forward output layout is
// the inverse input layout: a kernel may act on the spectrum in registers
// between the two without any exchange.
//
// Twiddles come from a table of N entries exp(-2 pi i m / N) (conjugated for
// the inverse); the small DFTs use compile-time constants.
#pragma once

#include "pse_internal.h"

namespace pse {

// ------------------------------------------------- compile-time constants --

constexpr double kPi = 3.14159265358979323846;

// sin and cos of 2 pi m / n by Taylor series on the reduced angle (exact to
// a few ulp for the small n used here).
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / n for even n, reduced to the first octant so
// that the series runs on |x| <= pi/4 and the special angles are exact.
// q = n - 4 m > 0 measures pi/2 - x in units of 2 pi / (4 n).
constexpr double first_quadrant(int m, int n, bool want_cos) {
  // 0 <= 2 pi m / n <= pi/2
  if (8 * m <= n) return want_cos ? taylor_cos(2.0 * kPi * m / n) : taylor_sin(2.0 * kPi * m / n);
  const double y = 2.0 * kPi * (n - 4 * m) / (4.0 * n);   // pi/2 - x
  return want_cos ? taylor_sin(y) : taylor_cos(y);
}
constexpr double root_cos(int m, int n) {
  m %= n;
  if (2 * m > n) m = n - m;             // cos is even: angle in [0, pi]
  if (4 * m <= n) return first_quadrant(m, n, true);
  return -first_quadrant(n / 2 - m, n, true);   // cos(pi - x) = -cos x
}
constexpr double root_sin(int m, int n) {
  m %= n;
  double sign = 1.0;
  if (2 * m > n) {                      // sin is odd: angle in [0, pi]
    m = n - m;
    sign = -1.0;
  }
  if (4 * m <= n) return sign * first_quadrant(m, n, false);
  return sign * first_quadrant(n / 2 - m, n, false);   // sin(pi - x) = sin x
}

template <int N> struct Roots {
  double c[N], s[N];
  constexpr Roots() : c(), s() {
    for (int m = 0; m < N; ++m) {
      c[m] = root_cos(m, N);
      s[m] = root_sin(m, N);
    }
  }
};

// -------------------------------------------------------- complex helpers --

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
// multiply by -i (forward, dir < 0) or +i (inverse)
template <typename C> __device__ __forceinline__ C rot(C a, int dir) {
  C c;
  if (dir < 0) { c.x = a.y; c.y = -a.x; }
  else         { c.x = -a.y; c.y = a.x; }
  return c;
}

// ------------------------------------------------------------ small DFTs --

template <typename T, int R> __device__ __forceinline__ void dft(cplx<T> *v, int dir);

// N = A * B by one Cooley-Tukey step: input n = B n1 + n2, output
// k = k1 + A k2; A-point DFTs over n1, twiddle W_N^(n2 k1), B-point DFTs
// over n2.
template <typename T, int A, int B>
__device__ __forceinline__ void dft_compose(cplx<T> *v, int dir) {
  using C = cplx<T>;
  constexpr int N = A * B;
  constexpr Roots<N> W{};
  C y[N];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    C a[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) a[n1] = v[B * n1 + n2];
    dft<T, A>(a, dir);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) y[n2 * A + k1] = a[k1];
  }
#pragma unroll
  for (int n2 = 1; n2 < B; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
      const int m = (n2 * k1) % N;
      C w;
      w.x = (T)W.c[m];
      w.y = (T)(dir < 0 ? -W.s[m] : W.s[m]);
      y[n2 * A + k1] = cmul(y[n2 * A + k1], w);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    C b[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) b[n2] = y[n2 * A + k1];
    dft<T, B>(b, dir);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = b[k2];
  }
}

template <typename T, int R> __device__ __forceinline__ void dft(cplx<T> *v, int dir) {
  using C = cplx<T>;
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T s = (T)0.86602540378443864676;
    C a = v[0];
    C t1 = cadd(v[1], v[2]);
    C t2; t2.x = a.x - (T)0.5 * t1.x; t2.y = a.y - (T)0.5 * t1.y;
    C t3 = rot(csub(v[1], v[2]), dir);
    t3.x *= s; t3.y *= s;
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  } else if constexpr (R == 4) {
    C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]), t3 = rot(csub(v[1], v[3]), dir);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 6) {
    dft_compose<T, 3, 2>(v, dir);
  } else if constexpr (R == 8) {
    dft_compose<T, 2, 4>(v, dir);
  } else if constexpr (R == 12) {
    dft_compose<T, 3, 4>(v, dir);
  } else if constexpr (R == 16) {
    dft_compose<T, 4, 4>(v, dir);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// ------------------------------------------------------------ the passes --

struct Radices {
  int np;
  int r[8];
};

// Greedy factorisation of n into radices that divide e (largest first);
// np = -1 when n has no such factorisation in at most 8 passes.
constexpr Radices factor(int n, int e) {
  Radices out{};
  const int cand[7] = {16, 12, 8, 6, 4, 3, 2};
  int m = n;
  while (m > 1 && out.np < 8) {
    int pick = 0;
    for (int i = 0; i < 7; ++i) {
      if (e % cand[i] == 0 && m % cand[i] == 0) {
        pick = cand[i];
        break;
      }
    }
    if (pick == 0) return Radices{-1, {}};
    out.r[out.np++] = pick;
    m /= pick;
  }
  if (m > 1) return Radices{-1, {}};
  return out;
}

template <int N, int E> struct Shape {
  static constexpr Radices RD = factor(N, E);
  static constexpr int NP = RD.np;
  static constexpr int TPL = N / E;
  static_assert(NP > 0, "no factorisation of N with radices dividing E");
  static constexpr int radix(int p, bool rev) { return RD.r[rev ? NP - 1 - p : p]; }
  static constexpr int first(bool rev) { return radix(0, rev); }
  static constexpr int last(bool rev) { return radix(NP - 1, rev); }
};

// Position of register (b, r) for a pass of radix R: t + b*TPL + r*N/R.
template <int N, int E, int R>
__device__ __forceinline__ int reg_pos(int t, int b, int r) {
  return t + b * (N / E) + r * (N / R);
}

// One Stockham pass of radix R; Ns is the product of the radices before it.
template <typename T, int N, int E, int R, int Ns>
__device__ __forceinline__ void reg_pass(cplx<T> (&v)[E], int t, const cplx<T> *__restrict__ tw,
                                         int dir) {
  using C = cplx<T>;
  constexpr int TPL = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    if constexpr (Ns > 1) {
      const int j = t + b * TPL;
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * (N / (Ns * R))];
        if (dir > 0) w.y = -w.y;
        v[b * R + r] = cmul(v[b * R + r], w);
      }
    }
    dft<T, R>(&v[b * R], dir);
  }
}

// LDS position with one pad element after every PADP positions (PADP = 0:
// none).  In the contiguous-line layouts (ps = 1) the first pass of radix R
// writes positions j R + r, a stride of R elements across the threads of a
// line; padding with PADP = R makes that stride R + 1 and spreads the
// accesses over the banks.
template <int PADP> __device__ __forceinline__ int padpos(int pos) {
  if constexpr (PADP > 0) return pos + pos / PADP;
  else return pos;
}

// Stride of a contiguous padded line of n elements (pad element every pad).
constexpr int xstride(int n, int pad) { return n + n / pad + 1; }

// Exchange through LDS after a pass of radix R (span Ns) into the input
// layout of a pass of radix R2.  Element at position pos lives at
// lds[padpos(pos) * ps + off].
template <typename T, int N, int E, int R, int Ns, int R2, int PADP>
__device__ __forceinline__ void reg_exchange(cplx<T> (&v)[E], int t, cplx<T> *lds, int ps,
                                             int off) {
  constexpr int TPL = N / E;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j = t + b * TPL;
    const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
    for (int r = 0; r < R; ++r) lds[padpos<PADP>(base + r * Ns) * ps + off] = v[b * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < E / R2; ++b)
#pragma unroll
    for (int r = 0; r < R2; ++r)
      v[b * R2 + r] = lds[padpos<PADP>(reg_pos<N, E, R2>(t, b, r)) * ps + off];
}

template <typename T, int N, int E, bool REV, int P, int Ns, int PADP>
__device__ __forceinline__ void reg_run(cplx<T> (&v)[E], int t, cplx<T> *lds, int ps, int off,
                                        const cplx<T> *__restrict__ tw, int dir) {
  using S = Shape<N, E>;
  constexpr int R = S::radix(P, REV);
  reg_pass<T, N, E, R, Ns>(v, t, tw, dir);
  if constexpr (P + 1 < S::NP) {
    constexpr int R2 = S::radix(P + 1, REV);
    reg_exchange<T, N, E, R, Ns, R2, PADP>(v, t, lds, ps, off);
    reg_run<T, N, E, REV, P + 1, Ns * R, PADP>(v, t, lds, ps, off, tw, dir);
  }
}

// Forward transform (exp(-2 pi i k n / N)) with the passes in factor order.
template <typename T, int N, int E, int PADP = 0>
__device__ __forceinline__ void reg_fft_forward(cplx<T> (&v)[E], int t, cplx<T> *lds, int ps,
                                                int off, const cplx<T> *__restrict__ tw) {
  reg_run<T, N, E, false, 0, 1, PADP>(v, t, lds, ps, off, tw, -1);
}

// Inverse (unnormalised, exp(+2 pi i k n / N)) with the passes reversed.
template <typename T, int N, int E, int PADP = 0>
__device__ __forceinline__ void reg_fft_inverse(cplx<T> (&v)[E], int t, cplx<T> *lds, int ps,
                                                int off, const cplx<T> *__restrict__ tw) {
  reg_run<T, N, E, true, 0, 1, PADP>(v, t, lds, ps, off, tw, +1);
}

// The twiddle table in LDS behind a kernel's exchange area: the transforms
// then read their twiddles with LDS loads.  Read from global memory inside a
// transform, each twiddle's first use waits on the in-order vector-memory
// counter, that is for every grid load and store issued before it, so no
// transform overlaps the grid traffic in flight.  A thread takes its entry
// before the grid loads (tw_fetch) and stores it after issuing them
// (tw_store); a transform's first pass uses no twiddles, so the first
// exchange's barrier orders these stores before any read.
template <typename C, int N>
__device__ __forceinline__ C tw_fetch(const C *__restrict__ tw) {
  return threadIdx.x < N ? tw[threadIdx.x] : C{};
}

template <typename C, int N>
__device__ __forceinline__ void tw_store(C *twl, C first, const C *__restrict__ tw) {
  if (threadIdx.x < N) twl[threadIdx.x] = first;
  for (int i = (int)(threadIdx.x + blockDim.x); i < N; i += blockDim.x) twl[i] = tw[i];
}

// Element counts per thread: line passes and the fused k-space kernel (which
// also keeps three complex numbers per element in registers, so it takes few
// elements: 4 for powers of two, 6 (radices 6, 3, 2) for 3 * 2^k lengths).
constexpr int line_e(int n) { return n % 3 == 0 ? 12 : (n >= 128 ? 16 : 8); }
constexpr int fused_e(int n) { return n % 3 == 0 ? 6 : 4; }

// Lines per workgroup: a power of two dividing `count`, at most max_threads
// threads (about 256 by default), LDS of tl * line_bytes within 64 KiB.
int lines_per_block(int n, int tpl, size_t line_bytes, size_t count, int max_threads = 256);

// Line lengths whose x-y plane fits one workgroup's LDS.
#define PSE_FOR_EACH_SMALL_N(X) X(32) X(48) X(64) X(96) X(128)

// Supported line lengths (the grid sizes accepted by the parameter rule).
#define PSE_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

}  // namespace pse
