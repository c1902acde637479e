// Stockham autosort FFT on lines staged in LDS (shared by the FFT passes and
// the fused k-space kernel).  LDS holds TL lines of length N laid out
// [position][line]; radix 4, 2 and 3 stages follow the Govindaraju et al.
// (SC'08) formulation, ping-ponging between two LDS buffers.
#pragma once

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

inline FftPlan make_plan(int n, size_t elem_bytes) {
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

}  // namespace pse
