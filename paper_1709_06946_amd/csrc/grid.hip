// Wave-space stages of the NUFFT mobility (Sec. II.C, Eq. WSops2) and of the
// wave-space square root (Sec. III.C, Eq. FFTsqrt).
//
// Grids: each of the G real components of one operator application has its
// own real grid [c][z][y][x]; the real FFT turns it in place into a half
// spectrum [c][kz][ky][kx < n/2] (fft.hip), so the k-space kernels act on one
// wave vector at a time and the other half follows by Hermitian symmetry.
//
// Gaussian kernel (Sec. II.C): K(r) = (2 xi^2/(pi eta_s))^(3/2)
// exp(-2 xi^2 r^2 / eta_s), truncated to the P^3 nearest grid points, whose
// Fourier transform is exp(-eta_s k^2 / 8 xi^2).  Spreading and
// interpolation each contribute that factor once; the k-space scaling
// divides both out again.
#include <mutex>
#include <type_traits>

#include "fftreg.h"

namespace pse {

// ---------------------------------------------------------------- helpers --

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// First stencil index and the grid offset of a particle coordinate.
__device__ __forceinline__ int stencil_start(double xc, double h, int P) {
  const double f = xc / h;
  return (P & 1) ? (int)floor(f + 0.5) - (P - 1) / 2 : (int)floor(f) - P / 2 + 1;
}

template <typename T> __device__ __forceinline__ T &part(cplx<T> &z, int k) {
  return (k & 1) ? z.y : z.x;
}

// ------------------------------------------------------------- spreading --

// One wavefront per particle; its lanes cover the P^3 stencil.
template <typename T>
__global__ void __launch_bounds__(256)
spread_kernel(const double *__restrict__ x, const double *__restrict__ q,
              Layout lq, CompSet cs, GridGeom g, const int *__restrict__ order,
              int64_t n, T *__restrict__ grids, size_t ngrid) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  const int64_t p = order ? order[t] : t;
  const double px = x[3 * p], py = x[3 * p + 1], pz = x[3 * p + 2];
  const int P = g.P, P3 = P * P * P;
  const int ix0 = stencil_start(px, g.h, P);
  const int iy0 = stencil_start(py, g.h, P);
  const int iz0 = stencil_start(pz, g.h, P);
  T qv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k)
    qv[k] = k < cs.n ? (T)q[p * lq.stride + cs.idx[k] - lq.off] : (T)0;
  const double kn3 = g.knorm * g.knorm * g.knorm;
  for (int s = lane; s < P3; s += 64) {
    const int a = s % P, b = (s / P) % P, c = s / (P * P);
    const double dx = (ix0 + a) * g.h - px;
    const double dy = (iy0 + b) * g.h - py;
    const double dz = (iz0 + c) * g.h - pz;
    const double r2 = g.def ? qform(g.G, dx, dy, dz) : dx * dx + dy * dy + dz * dz;
    const T w = (T)(kn3 * exp(-g.kcoef * r2));
    const size_t gi = ((size_t)wrapi(iz0 + c, g.ng) * g.ng + wrapi(iy0 + b, g.ng)) * g.ng
                      + wrapi(ix0 + a, g.ng);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k < cs.n) atomicAdd(grids + (size_t)k * ngrid + gi, w * qv[k]);
    }
  }
}

// Whether a stencil starting at grid index st (P points) meets the tile
// starting at t0 (S points) on a periodic axis of ng points.
__device__ __forceinline__ bool stencil_meets(int st, int t0, int P, int S, int ng) {
  int a = (t0 - st) % ng;
  a += a < 0 ? ng : 0;
  return a < P || a > ng - S;
}

// The candidate lists hold one record per (tile, particle) pair: the
// particle index (rp) and REC_W(S) doubles (rw): the one-dimensional Gaussian
// weights at the tile's S grid positions along x, y and z (zero outside the
// stencil), then per axis the offset d0 such that d0 + i h is the distance
// from the particle to tile position i wherever the weight is nonzero (the
// gradient weights of derivative gridding are -2 kcoef (d0 + i h) w_i).  They
// depend on the positions only, so they are formed once per position update,
// when the lists are built.
struct TileRecs {
  int *p;
  double *w;
};

// FILL = false: count each tile's candidates; true: write their records from
// start[tile] on, in bin order and ranked with a ballot.  One wavefront per
// tile enumerates the particles of the 27 bins around it 64 at a time (bins
// are tiles; a stencil reaches at most one tile beyond its particle's).
template <bool FILL>
__global__ void __launch_bounds__(256)
tile_list_kernel(const double *__restrict__ x, GridGeom g, int S, int nb,
                 const int *__restrict__ bstart, const int *__restrict__ bperm,
                 int *__restrict__ cnt, const int *__restrict__ start, TileRecs rec) {
  const int tile = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (tile >= nb * nb * nb) return;
  const int tc[3] = {tile % nb, (tile / nb) % nb, tile / (nb * nb)};
  const int P = g.P, ng = g.ng;
  int first, pre, total;
  nbr27_setup(lane, tc[0], tc[1], tc[2], nb, bstart, first, pre, total);
  int pos = FILL ? start[tile] : 0;
  int count = 0;
  for (int base = 0; base < total; base += 64) {
    const int idx = base + lane;
    const int s = nbr27_slot(idx, first, pre);
    bool ok = false;
    int p = 0, st[3] = {0, 0, 0};
    if (idx < total) {
      p = bperm[s];
      ok = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        st[d] = stencil_start(x[3 * p + d], g.h, P);
        ok = ok && stencil_meets(st[d], tc[d] * S, P, S, ng);
      }
    }
    if (!FILL) {
      count += ok ? 1 : 0;
    } else {
      const unsigned long long m = __ballot(ok);
      if (ok) {
        // the record's particle and, in its first offset slot, the tile's
        // index; tile_weights_kernel forms the weights and offsets (on every
        // lane, not on the lanes of a candidate batch that met the tile)
        const int e = pos + __popcll(m & ((1ull << lane) - 1ull));
        rec.p[e] = p;
        rec.w[(size_t)e * (3 * S + 3) + 3 * S] = (double)tile;
      }
      pos += __popcll(m);
    }
  }
  if (!FILL) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
    if (lane == 0) cnt[tile] = count;
  }
}

// Second half of the tile-list fill: for every record, the S
// one-dimensional weights of its particle at the tile's grid positions along
// each axis (zero outside its stencil) and the offset d0 of the first
// stencil point inside the tile from that position.  A workgroup takes
// TW_RECS records, one thread per (record, axis), forms their 3 S + 3
// numbers in LDS and writes them back as one contiguous block, so the stores
// are coalesced (written in place, each record's numbers stride 3 S + 3
// apart across the threads).
constexpr int TW_RECS = 64;

__global__ void __launch_bounds__(3 * TW_RECS)
tile_weights_kernel(const double *__restrict__ x, GridGeom g, int S, int nb,
                    const int *__restrict__ total, int64_t cap, TileRecs rec) {
  extern __shared__ double tw_block[];   // TW_RECS records of 3 S + 3
  const int RW = 3 * S + 3;
  const int64_t len = min((int64_t)total[0], cap);
  const int64_t e0 = (int64_t)blockIdx.x * TW_RECS;
  if (e0 >= len) return;
  const int nrec = (int)min((int64_t)TW_RECS, len - e0);
  const int tid = threadIdx.x;
  const int j = tid / 3, d = tid % 3;
  if (j < nrec) {
    const int64_t e = e0 + j;
    const int P = g.P, ng = g.ng;
    const int p = rec.p[e];
    // the tile's first grid index along the axis, from the tile index the
    // list fill left in the record
    const int tile = (int)rec.w[(size_t)e * RW + 3 * S];
    const int t0 = (d == 0 ? tile % nb : (d == 1 ? (tile / nb) % nb : tile / (nb * nb))) * S;
    const double xd = x[3 * p + d];
    const int st = stencil_start(xd, g.h, P);
    double d0 = 0.0;
    for (int i = 0; i < S; ++i) {
      int a = (t0 + i - st) % ng;
      a += a < 0 ? ng : 0;
      double wi = 0.0;
      if (a < P) {
        const double dx = (st + a) * g.h - xd;
        wi = g.knorm * exp(-g.kcoef * dx * dx);
        d0 = dx - i * g.h;
      }
      tw_block[j * RW + d * S + i] = wi;
    }
    tw_block[j * RW + 3 * S + d] = d0;
  }
  __syncthreads();
  double *dst = rec.w + (size_t)e0 * RW;
  for (int k = tid; k < nrec * RW; k += blockDim.x) dst[k] = tw_block[k];
}

// Gather form of the spreading sum: one workgroup per tile of S^3 grid
// points reads the tile's candidate records.  The Gaussian factorises over
// the axes, K = w_x w_y w_z, and the records carry the 1D weights, so a chunk
// of candidates is staged in LDS with one coalesced read of its weights and
// one gather of its moments.  Each thread owns ZPT points of one z-column of
// the tile and, per candidate, forms w_x w_y once and reads the moments once
// for all of them.  Every grid point is written exactly once: no atomics and
// no zeroing pass.
constexpr int GMAXC = 32;

template <typename T, int S, int NCM, int ZPT>
__global__ void __launch_bounds__(S * S * S / ZPT)
spread_list_kernel(const double *__restrict__ q, Layout lq, CompSet cs, GridGeom g, int nb,
                   const int *__restrict__ tstart, TileRecs rec, T *__restrict__ grids,
                   size_t ngrid) {
  constexpr int NT = S * S * S / ZPT;
  constexpr int RW = 3 * S + 3;
  constexpr int WPT = (GMAXC * RW + NT - 1) / NT;
  constexpr int NCMP = NCM + (NCM & 1);
  static_assert(GMAXC <= NT, "one candidate per thread in the moment gather");
  __shared__ T wts[GMAXC * RW];
  __shared__ T cq[GMAXC * NCMP];
  const int tile = blockIdx.x;
  const int tc[3] = {tile % nb, (tile / nb) % nb, tile / (nb * nb)};
  const int lo = tstart[tile];
  const int total = tstart[tile + 1] - lo;
  const int ng = g.ng;
  const int tid = threadIdx.x;
  const int lx = tid % S, ly = (tid / S) % S, z0 = (tid / (S * S)) * ZPT;
  T acc[ZPT][NCM];
#pragma unroll
  for (int z = 0; z < ZPT; ++z)
#pragma unroll
    for (int k = 0; k < NCM; ++k) acc[z][k] = (T)0;
  for (int c0 = 0; c0 < total; c0 += GMAXC) {
    const int nchunk = min(GMAXC, total - c0);
    const int nw = nchunk * RW;
    __syncthreads();
    const int pj = tid < nchunk ? rec.p[lo + c0 + tid] : 0;
    const double *wsrc = rec.w + (size_t)(lo + c0) * RW;
    double wv[WPT];
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int t = tid + i * NT;
      wv[i] = t < nw ? wsrc[t] : 0.0;
    }
    if (tid < nchunk) {
#pragma unroll
      for (int k = 0; k < NCM; ++k)
        if (k < cs.n) cq[tid * NCMP + k] = (T)q[(size_t)pj * lq.stride + cs.idx[k] - lq.off];
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int t = tid + i * NT;
      if (t < nw) wts[t] = (T)wv[i];
    }
    __syncthreads();
    for (int j = 0; j < nchunk; ++j) {
      const T *wj = wts + j * RW;
      const T wxy = wj[lx] * wj[S + ly];
      T qk[NCM];
#pragma unroll
      for (int k = 0; k < NCM; ++k) qk[k] = cq[j * NCMP + k];
#pragma unroll
      for (int z = 0; z < ZPT; ++z) {
        const T w = wxy * wj[2 * S + z0 + z];
#pragma unroll
        for (int k = 0; k < NCM; ++k)
          if (k < cs.n) acc[z][k] += w * qk[k];
      }
    }
  }
#pragma unroll
  for (int z = 0; z < ZPT; ++z) {
    const size_t gi = ((size_t)(tc[2] * S + z0 + z) * ng + tc[1] * S + ly) * ng
                      + tc[0] * S + lx;
#pragma unroll
    for (int k = 0; k < NCM; ++k)
      if (k < cs.n) grids[(size_t)k * ngrid + gi] = acc[z][k];
  }
}

// Derivative gridding of the couplets: three grids
// D_i(x_n) = sum_b sum_j C_b,ij dK/dx_j (x_n - x_b), with C_b = S_b + A_b the
// particle's couplet, S_b the symmetric traceless stresslet of its five
// components in the Y_q basis and A_b x = (1/2) L_b x x its torque.  Their
// transform is i C^ k K^, so the k-space factors of the stresslet column,
// -3 i f1(ka) Y_q k, and of the torque column, (3/2) i f1(ka) k x e_c,
// become one factor -3 f1(ka) on D^ (Eq. WSops with the gradient moved onto
// the Gaussian).  With HF the forces are spread as well, onto three grids
// ahead of the couplet grids: F_i K (x_n - x_b), the moment gridding of F.
// Input groups (forces 0-2, torques 3-5, stresslets 6-10) are either all in
// cs or absent (hasL, hasS).  Tiles, records and staging as
// spread_list_kernel; per candidate the gradient weights along each axis are
// g_i = -2 kcoef (d0 + i h) w_i, and per point dK/dx = g_x w_y w_z, etc.
template <typename T, int S, int ZPT, bool HF>
__global__ void __launch_bounds__(S * S * S / ZPT)
spread_deriv_kernel(const double *__restrict__ q, Layout lq, CompSet cs, int hasL, int hasS,
                    GridGeom g, int nb, const int *__restrict__ tstart, TileRecs rec,
                    const double *__restrict__ mu, T *__restrict__ grids, size_t ngrid) {
  constexpr int NT = S * S * S / ZPT;
  constexpr int RW = 3 * S + 3;
  constexpr int WPT = (GMAXC * RW + NT - 1) / NT;
  constexpr int NQ = HF ? 12 : 9;      // per candidate: C (9), then F (3)
  constexpr int NG = HF ? 6 : 3;
  static_assert(GMAXC <= NT, "one candidate per thread in the moment gather");
  __shared__ double raw[GMAXC * RW];
  __shared__ T wg[GMAXC * 6 * S];      // per candidate: w (3 S), then g (3 S)
  __shared__ T cq[GMAXC * NQ];
  __shared__ double cmu[GMAXC * 6];   // per candidate: mu (3), lambda (3)
  const int tile = blockIdx.x;
  const int tc[3] = {tile % nb, (tile / nb) % nb, tile / (nb * nb)};
  const int lo = tstart[tile];
  const int total = tstart[tile + 1] - lo;
  const int ng = g.ng;
  const int tid = threadIdx.x;
  const int lx = tid % S, ly = (tid / S) % S, z0 = (tid / (S * S)) * ZPT;
  const T r2 = (T)0.70710678118654752440, r6 = (T)0.40824829046386301637;
  // positions of the groups in cs (cs lists them in increasing order)
  const int kL = HF ? 3 : 0, kS = kL + (hasL ? 3 : 0);
  T acc[ZPT][NG];
#pragma unroll
  for (int z = 0; z < ZPT; ++z)
#pragma unroll
    for (int k = 0; k < NG; ++k) acc[z][k] = (T)0;
  for (int c0 = 0; c0 < total; c0 += GMAXC) {
    const int nchunk = min(GMAXC, total - c0);
    const int nw = nchunk * RW;
    __syncthreads();
    const int pj = tid < nchunk ? rec.p[lo + c0 + tid] : 0;
    const double *wsrc = rec.w + (size_t)(lo + c0) * RW;
    double wv[WPT];
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int t = tid + i * NT;
      wv[i] = t < nw ? wsrc[t] : 0.0;
    }
    if (tid < nchunk) {
      const double *qp = q + (size_t)pj * lq.stride - lq.off;
      T sq[5] = {(T)0, (T)0, (T)0, (T)0, (T)0}, lh[3] = {(T)0, (T)0, (T)0};
      if (hasS)
#pragma unroll
        for (int k = 0; k < 5; ++k) sq[k] = (T)qp[cs.idx[kS + k]];
      if (hasL)
#pragma unroll
        for (int k = 0; k < 3; ++k) lh[k] = (T)0.5 * (T)qp[cs.idx[kL + k]];
      const T sxy = r2 * sq[0], sxz = r2 * sq[1], syz = r2 * sq[2];
      T *o = cq + tid * NQ;
      o[0] = r2 * sq[3] + r6 * sq[4];          // Cxx
      o[1] = sxy - lh[2];                      // Cxy
      o[2] = sxz + lh[1];                      // Cxz
      o[3] = sxy + lh[2];                      // Cyx
      o[4] = -r2 * sq[3] + r6 * sq[4];         // Cyy
      o[5] = syz - lh[0];                      // Cyz
      o[6] = sxz - lh[1];                      // Czx
      o[7] = syz + lh[0];                      // Czy
      o[8] = (T)-2 * r6 * sq[4];               // Czz
      if constexpr (HF)
#pragma unroll
        for (int k = 0; k < 3; ++k) o[9 + k] = (T)qp[cs.idx[k]];
#pragma unroll
      for (int k = 0; k < 6; ++k) cmu[tid * 6 + k] = mu[6 * (size_t)pj + k];
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int t = tid + i * NT;
      if (t < nw) raw[t] = wv[i];
    }
    __syncthreads();
    for (int t = tid; t < nchunk * 3 * S; t += NT) {
      const int j = t / (3 * S), r = t % (3 * S), d = r / S, i = r % S;
      const double w = raw[j * RW + r];
      const double dx = raw[j * RW + 3 * S + d] + i * g.h;
      wg[j * 6 * S + r] = (T)w;
      wg[j * 6 * S + 3 * S + r] =
          (T)(cmu[j * 6 + 3 + d] * (-2.0 * g.kcoef * dx - cmu[j * 6 + d]) * w);
    }
    __syncthreads();
    for (int j = 0; j < nchunk; ++j) {
      const T *wj = wg + j * 6 * S, *gj = wj + 3 * S, *cj = cq + j * NQ;
      const T gxwy = gj[lx] * wj[S + ly], wxgy = wj[lx] * gj[S + ly], wxwy = wj[lx] * wj[S + ly];
      // D_i = (C_ix g_x w_y + C_iy w_x g_y) w_z + C_iz w_x w_y g_z: the two
      // brackets are constant along the thread's z-column
      T a[3], b[3], f[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        a[i] = cj[3 * i] * gxwy + cj[3 * i + 1] * wxgy;
        b[i] = cj[3 * i + 2] * wxwy;
      }
      if constexpr (HF)
#pragma unroll
        for (int i = 0; i < 3; ++i) f[i] = cj[9 + i] * wxwy;
#pragma unroll
      for (int z = 0; z < ZPT; ++z) {
        const T wz = wj[2 * S + z0 + z], gz = gj[2 * S + z0 + z];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          if constexpr (HF) acc[z][i] += f[i] * wz;
          acc[z][NG - 3 + i] += a[i] * wz + b[i] * gz;
        }
      }
    }
  }
#pragma unroll
  for (int z = 0; z < ZPT; ++z) {
    const size_t gi = ((size_t)(tc[2] * S + z0 + z) * ng + tc[1] * S + ly) * ng
                      + tc[0] * S + lx;
#pragma unroll
    for (int k = 0; k < NG; ++k) grids[(size_t)k * ngrid + gi] = acc[z][k];
  }
}

// --------------------------------------------------------- interpolation --

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const long long hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((hi << 32) | lo);
}

// Any support: lane l holds the one-dimensional factors exp(-kcoef d^2) at
// offset l along x, y and z (meaningful for l < P); stencil point (a, b, c)
// takes the product of the three, fetched from lanes a, b and c.  Every lane
// of the wavefront must call it and the shuffles (all lanes active).
__device__ __forceinline__ void factors1d(int lane, double px, double py, double pz, int ix0,
                                          int iy0, int iz0, const GridGeom &g, double f[3]) {
  const double dx = (ix0 + lane) * g.h - px, dy = (iy0 + lane) * g.h - py;
  const double dz = (iz0 + lane) * g.h - pz;
  f[0] = exp(-g.kcoef * dx * dx);
  f[1] = exp(-g.kcoef * dy * dy);
  f[2] = exp(-g.kcoef * dz * dz);
}

__device__ __forceinline__ double gauss_at(const double f[3], int a, int b, int c) {
  return __shfl(f[0], a & 63, 64) * __shfl(f[1], b & 63, 64) * __shfl(f[2], c & 63, 64);
}

// Support 8 (512 stencil points, 8 per lane): lane l covers the points
// (a, b) = (l % 8, l / 8) at every z index c, its point it being c = it.
// The Gaussian factorises, so a lane takes one exponential for its x-y
// factor and one for the z factor of c = l % 8; the z factor of point it is
// read from lane it.  Fills the grid offsets (within one grid: below 2^31
// for every supported length) and exp(-kcoef |d|^2) of the lane's eight
// points, and their offsets d along z (x and y are dx, dy); the weights and
// z offsets in the kernel's type T (FP32 kernels keep half the registers).
__device__ __forceinline__ float readlane_t(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_t(double v, int l) { return readlane_d(v, l); }

template <typename T>
__device__ __forceinline__ void stencil8(int lane, double px, double py, double pz, int ix0,
                                         int iy0, int iz0, const GridGeom &g, uint32_t gi[8],
                                         T e[8], T dz[8], double &dx, double &dy) {
  const int a = lane & 7, b = lane >> 3;
  dx = (ix0 + a) * g.h - px;
  dy = (iy0 + b) * g.h - py;
  const T exy = (T)exp(-g.kcoef * (dx * dx + dy * dy));
  const double dzl = (iz0 + a) * g.h - pz;
  const T ezl = (T)exp(-g.kcoef * dzl * dzl);
  const uint32_t gxy = (uint32_t)wrapi(iy0 + b, g.ng) * g.ng + wrapi(ix0 + a, g.ng);
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    dz[it] = (T)((iz0 + it) * g.h - pz);
    e[it] = exy * readlane_t(ezl, it);
    gi[it] = (uint32_t)wrapi(iz0 + it, g.ng) * g.ng * g.ng + gxy;
  }
}

// One wavefront per particle (particles in cell order, each XCD taking a
// contiguous range of them so that neighbouring stencils share its L2);
// lane s covers stencil points s, s + 64, ...
// With MAXIT = ceil(P^3 / 64) fixed at compile time, a lane first forms all
// its grid indices and weights and then issues every grid load at once, so
// that the loads of all stencil points and components are in flight
// together (MAXIT = 0: generic loop for large supports).
template <typename T, int MAXIT>
__global__ void __launch_bounds__(256)
interp_kernel(const double *__restrict__ x, const T *__restrict__ grids,
              size_t ngrid, CompSet cs, GridGeom g, const int *__restrict__ order,
              int64_t n, double *__restrict__ out, Layout lo, int accumulate,
              double scale) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  const int64_t p = order ? order[t] : t;
  const double px = x[3 * p], py = x[3 * p + 1], pz = x[3 * p + 2];
  const int P = g.P, P3 = P * P * P;
  const int ix0 = stencil_start(px, g.h, P);
  const int iy0 = stencil_start(py, g.h, P);
  const int iz0 = stencil_start(pz, g.h, P);
  T acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = (T)0;
  const double kn3 = g.knorm * g.knorm * g.knorm;
  if constexpr (MAXIT > 0) {
    uint32_t gi[MAXIT];
    T w[MAXIT];
    bool done = false;
    if constexpr (MAXIT == 8) {
      if (P == 8) {
        T e[8], dz[8];
        double dx, dy;
        stencil8<T>(lane, px, py, pz, ix0, iy0, iz0, g, gi, e, dz, dx, dy);
#pragma unroll
        for (int it = 0; it < 8; ++it) w[it] = (T)kn3 * e[it];
        done = true;
      }
    }
    if (!done) {
      double f[3];
      factors1d(lane, px, py, pz, ix0, iy0, iz0, g, f);
#pragma unroll
      for (int it = 0; it < MAXIT; ++it) {
        const int s = lane + 64 * it;
        const int a = s % P, b = (s / P) % P, c = s / (P * P);
        const bool in = s < P3;
        const double e = gauss_at(f, a, b, c);
        w[it] = in ? (T)(kn3 * e) : (T)0;
        gi[it] = in ? ((uint32_t)wrapi(iz0 + c, g.ng) * g.ng + wrapi(iy0 + b, g.ng)) * g.ng
                          + wrapi(ix0 + a, g.ng)
                    : 0;
      }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k < cs.n) {
        const T *gk = grids + (size_t)k * ngrid;
        T v[MAXIT];
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) v[it] = gk[gi[it]];
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) acc[k] += w[it] * v[it];
      }
    }
  } else {
    for (int s = lane; s < P3; s += 64) {
      const int a = s % P, b = (s / P) % P, c = s / (P * P);
      const double dx = (ix0 + a) * g.h - px;
      const double dy = (iy0 + b) * g.h - py;
      const double dz = (iz0 + c) * g.h - pz;
      const double r2 = g.def ? qform(g.G, dx, dy, dz) : dx * dx + dy * dy + dz * dz;
      const T w = (T)(kn3 * exp(-g.kcoef * r2));
      const size_t gi = ((size_t)wrapi(iz0 + c, g.ng) * g.ng + wrapi(iy0 + b, g.ng)) * g.ng
                        + wrapi(ix0 + a, g.ng);
#pragma unroll
      for (int k = 0; k < NC; ++k)
        if (k < cs.n) acc[k] += w * grids[(size_t)k * ngrid + gi];
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k < cs.n) {
      T v = acc[k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[k] = v;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k < cs.n) {
        double *o = out + p * lo.stride + cs.idx[k] - lo.off;
        const double v = scale * (double)acc[k];
        *o = accumulate ? *o + v : v;
      }
    }
  }
}

// ------------------------------------------------------ k-space kernels --

// Wave vector of grid index i (FFT order).
__device__ __forceinline__ int kidx(int i, int n) { return i < n / 2 ? i : i - n; }

// Shape factors j0(x) = sin x / x and f1(x) = (sin x - x cos x)/x^3
// (Eq. WSops); series below x = 0.1 where the closed form cancels.
__device__ __forceinline__ void shape_factors(double x, double &j0, double &f1) {
  if (x < 0.1) {
    const double x2 = x * x;
    j0 = 1.0 - x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0));
    f1 = 1.0 / 3.0 - x2 / 30.0 * (1.0 - x2 / 28.0 * (1.0 - x2 / 54.0));
  } else {
    double s, c;
    sincos(x, &s, &c);
    j0 = s / x;
    f1 = (s - x * c) / (x * x * x);
  }
}

// k-table entry type per precision: double4 for the FP64 kernels, float4
// (the same values rounded) for the FP32 ones.
template <typename T> struct TabT;
template <> struct TabT<double> { using type = double4; };
template <> struct TabT<float> { using type = float4; };

struct KGeom {
  int ng;
  double twopi_L;     // 2 pi / L
  double a;
  double inv4xi2;     // 1 / (4 xi^2)
  double one_m_etas;  // 1 - eta_s
  double pref_m;      // mobility: h^6 / (V eta)
  double pref_n;      // noise: h^3 / sqrt(V eta)
  int def;            // deformed lattice: k = (2 pi / L) A^-T n
  double Ai[9];       // A^-1 (row-major)
};

// Wave vector of the integer index (i, j, l): (2 pi / L) A^-T (i, j, l).
__device__ __forceinline__ void deformed_k(const KGeom &kg, int i, int j, int l, double *kv) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    kv[r] = kg.twopi_L * (kg.Ai[r] * i + kg.Ai[3 + r] * j + kg.Ai[6 + r] * l);
}

// Every stored wave vector is k = (2 pi / L) (i, j, l) with integers, so all
// radial factors depend on |k|^2 only through the integer n2 = i^2 + j^2 + l^2
// <= 3 (N/2)^2.  The table holds, per n2:
//   x = j0(ka), y = f1(ka), z = h^6/(V eta) (1 + u) e^{-(1 - eta_s) u} / k^2,
//   w = h^3/sqrt(V eta) sqrt(1 + u) e^{-(1 - eta_s) u / 2} / k,  u = k^2 / 4 xi^2
// (the mobility scaling of Eq. WSops2 with both Gaussian factors divided out,
// and the amplitude of Eq. FFTsqrt).  Entry 0 (k = 0) is zero.
// Radial factors of one wave number k^2 (the entries of the |k|^2 table):
// j0(ka), f1(ka), the mobility scale and the noise amplitude.
__device__ __forceinline__ double4 radial_factors(const KGeom &kg, double k2) {
  const double k = sqrt(k2);
  double j0, f1;
  shape_factors(k * kg.a, j0, f1);
  const double u = k2 * kg.inv4xi2;
  const double mob = kg.pref_m * (1.0 + u) * exp(-kg.one_m_etas * u) / k2;
  const double amp = kg.pref_n * sqrt(1.0 + u) * exp(-0.5 * kg.one_m_etas * u) / k;
  return double4{j0, f1, mob, amp};
}

__global__ void __launch_bounds__(256)
ktable_kernel(KGeom kg, int len, double4 *__restrict__ tab) {
  const int n2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (n2 >= len) return;
  if (n2 == 0) {
    tab[0] = double4{0, 0, 0, 0};
    return;
  }
  const double k2 = kg.twopi_L * kg.twopi_L * (double)n2;
  const double k = sqrt(k2);
  double j0, f1;
  shape_factors(k * kg.a, j0, f1);
  const double u = k2 * kg.inv4xi2;
  const double mob = kg.pref_m * (1.0 + u) * exp(-kg.one_m_etas * u) / k2;
  const double amp = kg.pref_n * sqrt(1.0 + u) * exp(-0.5 * kg.one_m_etas * u) / k;
  tab[n2] = double4{j0, f1, mob, amp};
}

// Column of P(k) for moment component c (0..10), as (coef, col): the
// contribution to rho is coef * col * g with coef real for F (j0) and
// imaginary for L and s:
//   F_c:  j0 e_c;   L_l: (3i/2) f1 (k x e_l);   s_q: -3i f1 Y_q k.
// R is the arithmetic type (double, or float in the FP32 kernels).
template <typename R>
__device__ __forceinline__ void p_column(int c, R kx, R ky, R kz, R j0, R f1, bool &imag,
                                         R &cx, R &cy, R &cz) {
  const R r2 = (R)0.70710678118654752440, r6 = (R)0.40824829046386301637;
  imag = c >= 3;
  const R a = (R)1.5 * f1, b = (R)-3.0 * f1;
  switch (c) {
    case 0: cx = j0;  cy = 0;   cz = 0;   break;
    case 1: cx = 0;   cy = j0;  cz = 0;   break;
    case 2: cx = 0;   cy = 0;   cz = j0;  break;
    case 3: cx = 0;   cy = a * kz;  cz = -a * ky; break;       // k x e_x
    case 4: cx = -a * kz; cy = 0;   cz = a * kx;  break;       // k x e_y
    case 5: cx = a * ky;  cy = -a * kx; cz = 0;   break;       // k x e_z
    case 6: cx = b * r2 * ky; cy = b * r2 * kx; cz = 0; break;
    case 7: cx = b * r2 * kz; cy = 0; cz = b * r2 * kx; break;
    case 8: cx = 0; cy = b * r2 * kz; cz = b * r2 * ky; break;
    case 9: cx = b * r2 * kx; cy = -b * r2 * ky; cz = 0; break;
    default: cx = b * r6 * kx; cy = b * r6 * ky; cz = (R)-2.0 * b * r6 * kz; break;
  }
}

// rho += P_c(k) g
template <typename C, typename R>
__device__ __forceinline__ void add_P(int c, C gv, const R *kv, R j0, R f1, C *rho) {
  bool imag;
  R cx, cy, cz;
  p_column<R>(c, kv[0], kv[1], kv[2], j0, f1, imag, cx, cy, cz);
  const R gx = (R)gv.x, gy = (R)gv.y;
  if (!imag) {
    rho[0].x += cx * gx; rho[0].y += cx * gy;
    rho[1].x += cy * gx; rho[1].y += cy * gy;
    rho[2].x += cz * gx; rho[2].y += cz * gy;
  } else {
    // i col g = col (-g.y, g.x)
    rho[0].x -= cx * gy; rho[0].y += cx * gx;
    rho[1].x -= cy * gy; rho[1].y += cy * gx;
    rho[2].x -= cz * gy; rho[2].y += cz * gx;
  }
}

// W_c = P_c^+ u = conj(coef) col . u
template <typename C, typename R>
__device__ __forceinline__ C apply_Pdag(int c, const C *u, const R *kv, R j0, R f1) {
  bool imag;
  R cx, cy, cz;
  p_column<R>(c, kv[0], kv[1], kv[2], j0, f1, imag, cx, cy, cz);
  const R re = cx * (R)u[0].x + cy * (R)u[1].x + cz * (R)u[2].x;
  const R im = cx * (R)u[0].y + cy * (R)u[1].y + cz * (R)u[2].y;
  C w;
  if (!imag) {
    w.x = re;
    w.y = im;
  } else {
    // conj(i) = -i: -i (re + i im) = im - i re
    w.x = im;
    w.y = -re;
  }
  return w;
}

// Stored half-spectrum mode (ix < n/2, iy, iz) that is zeroed: a Nyquist
// index in y or z, or k = 0 (the x Nyquist column is not stored).
__device__ __forceinline__ bool zero_mode(int ix, int iy, int iz, int n) {
  const int h = n / 2;
  return iy == h || iz == h || (ix == 0 && iy == 0 && iz == 0);
}

// Fused z transform + k-space kernel + inverse z transform (Eq. WSops2 from
// the half spectra after the x and y transforms back to them).  A workgroup
// owns TL neighbouring kx columns at one ky, i.e. TL z-lines, each
// transformed by TPL threads that hold E modes in registers.  For every input
// component the z transform runs in registers and the mode is folded at
// once into rho(k) = sum_c P_c(k) G_c(k) (three complex numbers per mode,
// kept in registers), so the inputs stream through one at a time.  Then
// u = scale (I - k^k^) rho, and for every output component P_q^+ u is formed
// in the same registers -- the inverse transform runs the passes in reverse
// order, so its input layout is the forward output layout -- transformed back
// along z and stored.  One read of the inputs and one write of the outputs.
// DG (derivative gridding): the components are grid codes, 0-2 the force
// grids F^ (factor j0(ka)) and 3-5 the couplet grids D^ spread with the
// Gaussian's gradient (factor -3 f1(ka)) on input, so rho = j0 F^ - 3 f1 D^;
// on output 0-2 the velocity grids j0(ka) u^ and 3-5 the grids
// v^ = 3 f1(ka) u^ whose gradient the interpolation takes.
template <typename T, int N, bool DG>
__global__ void __launch_bounds__(512)
kspace_fused_kernel(const cplx<T> *__restrict__ in, CompSet cin, cplx<T> *__restrict__ out,
                    CompSet cout, KGeom kg, const typename TabT<T>::type *__restrict__ ktab,
                    const cplx<T> *__restrict__ tw, int TL) {
  using C = cplx<T>;
  constexpr int E = fused_e(N), M = N / 2;
  using S = Shape<N, E>;
  constexpr int R0 = S::first(false), RL = S::last(false);
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  const int tiles = M / TL;
  // neighbouring x tiles share the cache lines of their row segments (TL
  // complex numbers, 32 or 64 bytes at long lines): they run on one XCD, so
  // its L2 fetches each line once (at 512^3 in FP32 the HBM reads were five
  // times the data with tiles spread over the XCDs)
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int xt = lb % tiles, iy = lb / tiles;
  const int line = threadIdx.x % TL, t = threadIdx.x / TL;
  const int ix = xt * TL + line;
  const int ky = kidx(iy, N);
  const size_t hsz = (size_t)M * N * N, plane = (size_t)N * M;
  const size_t base = (size_t)iy * M + ix;
  const T tp = (T)kg.twopi_L;
  C rho[E][3];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int m = 0; m < 3; ++m) rho[e][m] = C{(T)0, (T)0};
  // radial factors of this thread's modes: j0 (x), f1 (y) and the
  // projection's scale (z).  With four modes per thread they are read from
  // the table once for all components; with six the registers they would
  // hold cost more than the repeated (cached) table reads.
  constexpr bool HOIST = E <= 4;
  const auto entry = [&](int e) {
    const int iz = reg_pos<N, E, RL>(t, e / RL, e % RL);
    const int kz = kidx(iz, N);
    return ktab[ix * ix + ky * ky + kz * kz];
  };
  T tj0[HOIST ? E : 1], tf1[HOIST ? E : 1], tsc[HOIST ? E : 1];
  if constexpr (HOIST) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const auto tb = entry(e);
      tj0[e] = (T)tb.x;
      tf1[e] = (T)tb.y;
      tsc[e] = (T)tb.z;
    }
  }
  // Without hoisting, FP32 kernels up to 384 points (BATCH) load the factors
  // where nothing else is in flight that their use would wait for (the
  // vector-memory counter is in order): in each input step before the next
  // component's prefetch, and for the fold and the output steps once, before
  // the first store; the others (registers) read them at each use.
  constexpr bool BATCH = !HOIST && sizeof(T) == 4 && N <= 384;
  // the next component's z-line is loaded while the current one is
  // transformed (the barriers of the exchanges wait on LDS traffic only)
  const C tw0 = tw_fetch<C, N>(tw);
  C v[E], vn[E];
#pragma unroll
  for (int b = 0; b < E / R0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) vn[b * R0 + r] = in[base + reg_pos<N, E, R0>(t, b, r) * plane];
  C *twl = lds + (size_t)TL * N;
  tw_store<C, N>(twl, tw0, tw);
  for (int p = 0; p < cin.n; ++p) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vn[e];
    T pj0[BATCH ? E : 1], pf1[BATCH ? E : 1];
    if constexpr (BATCH) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const auto tb = entry(e);
        pj0[e] = (T)tb.x;
        pf1[e] = (T)tb.y;
      }
    }
    const auto j0_at = [&](int e) -> T {
      if constexpr (HOIST) return tj0[e];
      else if constexpr (BATCH) return pj0[e];
      else return (T)entry(e).x;
    };
    const auto f1_at = [&](int e) -> T {
      if constexpr (HOIST) return tf1[e];
      else if constexpr (BATCH) return pf1[e];
      else return (T)entry(e).y;
    };
    if (p + 1 < cin.n) {
      const C *src = in + (size_t)(p + 1) * hsz + base;
#pragma unroll
      for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) vn[b * R0 + r] = src[reg_pos<N, E, R0>(t, b, r) * plane];
    }
    reg_fft_forward<T, N, E>(v, t, lds, TL, line, twl);
    const int c = cin.idx[p];
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int iz = reg_pos<N, E, RL>(t, b, r);
        if (zero_mode(ix, iy, iz, N)) continue;
        if constexpr (DG) {
          const T f = c < 3 ? j0_at(b * RL + r) : (T)-3 * f1_at(b * RL + r);
          const C vv = v[b * RL + r];
#pragma unroll
          for (int m = 0; m < 3; ++m)
            if (m == c % 3) {
              rho[b * RL + r][m].x += f * vv.x;
              rho[b * RL + r][m].y += f * vv.y;
            }
        } else {
          const T kv[3] = {tp * ix, tp * ky, tp * kidx(iz, N)};
          add_P<C, T>(c, v[b * RL + r], kv, j0_at(b * RL + r), f1_at(b * RL + r), rho[b * RL + r]);
        }
      }
  }
  T oj0[BATCH ? E : 1], of1[BATCH ? E : 1], osc[BATCH ? E : 1];
  if constexpr (BATCH) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const auto tb = entry(e);
      oj0[e] = (T)tb.x;
      of1[e] = (T)tb.y;
      osc[e] = (T)tb.z;
    }
  }
  const auto j0_at = [&](int e) -> T {
    if constexpr (HOIST) return tj0[e];
    else if constexpr (BATCH) return oj0[e];
    else return (T)entry(e).x;
  };
  const auto f1_at = [&](int e) -> T {
    if constexpr (HOIST) return tf1[e];
    else if constexpr (BATCH) return of1[e];
    else return (T)entry(e).y;
  };
  const auto sc_at = [&](int e) -> T {
    if constexpr (HOIST) return tsc[e];
    else if constexpr (BATCH) return osc[e];
    else return (T)entry(e).z;
  };
  // u = scale (I - k^k^) rho
#pragma unroll
  for (int b = 0; b < E / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int e = b * RL + r;
      const int iz = reg_pos<N, E, RL>(t, b, r);
      const int kz = kidx(iz, N);
      const int n2 = ix * ix + ky * ky + kz * kz;
      if (zero_mode(ix, iy, iz, N)) {
#pragma unroll
        for (int m = 0; m < 3; ++m) rho[e][m] = C{(T)0, (T)0};
        continue;
      }
      const T scale = sc_at(e);
      const T kv[3] = {(T)ix, (T)ky, (T)kz};
      const T inv = (T)1 / (T)n2;
      T krx = 0, kry = 0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        krx += kv[m] * rho[e][m].x;
        kry += kv[m] * rho[e][m].y;
      }
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        rho[e][m].x = scale * (rho[e][m].x - kv[m] * krx * inv);
        rho[e][m].y = scale * (rho[e][m].y - kv[m] * kry * inv);
      }
    }
  for (int q = 0; q < cout.n; ++q) {
    const int c = cout.idx[q];
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int e = b * RL + r;
        const int iz = reg_pos<N, E, RL>(t, b, r);
        if (zero_mode(ix, iy, iz, N)) {
          v[e] = C{(T)0, (T)0};
          continue;
        }
        if constexpr (DG) {
          const T f = c < 3 ? j0_at(e) : (T)3 * f1_at(e);
          v[e] = C{(T)0, (T)0};
#pragma unroll
          for (int m = 0; m < 3; ++m)
            if (m == c % 3) v[e] = C{f * rho[e][m].x, f * rho[e][m].y};
        } else {
          const T kv[3] = {tp * ix, tp * ky, tp * kidx(iz, N)};
          v[e] = apply_Pdag<C, T>(c, rho[e], kv, j0_at(e), f1_at(e));
        }
      }
    reg_fft_inverse<T, N, E>(v, t, lds, TL, line, twl);
    C *dst = out + (size_t)q * hsz + base;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) dst[reg_pos<N, E, R0>(t, b, r) * plane] = v[b * R0 + r];
  }
}

// Derivative gridding on long lines with all three grids in registers: a
// workgroup owns TL neighbouring kx columns at one ky (row segments of up to
// 128 bytes), and the TPL threads of a line hold E modes of each of the
// three couplet grids D^.  Every load is issued before the first transform; the
// three forward z transforms run one after the other through one LDS area;
// each mode is then folded with its three components at hand,
// out = -9 f1^2 scale (I - k^k^) D^; and the three inverse transforms
// follow.  No accumulator and no prefetch copy: 3 E complex numbers per
// thread, so E can be as large as the line passes' (fewer exchanges).
template <typename T, int N, int E>
__global__ void __launch_bounds__(512)
kspace_dg3_kernel(const cplx<T> *__restrict__ in, cplx<T> *__restrict__ out, KGeom kg,
                  const T *__restrict__ kdg, const cplx<T> *__restrict__ tw, int TL) {
  using C = cplx<T>;
  constexpr int M = N / 2;
  using S = Shape<N, E>;
  constexpr int R0 = S::first(false), RL = S::last(false);
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  const int tiles = M / TL;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int xt = lb % tiles, iy = lb / tiles;
  const int line = threadIdx.x % TL, t = threadIdx.x / TL;
  const int ix = xt * TL + line;
  const int ky = kidx(iy, N);
  const size_t hsz = (size_t)M * N * N, plane = (size_t)N * M;
  const size_t base = (size_t)iy * M + ix;
  const C tw0 = tw_fetch<C, N>(tw);
  C v[3][E];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        v[m][b * R0 + r] = in[m * hsz + base + reg_pos<N, E, R0>(t, b, r) * plane];
  C *twl = lds + (size_t)TL * N;
  tw_store<C, N>(twl, tw0, tw);
#pragma unroll
  for (int m = 0; m < 3; ++m) reg_fft_forward<T, N, E>(v[m], t, lds, TL, line, twl);
  // the factors of the thread's modes are loaded in groups of KG before
  // their first use (every mode's |k|^2 is inside the table, the zeroed
  // modes' included) instead of one round trip per mode
  constexpr int KG = sizeof(T) == 8 ? 2 : (E < 8 ? E : 8);
#pragma unroll
  for (int g0 = 0; g0 < E; g0 += KG) {
    T sk[KG];
#pragma unroll
    for (int i = 0; i < KG; ++i) {
      const int e = g0 + i;
      const int kz = kidx(reg_pos<N, E, RL>(t, e / RL, e % RL), N);
      sk[i] = kdg[ix * ix + ky * ky + kz * kz];
    }
#pragma unroll
    for (int i = 0; i < KG; ++i) {
      const int e = g0 + i;
      const int iz = reg_pos<N, E, RL>(t, e / RL, e % RL);
      if (zero_mode(ix, iy, iz, N)) {
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][e] = C{(T)0, (T)0};
        continue;
      }
      const int kz = kidx(iz, N);
      const int n2 = ix * ix + ky * ky + kz * kz;
      const T s = sk[i];
      const T kv[3] = {(T)ix, (T)ky, (T)kz};
      const T inv = (T)1 / (T)n2;
      T krx = 0, kry = 0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        krx += kv[m] * v[m][e].x;
        kry += kv[m] * v[m][e].y;
      }
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        v[m][e].x = s * (v[m][e].x - kv[m] * krx * inv);
        v[m][e].y = s * (v[m][e].y - kv[m] * kry * inv);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    reg_fft_inverse<T, N, E>(v[m], t, lds, TL, line, twl);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        out[m * hsz + base + reg_pos<N, E, R0>(t, b, r) * plane] = v[m][b * R0 + r];
  }
}

// ----------------------------------------------------- Philox4x32-10 RNG --
// Counter-based generator of Salmon, Moraes, Dror & Shaw (SC'11), written
// from its published definition.

struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox4x32_10(u4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Four standard normals from one Philox block (Box-Muller).
__device__ __forceinline__ void normals4(u4 r, double *z) {
  const double s = 2.3283064365386963e-10;  // 2^-32
  const double u1 = ((double)r.x + 0.5) * s, u2 = ((double)r.y + 0.5) * s;
  const double u3 = ((double)r.z + 0.5) * s, u4v = ((double)r.w + 0.5) * s;
  const double ra = sqrt(-2.0 * log(u1)), rb = sqrt(-2.0 * log(u3));
  double sa, ca, sb, cb;
  sincospi(2.0 * u2, &sa, &ca);
  sincospi(2.0 * u4v, &sb, &cb);
  z[0] = ra * ca; z[1] = ra * sa; z[2] = rb * cb; z[3] = rb * sb;
}

// The same in FP32 (the wave noise of mixed-precision handles, whose grids
// are FP32): u in (0, 1] from the same 32-bit words.
__device__ __forceinline__ void normals4f(u4 r, double *z) {
  const float s = 2.3283064365386963e-10f;  // 2^-32
  const float u1 = ((float)r.x + 0.5f) * s, u2 = ((float)r.y + 0.5f) * s;
  const float u3 = ((float)r.z + 0.5f) * s, u4v = ((float)r.w + 0.5f) * s;
  const float ra = sqrtf(-2.0f * logf(u1)), rb = sqrtf(-2.0f * logf(u3));
  float sa, ca, sb, cb;
  sincospif(2.0f * u2, &sa, &ca);
  sincospif(2.0f * u4v, &sb, &cb);
  z[0] = ra * ca; z[1] = ra * sa; z[2] = rb * cb; z[3] = rb * sb;
}

template <bool F32 = false>
__device__ __forceinline__ void philox_normals(uint64_t seed, uint64_t counter,
                                               uint32_t stream, uint32_t index,
                                               int nblk, double *z) {
  for (int b = 0; b < nblk; ++b) {
    u4 c{index, stream * 16u + (uint32_t)b, (uint32_t)counter, (uint32_t)(counter >> 32)};
    const u4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    if constexpr (F32) normals4f(r, z + 4 * b);
    else normals4(r, z + 4 * b);
  }
}

enum : uint32_t { STREAM_REAL = 1, STREAM_WAVE = 2 };

// u(k) of the wave noise at stored mode (ix, iy, iz) (not a zeroed mode) and
// its radial factors tb and wave vector kv (see kspace_noise_kernel).
template <bool F32>
__device__ __forceinline__ void noise_mode(const double2 *__restrict__ psi, uint64_t seed,
                                           uint64_t counter, const KGeom &kg,
                                           const double4 *__restrict__ ktab, int ix, int iy,
                                           int iz, double2 uu[3], double4 &tb, double kv[3]) {
  const int n = kg.ng, hx = n / 2, hp = n / 2 + 1;
  // canonical member: kx > 0; or kx = 0 and ky in (0, n/2); or kx = ky = 0, kz in (0, n/2)
  const bool canon = ix > 0 || (iy > 0 && iy < hx) || (iy == 0 && iz < hx);
  const int cy = canon ? iy : (n - iy) % n, cz = canon ? iz : (n - iz) % n;
  const size_t cidx = ((size_t)cz * n + cy) * hp + ix;   // index in the noise layout
  double2 ps[3];
  if (psi) {
    const size_t psz = (size_t)n * n * hp;
    for (int m = 0; m < 3; ++m) ps[m] = psi[m * psz + cidx];
  } else {
    double z[8];
    philox_normals<F32>(seed, counter, STREAM_WAVE, (uint32_t)cidx, 2, z);
    const double s = 0.70710678118654752440;
    for (int m = 0; m < 3; ++m) ps[m] = double2{s * z[2 * m], s * z[2 * m + 1]};
  }
  if (!canon)
    for (int m = 0; m < 3; ++m) ps[m].y = -ps[m].y;
  const int ky = kidx(iy, n), kz = kidx(iz, n);
  double iv[3], inv;
  if (kg.def) {
    // deformed lattice: the projection and the radial factors of the true k
    deformed_k(kg, ix, ky, kz, kv);
    const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
    tb = radial_factors(kg, k2);
    for (int m = 0; m < 3; ++m) iv[m] = kv[m];
    inv = 1.0 / k2;
  } else {
    const int n2 = ix * ix + ky * ky + kz * kz;
    tb = ktab[n2];
    kv[0] = kg.twopi_L * ix;
    kv[1] = kg.twopi_L * ky;
    kv[2] = kg.twopi_L * kz;
    iv[0] = (double)ix;
    iv[1] = (double)ky;
    iv[2] = (double)kz;
    inv = 1.0 / (double)n2;
  }
  double2 kr{0, 0};
  for (int m = 0; m < 3; ++m) {
    kr.x += iv[m] * ps[m].x;
    kr.y += iv[m] * ps[m].y;
  }
  for (int m = 0; m < 3; ++m) {
    uu[m].x = tb.w * (ps[m].x - iv[m] * kr.x * inv);
    uu[m].y = tb.w * (ps[m].y - iv[m] * kr.y * inv);
  }
}

// Wave-space square root (Eq. FFTsqrt): for each stored mode k,
//   u(k) = h^3 / sqrt(V eta) sqrt(1 + k^2/4xi^2) exp(-(1 - eta_s) k^2/8xi^2) / k
//          (I - kk) psi(k),   W_c(k) = P_c^+(k) u(k),
// with psi read (or drawn) at the canonical member of {k, -k}; the stored
// modes with kx = 0 outside the canonical half take conj psi(-k), so that the
// spectrum is Hermitian.
template <typename T>
__global__ void __launch_bounds__(256)
kspace_noise_kernel(const double2 *__restrict__ psi, uint64_t seed, uint64_t counter,
                    cplx<T> *__restrict__ out, CompSet cout, int dg, KGeom kg,
                    const double4 *__restrict__ ktab, const uint64_t *counter_dev) {
  using C = cplx<T>;
  const int n = kg.ng, hx = n / 2, hp = n / 2 + 1;
  const size_t hsz = (size_t)hx * n * n;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= hsz) return;
  if (counter_dev) counter = *counter_dev;
  const int ix = (int)(tid % hx);
  const int iy = (int)((tid / hx) % n);
  const int iz = (int)(tid / ((size_t)hx * n));
  if (zero_mode(ix, iy, iz, n)) {
    for (int q = 0; q < cout.n; ++q) out[q * hsz + tid] = C{(T)0, (T)0};
    return;
  }
  double2 uu[3];
  double4 tb;
  double kv[3];
  noise_mode<sizeof(T) == 4>(psi, seed, counter, kg, ktab, ix, iy, iz, uu, tb, kv);
  for (int q = 0; q < cout.n; ++q) {
    const int c = cout.idx[q];
    double2 w;
    if (dg) {
      // grid codes of derivative gridding: j0(ka) u^ (0-2), 3 f1(ka) u^ (3-5)
      const double f = c < 3 ? tb.x : 3.0 * tb.y;
      w = double2{f * uu[c % 3].x, f * uu[c % 3].y};
    } else {
      w = apply_Pdag<double2, double>(c, uu, kv, tb.x, tb.y);
    }
    out[q * hsz + tid] = C{(T)w.x, (T)w.y};
  }
}


// The wave noise of derivative gridding with the inverse z transform fused
// (cubic lattice, long lines): a workgroup owns TL neighbouring kx columns
// at one ky as the k-space kernels do; each thread forms u(k) of its E modes
// (noise_mode), keeps them with the factors j0(ka) and 3 f1(ka), and for
// every output grid code (0-2: j0 u^, 3-5: 3 f1 u^) transforms the line back
// along z and stores it -- the grids the y and x passes take next, without
// the round trip through HBM of a separate noise kernel and z pass.
template <typename T, int N, int E>
__global__ void __launch_bounds__(512)
kspace_noise_z_kernel(const double2 *__restrict__ psi, uint64_t seed, uint64_t counter,
                      cplx<T> *__restrict__ out, CompSet cout, KGeom kg,
                      const double4 *__restrict__ ktab, const cplx<T> *__restrict__ tw, int TL,
                      const uint64_t *counter_dev) {
  using C = cplx<T>;
  constexpr int M = N / 2;
  using S = Shape<N, E>;
  constexpr int R0 = S::first(false), RL = S::last(false);
  extern __shared__ unsigned char smem_raw[];
  C *lds = reinterpret_cast<C *>(smem_raw);
  if (counter_dev) counter = *counter_dev;
  const int tiles = M / TL;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int xt = lb % tiles, iy = lb / tiles;
  const int line = threadIdx.x % TL, t = threadIdx.x / TL;
  const int ix = xt * TL + line;
  const size_t hsz = (size_t)M * N * N, plane = (size_t)N * M;
  const size_t base = (size_t)iy * M + ix;
  C *twl = lds + (size_t)TL * N;
  tw_store<C, N>(twl, tw_fetch<C, N>(tw), tw);
  C u[3][E];
  T fj[E], ff[E];
#pragma unroll
  for (int b = 0; b < E / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int e = b * RL + r;
      const int iz = reg_pos<N, E, RL>(t, b, r);
      if (zero_mode(ix, iy, iz, N)) {
#pragma unroll
        for (int m = 0; m < 3; ++m) u[m][e] = C{(T)0, (T)0};
        fj[e] = ff[e] = (T)0;
        continue;
      }
      double2 uu[3];
      double4 tb;
      double kv[3];
      noise_mode<sizeof(T) == 4>(psi, seed, counter, kg, ktab, ix, iy, iz, uu, tb, kv);
#pragma unroll
      for (int m = 0; m < 3; ++m) u[m][e] = C{(T)uu[m].x, (T)uu[m].y};
      fj[e] = (T)tb.x;
      ff[e] = (T)(3.0 * tb.y);
    }
  for (int q = 0; q < cout.n; ++q) {
    const int c = cout.idx[q];
    C v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T f = c < 3 ? fj[e] : ff[e];
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m == c % 3) v[e] = C{f * u[m][e].x, f * u[m][e].y};
    }
    reg_fft_inverse<T, N, E>(v, t, lds, TL, line, twl);
    C *dst = out + (size_t)q * hsz + base;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) dst[reg_pos<N, E, R0>(t, b, r) * plane] = v[b * R0 + r];
  }
}

// k-space kernel of a deformed lattice on full 3D half spectra (x, y and z
// transformed): per stored mode, rho = sum_c P_c(k) G_c, u = scale
// (I - k^k^) rho, W_q = P_q^+ u, with k = (2 pi / L) A^-T n and the radial
// factors of that k (no |k|^2 table: k^2 is no longer an integer multiple
// of (2 pi / L)^2).  One thread per mode; in and out may be the same.
template <typename T>
__global__ void __launch_bounds__(256)
kspace_deformed_kernel(const cplx<T> *__restrict__ in, CompSet cin, cplx<T> *__restrict__ out,
                       CompSet cout, KGeom kg) {
  using C = cplx<T>;
  const int n = kg.ng, hx = n / 2;
  const size_t hsz = (size_t)hx * n * n;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= hsz) return;
  const int ix = (int)(tid % hx);
  const int iy = (int)((tid / hx) % n);
  const int iz = (int)(tid / ((size_t)hx * n));
  if (zero_mode(ix, iy, iz, n)) {
    for (int q = 0; q < cout.n; ++q) out[q * hsz + tid] = C{(T)0, (T)0};
    return;
  }
  double kv[3];
  deformed_k(kg, ix, kidx(iy, n), kidx(iz, n), kv);
  const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
  const double4 tb = radial_factors(kg, k2);
  double2 rho[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int p = 0; p < cin.n; ++p) {
    const C g = in[p * hsz + tid];
    add_P<double2, double>(cin.idx[p], double2{(double)g.x, (double)g.y}, kv, tb.x, tb.y, rho);
  }
  double2 kr{0, 0};
  for (int m = 0; m < 3; ++m) {
    kr.x += kv[m] * rho[m].x;
    kr.y += kv[m] * rho[m].y;
  }
  for (int m = 0; m < 3; ++m) {
    rho[m].x = tb.z * (rho[m].x - kv[m] * kr.x / k2);
    rho[m].y = tb.z * (rho[m].y - kv[m] * kr.y / k2);
  }
  for (int q = 0; q < cout.n; ++q) {
    const double2 w = apply_Pdag<double2, double>(cout.idx[q], rho, kv, tb.x, tb.y);
    out[q * hsz + tid] = C{(T)w.x, (T)w.y};
  }
}

// Real-space noise psi1 ~ N(0, I), 11 per particle, from Philox.
__global__ void real_noise_kernel(uint64_t seed, uint64_t counter, int64_t n, int ncomp,
                                  double *__restrict__ out, const uint64_t *counter_dev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (counter_dev) counter = *counter_dev;
  double z[12];
  philox_normals(seed, counter, STREAM_REAL, (uint32_t)i, 3, z);
  for (int c = 0; c < ncomp; ++c) out[i * ncomp + c] = z[c];
}

// --------------------------------------------------------- small kernels --

template <typename T>
__global__ void zero_kernel(T *g, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = (T)0;
}

template <typename T>
__global__ void from_double_kernel(const double *src, size_t n, T *dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

template <typename T>
__global__ void to_double_kernel(const T *src, size_t n, double *dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// ----------------------------------------------------------- host side --

static GridGeom geom(const Handle &h) {
  GridGeom g;
  g.ng = h.d.grid;
  g.P = h.d.support;
  g.L = h.p.box;
  g.h = h.d.h;
  const double xi2 = h.d.xi * h.d.xi;
  g.kcoef = 2.0 * xi2 / h.d.eta_s;
  g.knorm = sqrt(2.0 * xi2 / (M_PI * h.d.eta_s));
  g.def = h.def.on;
  for (int i = 0; i < 6; ++i) g.G[i] = h.def.G[i];
  return g;
}

static KGeom kgeom(const Handle &h) {
  KGeom k;
  k.ng = h.d.grid;
  k.twopi_L = 2.0 * M_PI / h.p.box;
  k.a = h.p.radius;
  k.inv4xi2 = 1.0 / (4.0 * h.d.xi * h.d.xi);
  k.one_m_etas = 1.0 - h.d.eta_s;
  const double V = h.p.box * h.p.box * h.p.box;
  const double h3 = h.d.h * h.d.h * h.d.h;
  k.pref_n = h3 / sqrt(V * h.p.viscosity);
  k.pref_m = h3 * h3 / (V * h.p.viscosity);
  k.def = h.def.on;
  for (int i = 0; i < 9; ++i) k.Ai[i] = h.def.Ai[i];
  return k;
}

int ktable_len(int grid) { return 3 * (grid / 2) * (grid / 2) + 1; }

__global__ void __launch_bounds__(256)
ktable_to_float_kernel(const double4 *__restrict__ src, int len, float4 *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = float4{(float)src[i].x, (float)src[i].y, (float)src[i].z, (float)src[i].w};
}

// The constraint operator's k-space factor of derivative gridding,
// -9 f1(ka)^2 times the mobility factor, one number per |k|^2 (the fold of
// kspace_dg3_kernel reads only this; a quarter of the four-factor entry).
__global__ void __launch_bounds__(256)
kdg_table_kernel(const double4 *__restrict__ tab, int len, double *__restrict__ d,
                 float *__restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double4 t = tab[i];
  const double v = -9.0 * t.y * t.y * t.z;
  d[i] = v;
  if (f) f[i] = (float)v;
}

void build_ktable(Handle &h) {
  const int len = ktable_len(h.d.grid);
  hipLaunchKernelGGL(ktable_kernel, dim3(nblocks(len, 256)), dim3(256), 0, h.stream, kgeom(h),
                     len, (double4 *)h.ktab);
  PSE_LAUNCH_CHECK();
  if (h.ktab32) {
    hipLaunchKernelGGL(ktable_to_float_kernel, dim3(nblocks(len, 256)), dim3(256), 0, h.stream,
                       (const double4 *)h.ktab, len, (float4 *)h.ktab32);
    PSE_LAUNCH_CHECK();
  }
  if (h.kdg) {
    hipLaunchKernelGGL(kdg_table_kernel, dim3(nblocks(len, 256)), dim3(256), 0, h.stream,
                       (const double4 *)h.ktab, len, h.kdg, h.kdg32);
    PSE_LAUNCH_CHECK();
  }
}

namespace {

// The record arrays inside the handle's tile-record allocation: tl_cap
// particle indices, then (from a 256-byte boundary) tl_cap x 3 S weights.
TileRecs tile_recs(const Handle &h) {
  const size_t off = (h.tl_cap * sizeof(int) + 255) / 256 * 256;
  return TileRecs{(int *)h.tl_rec, (double *)((char *)h.tl_rec + off)};
}

}  // namespace

// Candidate lists of the spreading tiles for wrapped positions xw (after the
// spreading bins are current).
// The capacity N * (ceil((P-1)/S) + 1)^3 is the most tiles a stencil can
// meet, so the lists never overflow.
void build_tile_lists(Handle &h, const double *xw) {
  if (!h.stile) return;
  const GridGeom g = geom(h);
  const int nb = h.sbins.nc;
  const int ntile = nb * nb * nb;
  const unsigned blocks = (unsigned)((ntile + 3) / 4);
  hipLaunchKernelGGL((tile_list_kernel<false>), dim3(blocks), dim3(256), 0, h.stream, xw, g,
                     h.stile, nb, (const int *)h.sbins.start, (const int *)h.sbins.perm,
                     h.tl_cnt, nullptr, TileRecs{nullptr, nullptr});
  PSE_LAUNCH_CHECK();
  exclusive_scan(h, h.tl_cnt, h.tl_start, h.tl_scan, ntile);
  hipLaunchKernelGGL((tile_list_kernel<true>), dim3(blocks), dim3(256), 0, h.stream, xw, g,
                     h.stile, nb, (const int *)h.sbins.start, (const int *)h.sbins.perm, nullptr,
                     (const int *)h.tl_start, tile_recs(h));
  PSE_LAUNCH_CHECK();
  // grid over the capacity; the kernel reads the list's length on the device
  hipLaunchKernelGGL(tile_weights_kernel, dim3(nblocks(h.tl_cap, TW_RECS)), dim3(3 * TW_RECS),
                     (size_t)TW_RECS * (3 * h.stile + 3) * sizeof(double), h.stream, xw, g,
                     h.stile, nb, (const int *)h.tl_start + ntile, (int64_t)h.tl_cap,
                     tile_recs(h));
  PSE_LAUNCH_CHECK();
}

// Moment correction of the gradient weights of derivative gridding.  On the
// grid the gradient of the truncated Gaussian does not have the moments of
// the continuous one: along axis d its one-dimensional weights
// g_i = dK1/dx (x_i - x) sum to mu_d times the Gaussian's, sum_i g_i =
// mu_d sum_i w_i, with mu_d a small number that depends on the particle's
// offset from the grid, and their first moment sum_i d_i g_i (d_i = x_i - x)
// differs from -sum_i w_i, its continuous value.  A spread couplet then
// leaves a spurious monopole in the smallest wave numbers, where the Stokes
// kernel amplifies it, and the interpolated gradient of a smooth field picks
// up the field itself.  Spreading and interpolation take instead
// lambda_d (g_i - mu_d w_i), still separable, whose discrete sum is zero and
// whose first moment is -sum_i w_i: the gradient of a constant field is
// zero and that of a linear field exact, relative to the Gaussian's own
// normalisation.  mu and lambda (three each per particle) are formed once
// per position update.
__global__ void __launch_bounds__(256)
dg_mu_kernel(const double *__restrict__ x, int64_t n, GridGeom g, double *__restrict__ mu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const double xc = x[t];
  const int i0 = stencil_start(xc, g.h, g.P);
  double s0 = 0.0, s1 = 0.0, sd = 0.0, sd1 = 0.0;
  for (int i = 0; i < g.P; ++i) {
    const double d = (i0 + i) * g.h - xc;
    const double w = exp(-g.kcoef * d * d);
    const double gi = -2.0 * g.kcoef * d * w;
    s0 += w;
    s1 += gi;
    sd += d * w;
    sd1 += d * gi;
  }
  const double m = s1 / s0;
  // sum_i d_i (g_i - m w_i) = sd1 - m sd
  const int64_t p = t / 3, ax = t % 3;
  mu[6 * p + ax] = m;
  mu[6 * p + 3 + ax] = -s0 / (sd1 - m * sd);
}

void build_dg_mu(Handle &h, const double *xw) {
  if (!h.deriv) return;
  hipLaunchKernelGGL(dg_mu_kernel, dim3(nblocks(3 * (size_t)h.n, 256)), dim3(256), 0, h.stream,
                     xw, h.n, geom(h), h.dg_mu);
  PSE_LAUNCH_CHECK();
}

size_t tile_record_bytes(int S) { return sizeof(int) + (3 * (size_t)S + 3) * sizeof(double); }

namespace {

// Component-count buckets: kernels keep NCM accumulators per point.
template <typename F> void with_ncm(int n, F f) {
  if (n <= 3) f(std::integral_constant<int, 3>());
  else if (n <= 5) f(std::integral_constant<int, 5>());
  else if (n <= 6) f(std::integral_constant<int, 6>());
  else f(std::integral_constant<int, NC>());
}

}  // namespace

// Rotation and strain from derivative gridding: with v = the three velocity
// grids of the k-space factor 3 f1(ka) u^, and the sums
// G_ij = sum_n v_i(x_n) dK/dx_j (x_n - x_p) = -(d v_i / d x_j)(x_p) (the
// interpolation of grad v with the gradient moved onto the Gaussian), the
// strain is e_q = Y_q : grad v and the rotation curl v / 2 (the adjoints of
// the stresslet and torque columns).  With HU the three grids of j0(ka) u^
// come first and give the velocity by plain interpolation.  One wavefront
// per particle as interp_kernel; per stencil point the gradient weight is
// lambda (-2 kcoef d - mu) K(d), d = x_n - x_p, with the moment corrections
// mu, lambda of the particle (see dg_mu_kernel).  cs: the output components (velocity 0-2
// with HU, rotation 3-5, strain 6-10), any subset.
template <typename T, int MAXIT, bool HU>
__global__ void __launch_bounds__(256)
interp_deriv_kernel(const double *__restrict__ x, const T *__restrict__ grids, size_t ngrid,
                    CompSet cs, int rot, GridGeom g, const int *__restrict__ order, int64_t n,
                    const double *__restrict__ mu, double *__restrict__ out, Layout lo,
                    int accumulate, double scale) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  const int64_t p = order ? order[t] : t;
  const double px = x[3 * p], py = x[3 * p + 1], pz = x[3 * p + 2];
  const int P = g.P, P3 = P * P * P;
  const int ix0 = stencil_start(px, g.h, P);
  const int iy0 = stencil_start(py, g.h, P);
  const int iz0 = stencil_start(pz, g.h, P);
  const double kn3 = g.knorm * g.knorm * g.knorm;
  const double mx = mu[6 * p], my = mu[6 * p + 1], mz = mu[6 * p + 2];
  const double lx = mu[6 * p + 3], ly = mu[6 * p + 4], lz = mu[6 * p + 5];
  const T *vg = grids + (HU ? 3 * ngrid : 0);
  // G (row-major, 9) and the velocity (3)
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = (T)0;
  bool done = false;
  if constexpr (MAXIT == 8) {
    if (P == 8) {
      // the lane's points share x and y: with dK/dx_i = c d_i e (c = -2
      // kcoef knorm^3, e the Gaussian), the column sums s_k = sum v_k e and
      // z_k = sum v_k e dz give every G_ij
      uint32_t gi[8];
      T e[8], dz[8];
      double dx, dy;
      stencil8<T>(lane, px, py, pz, ix0, iy0, iz0, g, gi, e, dz, dx, dy);
      T v[3][8], u[HU ? 3 : 1][8];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int it = 0; it < 8; ++it) v[k][it] = vg[(size_t)k * ngrid + gi[it]];
      if constexpr (HU)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int it = 0; it < 8; ++it) u[k][it] = grids[(size_t)k * ngrid + gi[it]];
      // moment correction: lambda_i (dK/dx_i - mu_i K) = lambda_i c (d_i - mu_i / (-2 kcoef)) e
      T sk[3] = {(T)0, (T)0, (T)0}, zk[3] = {(T)0, (T)0, (T)0}, uk[3] = {(T)0, (T)0, (T)0};
      const double sh = 1.0 / (-2.0 * g.kcoef);
      dx -= mx * sh;
      dy -= my * sh;
      const T mzs = (T)(mz * sh);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const T et = e[it], dzt = dz[it] - mzs;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T ve = v[k][it] * et;
          sk[k] += ve;
          zk[k] += ve * dzt;
          if constexpr (HU) uk[k] += u[k][it] * et;
        }
      }
      const double c = -2.0 * g.kcoef * kn3;
      const T c0 = (T)(c * lz), cx = (T)(c * lx * dx), cy = (T)(c * ly * dy);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        acc[3 * k] = cx * sk[k];
        acc[3 * k + 1] = cy * sk[k];
        acc[3 * k + 2] = c0 * zk[k];
        if constexpr (HU) acc[9 + k] = (T)kn3 * uk[k];
      }
      done = true;
    }
  }
  if (!done) {
    uint32_t gi[MAXIT];
    T gw[MAXIT][3], w0[MAXIT];
    double f1[3];
    factors1d(lane, px, py, pz, ix0, iy0, iz0, g, f1);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int s = lane + 64 * it;
      const int a = s % P, b = (s / P) % P, c = s / (P * P);
      const double dx = (ix0 + a) * g.h - px;
      const double dy = (iy0 + b) * g.h - py;
      const double dz = (iz0 + c) * g.h - pz;
      const bool in = s < P3;
      const double e = gauss_at(f1, a, b, c);
      const double f = in ? kn3 * e : 0.0;
      gw[it][0] = (T)(f * lx * (-2.0 * g.kcoef * dx - mx));
      gw[it][1] = (T)(f * ly * (-2.0 * g.kcoef * dy - my));
      gw[it][2] = (T)(f * lz * (-2.0 * g.kcoef * dz - mz));
      w0[it] = (T)f;
      gi[it] = in ? ((uint32_t)wrapi(iz0 + c, g.ng) * g.ng + wrapi(iy0 + b, g.ng)) * g.ng
                        + wrapi(ix0 + a, g.ng)
                  : 0;
    }
    T v[3][MAXIT];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int it = 0; it < MAXIT; ++it) v[k][it] = vg[(size_t)k * ngrid + gi[it]];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[3 * k + j] += v[k][it] * gw[it][j];
    if constexpr (HU) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T u[MAXIT];
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) u[it] = grids[(size_t)k * ngrid + gi[it]];
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) acc[9 + k] += w0[it] * u[it];
      }
    }
  }
  // wavefront sums: the symmetric part always, the antisymmetric part for a
  // rotation, the velocity with HU
  T r[12];
  r[0] = acc[0];                 // Gxx
  r[1] = acc[4];                 // Gyy
  r[2] = acc[8];                 // Gzz
  r[3] = acc[1] + acc[3];        // Gxy + Gyx
  r[4] = acc[2] + acc[6];        // Gxz + Gzx
  r[5] = acc[5] + acc[7];        // Gyz + Gzy
  r[6] = acc[7] - acc[5];        // Gzy - Gyz
  r[7] = acc[2] - acc[6];        // Gxz - Gzx
  r[8] = acc[3] - acc[1];        // Gyx - Gxy
  r[9] = acc[9];
  r[10] = acc[10];
  r[11] = acc[11];
  const int nr = HU ? 12 : (rot ? 9 : 6);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    if (k < nr) {
      T w = r[k];
      for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
      r[k] = w;
    }
  }
  if (lane == 0) {
    const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637;
    for (int k = 0; k < cs.n; ++k) {
      const int c = cs.idx[k];
      double val;
      if (c < 3) val = (double)r[9 + c];
      else if (c < 6) val = -0.5 * (double)r[3 + c];   // rotation: -(G_ji - G_ij) / 2
      else if (c < 9) val = -r2 * (double)r[c - 3];
      else if (c == 9) val = -r2 * ((double)r[0] - (double)r[1]);
      else val = -r6 * ((double)r[0] + (double)r[1] - 2.0 * (double)r[2]);
      double *o = out + p * lo.stride + c - lo.off;
      val *= scale;
      *o = accumulate ? *o + val : val;
    }
  }
}

template <typename T>
void spread(Handle &h, const double *x, const double *q, Layout lq, const CompSet &cs,
            T *grids) {
  const GridGeom g = geom(h);
  if (h.stile) {
    if (!h.tiles_current)
      throw Error{PSE_ERR_INVALID, "spreading tile lists not built for these positions"};
    ProfScope ps(h, PK_SPREAD, (double)cs.n * h.ngrid * sizeof(T) + (double)h.n * (3 + cs.n) * 8);
    const int nb = h.sbins.nc;
    const unsigned tiles = (unsigned)nb * nb * nb;
    const TileRecs rec = tile_recs(h);
    const int *ts = (const int *)h.tl_start;
    with_ncm(cs.n, [&](auto ncm) {
      constexpr int M = decltype(ncm)::value;
      // z points per thread: a whole column of the tile while the
      // accumulators fit, half of it for the 11-component product
      constexpr int Z8 = M <= 6 ? 8 : 4;
      if (h.stile == 4)
        hipLaunchKernelGGL((spread_list_kernel<T, 4, M, 1>), dim3(tiles), dim3(64), 0,
                           h.stream, q, lq, cs, g, nb, ts, rec, grids, h.ngrid);
      else if (h.stile == 8)
        hipLaunchKernelGGL((spread_list_kernel<T, 8, M, Z8>), dim3(tiles), dim3(512 / Z8), 0,
                           h.stream, q, lq, cs, g, nb, ts, rec, grids, h.ngrid);
      else
        throw Error{PSE_ERR_INVALID, "unsupported spreading tile"};
    });
    PSE_LAUNCH_CHECK();
    return;
  }
  zero_grids<T>(h, grids, cs.n);
  ProfScope ps(h, PK_SPREAD, (double)cs.n * h.ngrid * sizeof(T) + (double)h.n * (3 + cs.n) * 8);
  hipLaunchKernelGGL(spread_kernel<T>, dim3(nblocks(h.n, 4)), dim3(256), 0,
                     h.stream, x, q, lq, cs, g, (const int *)h.cells.perm, h.n,
                     grids, h.ngrid);
  PSE_LAUNCH_CHECK();
}

template <typename T>
void interpolate(Handle &h, const double *x, const T *grids, const CompSet &cs, double *out,
                 Layout lo, bool accumulate, double scale) {
  const GridGeom g = geom(h);
  const int acc = accumulate ? 1 : 0;
  ProfScope ps(h, PK_INTERP, (double)cs.n * h.ngrid * sizeof(T) + (double)h.n * (3 + cs.n) * 8);
  const int P3 = g.P * g.P * g.P;
  const dim3 grid(nblocks(h.n, 4)), block(256);
  const int *order = (const int *)h.cells.trav;
  if (g.def)   // the Gaussian does not factorise over the lattice axes
    hipLaunchKernelGGL((interp_kernel<T, 0>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  else if (P3 <= 128)
    hipLaunchKernelGGL((interp_kernel<T, 2>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  else if (P3 <= 256)
    hipLaunchKernelGGL((interp_kernel<T, 4>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  else if (P3 <= 384)
    hipLaunchKernelGGL((interp_kernel<T, 6>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  else if (P3 <= 512)
    hipLaunchKernelGGL((interp_kernel<T, 8>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  else if (P3 <= 1024)
    hipLaunchKernelGGL((interp_kernel<T, 16>), grid, block, 0, h.stream, x, grids, h.ngrid, cs,
                       g, order, h.n, out, lo, acc, scale);
  else
    hipLaunchKernelGGL((interp_kernel<T, 0>), grid, block, 0, h.stream, x, grids, h.ngrid, cs, g,
                       order, h.n, out, lo, acc, scale);
  PSE_LAUNCH_CHECK();
}

// Derivative gridding of the constraint operator (tile lists required): the
// stresslet components cs (five, in the Y_q basis) of q in layout lq spread
// onto three grids with the Gaussian's gradient.
template <typename T>
void spread_deriv(Handle &h, const double *q, Layout lq, const CompSet &cs, bool hf, bool hasL,
                  bool hasS, T *grids) {
  if (!h.stile) throw Error{PSE_ERR_INVALID, "derivative gridding unavailable"};
  if (!h.tiles_current)
    throw Error{PSE_ERR_INVALID, "spreading tile lists not built for these positions"};
  const GridGeom g = geom(h);
  const int ng = hf ? 6 : 3;
  ProfScope ps(h, PK_SPREAD, (double)ng * h.ngrid * sizeof(T) + (double)h.n * (3 + cs.n) * 8);
  const int nb = h.sbins.nc;
  const unsigned tiles = (unsigned)nb * nb * nb;
  const TileRecs rec = tile_recs(h);
  const int *ts = (const int *)h.tl_start;
  const int L = hasL ? 1 : 0, S3 = hasS ? 1 : 0;
  if (h.stile == 4) {
    if (hf)
      hipLaunchKernelGGL((spread_deriv_kernel<T, 4, 1, true>), dim3(tiles), dim3(64), 0,
                         h.stream, q, lq, cs, L, S3, g, nb, ts, rec, h.dg_mu, grids, h.ngrid);
    else
      hipLaunchKernelGGL((spread_deriv_kernel<T, 4, 1, false>), dim3(tiles), dim3(64), 0,
                         h.stream, q, lq, cs, L, S3, g, nb, ts, rec, h.dg_mu, grids, h.ngrid);
  } else if (h.stile == 8) {
    if (hf)
      hipLaunchKernelGGL((spread_deriv_kernel<T, 8, 4, true>), dim3(tiles), dim3(128), 0,
                         h.stream, q, lq, cs, L, S3, g, nb, ts, rec, h.dg_mu, grids, h.ngrid);
    else
      hipLaunchKernelGGL((spread_deriv_kernel<T, 8, 4, false>), dim3(tiles), dim3(128), 0,
                         h.stream, q, lq, cs, L, S3, g, nb, ts, rec, h.dg_mu, grids, h.ngrid);
  } else {
    throw Error{PSE_ERR_INVALID, "unsupported spreading tile"};
  }
  PSE_LAUNCH_CHECK();
}

// Velocity (with hu), rotation and strain components cs of out in layout lo
// from the grids of derivative gridding (see interp_deriv_kernel).
template <typename T>
void interp_deriv(Handle &h, const double *x, const T *grids, bool hu, const CompSet &cs,
                  double *out, Layout lo, bool accumulate, double scale) {
  const GridGeom g = geom(h);
  const int acc = accumulate ? 1 : 0;
  int rot = 0;
  for (int k = 0; k < cs.n; ++k) rot |= cs.idx[k] >= 3 && cs.idx[k] < 6;
  ProfScope ps(h, PK_INTERP, (hu ? 6.0 : 3.0) * h.ngrid * sizeof(T) + (double)h.n * (3 + cs.n) * 8);
  const int P3 = g.P * g.P * g.P;
  const dim3 grid(nblocks(h.n, 4)), block(256);
  const int *order = (const int *)h.cells.trav;
  const auto launch = [&](auto maxit) {
    constexpr int MI = decltype(maxit)::value;
    if (hu)
      hipLaunchKernelGGL((interp_deriv_kernel<T, MI, true>), grid, block, 0, h.stream, x, grids,
                         h.ngrid, cs, rot, g, order, h.n, h.dg_mu, out, lo, acc, scale);
    else
      hipLaunchKernelGGL((interp_deriv_kernel<T, MI, false>), grid, block, 0, h.stream, x, grids,
                         h.ngrid, cs, rot, g, order, h.n, h.dg_mu, out, lo, acc, scale);
  };
  if (P3 <= 256) launch(std::integral_constant<int, 4>());
  else if (P3 <= 384) launch(std::integral_constant<int, 6>());
  else if (P3 <= 512) launch(std::integral_constant<int, 8>());
  else if (P3 <= 1024) launch(std::integral_constant<int, 16>());
  else throw Error{PSE_ERR_INVALID, "derivative gridding supports P <= 10"};
  PSE_LAUNCH_CHECK();
}

namespace {

template <typename T, int N>
void launch_fused(Handle &h, const cplx<T> *in, const CompSet &cin, cplx<T> *out,
                  const CompSet &cout, const cplx<T> *tw, bool dg) {
  using Tab = typename TabT<T>::type;
  const Tab *tab = sizeof(T) == 8 ? (const Tab *)h.ktab : (const Tab *)h.ktab32;
  // the constraint operator's derivative gridding at 512 (couplet grids
  // each way): all three grids in registers, 128-byte row
  // segments (measured 1.63 -> 1.32 ms per FP32 launch at 512^3, and 3.10 ->
  // 2.65 ms in FP64, against the accumulating form below; at 256 the FP32
  // form spills)
  const auto couplet3 = [](const CompSet &c) {
    return c.n == 3 && c.idx[0] == 3 && c.idx[1] == 4 && c.idx[2] == 5;
  };
  if constexpr (N == 512) {
    if (dg && couplet3(cin) && couplet3(cout)) {
      // the line passes' element count in FP32, half of it in FP64
      constexpr int E = sizeof(T) == 4 ? line_e(N) : line_e(N) / 2;
      constexpr int TPL = N / E;
      int tl = (int)(128 / sizeof(cplx<T>));
      // exchange area of tl lines and the twiddle table
      const auto lds_of = [](int l) { return (size_t)(l + 1) * N * sizeof(cplx<T>); };
      while (tl > 1 && (tl * TPL > 512 || lds_of(tl) > (size_t)h.max_lds)) tl /= 2;
      const size_t lds = lds_of(tl);
      const unsigned nb = (unsigned)(N * (N / 2 / tl));
      const T *kdg = sizeof(T) == 8 ? (const T *)h.kdg : (const T *)h.kdg32;
      if (!kdg) throw Error{PSE_ERR_INVALID, "k-space factor of derivative gridding missing"};
      hipLaunchKernelGGL((kspace_dg3_kernel<T, N, E>), dim3(nb), dim3(tl * TPL), lds, h.stream,
                         in, out, kgeom(h), kdg, tw, tl);
      PSE_LAUNCH_CHECK();
      return;
    }
  }
  constexpr int TPL = N / fused_e(N);
  // at least four z-lines (64-byte row segments) per workgroup on long lines
  const int tl = lines_per_block(N, TPL, N * sizeof(cplx<T>), (size_t)N / 2,
                                 TPL >= 128 ? 512 : 256);
  // exchange area and the twiddle table
  const size_t lds = (size_t)(tl + 1) * N * sizeof(cplx<T>);
  if (lds > (size_t)h.max_lds)
    throw Error{PSE_ERR_HIP, "k-space kernel: LDS beyond the device's per-workgroup limit"};
  const unsigned nb = (unsigned)(N * (N / 2 / tl));
  if (dg)
    hipLaunchKernelGGL((kspace_fused_kernel<T, N, true>), dim3(nb), dim3(tl * TPL), lds,
                       h.stream, in, cin, out, cout, kgeom(h), tab, tw, tl);
  else
    hipLaunchKernelGGL((kspace_fused_kernel<T, N, false>), dim3(nb), dim3(tl * TPL), lds,
                       h.stream, in, cin, out, cout, kgeom(h), tab, tw, tl);
  PSE_LAUNCH_CHECK();
}

}  // namespace

#define PSE_CASE_F(NN) case NN: launch_fused<T, NN>(h, in, cin, out, cout, tw, dg); break;

template <typename T>
void kspace_fused(Handle &h, const cplx<T> *in, const CompSet &cin, cplx<T> *out,
                  const CompSet &cout, const cplx<T> *tw, bool dg) {
  const size_t hsz = h.ngrid / 2;
  ProfScope ps(h, PK_KSPACE, (double)(cin.n + cout.n) * hsz * sizeof(cplx<T>));
  switch (h.d.grid) {
    PSE_FOR_EACH_N(PSE_CASE_F)
    default: throw Error{PSE_ERR_INVALID, "unsupported FFT length"};
  }
}

template <typename T>
void kspace_deformed(Handle &h, const cplx<T> *in, const CompSet &cin, cplx<T> *out,
                     const CompSet &cout) {
  const size_t hsz = h.ngrid / 2;
  ProfScope ps(h, PK_KSPACE, (double)(cin.n + cout.n) * hsz * sizeof(cplx<T>));
  hipLaunchKernelGGL(kspace_deformed_kernel<T>, dim3(nblocks(hsz, 256)), dim3(256), 0,
                     h.stream, in, cin, out, cout, kgeom(h));
  PSE_LAUNCH_CHECK();
}

template <typename T>
bool kspace_noise_z(Handle &h, const double *psi, uint64_t seed, uint64_t counter,
                    cplx<T> *out, const CompSet &cout, const cplx<T> *tw) {
  // long power-of-two lines of a cubic lattice (measured at 512)
  if (h.def.on || h.d.grid != 512) return false;
  constexpr int N = 512, E = 8, TPL = N / E;
  const int tl = 512 / TPL;
  const size_t hsz = h.ngrid / 2;
  ProfScope ps(h, PK_NOISE, (double)cout.n * hsz * sizeof(cplx<T>) + (psi ? 3.0 * hsz * 16 : 0.0));
  // exchange area and the twiddle table
  const size_t lds = (size_t)(tl + 1) * N * sizeof(cplx<T>);
  if (lds > (size_t)h.max_lds) return false;
  const unsigned nb = (unsigned)(N * (N / 2 / tl));
  hipLaunchKernelGGL((kspace_noise_z_kernel<T, N, E>), dim3(nb), dim3(tl * TPL), lds,
                     h.stream, (const double2 *)psi, seed, counter, out, cout, kgeom(h),
                     (const double4 *)h.ktab, tw, tl, h.counter_dev);
  PSE_LAUNCH_CHECK();
  return true;
}

template <typename T>
void kspace_noise(Handle &h, const double *psi, uint64_t seed, uint64_t counter,
                  cplx<T> *out, const CompSet &cout, bool dg) {
  const size_t hsz = h.ngrid / 2;
  ProfScope ps(h, PK_NOISE, (double)cout.n * hsz * sizeof(cplx<T>) + (psi ? 3.0 * hsz * 16 : 0.0));
  hipLaunchKernelGGL(kspace_noise_kernel<T>, dim3(nblocks(hsz, 256)), dim3(256),
                     0, h.stream, (const double2 *)psi, seed, counter, out, cout, dg ? 1 : 0,
                     kgeom(h), (const double4 *)h.ktab, h.counter_dev);
  PSE_LAUNCH_CHECK();
}

void real_noise(Handle &h, uint64_t seed, uint64_t counter, double *out, int ncomp) {
  hipLaunchKernelGGL(real_noise_kernel, dim3(nblocks(h.n, 256)), dim3(256), 0,
                     h.stream, seed, counter, h.n, ncomp, out, h.counter_dev);
  PSE_LAUNCH_CHECK();
}

template <typename T> void zero_grids(Handle &h, T *g, int ncomp) {
  const size_t n = (size_t)ncomp * h.ngrid;
  ProfScope ps(h, PK_ZERO, (double)n * sizeof(T));
  hipLaunchKernelGGL(zero_kernel<T>, dim3(nblocks(n, 256)), dim3(256), 0, h.stream, g, n);
  PSE_LAUNCH_CHECK();
}

template <typename T> void from_double(Handle &h, const double *src, size_t n, T *dst) {
  hipLaunchKernelGGL(from_double_kernel<T>, dim3(nblocks(n, 256)), dim3(256), 0, h.stream,
                     src, n, dst);
  PSE_LAUNCH_CHECK();
}

template <typename T> void to_double(Handle &h, const T *src, size_t n, double *dst) {
  hipLaunchKernelGGL(to_double_kernel<T>, dim3(nblocks(n, 256)), dim3(256), 0, h.stream,
                     src, n, dst);
  PSE_LAUNCH_CHECK();
}

#define INST(T)                                                                 \
  template void spread<T>(Handle &, const double *, const double *, Layout,      \
                          const CompSet &, T *);                                 \
  template void interpolate<T>(Handle &, const double *, const T *,              \
                               const CompSet &, double *, Layout, bool, double); \
  template void kspace_deformed<T>(Handle &, const cplx<T> *, const CompSet &,   \
                                   cplx<T> *, const CompSet &);                  \
  template void kspace_noise<T>(Handle &, const double *, uint64_t, uint64_t,    \
                                cplx<T> *, const CompSet &, bool);               \
  template bool kspace_noise_z<T>(Handle &, const double *, uint64_t, uint64_t,  \
                                  cplx<T> *, const CompSet &, const cplx<T> *);  \
  template void kspace_fused<T>(Handle &, const cplx<T> *, const CompSet &,      \
                                cplx<T> *, const CompSet &, const cplx<T> *,     \
                                bool);                                           \
  template void spread_deriv<T>(Handle &, const double *, Layout, const CompSet &, \
                                bool, bool, bool, T *);                          \
  template void interp_deriv<T>(Handle &, const double *, const T *, bool,       \
                                const CompSet &, double *, Layout, bool, double); \
  template void zero_grids<T>(Handle &, T *, int);                               \
  template void from_double<T>(Handle &, const double *, size_t, T *);           \
  template void to_double<T>(Handle &, const T *, size_t, double *);
INST(double)
INST(float)
#undef INST

}  // namespace pse
