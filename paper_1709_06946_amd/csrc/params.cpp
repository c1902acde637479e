// Parameter derivation and device footprint (host only, no GPU calls).
//
// Rules (Sec. II.C):
//  * Eq. bound with lambda_max = 1: setting the two error terms equal with
//    erfc(x) <= exp(-x^2) gives m = sqrt(pi P), each term exp(-pi P / 2), and
//    2 exp(-pi P/2) <= eps_q gives P = ceil((2/pi) ln(2/eps_q)).
//    The bound carries unknown O(1) constants.  Measured against the exact
//    Ewald sum, eps_q = eps leaves gridding errors of 2e-3 to 2e-2 on the
//    couplet blocks (Omega, E) at eps = 1e-3, dominated by aliasing near the
//    Nyquist wave number; the wave-space square root, whose error follows
//    the square root of the damping at the Nyquist shell, needs still more.
//    The library therefore uses eps_q = eps / 20,
//    truncates the Gaussian at 0.85 of the balanced number of standard
//    deviations (m = 0.85 sqrt(pi P): for the same P a wider Gaussian in grid
//    units, hence less aliasing), and a splitting parameter that damps the
//    Nyquist mode further.
//  * eta_s = (h P xi / m)^2 (Gaussian shape, must be < 1 so that the
//    remaining factor exp(-(1 - eta_s) k^2 / 4 xi^2) still decays).
//  * xi from the grid: the Hasimoto factor exp(-k^2/4xi^2) at the Nyquist
//    wave number pi Ng / L equals exp(-u_N) with u_N = ln(1/eps) + 9, i.e.
//    xi = pi Ng / (2 L sqrt(u_N)).
//  * Real-space cutoff: the real-space functions decay like
//    exp(-xi^2 (r - 2a)^2) beyond contact (Appendix A), so
//    rcut = 2a + sqrt(ln(1/eps)) / xi.
#include <cmath>
#include <cstdio>

#include "pse_internal.h"

namespace pse {

static bool grid_supported(int ng) {
  if (ng < 8 || ng > 1024 || (ng & 1)) return false;
  int m = ng;
  if (m % 3 == 0) m /= 3;
  return (m & (m - 1)) == 0;
}

static int next_supported(int n) {
  for (int g = std::max(n, 8); g <= 1024; ++g)
    if (grid_supported(g)) return g;
  return -1;
}

static void fail(const char *msg) { throw Error{PSE_ERR_INVALID, msg}; }

// All zero (unset) or the identity: the cube.
static bool lattice_deformed(const pse_params &p) {
  bool any = false, ident = true;
  for (int i = 0; i < 9; ++i) {
    if (p.deform[i] != 0.0) any = true;
    if (p.deform[i] != ((i % 4 == 0) ? 1.0 : 0.0)) ident = false;
  }
  return any && !ident;
}

// Largest eigenvalue of the symmetric 3x3 matrix S (cyclic Jacobi rotations).
static double sym3_lambda_max(double S[3][3]) {
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 3; ++q) off += S[p][q] * S[p][q];
    if (off < 1e-30) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (S[p][q] == 0.0) continue;
        const double th = 0.5 * (S[q][q] - S[p][p]) / S[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double a = S[k][p], b = S[k][q];
          S[k][p] = c * a - s * b;
          S[k][q] = s * a + c * b;
        }
        for (int k = 0; k < 3; ++k) {
          const double a = S[p][k], b = S[q][k];
          S[p][k] = c * a - s * b;
          S[q][k] = s * a + c * b;
        }
      }
  }
  return std::max(S[0][0], std::max(S[1][1], S[2][2]));
}

void deformation(const pse_params &p, Deform &df) {
  df = Deform{};
  df.on = lattice_deformed(p) ? 1 : 0;
  double A[9];
  for (int i = 0; i < 9; ++i) A[i] = df.on ? p.deform[i] : ((i % 4 == 0) ? 1.0 : 0.0);
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!(std::fabs(det - 1.0) < 1e-9)) fail("the lattice deformation must have det A = 1");
  // inverse (det = 1: the adjugate)
  double Ai[9] = {A[4] * A[8] - A[5] * A[7], A[2] * A[7] - A[1] * A[8], A[1] * A[5] - A[2] * A[4],
                  A[5] * A[6] - A[3] * A[8], A[0] * A[8] - A[2] * A[6], A[2] * A[3] - A[0] * A[5],
                  A[3] * A[7] - A[4] * A[6], A[1] * A[6] - A[0] * A[7], A[0] * A[4] - A[1] * A[3]};
  for (int i = 0; i < 9; ++i) {
    df.A[i] = A[i];
    df.Ai[i] = Ai[i] / det;
  }
  double S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += A[3 * k + i] * A[3 * k + j];
      S[i][j] = v;
    }
  df.G[0] = S[0][0];
  df.G[1] = S[1][1];
  df.G[2] = S[2][2];
  df.G[3] = S[0][1];
  df.G[4] = S[0][2];
  df.G[5] = S[1][2];
  df.lambda_max = df.on ? sym3_lambda_max(S) : 1.0;
  // thinnest width of the cell, in units of L: 1 / max_i |row i of A^-1|
  double rmax = 0.0;
  for (int i = 0; i < 3; ++i)
    rmax = std::max(rmax, std::sqrt(df.Ai[3 * i] * df.Ai[3 * i] +
                                    df.Ai[3 * i + 1] * df.Ai[3 * i + 1] +
                                    df.Ai[3 * i + 2] * df.Ai[3 * i + 2]));
  df.width = 1.0 / rmax;
}

void derive(const pse_params &p, pse_derived &d) {
  if (p.n <= 0) fail("n must be positive");
  if (!(p.radius > 0)) fail("radius must be positive");
  if (!(p.viscosity > 0)) fail("viscosity must be positive");
  if (!(p.kT > 0)) fail("kT must be positive");
  if (!(p.box > 4 * p.radius)) fail("box must exceed 4 radii");
  if (!(p.tol > 0 && p.tol <= 0.1)) fail("tol must be in (0, 0.1]");
  if (p.precision != PSE_FP64 && p.precision != PSE_MIXED)
    fail("precision must be PSE_FP64 or PSE_MIXED");
  const double L = p.box, a = p.radius, eps = p.tol;
  const double lg = std::sqrt(std::log(1.0 / eps));
  Deform df;
  deformation(p, df);
  // deformed lattices: the shortest Nyquist wave vector is sqrt(lambda_max)
  // times shorter, so xi is that much smaller for the same damping there
  const double un = std::sqrt(std::log(1.0 / eps) + 9.0) * std::sqrt(df.lambda_max);
  d = pse_derived{};
  d.lambda_max = df.lambda_max;
  if (p.grid > 0) {
    if (!grid_supported(p.grid)) fail("grid must be 2^j or 3*2^j in [8, 1024]");
    d.grid = p.grid;
    d.xi = p.xi > 0 ? p.xi : M_PI * p.grid / (2.0 * L * un);
  } else if (p.xi > 0) {
    d.xi = p.xi;
    d.grid = next_supported((int)std::ceil(2.0 * p.xi * L * un / M_PI));
    if (d.grid < 0) fail("grid needed for this xi exceeds 1024");
  } else {
    fail("set grid or xi");
  }
  if (p.deriv_gridding < 0 || p.deriv_gridding > 2) fail("deriv_gridding must be 0, 1 or 2");
  const double eps_q = eps / 20.0;
  d.support = p.support > 0 ? p.support
                            : (int)std::ceil(df.lambda_max * 2.0 / M_PI * std::log(2.0 / eps_q));
  // Derivative gridding: the gradient of the truncated Gaussian carries a
  // larger quadrature error than the Gaussian at equal support (each further
  // point divides both by about 3.5), so with an automatic support it takes
  // one more point (with the moment-corrected gradient weights the couplings
  // then measure 0.5 to 1.5 times the moment gridding's errors at eps =
  // 1e-3); it needs the spreading tiles and at most 10 points, else the
  // moment gridding is used.
  // By default it is used where it pays: it moves two fifths of the grid
  // traffic of M_ES and about half of that of the whole product but spreads
  // and interpolates over (P+1)^3 points, so it is faster while the stencil
  // points per grid point, N (P+1)^3 / Ng^3, stay below about 20 (measured
  // on M_ES: faster at 2.4, 3.8, 12 and 14.5, slower at 33).
  d.deriv_gridding = 1;
  if (p.deriv_gridding != 1 && !df.on) {   // 0 (default) or 2; cube only
    const int pd = p.support > 0 ? d.support : d.support + 1;
    const double dens = (double)p.n * pd * pd * pd / ((double)d.grid * d.grid * d.grid);
    if (pd <= 10 && spread_tile(d.grid, pd) != 0 && (p.deriv_gridding == 2 || dens <= 20.0)) {
      d.support = pd;
      d.deriv_gridding = 2;
    }
  }
  if (d.support < 2 || d.support > 16) fail("support must be in [2, 16]");
  if (d.support > d.grid) fail("support larger than the grid");
  d.m = 0.85 * std::sqrt(M_PI * d.support);
  d.h = L / d.grid;
  d.eta_s = std::pow(d.h * d.support * d.xi / d.m, 2);
  if (!(d.eta_s < 1.0)) fail("eta_s = (h P xi / m)^2 must be < 1: refine the grid or lower xi");
  d.rcut = p.rcut > 0 ? p.rcut : 2.0 * a + lg / d.xi;
  if (d.rcut > df.width * L / 3.0)
    fail("rcut exceeds a third of the cell's thinnest width: raise xi or use a larger box");
  d.cells = (int)std::floor(df.width * L / d.rcut);
  if (d.cells < 3) fail("fewer than 3 cells per side");
  if (d.cells > 1024) d.cells = 1024;
  d.lanczos_tol = p.lanczos_tol > 0 ? p.lanczos_tol : 1e-3;
  d.gmres_tol = p.gmres_tol > 0 ? p.gmres_tol : 1e-6;
  if (p.async_calls) {
    // device-checked solves run exactly maxit iterations: modest defaults,
    // and GMRES without restarts (its basis holds every iteration)
    d.lanczos_maxit = p.lanczos_maxit > 0 ? p.lanczos_maxit : 16;
    d.gmres_maxit = p.gmres_maxit > 0 ? p.gmres_maxit : 32;
    d.gmres_restart = d.gmres_maxit;
    d.refine_passes = p.refine_passes > 0 ? p.refine_passes : 1;
  } else {
    d.lanczos_maxit = p.lanczos_maxit > 0 ? p.lanczos_maxit : 100;
    d.gmres_restart = p.gmres_restart > 0 ? p.gmres_restart : 30;
    d.gmres_maxit = p.gmres_maxit > 0 ? p.gmres_maxit : 200;
    d.refine_passes = p.refine_passes > 0 ? p.refine_passes : 3;
  }
  if (d.lanczos_maxit > 500 || d.gmres_restart > 200)
    fail("Krylov basis limits too large");
}

size_t footprint(const pse_params &p, const pse_derived &d) {
  const size_t ng3 = (size_t)d.grid * d.grid * d.grid;
  const size_t n = (size_t)p.n;
  const size_t ncell3 = (size_t)d.cells * d.cells * d.cells;
  size_t bytes = 0;
  // FP64 grids are always present (the FP64 path; in mixed handles only the
  // five-component sets of the FP64 residual of the constraint solve); FP32
  // grids only for mixed handles.
  const bool mixed = p.precision == PSE_MIXED;
  bytes += 2 * (size_t)(mixed ? MIXED_FP64_PACK : MAX_PACK) * ng3 * sizeof(double2)
           + d.grid * sizeof(double2);
  if (mixed) bytes += 2 * MAX_PACK * ng3 * sizeof(float2) + d.grid * sizeof(float2);
  // the per-|k|^2 tables: four radial factors (FP64, and FP32 in mixed
  // handles), and with derivative gridding the constraint operator's factor
  const size_t nk = (size_t)(3 * (d.grid / 2) * (d.grid / 2) + 1);
  bytes += nk * 4 * (sizeof(double) + (mixed ? sizeof(float) : 0));
  if (d.deriv_gridding == 2) bytes += nk * (sizeof(double) + (mixed ? sizeof(float) : 0));
  bytes += (p.async_calls ? 2 : 1) * pair_capacity(p, d) * pair_entry_bytes(mixed)
           + (2 * n + n / 1024 + 16) * sizeof(int);
  const size_t ntab = (size_t)(2048.0 * d.rcut / (2 * p.radius)) + 16;
  bytes += ntab * NCOEF * (sizeof(double) + sizeof(float));
  const int S = spread_tile(d.grid, d.support);
  const size_t tiles3 = S ? ng3 / ((size_t)S * S * S) : 0;
  if (S) {
    // tile CSR and one record per (tile, particle) pair: the particle index,
    // 3 S one-dimensional weights and 3 offsets
    const size_t cap = n * tiles_per_particle(d.support, S);
    bytes += (2 * tiles3 + tiles3 / 1024 + 16) * sizeof(int)
             + cap * (sizeof(int) + (3 * (size_t)S + 3) * sizeof(double)) + 256;
  }
  bytes += (2 * (ncell3 + tiles3) + 4 + (ncell3 + tiles3) / 1024 + 16) * sizeof(int)
           + 8 * n * sizeof(int);
  bytes += (2 * 3 * n + 6 * NC * n + 5 * 5 * n) * sizeof(double);
  if (d.deriv_gridding == 2) bytes += 6 * n * sizeof(double);
  bytes += 12 * n * sizeof(double);   // packed moments of the pair sums
  bytes += (size_t)(d.lanczos_maxit + 1) * NC * n * sizeof(double);
  bytes += (size_t)(d.gmres_restart + 1) * 5 * n * sizeof(double);
  const size_t small = 4 * (size_t)(d.gmres_restart + 2) * (d.gmres_restart + 2)
                       + 10 * (size_t)(d.lanczos_maxit + 2) * (d.lanczos_maxit + 2) + 64;
  bytes += small * sizeof(double);
  bytes += (size_t)4096 * (std::max(d.lanczos_maxit, d.gmres_restart) + 2) * sizeof(double);
  return bytes;
}

}  // namespace pse
