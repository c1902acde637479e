/* Seeded hard-sphere packings for the synthetic inputs (host C, no GPU).
 *
 * Not part of the method: it only places non-overlapping spheres of radius a
 * in a periodic cube, standing in for the random hard-sphere suspensions of
 * the paper's performance measurements.
 *
 *   pack_rsa:        random sequential addition (uniform candidates, each
 *                    kept when it overlaps no placed sphere).
 *   pack_compressed: random sequential addition at a reduced radius (volume
 *                    fraction phi_rsa), then compression: the radius is set
 *                    to a and overlapping pairs are pushed apart along their
 *                    line of centres (Gauss-Seidel sweeps over a cell list)
 *                    until every pair is at least 2a (1 + 1e-6) apart.  The
 *                    result is a random, non-crystalline packing at the
 *                    target fraction; fifty sweeps of hard-sphere Monte Carlo
 *                    moves then lift the pairs left at contact.  (Growing the radius in small steps
 *                    with a relaxation after each ends in the same kind of
 *                    packing and takes many more sweeps.)
 *
 * Random numbers: splitmix64 (Steele, Lea & Flood, OOPSLA 2014) on the seed;
 * uniform doubles from the top 53 bits.  Everything is sequential double
 * arithmetic, so the output depends only on (N, L, a, seed).
 *
 * Return value 0 on success, -1 on bad arguments or exhausted attempts,
 * -2 on host allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double sm_uniform(uint64_t *s) { return (double)(sm_next(s) >> 11) * 0x1.0p-53; }

static double wrap(double v, double L) {
  v -= L * floor(v / L);
  if (v >= L) v -= L;
  if (v < 0) v = 0;
  return v;
}

static double mind(double d, double L) { return d - L * nearbyint(d / L); }

/* Cell grid of side >= cmin over the box: head/next linked lists. */
typedef struct {
  int nc;
  double cs;
  int *head, *next;
} Grid;

static int grid_init(Grid *g, int64_t n, double L, double cmin) {
  g->nc = (int)floor(L / cmin);
  if (g->nc < 1) g->nc = 1;
  if (g->nc > 512) g->nc = 512;
  g->cs = L / g->nc;
  const size_t nc3 = (size_t)g->nc * g->nc * g->nc;
  g->head = (int *)malloc(nc3 * sizeof(int));
  g->next = (int *)malloc((size_t)n * sizeof(int));
  if (!g->head || !g->next) return -2;
  for (size_t i = 0; i < nc3; ++i) g->head[i] = -1;
  return 0;
}

static void grid_free(Grid *g) {
  free(g->head);
  free(g->next);
}

static int cell_of(const Grid *g, double v) {
  int c = (int)(v / g->cs);
  return c >= g->nc ? g->nc - 1 : (c < 0 ? 0 : c);
}

static size_t cell_index(const Grid *g, const double *p) {
  return ((size_t)cell_of(g, p[2]) * g->nc + cell_of(g, p[1])) * g->nc + cell_of(g, p[0]);
}

static void grid_insert(Grid *g, const double *x, int i) {
  const size_t c = cell_index(g, x + 3 * (size_t)i);
  g->next[i] = g->head[c];
  g->head[c] = i;
}

static void grid_rebuild(Grid *g, const double *x, int64_t n) {
  const size_t nc3 = (size_t)g->nc * g->nc * g->nc;
  for (size_t i = 0; i < nc3; ++i) g->head[i] = -1;
  for (int64_t i = n - 1; i >= 0; --i) grid_insert(g, x, (int)i);
}

/* 1 if p overlaps (centre distance below dmin) a sphere in the grid. */
static int overlaps(const Grid *g, const double *x, const double *p, double L, double dmin) {
  const int nc = g->nc, r = nc >= 3 ? 1 : 0;
  const int cx = cell_of(g, p[0]), cy = cell_of(g, p[1]), cz = cell_of(g, p[2]);
  const double d2 = dmin * dmin;
  for (int dz = -r; dz <= r; ++dz)
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const int bx = (cx + dx + nc) % nc, by = (cy + dy + nc) % nc, bz = (cz + dz + nc) % nc;
        for (int j = g->head[((size_t)bz * nc + by) * nc + bx]; j >= 0; j = g->next[j]) {
          const double ex = mind(p[0] - x[3 * (size_t)j], L);
          const double ey = mind(p[1] - x[3 * (size_t)j + 1], L);
          const double ez = mind(p[2] - x[3 * (size_t)j + 2], L);
          if (ex * ex + ey * ey + ez * ez < d2) return 1;
        }
      }
  return 0;
}

static int rsa(int64_t n, double L, double a, uint64_t *st, double *x) {
  if (n <= 0 || !(L > 4 * a) || !(a > 0)) return -1;
  Grid g;
  int rc = grid_init(&g, n, L, 2.0 * a);
  if (rc) {
    grid_free(&g);
    return rc;
  }
  const int64_t max_tries = 2000 * n + 1000000;
  int64_t placed = 0, tries = 0;
  while (placed < n) {
    if (++tries > max_tries) {
      grid_free(&g);
      return -1;
    }
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = sm_uniform(st) * L;
    for (int d = 0; d < 3; ++d) p[d] = wrap(p[d], L);
    if (overlaps(&g, x, p, L, 2.0 * a)) continue;
    memcpy(x + 3 * placed, p, sizeof(p));
    grid_insert(&g, x, (int)placed);
    ++placed;
  }
  grid_free(&g);
  return 0;
}

int pack_rsa(int64_t n, double L, double a, uint64_t seed, double *x) {
  uint64_t st = seed;
  return rsa(n, L, a, &st, x);
}

/* One Gauss-Seidel sweep: every pair closer than thr is pushed apart along
 * its line of centres, each sphere by half of what separates the pair from
 * target (> thr).  Returns the number of pairs pushed: a sweep that pushes
 * none leaves every pair at least thr apart. */
static int64_t relax_sweep(Grid *g, double *x, int64_t n, double L, double thr,
                           double target) {
  const int nc = g->nc, r = nc >= 3 ? 1 : 0;
  int64_t pushed = 0;
  grid_rebuild(g, x, n);
  for (int64_t i = 0; i < n; ++i) {
    double *pi = x + 3 * (size_t)i;
    const int cx = cell_of(g, pi[0]), cy = cell_of(g, pi[1]), cz = cell_of(g, pi[2]);
    for (int dz = -r; dz <= r; ++dz)
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          const int bx = (cx + dx + nc) % nc, by = (cy + dy + nc) % nc,
                    bz = (cz + dz + nc) % nc;
          for (int j = g->head[((size_t)bz * nc + by) * nc + bx]; j >= 0; j = g->next[j]) {
            if (j <= i) continue;
            double *pj = x + 3 * (size_t)j;
            const double ex = mind(pi[0] - pj[0], L), ey = mind(pi[1] - pj[1], L),
                         ez = mind(pi[2] - pj[2], L);
            const double d = sqrt(ex * ex + ey * ey + ez * ez);
            if (d >= thr) continue;
            ++pushed;
            double u[3];
            if (d > 1e-12) {
              u[0] = ex / d;
              u[1] = ey / d;
              u[2] = ez / d;
            } else {
              u[0] = 1.0;
              u[1] = 0.0;
              u[2] = 0.0;
            }
            const double s = 0.5 * (target - d);
            for (int k = 0; k < 3; ++k) {
              pi[k] = wrap(pi[k] + s * u[k], L);
              pj[k] = wrap(pj[k] - s * u[k], L);
            }
          }
        }
  }
  return pushed;
}

int pack_compressed(int64_t n, double L, double a, double phi_rsa, uint64_t seed, double *x) {
  if (n <= 0 || !(L > 4 * a) || !(a > 0) || !(phi_rsa > 0)) return -1;
  const double phi = (double)n * 4.0 / 3.0 * 3.14159265358979323846 * a * a * a / (L * L * L);
  if (!(phi < 0.55)) return -1;
  uint64_t st = seed;
  double r = phi_rsa < phi ? a * cbrt(phi_rsa / phi) : a;
  int rc = rsa(n, L, r, &st, x);
  if (rc) return rc;
  if (r >= a) return 0;
  Grid g;
  rc = grid_init(&g, n, L, 2.0 * a * 1.001);
  if (rc) {
    grid_free(&g);
    return rc;
  }
  const double thr = 2.0 * a * (1.0 + 1e-6), target = 2.0 * a * (1.0 + 2e-6);
  int sweeps = 0;
  while (relax_sweep(&g, x, n, L, thr, target) > 0) {
    if (++sweeps > 200000) {
      grid_free(&g);
      return -1;
    }
  }
  /* hard-sphere Monte Carlo sweeps: each sphere in turn tries a uniform
   * displacement of up to 0.1a per axis, kept when it overlaps no other;
   * this lifts the pairs the pushes left at contact */
  for (int sweep = 0; sweep < 50; ++sweep) {
    grid_rebuild(&g, x, n);
    for (int64_t i = 0; i < n; ++i) {
      double p[3], *pi = x + 3 * (size_t)i;
      for (int d = 0; d < 3; ++d) p[d] = wrap(pi[d] + 0.1 * a * (2.0 * sm_uniform(&st) - 1.0), L);
      if (cell_index(&g, p) != cell_index(&g, pi)) continue;   /* stay in the cell */
      const double keep[3] = {pi[0], pi[1], pi[2]};
      pi[0] = NAN;   /* not its own neighbour (a NaN distance is no overlap) */
      const int hit = overlaps(&g, x, p, L, thr);
      memcpy(pi, hit ? keep : p, sizeof(p));
    }
  }
  grid_free(&g);
  return 0;
}
