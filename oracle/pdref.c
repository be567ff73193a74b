/*
 * pdref.c -- plain FP64 CPU oracle of the explicit peridynamic grain-aggregate step.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
 * benchmark's CPU-baseline leg are its only users.  It shares no code with the
 * HIP library.  Every function follows the paper's definitions written out in
 * the plainest order; see pdref.h for the list of sections it follows.
 *
 * Readings of points the paper leaves open (each is also listed in the design notes):
 *   R1 constant micromodulus c = 18K/(pi delta^4) and s0 = sqrt(5 Gc/(9 K delta))
 *      (conic, PDREF_CONIC: c0 = 90K/(pi delta^4), s0 = sqrt(2 Gc/(3 K delta))):
 *      the values for which a uniform small strain reproduces the strain-energy
 *      density 9Ks^2/2 and breaking every bond across a unit area costs G_c
 *      (Sec. 3.1.1 states both calibrations; the 3-D row of its table carries a
 *      2-D (1-nu) factor).  PDREF_TABLE_LITERAL selects the printed row.
 *   R2 the horizon is the inclusive integer shell 0 < |d ijk|^2 <= m^2.
 *   R3 bonds break in tension, s > s0 (the formal definition of gamma);
 *      PDREF_ABS_STRETCH selects |s| > s0.  A bond that exceeds s0 in an
 *      evaluation contributes no force in that evaluation and stays broken.
 *   R4 damage = 1 - intact/initial (the text states the inverted ratio).
 *   R5 eps in K_n is the horizon; walls use the true spherical-cap volume
 *      (pi/3)(Rc-d)^2(2Rc+d), the one consistent with the printed centroid;
 *      several walls are summed.
 *   R6 velocity Verlet in position form; fixed nodes keep u and have v = a = 0.
 *   R15 normal damping (Sec. 3.4) is linear in the normal relative velocity,
 *      -beta_d (w . e) e with w the velocity of the node relative to its partner
 *      (the sign that dissipates): the text calls the law linear and likens it
 *      to a viscoelastic spring, while the printed formula normalises w.  The
 *      velocity is the mid-step value v_n + dt/2 a_n, the one known when the
 *      force at u_{n+1} is evaluated (v_0 in the first evaluation).  Against a
 *      wall the partner moves with the wall's rate along its normal.
 *   R17 stick-slip friction (Sec. 3.3) acts per contact pair on the pair's force
 *      density: f_r is the repulsive force density the partner exerts on the
 *      node (K_n (R_c - d) V_j; against a wall K_n (R_c - |c - p|) |S|), so that
 *      v_thr = mu f_r dt / rho is a speed and the stick force (rho/dt) |w_t|
 *      meets the slip force mu f_r at the threshold.  The force opposes the
 *      node's own tangential relative velocity w_t (the prose; the printed
 *      e_perp(y,x) would push along it).  rho is the node's density; the
 *      velocities are the mid-step ones of R15; f_r excludes the damping term.
 *   R18 self-contact (Sec. 5, PDREF_SELF_CONTACT): every pair of nodes of one
 *      grain with no intact bond at the evaluation (broken in this or an
 *      earlier evaluation, removed by a cut, or never in the horizon) and
 *      current distance d < R_c repels.  Reference length |xi| < R_c: the
 *      repulsive-only bond K_n R_c (|xi| - d)/|xi| for d < |xi|; otherwise the
 *      contact spring K_n (R_c - d) (c_w = K_n R_c), both times V_j, with the
 *      damping and friction of R15/R17 on top.  The paper's assumption
 *      eps <= R_c is not needed for this case split and is not made.  With
 *      self-contact the skin guard applies to a single grain as well.
 *   R12 contact pairs (Sec. 3.2) are found among candidates within R_c + skin,
 *      rebuilt every rebuild_every steps; a node that moved more than skin/2
 *      since the last rebuild may have missed a pair, which the guard reports.
 *      PDREF_ADAPTIVE_REBUILD instead rebuilds before any evaluation at which
 *      that happened: the forces do not depend on when the candidates were
 *      built as long as they hold every pair within R_c, so the result is that
 *      of a rebuild before every evaluation.
 *   R19 several walls (Sec. 4.1.1, PDREF_WALL_CORNERS): inclusion-exclusion
 *      over the walls a node touches, pairs counted once (the printed sum over
 *      i != j would count each twice) and the triple term without the stray
 *      factor V_x; the intersection volumes and centroids, which the paper does
 *      not give, are integrated over slices of the ball.  Only mutually
 *      orthogonal walls (a box) form pairs and triples.  The damping and
 *      friction of each wall stay per wall.  Each wall's reaction takes the
 *      corrections' components along its normal.
 */
#include "pdref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

typedef struct {
  double n[3], offset0, offset, velocity, lo[3], hi[3];
  int mode;
  double target, gain, area;
  double rate;       /* d(offset)/dt over the step that led to the current offset */
  double force[3];   /* reaction on the wall, -sum_i V_i F_wall,i */
  double impulse[3]; /* sum over completed steps of force * dt */
} wall_t;

typedef struct {
  int64_t kind, grain, plane[4], lo[3], hi[3], c[3], r2;
} cut_t;

struct pdref {
  int64_t n;
  double *X, *u, *v, *a, *F;
  int32_t* ijk;
  uint8_t* fixed;
  int32_t n_grains;
  int64_t* grain_begin;
  int32_t* grain_of; /* node -> grain */
  int32_t* gmat;
  double* gh;
  double *gc, *gs0, *gV, *grho, *gK; /* per grain */
  int32_t n_mat;
  double* mat;
  int m;
  double Rc, eps, skin, dt, g[3];
  double beta;   /* normal damping coefficient beta_d, Sec. 3.4 */
  double mu;     /* friction coefficient of the stick-slip law, Sec. 3.3 */
  double* vh;    /* velocity the damping and friction laws see: v + dt/2 a (v at the build) */
  int rebuild_every;
  int32_t n_walls;
  wall_t* walls;
  int32_t n_cuts;
  cut_t* cuts;
  int32_t flags;
  /* bonds */
  int64_t* row_ptr;
  int32_t* col;
  uint8_t* broken;
  int32_t* n0;
  /* contact candidates */
  int64_t* cand_ptr;
  int32_t* cand;
  double* u_at_build;
  int64_t step;
  int64_t early_rebuilds; /* PDREF_ADAPTIVE_REBUILD rebuilds between the cadence ones */
  double* margin; /* [nnz] min over the bond's evaluations of its break margin */
  double min_margin;
  int built;
};

/* ------------------------------------------------------------------------- */
/* constants                                                                 */
/* ------------------------------------------------------------------------- */

/* Sec. 3.1.1 and its table.  Calibrated (R1): the strain-energy density of a
 * uniform stretch s, (1/2) int_H (1/2) c w(r) s^2 r dV = 9 K s^2 / 2, and the
 * energy of all bonds across a unit area at s0 equal to G_c:
 *   constant w = 1:          pi c delta^4 / 4  = 9K/2,  pi c s0^2 delta^5 / 10 = G_c;
 *   conic    w = 1 - r/delta: pi c delta^4 / 20 = 9K/2,  pi c s0^2 delta^5 / 60 = G_c.
 * PDREF_TABLE_LITERAL takes the printed 3-D rows instead (nu = 1/4, E = 3K(1-2nu)). */
void pdref_constants(double K, double Gc, double delta, int32_t flags, double* c, double* s0) {
  const int conic = (flags & PDREF_CONIC) != 0;
  if (flags & PDREF_TABLE_LITERAL) {
    double nu = 0.25;
    double E = 3.0 * K * (1.0 - 2.0 * nu);
    if (conic) {
      /* 60 E (delta - r) / (pi delta^5 (1 - nu)) = c0 (1 - r/delta) */
      *c = 60.0 * E / (PI * pow(delta, 4) * (1.0 - nu));
      *s0 = sqrt(7.0 * PI * Gc / (12.0 * E * delta));
    } else {
      *c = 12.0 * E / (PI * pow(delta, 4) * (1.0 - nu));
      *s0 = sqrt(5.0 * PI * Gc / (12.0 * E * delta));
    }
  } else if (conic) {
    *c = 90.0 * K / (PI * pow(delta, 4));
    *s0 = sqrt(2.0 * Gc / (3.0 * K * delta));
  } else {
    *c = 18.0 * K / (PI * pow(delta, 4));
    *s0 = sqrt(5.0 * Gc / (9.0 * K * delta));
  }
}

/* micromodulus weight w(|xi|) of a bond in grain g */
static double bond_weight(const pdref* s, int32_t g, double l0) {
  return (s->flags & PDREF_CONIC) ? 1.0 - l0 / (s->m * s->gh[g]) : 1.0;
}

double pdref_contact_stiffness(double k_a, double k_b, double eps) {
  double k = 2.0 * k_a * k_b / (k_a + k_b);
  return 18.0 * k / (PI * pow(eps, 5));
}

void pdref_wall_cap(double Rc, double d, double* volume, double* centroid) {
  /* cap of the ball B_Rc(p) on the far side of a plane at signed distance d */
  *volume = PI / 3.0 * (Rc - d) * (Rc - d) * (2.0 * Rc + d);
  *centroid = (PI / 4.0) * (Rc * Rc - d * d) * (Rc * Rc - d * d) / *volume;
}

/* ------------------------------------------------------------------------- */
/* several walls at a corner (Sec. 4.1.1, R19)                               */
/* ------------------------------------------------------------------------- */

/* Area and first moments of the plane region {v > b, w > c, v^2 + w^2 < r^2}
   (c = -INFINITY: the circular segment v > b), integrated over v in closed
   form.  For a given v the region spans w in (max(c, -s), s), s = sqrt(r^2 - v^2). */
static double seg_S0(double r, double x) { /* int sqrt(r^2 - v^2) dv */
  const double sx = sqrt(fmax(r * r - x * x, 0.0));
  return 0.5 * (x * sx + r * r * asin(fmax(-1.0, fmin(1.0, x / r))));
}
static double seg_S1(double r, double x) { /* int v sqrt(r^2 - v^2) dv */
  const double q = fmax(r * r - x * x, 0.0);
  return -q * sqrt(q) / 3.0;
}
static double seg_S2(double r, double x) { /* int (r^2 - v^2) dv */
  return r * r * x - x * x * x / 3.0;
}
static void region2d(double r, double b, double c, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (!(r > 0.0) || b >= r || c >= r) return;
  const double v0 = fmax(b, -r);
  /* pieces of the v axis: |v| < e where the lower bound is c (s > -c), and
     e <= |v| < r where it is -s; with c >= 0 only |v| < e is non-empty */
  double e = r;
  if (c > -r) e = sqrt(r * r - c * c);
  double lo[3] = {-r, -e, e}, hi[3] = {-e, e, r};
  int kind[3] = {2, 1, 2}; /* 1: length s - c, 2: length 2s */
  if (c >= 0.0) kind[0] = kind[2] = 0;
  if (!(c > -r)) { kind[1] = 2; }
  for (int k = 0; k < 3; ++k) {
    if (!kind[k]) continue;
    double x0 = fmax(lo[k], v0), x1 = hi[k];
    if (!(x1 > x0)) continue;
    if (kind[k] == 1) {
      out[0] += seg_S0(r, x1) - seg_S0(r, x0) - c * (x1 - x0);
      out[1] += seg_S1(r, x1) - seg_S1(r, x0) - 0.5 * c * (x1 * x1 - x0 * x0);
      out[2] += 0.5 * (seg_S2(r, x1) - seg_S2(r, x0) - c * c * (x1 - x0));
    } else {
      out[0] += 2.0 * (seg_S0(r, x1) - seg_S0(r, x0));
      out[1] += 2.0 * (seg_S1(r, x1) - seg_S1(r, x0));
    }
  }
}

/* integrand over u: [A, u A, M_v, M_w] of the slice of the ball at height u */
static void corner_slice(double R, double b, double c, double u, double f[4]) {
  double m[3];
  region2d(sqrt(fmax(R * R - u * u, 0.0)), b, c, m);
  f[0] = m[0];
  f[1] = u * m[0];
  f[2] = m[1];
  f[3] = m[2];
}

/* tanh-sinh (double-exponential) quadrature of the four integrands on
   [x0, x1] (Takahasi and Mori): x = mid + half tanh((pi/2) sinh t) on a step
   of t halved until two levels agree; it is exact to rounding for integrands
   that are smooth inside the interval, whatever their behaviour at its ends. */
static void tanh_sinh4(double R, double b, double c, double x0, double x1, double out[4]) {
  const double mid = 0.5 * (x0 + x1), half = 0.5 * (x1 - x0);
  double prev[4] = {0.0, 0.0, 0.0, 0.0}, sum[4] = {0.0, 0.0, 0.0, 0.0};
  double step = 0.5;
  /* level 0: t = k step for |t| <= 4, then odd multiples of each halved step */
  for (int level = 0; level < 9; ++level) {
    const int stride = level == 0 ? 1 : 2;
    const int first = level == 0 ? 0 : 1;
    for (int k = first; k * step <= 4.0; k += stride) {
      const double t = k * step;
      const double sh = (PI / 2.0) * sinh(t), ch = cosh(sh);
      const double w = (PI / 2.0) * cosh(t) / (ch * ch);
      const double x = tanh(sh);
      double f[4];
      corner_slice(R, b, c, mid + half * x, f);
      for (int q = 0; q < 4; ++q) sum[q] += w * f[q];
      if (k > 0) {
        corner_slice(R, b, c, mid - half * x, f);
        for (int q = 0; q < 4; ++q) sum[q] += w * f[q];
      }
    }
    double est[4], diff = 0.0, scale = 0.0;
    for (int q = 0; q < 4; ++q) {
      est[q] = half * step * sum[q];
      diff = fmax(diff, fabs(est[q] - prev[q]));
      scale = fmax(scale, fabs(est[q]));
      prev[q] = est[q];
    }
    if (level >= 3 && diff <= 1e-15 * scale) break;
    step *= 0.5;
  }
  for (int q = 0; q < 4; ++q) out[q] += prev[q];
}

/* Volume and centroid of {x : |x| < R, x_u > a, x_v > b, x_w > c} (c = -INFINITY
   for two planes): V = int A(u) du over the slices u = const, each a disk of
   radius sqrt(R^2 - u^2) cut by the other planes.  The u axis is split where a
   slice changes shape, and each piece is integrated by tanh-sinh quadrature. */
void pdref_corner_region(double R, double a, double b, double c, double* volume, double centroid[3]) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const double u0 = fmax(a, -R);
  double cuts[8]; /* u0, R and up to two points for each of three radii */
  int nc = 0;
  cuts[nc++] = u0;
  const double rr[3] = {fabs(b), fabs(c), sqrt(b * b + c * c)};
  for (int k = 0; k < 3; ++k)
    if (rr[k] < R && isfinite(rr[k])) {
      const double uk = sqrt(R * R - rr[k] * rr[k]);
      if (uk > u0 && uk < R) cuts[nc++] = uk;
      if (-uk > u0 && -uk < R) cuts[nc++] = -uk;
    }
  cuts[nc++] = R;
  for (int i = 1; i < nc; ++i) /* sort the break points */
    for (int j = i; j > 0 && cuts[j] < cuts[j - 1]; --j) {
      const double t = cuts[j];
      cuts[j] = cuts[j - 1];
      cuts[j - 1] = t;
    }
  for (int k = 0; k + 1 < nc; ++k) {
    const double x0 = cuts[k], x1 = cuts[k + 1];
    if (!(x1 > x0)) continue;
    tanh_sinh4(R, b, c, x0, x1, acc);
  }
  *volume = acc[0];
  for (int q = 0; q < 3; ++q) centroid[q] = acc[0] > 0.0 ? acc[q + 1] / acc[0] : 0.0;
}

/* ------------------------------------------------------------------------- */
/* set-up                                                                    */
/* ------------------------------------------------------------------------- */

static double* dup_d(const double* src, int64_t n) {
  double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (src)
    memcpy(p, src, sizeof(double) * (size_t)n);
  else
    memset(p, 0, sizeof(double) * (size_t)(n > 0 ? n : 1));
  return p;
}

pdref* pdref_create(int64_t n, const double* X, const int32_t* ijk, const double* u0,
                    const double* v0, const uint8_t* fixed, int32_t n_grains,
                    const int64_t* grain_begin, const int32_t* grain_material,
                    const double* grain_h, int32_t n_mat, const double* mat,
                    const double* params, int32_t n_walls, const double* walls, int32_t n_cuts,
                    const int64_t* cuts, int32_t flags) {
  pdref* s = (pdref*)calloc(1, sizeof(pdref));
  s->n = n;
  s->X = dup_d(X, 3 * n);
  s->u = dup_d(u0, 3 * n);
  s->v = dup_d(v0, 3 * n);
  s->a = dup_d(NULL, 3 * n);
  s->vh = dup_d(NULL, 3 * n);
  s->F = dup_d(NULL, 3 * n);
  s->u_at_build = dup_d(NULL, 3 * n);
  s->ijk = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * n + 1));
  memcpy(s->ijk, ijk, sizeof(int32_t) * (size_t)(3 * n));
  s->fixed = (uint8_t*)calloc((size_t)n + 1, 1);
  if (fixed) memcpy(s->fixed, fixed, (size_t)n);
  s->n_grains = n_grains;
  s->grain_begin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_grains + 1));
  memcpy(s->grain_begin, grain_begin, sizeof(int64_t) * (size_t)(n_grains + 1));
  s->gmat = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_grains);
  memcpy(s->gmat, grain_material, sizeof(int32_t) * (size_t)n_grains);
  s->gh = dup_d(grain_h, n_grains);
  s->n_mat = n_mat;
  s->mat = dup_d(mat, 3 * n_mat);
  s->m = (int)params[0];
  s->Rc = params[1];
  s->eps = params[2];
  s->skin = params[3];
  s->rebuild_every = (int)params[4];
  if (s->rebuild_every < 1) s->rebuild_every = 1;
  s->dt = params[5];
  s->g[0] = params[6];
  s->g[1] = params[7];
  s->g[2] = params[8];
  s->beta = params[9];
  s->mu = params[10];
  s->flags = flags;
  s->grain_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  for (int32_t g = 0; g < n_grains; ++g)
    for (int64_t i = grain_begin[g]; i < grain_begin[g + 1]; ++i) s->grain_of[i] = g;
  s->gc = dup_d(NULL, n_grains);
  s->gs0 = dup_d(NULL, n_grains);
  s->gV = dup_d(NULL, n_grains);
  s->grho = dup_d(NULL, n_grains);
  s->gK = dup_d(NULL, n_grains);
  for (int32_t g = 0; g < n_grains; ++g) {
    const double* mt = s->mat + 3 * s->gmat[g];
    double delta = s->m * s->gh[g];
    pdref_constants(mt[0], mt[2], delta, flags, &s->gc[g], &s->gs0[g]);
    s->gV[g] = s->gh[g] * s->gh[g] * s->gh[g];
    s->grho[g] = mt[1];
    s->gK[g] = mt[0];
  }
  s->n_walls = n_walls;
  s->walls = (wall_t*)calloc((size_t)(n_walls > 0 ? n_walls : 1), sizeof(wall_t));
  for (int32_t w = 0; w < n_walls; ++w) {
    const double* r = walls + PDREF_WALL_DOUBLES * w;
    wall_t* W = &s->walls[w];
    W->n[0] = r[0]; W->n[1] = r[1]; W->n[2] = r[2];
    W->offset0 = W->offset = r[3];
    W->velocity = r[4];
    W->lo[0] = r[5]; W->lo[1] = r[6]; W->lo[2] = r[7];
    W->hi[0] = r[8]; W->hi[1] = r[9]; W->hi[2] = r[10];
    W->mode = (int)r[11];
    W->target = r[12];
    W->gain = r[13];
    W->area = r[14];
    W->rate = W->mode == 1 ? W->velocity : 0.0;
  }
  s->n_cuts = n_cuts;
  s->cuts = (cut_t*)calloc((size_t)(n_cuts > 0 ? n_cuts : 1), sizeof(cut_t));
  for (int32_t k = 0; k < n_cuts; ++k) {
    const int64_t* r = cuts + PDREF_CUT_INTS * k;
    cut_t* C = &s->cuts[k];
    C->kind = r[0]; C->grain = r[1];
    for (int q = 0; q < 4; ++q) C->plane[q] = r[2 + q];
    for (int q = 0; q < 3; ++q) { C->lo[q] = r[6 + q]; C->hi[q] = r[9 + q]; C->c[q] = r[12 + q]; }
    C->r2 = r[15];
  }
  s->min_margin = INFINITY;
  return s;
}

void pdref_destroy(pdref* s) {
  if (!s) return;
  free(s->X); free(s->u); free(s->v); free(s->a); free(s->vh); free(s->F); free(s->u_at_build);
  free(s->ijk); free(s->fixed); free(s->grain_begin); free(s->gmat); free(s->gh);
  free(s->mat); free(s->grain_of); free(s->gc); free(s->gs0); free(s->gV); free(s->grho);
  free(s->gK); free(s->walls); free(s->cuts); free(s->row_ptr); free(s->col); free(s->broken);
  free(s->n0); free(s->cand_ptr); free(s->cand); free(s->margin);
  free(s);
}

void pdref_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* bond family and bond removal (Sec. 3.1, Sec. 6.3)                         */
/* ------------------------------------------------------------------------- */

#define HALF_UNBOUNDED (((int64_t)1) << 50)

/* Sec. 6.3.1: the bond P1->P2 crosses the plane at a parameter 0 < t < 1,
   and the crossing point lies inside the cut's bounds.  Exact integer test. */
static int notch_removes(const cut_t* C, const int64_t P1[3], const int64_t P2[3]) {
  int64_t f1 = C->plane[0] * P1[0] + C->plane[1] * P1[1] + C->plane[2] * P1[2] + C->plane[3];
  int64_t f2 = C->plane[0] * P2[0] + C->plane[1] * P2[1] + C->plane[2] * P2[2] + C->plane[3];
  if (!((f1 < 0 && f2 > 0) || (f1 > 0 && f2 < 0))) return 0;
  /* t = f1 / (f1 - f2); crossing Q = P1 + t (P2 - P1); scale by den = f1 - f2 */
  int64_t num = f1, den = f1 - f2;
  if (den < 0) { num = -num; den = -den; }
  for (int q = 0; q < 3; ++q) {
    int64_t Qs = P1[q] * den + num * (P2[q] - P1[q]); /* Q_q * den */
    if (C->lo[q] > -HALF_UNBOUNDED && Qs < C->lo[q] * den) return 0;
    if (C->hi[q] < HALF_UNBOUNDED && Qs > C->hi[q] * den) return 0;
  }
  return 1;
}

static int64_t dist2_i(const int64_t A[3], const int64_t B[3]) {
  int64_t d0 = A[0] - B[0], d1 = A[1] - B[1], d2 = A[2] - B[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}

/* Sec. 6.3.2: remove a bond with an endpoint strictly inside the inner sphere */
static int cavity_endpoint_removes(const cut_t* C, const int64_t P1[3], const int64_t P2[3]) {
  return dist2_i(P1, C->c) < C->r2 || dist2_i(P2, C->c) < C->r2;
}

/* chord variant: remove a bond whose segment passes strictly inside the sphere */
static int cavity_chord_removes(const cut_t* C, const int64_t P1[3], const int64_t P2[3]) {
  int64_t D[3] = {P2[0] - P1[0], P2[1] - P1[1], P2[2] - P1[2]};
  int64_t W[3] = {C->c[0] - P1[0], C->c[1] - P1[1], C->c[2] - P1[2]};
  int64_t DD = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
  int64_t WD = W[0] * D[0] + W[1] * D[1] + W[2] * D[2];
  if (WD <= 0) return dist2_i(P1, C->c) < C->r2;
  if (WD >= DD) return dist2_i(P2, C->c) < C->r2;
  int64_t WW = W[0] * W[0] + W[1] * W[1] + W[2] * W[2];
  /* squared distance to the line, times DD */
  return WW * DD - WD * WD < C->r2 * DD;
}

static int bond_removed(const pdref* s, int32_t g, int64_t i, int64_t j) {
  int64_t P1[3], P2[3];
  for (int q = 0; q < 3; ++q) {
    P1[q] = 2 * (int64_t)s->ijk[q * s->n + i];
    P2[q] = 2 * (int64_t)s->ijk[q * s->n + j];
  }
  for (int32_t k = 0; k < s->n_cuts; ++k) {
    const cut_t* C = &s->cuts[k];
    if (C->grain != g) continue;
    if (C->kind == 0 && notch_removes(C, P1, P2)) return 1;
    if (C->kind == 1 && cavity_endpoint_removes(C, P1, P2)) return 1;
    if (C->kind == 2 && cavity_chord_removes(C, P1, P2)) return 1;
  }
  return 0;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* bond rows: for node i every node j of the same grain at lattice offset d with
   0 < |d|^2 <= m^2 (the horizon H_eps(x) intersected with P_i), minus cut bonds;
   rows sorted ascending. */
static void build_bonds(pdref* s) {
  const int64_t n = s->n;
  const int m = s->m;
  s->row_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  s->n0 = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int64_t cap = 1024, nnz = 0;
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  for (int32_t g = 0; g < s->n_grains; ++g) {
    int64_t b = s->grain_begin[g], e = s->grain_begin[g + 1];
    if (e <= b) continue;
    int32_t lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int64_t i = b; i < e; ++i)
      for (int q = 0; q < 3; ++q) {
        int32_t v = s->ijk[q * n + i];
        if (v < lo[q]) lo[q] = v;
        if (v > hi[q]) hi[q] = v;
      }
    int64_t ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    int64_t* map = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ex * ey * ez));
    for (int64_t k = 0; k < ex * ey * ez; ++k) map[k] = -1;
    for (int64_t i = b; i < e; ++i) {
      int64_t x = s->ijk[i] - lo[0], y = s->ijk[n + i] - lo[1], z = s->ijk[2 * n + i] - lo[2];
      map[(x * ey + y) * ez + z] = i;
    }
    for (int64_t i = b; i < e; ++i) {
      s->row_ptr[i] = nnz;
      int64_t x = s->ijk[i] - lo[0], y = s->ijk[n + i] - lo[1], z = s->ijk[2 * n + i] - lo[2];
      for (int dx = -m; dx <= m; ++dx)
        for (int dy = -m; dy <= m; ++dy)
          for (int dz = -m; dz <= m; ++dz) {
            int d2 = dx * dx + dy * dy + dz * dz;
            if (d2 == 0 || d2 > m * m) continue;
            int64_t X2 = x + dx, Y2 = y + dy, Z2 = z + dz;
            if (X2 < 0 || Y2 < 0 || Z2 < 0 || X2 >= ex || Y2 >= ey || Z2 >= ez) continue;
            int64_t j = map[(X2 * ey + Y2) * ez + Z2];
            if (j < 0) continue;
            if (bond_removed(s, g, i, j)) continue;
            if (nnz == cap) {
              cap *= 2;
              col = (int32_t*)realloc(col, sizeof(int32_t) * (size_t)cap);
            }
            col[nnz++] = (int32_t)j;
          }
      if (nnz > s->row_ptr[i]) qsort(col + s->row_ptr[i], (size_t)(nnz - s->row_ptr[i]), sizeof(int32_t), cmp_i32);
      s->n0[i] = (int32_t)(nnz - s->row_ptr[i]);
    }
    free(map);
  }
  s->row_ptr[n] = nnz;
  s->col = col;
  s->broken = (uint8_t*)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
  s->margin = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t e = 0; e < nnz; ++e) s->margin[e] = INFINITY;
}

/* ------------------------------------------------------------------------- */
/* contact candidates (Sec. 3.2): nodes of other grains within R_c + skin     */
/* ------------------------------------------------------------------------- */

/* squared current distance |p_j - p_i|^2 with p_j - p_i = (X_j - X_i) + (u_j - u_i) */
static double pair_dist2(const pdref* s, int64_t i, int64_t j, double y[3]) {
  const int64_t n = s->n;
  for (int q = 0; q < 3; ++q)
    y[q] = (s->X[q * n + j] - s->X[q * n + i]) + (s->u[q * n + j] - s->u[q * n + i]);
  return (y[0] * y[0] + y[1] * y[1]) + y[2] * y[2];
}

typedef struct {
  int32_t* v;
  int64_t len, cap;
} ivec;

static void ivec_push(ivec* a, int32_t x) {
  if (a->len == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 256;
    a->v = (int32_t*)realloc(a->v, sizeof(int32_t) * (size_t)a->cap);
  }
  a->v[a->len++] = x;
}

/* pairs the contact search keeps: nodes of other grains, and with self-contact
   every other node of the same grain (whether bonded is decided at the force) */
static int contact_kind_pair(const pdref* s, int64_t i, int64_t j) {
  if (j == i) return 0;
  if (s->grain_of[j] != s->grain_of[i]) return 1;
  return (s->flags & PDREF_SELF_CONTACT) != 0;
}

static void build_candidates(pdref* s) {
  const int64_t n = s->n;
  const double cut = s->Rc + s->skin, cut2 = cut * cut;
  free(s->cand_ptr);
  free(s->cand);
  s->cand_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  ivec out = {0, 0, 0};
  double y[3];
  if (!(s->flags & PDREF_CELL_LIST)) {
    for (int64_t i = 0; i < n; ++i) {
      s->cand_ptr[i] = out.len;
      for (int64_t j = 0; j < n; ++j) {
        if (!contact_kind_pair(s, i, j)) continue;
        if (pair_dist2(s, i, j, y) < cut2) ivec_push(&out, (int32_t)j);
      }
    }
  } else {
    /* plain uniform cell list over the bounding box of p = X + u */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < 3; ++q) {
        double p = s->X[q * n + i] + s->u[q * n + i];
        if (p < lo[q]) lo[q] = p;
        if (p > hi[q]) hi[q] = p;
      }
    double cell = cut * 1.01;
    int64_t dim[3];
    for (int q = 0; q < 3; ++q) dim[q] = (n > 0) ? (int64_t)floor((hi[q] - lo[q]) / cell) + 1 : 1;
    int64_t ncell = dim[0] * dim[1] * dim[2];
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* cidx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * n + 1));
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
      int64_t c3[3];
      for (int q = 0; q < 3; ++q) {
        double p = s->X[q * n + i] + s->u[q * n + i];
        c3[q] = (int64_t)floor((p - lo[q]) / cell);
        if (c3[q] < 0) c3[q] = 0;
        if (c3[q] >= dim[q]) c3[q] = dim[q] - 1;
        cidx[3 * i + q] = c3[q];
      }
      int64_t c = (c3[0] * dim[1] + c3[1]) * dim[2] + c3[2];
      next[i] = head[c];
      head[c] = i;
    }
    for (int64_t i = 0; i < n; ++i) {
      s->cand_ptr[i] = out.len;
      int64_t start = out.len;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int64_t cx = cidx[3 * i] + dx, cy = cidx[3 * i + 1] + dy, cz = cidx[3 * i + 2] + dz;
            if (cx < 0 || cy < 0 || cz < 0 || cx >= dim[0] || cy >= dim[1] || cz >= dim[2]) continue;
            for (int64_t j = head[(cx * dim[1] + cy) * dim[2] + cz]; j >= 0; j = next[j]) {
              if (!contact_kind_pair(s, i, j)) continue;
              if (pair_dist2(s, i, j, y) < cut2) ivec_push(&out, (int32_t)j);
            }
          }
      if (out.len > start) qsort(out.v + start, (size_t)(out.len - start), sizeof(int32_t), cmp_i32);
    }
    free(head);
    free(next);
    free(cidx);
  }
  s->cand_ptr[n] = out.len;
  s->cand = out.v ? out.v : (int32_t*)malloc(sizeof(int32_t));
  memcpy(s->u_at_build, s->u, sizeof(double) * (size_t)(3 * n));
}

/* ------------------------------------------------------------------------- */
/* force density at the current u                                           */
/* ------------------------------------------------------------------------- */

/* Bond stretch s = (|xi + eta| - |xi|) / |xi| (Sec. 3.1).  The numerator is
   evaluated as (|xi+eta|^2 - |xi|^2) / (|xi+eta| + |xi|) with the squared
   difference formed directly as eta . (2 xi + eta): the same quantity, without
   the cancellation of two nearly equal rounded lengths (|eta| << |xi|). */
static double stretch(const double xi[3], const double eta[3], double l0, double l) {
  double dd = (eta[0] * (2.0 * xi[0] + eta[0]) + eta[1] * (2.0 * xi[1] + eta[1])) +
              eta[2] * (2.0 * xi[2] + eta[2]);
  return dd / (l0 * (l + l0));
}

/* returns nonzero when an instability was seen (NaN force, wall penetration) */

/* Regularised Coulomb friction, Sec. 3.3, eq. (regularized-friction), added to F.
 * wt: tangential velocity of the node relative to its partner; fr: magnitude of
 * the repulsive force density the partner exerts on the node; rho: the node's
 * density.  Slip (|wt| above v_thr = mu fr dt / rho): magnitude mu fr against wt.
 * Stick: -(1/eps_f) wt with eps_f = dt / rho, the force that stops wt in one step. */
static void add_friction(double mu, double fr, double rho, double dt, const double wt[3],
                         double F[3]) {
  const double vt = sqrt((wt[0] * wt[0] + wt[1] * wt[1]) + wt[2] * wt[2]);
  const double vthr = mu * fr * dt / rho;
  if (vt > vthr) {
    for (int q = 0; q < 3; ++q) F[q] -= mu * fr * wt[q] / vt;
  } else {
    const double eps_f = dt / rho;
    for (int q = 0; q < 3; ++q) F[q] -= wt[q] / eps_f;
  }
}

/* Inclusion-exclusion over the walls node i touches (Sec. 4.1.1): the force
   sum_l F_l - sum_{pairs} F_{l l'} + F_{l l' l''} of terms
   -K_n (R_c - |c_S - p|) |S| e_S, e_S = (c_S - p)/|c_S - p|, S the part of the
   contact ball beyond every wall of the term.  Pairs and triples are those of
   mutually orthogonal walls (the corners of a box; the regions of other pairs
   have no closed description here and their terms are left out).  Wall l takes
   the component of each correction along its normal, so the corrections land
   in the per-wall magnitudes: corr[l][i] += (sign F_S) . n_l. */
static void wall_corners(const pdref* s, int64_t i, double* corr) {
  const int64_t n = s->n;
  const double Rc = s->Rc;
  int hit[3], nh = 0;
  double dl[3];
  double p[3];
  for (int q = 0; q < 3; ++q) p[q] = s->X[q * n + i] + s->u[q * n + i];
  for (int32_t w = 0; w < s->n_walls && nh < 3; ++w) {
    const wall_t* W = &s->walls[w];
    int in = 1;
    for (int q = 0; q < 3; ++q)
      if (p[q] < W->lo[q] || p[q] > W->hi[q]) in = 0;
    if (!in) continue;
    double d = (W->n[0] * p[0] + W->n[1] * p[1]) + W->n[2] * p[2] - W->offset;
    if (!(d < Rc) || d <= -Rc) continue;
    hit[nh] = w;
    dl[nh] = d;
    ++nh;
  }
  if (nh < 2) return;
  const int32_t g = s->grain_of[i];
  const double Kn = pdref_contact_stiffness(s->gK[g], s->gK[g], s->eps);
  int orth[3][3];
  for (int x = 0; x < nh; ++x)
    for (int y = 0; y < nh; ++y) {
      const double* a = s->walls[hit[x]].n;
      const double* b = s->walls[hit[y]].n;
      orth[x][y] = fabs((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) < 1e-12;
    }
  /* terms: the pairs (minus) and the triple (plus) */
  for (int x = 0; x < nh; ++x)
    for (int y = x + 1; y < nh; ++y)
      for (int z = y + 1; z <= nh; ++z) {
        const int triple = z < nh;
        if (!orth[x][y] || (triple && (!orth[x][z] || !orth[y][z]))) continue;
        if (!triple && z != nh) continue;
        const int m[3] = {x, y, triple ? z : -1};
        double vol, cen[3];
        pdref_corner_region(Rc, dl[x], dl[y], triple ? dl[z] : -INFINITY, &vol, cen);
        if (!(vol > 0.0)) continue;
        /* c - p along the outward directions t_l = -n_l */
        double cp[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < (triple ? 3 : 2); ++k)
          for (int q = 0; q < 3; ++q) cp[q] -= cen[k] * s->walls[hit[m[k]]].n[q];
        const double ell = sqrt((cp[0] * cp[0] + cp[1] * cp[1]) + cp[2] * cp[2]);
        if (!(ell > 0.0)) continue;
        const double sign = triple ? 1.0 : -1.0;
        for (int k = 0; k < (triple ? 3 : 2); ++k) {
          const double* nl = s->walls[hit[m[k]]].n;
          /* F_S . n_l with F_S = -K_n (R_c - ell) vol cp / ell */
          const double fn = -Kn * (Rc - ell) * vol * ((cp[0] * nl[0] + cp[1] * nl[1]) + cp[2] * nl[2]) / ell;
          corr[hit[m[k]] * n + i] += sign * fn;
        }
      }
}

/* bond memory of the pair: 1 when j is in i's bond row and that bond is intact */
static int bond_intact(const pdref* s, int64_t i, int64_t j) {
  for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e)
    if (s->col[e] == j) return !s->broken[e];
  return 0;
}

/* reference distance |X_j - X_i| */
static double self_ref_length(const pdref* s, int64_t i, int64_t j) {
  const int64_t n = s->n;
  double xi[3];
  for (int q = 0; q < 3; ++q) xi[q] = s->X[q * n + j] - s->X[q * n + i];
  return sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
}

static int eval_force(pdref* s) {
  const int64_t n = s->n;
  const double Rc = s->Rc;
  double margin = INFINITY;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(min : margin) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t g = s->grain_of[i];
    const double c = s->gc[g], s0 = s->gs0[g];
    double Fi[3] = {0.0, 0.0, 0.0};
    /* peridynamic bond force with bond memory, Sec. 3.1.1 eq. (peri-damage) */
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      if (s->broken[e]) continue;
      const int64_t j = s->col[e];
      const double Vj = s->gV[s->grain_of[j]];
      double xi[3], eta[3], y[3];
      for (int q = 0; q < 3; ++q) {
        xi[q] = s->X[q * n + j] - s->X[q * n + i];
        eta[q] = s->u[q * n + j] - s->u[q * n + i];
        y[q] = xi[q] + eta[q];
      }
      double l0 = sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
      double l = sqrt((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]);
      double st = stretch(xi, eta, l0, l);
      const int absr = (s->flags & PDREF_ABS_STRETCH) != 0;
      /* how far this evaluation's break decision is from the threshold, relative
         to s0: |s/s0 - 1| for the tension test, ||s|/s0 - 1| for the |s| test;
         recorded at every evaluation, the one that breaks the bond included */
      double r = fabs((absr ? fabs(st) : st) / s0 - 1.0);
      if (r < s->margin[e]) s->margin[e] = r;
      if (r < margin) margin = r;
      int over = absr ? (fabs(st) > s0) : (st > s0);
      if (over) {
        s->broken[e] = 1;
        continue;
      }
      double coef = c * bond_weight(s, g, l0) * st * Vj / l;
      for (int q = 0; q < 3; ++q) Fi[q] += coef * y[q];
    }
    /* repulsive contact with nodes of other grains, Sec. 3.2, and with nodes of
       the same grain that have no intact bond to i, Sec. 5 (R18) */
    for (int64_t e = s->cand_ptr[i]; e < s->cand_ptr[i + 1]; ++e) {
      const int64_t j = s->cand[e];
      double y[3];
      double d2 = pair_dist2(s, i, j, y);
      if (!(d2 < Rc * Rc)) continue;
      double d = sqrt(d2);
      if (d == 0.0) continue;
      const int32_t gj = s->grain_of[j];
      double Kn = pdref_contact_stiffness(s->gK[g], s->gK[gj], s->eps);
      double fr = Kn * (Rc - d) * s->gV[gj]; /* repulsive force density, along -y/d */
      if (gj == g) {
        if (bond_intact(s, i, j)) continue;
        double l0 = self_ref_length(s, i, j);
        if (l0 < Rc) {
          if (!(d < l0)) continue;
          fr = Kn * Rc * (l0 - d) / l0 * s->gV[gj];
        }
      }
      double coef = -fr / d;
      if (s->beta > 0.0) {
        /* normal damping, Sec. 3.4 (linear reading): -beta (w . e) e V_j with w the
           velocity of i relative to j and e = y/d pointing from i to j */
        double w = 0.0;
        for (int q = 0; q < 3; ++q) w += (s->vh[q * n + i] - s->vh[q * n + j]) * y[q];
        coef -= s->beta * s->gV[gj] * w / d2;
      }
      for (int q = 0; q < 3; ++q) Fi[q] += coef * y[q];
      if (s->mu > 0.0) {
        /* stick-slip friction, Sec. 3.3: the tangential part of the velocity of i
           relative to j, against the repulsive force density K_n (R_c - d) V_j */
        double e[3], w[3], wt[3], wn = 0.0;
        for (int q = 0; q < 3; ++q) {
          e[q] = y[q] / d;
          w[q] = s->vh[q * n + i] - s->vh[q * n + j];
          wn += w[q] * e[q];
        }
        for (int q = 0; q < 3; ++q) wt[q] = w[q] - wn * e[q];
        add_friction(s->mu, fr, s->grho[g], s->dt, wt, Fi);
      }
    }
    for (int q = 0; q < 3; ++q) {
      s->F[q * n + i] = Fi[q];
      if (isnan(Fi[q]) || isinf(Fi[q])) bad = 1;
    }
  }
  if (margin < s->min_margin) s->min_margin = margin;
  /* several walls at a corner (Sec. 4.1.1, R19): corrections of the normal
     magnitude each wall applies to each node */
  double* corr = NULL;
  if ((s->flags & PDREF_WALL_CORNERS) && s->n_walls > 1) {
    corr = (double*)calloc((size_t)(s->n_walls * n), sizeof(double));
    for (int64_t i = 0; i < n; ++i) wall_corners(s, i, corr);
  }
  /* rigid walls, Sec. 4.1 (sequential pass so the reaction sum runs in ascending i) */
  for (int32_t w = 0; w < s->n_walls; ++w) {
    wall_t* W = &s->walls[w];
    W->force[0] = W->force[1] = W->force[2] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double p[3];
      for (int q = 0; q < 3; ++q) p[q] = s->X[q * n + i] + s->u[q * n + i];
      int in = 1;
      for (int q = 0; q < 3; ++q)
        if (p[q] < W->lo[q] || p[q] > W->hi[q]) in = 0;
      if (!in) continue;
      double d = (W->n[0] * p[0] + W->n[1] * p[1]) + W->n[2] * p[2] - W->offset;
      if (!(d < Rc)) continue;
      if (d <= -Rc) {
        bad = 1;
        continue;
      }
      const int32_t g = s->grain_of[i];
      double Kn = pdref_contact_stiffness(s->gK[g], s->gK[g], s->eps);
      double vol, ell;
      pdref_wall_cap(Rc, d, &vol, &ell);
      /* -K_n (R_c - |c_l - p|) |S_l| e_l with e_l = -n (towards the wall) */
      double mag = Kn * (Rc - ell) * vol;
      if (corr) mag += corr[w * n + i];
      if (s->beta > 0.0) {
        /* damping against the wall (Sec. 4.1 with V_y -> |S_l|): the relative
           normal velocity is v . n minus the wall's own rate along n */
        double vn = (W->n[0] * s->vh[i] + W->n[1] * s->vh[n + i]) + W->n[2] * s->vh[2 * n + i];
        mag -= s->beta * (vn - W->rate) * vol;
      }
      double f[3];
      for (int q = 0; q < 3; ++q) f[q] = mag * W->n[q];
      if (s->mu > 0.0) {
        /* friction against the wall (Sec. 4.1 with V_y -> |S_l|): the partner moves
           with the wall's rate along n, so only v's tangential part counts */
        double w[3], wt[3], wn = 0.0;
        for (int q = 0; q < 3; ++q) {
          w[q] = s->vh[q * n + i] - W->rate * W->n[q];
          wn += w[q] * W->n[q];
        }
        for (int q = 0; q < 3; ++q) wt[q] = w[q] - wn * W->n[q];
        add_friction(s->mu, Kn * (Rc - ell) * vol, s->grho[g], s->dt, wt, f);
      }
      for (int q = 0; q < 3; ++q) {
        s->F[q * n + i] += f[q];
        W->force[q] -= s->gV[g] * f[q];
      }
    }
  }
  free(corr);
  return bad;
}

static void set_accel(pdref* s, double* a) {
  const int64_t n = s->n;
  for (int64_t i = 0; i < n; ++i) {
    const double rho = s->grho[s->grain_of[i]];
    for (int q = 0; q < 3; ++q) a[q * n + i] = s->fixed[i] ? 0.0 : s->F[q * n + i] / rho + s->g[q];
  }
}

/* wall positions at the current step (prescribed or servo) */
static void advance_walls(pdref* s) {
  const double t = (double)s->step * s->dt;
  for (int32_t w = 0; w < s->n_walls; ++w) {
    wall_t* W = &s->walls[w];
    if (W->mode == 1) {
      W->offset = W->offset0 + W->velocity * t;
      W->rate = W->velocity;
    } else if (W->mode == 2) {
      /* servo: stress from the previous step's reaction; move into the domain when low */
      double sigma = -((W->force[0] * W->n[0] + W->force[1] * W->n[1]) + W->force[2] * W->n[2]) / W->area;
      W->rate = W->gain * (W->target - sigma);
      W->offset += s->dt * W->rate;
    }
  }
}

static int skin_exceeded(const pdref* s) {
  const int64_t n = s->n;
  const double lim2 = 0.25 * s->skin * s->skin;
  for (int64_t i = 0; i < n; ++i) {
    double d[3];
    for (int q = 0; q < 3; ++q) d[q] = s->u[q * n + i] - s->u_at_build[q * n + i];
    if ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] > lim2) return 1;
  }
  return 0;
}

int32_t pdref_build(pdref* s) {
  build_bonds(s);
  build_candidates(s);
  s->step = 0;
  /* the first evaluation sees the initial velocity (zero on fixed nodes) */
  for (int64_t i = 0; i < s->n; ++i)
    for (int q = 0; q < 3; ++q) s->vh[q * s->n + i] = s->fixed[i] ? 0.0 : s->v[q * s->n + i];
  int bad = eval_force(s);
  set_accel(s, s->a);
  for (int64_t i = 0; i < s->n; ++i)
    if (s->fixed[i])
      for (int q = 0; q < 3; ++q) s->v[q * s->n + i] = 0.0;
  s->built = 1;
  return bad ? -5 : 0;
}

int32_t pdref_step(pdref* s, int64_t nsteps) {
  const int64_t n = s->n;
  const double dt = s->dt, hdt2 = 0.5 * dt * dt;
  double* anew = (double*)malloc(sizeof(double) * (size_t)(3 * n + 1));
  int bad = 0;
  for (int64_t k = 0; k < nsteps && !bad; ++k) {
    /* Sec. 6.2: positions from the current velocity and acceleration */
    for (int64_t i = 0; i < n; ++i) {
      if (s->fixed[i]) continue;
      for (int q = 0; q < 3; ++q)
        s->u[q * n + i] = s->u[q * n + i] + dt * s->v[q * n + i] + hdt2 * s->a[q * n + i];
    }
    s->step += 1;
    advance_walls(s);
    /* the skin guard protects contact pairs; a single grain without
       self-contact has none to miss */
    const int contacts = s->n_grains > 1 || (s->flags & PDREF_SELF_CONTACT);
    const int adaptive = (s->flags & PDREF_ADAPTIVE_REBUILD) != 0;
    if (s->step % s->rebuild_every == 0) {
      if (contacts && !adaptive && skin_exceeded(s)) bad = 1;
      build_candidates(s);
    } else if (contacts && adaptive && skin_exceeded(s)) {
      build_candidates(s); /* the list may miss a pair within R_c at these positions */
      s->early_rebuilds += 1;
    }
    /* new accelerations at the new positions, then the velocity update; the
       damping law sees the mid-step velocity v_n + dt/2 a_n */
    for (int64_t k3 = 0; k3 < 3 * n; ++k3) s->vh[k3] = s->v[k3] + 0.5 * dt * s->a[k3];
    bad |= eval_force(s);
    for (int32_t w = 0; w < s->n_walls; ++w)
      for (int q = 0; q < 3; ++q) s->walls[w].impulse[q] += s->walls[w].force[q] * dt;
    set_accel(s, anew);
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < 3; ++q) {
        const int64_t k3 = q * n + i;
        s->v[k3] = s->fixed[i] ? 0.0 : s->v[k3] + 0.5 * dt * (s->a[k3] + anew[k3]);
        s->a[k3] = anew[k3];
      }
  }
  free(anew);
  return bad ? -5 : 0;
}

/* ------------------------------------------------------------------------- */
/* queries                                                                   */
/* ------------------------------------------------------------------------- */

int64_t pdref_nnz(const pdref* s) { return s->row_ptr ? s->row_ptr[s->n] : 0; }
int64_t pdref_step_count(const pdref* s) { return s->step; }

void pdref_get_bonds(const pdref* s, int64_t* row_ptr, int32_t* col, uint8_t* broken) {
  int64_t nnz = pdref_nnz(s);
  if (row_ptr) memcpy(row_ptr, s->row_ptr, sizeof(int64_t) * (size_t)(s->n + 1));
  if (col) memcpy(col, s->col, sizeof(int32_t) * (size_t)nnz);
  if (broken) memcpy(broken, s->broken, (size_t)nnz);
}

void pdref_get_state(const pdref* s, double* u, double* v, double* a, double* F) {
  size_t b = sizeof(double) * (size_t)(3 * s->n);
  if (u) memcpy(u, s->u, b);
  if (v) memcpy(v, s->v, b);
  if (a) memcpy(a, s->a, b);
  if (F) memcpy(F, s->F, b);
}

void pdref_get_damage(const pdref* s, double* damage, int32_t* intact, int32_t* n0) {
  for (int64_t i = 0; i < s->n; ++i) {
    int32_t cnt = 0;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) cnt += !s->broken[e];
    if (intact) intact[i] = cnt;
    if (n0) n0[i] = s->n0[i];
    if (damage) damage[i] = s->n0[i] > 0 ? 1.0 - (double)cnt / (double)s->n0[i] : 0.0;
  }
}

void pdref_get_walls(const pdref* s, double* force, double* offset) {
  for (int32_t w = 0; w < s->n_walls; ++w) {
    for (int q = 0; q < 3; ++q)
      if (force) force[3 * w + q] = s->walls[w].force[q];
    if (offset) offset[w] = s->walls[w].offset;
  }
}

void pdref_get_wall_impulse(const pdref* s, double* impulse) {
  for (int32_t w = 0; w < s->n_walls; ++w)
    for (int q = 0; q < 3; ++q) impulse[3 * w + q] = s->walls[w].impulse[q];
}

int64_t pdref_n_candidates(const pdref* s) { return s->cand_ptr ? s->cand_ptr[s->n] : 0; }

void pdref_get_candidates(const pdref* s, int64_t* row_ptr, int32_t* col) {
  if (row_ptr) memcpy(row_ptr, s->cand_ptr, sizeof(int64_t) * (size_t)(s->n + 1));
  if (col) memcpy(col, s->cand, sizeof(int32_t) * (size_t)pdref_n_candidates(s));
}

void pdref_energy_density(const pdref* s, double* W) {
  const int64_t n = s->n;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t g = s->grain_of[i];
    double acc = 0.0;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      if (s->broken[e]) continue;
      const int64_t j = s->col[e];
      double xi[3], eta[3], y[3];
      for (int q = 0; q < 3; ++q) {
        xi[q] = s->X[q * n + j] - s->X[q * n + i];
        eta[q] = s->u[q * n + j] - s->u[q * n + i];
        y[q] = xi[q] + eta[q];
      }
      double l0 = sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
      double l = sqrt((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]);
      double st = stretch(xi, eta, l0, l);
      /* micropotential 1/2 c s^2 |xi| per unit volume squared */
      acc += 0.5 * s->gc[g] * bond_weight(s, g, l0) * st * st * l0 * s->gV[s->grain_of[j]];
    }
    W[i] = 0.5 * acc;
  }
}

void pdref_energy(const pdref* s, double* out4) {
  const int64_t n = s->n;
  double ke = 0.0, el = 0.0, ct = 0.0, gp = 0.0;
  double* W = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  pdref_energy_density(s, W);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t g = s->grain_of[i];
    const double V = s->gV[g], rho = s->grho[g];
    double v2 = 0.0;
    for (int q = 0; q < 3; ++q) v2 += s->v[q * n + i] * s->v[q * n + i];
    ke += 0.5 * rho * V * v2;
    el += V * W[i];
    for (int q = 0; q < 3; ++q) gp -= rho * V * s->g[q] * s->u[q * n + i];
    for (int64_t e = s->cand_ptr[i]; e < s->cand_ptr[i + 1]; ++e) {
      const int64_t j = s->cand[e];
      double y[3];
      double d2 = pair_dist2(s, i, j, y);
      if (!(d2 < s->Rc * s->Rc)) continue;
      double d = sqrt(d2);
      const int32_t gj = s->grain_of[j];
      double Kn = pdref_contact_stiffness(s->gK[g], s->gK[gj], s->eps);
      /* pair potential 1/2 K_n (R_c - d)^2, each pair seen from both ends; the
         repulsive-only bond of a short same-grain pair 1/2 K_n R_c (|xi| - d)^2 / |xi| */
      double pot = 0.5 * Kn * (s->Rc - d) * (s->Rc - d);
      if (gj == g) {
        if (bond_intact(s, i, j)) continue;
        double l0 = self_ref_length(s, i, j);
        if (l0 < s->Rc) pot = d < l0 ? 0.5 * Kn * s->Rc * (l0 - d) * (l0 - d) / l0 : 0.0;
      }
      ct += 0.5 * V * pot * s->gV[gj];
    }
  }
  free(W);
  out4[0] = ke;
  out4[1] = el;
  out4[2] = ct;
  out4[3] = gp;
}

double pdref_min_margin(const pdref* s) { return s->min_margin; }

void pdref_bond_margin(const pdref* s, double* out) {
  const int64_t nnz = pdref_nnz(s);
  if (out && nnz > 0) memcpy(out, s->margin, sizeof(double) * (size_t)nnz);
}

int32_t pdref_skin_exceeded(const pdref* s) { return skin_exceeded(s); }
int64_t pdref_early_rebuilds(const pdref* s) { return s->early_rebuilds; }

void pdref_set_u(pdref* s, const double* u) {
  memcpy(s->u, u, sizeof(double) * (size_t)(3 * s->n));
  build_candidates(s);
}

void pdref_rebuild_candidates(pdref* s) { build_candidates(s); }
