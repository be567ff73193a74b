/*
 * pdref.h -- plain FP64 CPU oracle of the explicit peridynamic grain-aggregate step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this code; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source with the HIP library.
 *
 * What it computes (the paper's method, in the paper's order):
 *   - bond family: same-grain lattice neighbours with 0 < |d ijk|^2 <= m^2
 *     (horizon delta = m h, Sec. 3.1 eq. (peri)); bonds removed by notch planes
 *     (Sec. 6.3.1) and cavities (Sec. 6.3.2);
 *   - PMB bond force c s (xi+eta)/|xi+eta| with irreversible breaking when the
 *     stretch exceeds s0 (Sec. 3.1 eq. (pmb), Sec. 3.1.1 bond memory gamma,
 *     eq. (peri-damage)), nodal quadrature V_j = h^3 (Sec. 6.1);
 *   - damage 1 - intact/initial (Sec. 3.1.1);
 *   - repulsive contact -K_n (R_c - |p_y - p_x|) e between nodes of different
 *     grains (Sec. 3.2 eq. (repulsive-force)), K_n = 18 k / (pi eps^5) with the
 *     harmonic-mean bulk modulus; with PDREF_SELF_CONTACT the same law (and a
 *     repulsive-only bond for pairs shorter than R_c) between nodes of one grain
 *     that have no intact bond (Sec. 5);
 *   - normal contact damping (Sec. 3.4 eq. (damping-force)) and regularised
 *     stick-slip friction (Sec. 3.3 eq. (regularized-friction)) on the mid-step
 *     velocity, between grains and against walls;
 *   - rigid planar walls, spherical-cap law (Sec. 4.1), walls summed (Sec. 4.1.1);
 *   - body force (Sec. 5.1 eq. (intra_particle)) and velocity Verlet (Sec. 6.2).
 *
 * Arrays are SoA: a (3,N) field is x[0..N), y[N..2N), z[2N..3N).
 * Compile with -O2 -fno-fast-math -ffp-contract=off.
 */
#ifndef PDREF_H
#define PDREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flags */
#define PDREF_TABLE_LITERAL 1 /* 3-D constants exactly as printed in the paper's table */
#define PDREF_ABS_STRETCH 2   /* break when |s| > s0 (the paper's prose) instead of s > s0 */
#define PDREF_CELL_LIST 4     /* contact candidates from a cell list instead of an O(N^2) scan */
#define PDREF_CONIC 8         /* conic micromodulus c0 (1 - |xi|/delta) instead of a constant one */
#define PDREF_SELF_CONTACT 16 /* contact between nodes of one grain with no intact bond (Sec. 5) */
#define PDREF_WALL_CORNERS 32 /* inclusion-exclusion of orthogonal walls at a corner (Sec. 4.1.1) */
#define PDREF_ADAPTIVE_REBUILD 64 /* rebuild the contact candidates before any evaluation at which a
                                     node has moved more than skin/2 since the last rebuild */

/* packed wall record (15 doubles):
 *   nx ny nz offset velocity lox loy loz hix hiy hiz mode target_stress servo_gain area */
#define PDREF_WALL_DOUBLES 15
/* packed cut record (16 int64):
 *   kind grain a b c d lox loy loz hix hiy hiz cx cy cz radius2     (half-lattice units) */
#define PDREF_CUT_INTS 16
/* params (11 doubles): m R_c eps skin rebuild_every dt gx gy gz beta_d mu */
#define PDREF_PARAM_DOUBLES 11

typedef struct pdref pdref;

/* 3-D micromodulus constants: c [N/m^6] (c0 of the conic form with PDREF_CONIC) and s0 */
void pdref_constants(double K, double Gc, double delta, int32_t flags, double* c, double* s0);
/* K_n = 18 k_eff / (pi eps^5), k_eff = 2 k_a k_b / (k_a + k_b) */
double pdref_contact_stiffness(double k_a, double k_b, double eps);
/* spherical cap of B_Rc(p) beyond a plane at signed distance d: volume and centroid distance */
void pdref_wall_cap(double Rc, double d, double* volume, double* centroid);
/* volume and centroid (coordinates along the three plane normals) of the part
   of the ball |x| < R with x_u > a, x_v > b and x_w > c (c = -INFINITY: two planes) */
void pdref_corner_region(double R, double a, double b, double c, double* volume, double centroid[3]);

pdref* pdref_create(int64_t n, const double* X, const int32_t* ijk, const double* u0,
                    const double* v0, const uint8_t* fixed, int32_t n_grains,
                    const int64_t* grain_begin, const int32_t* grain_material,
                    const double* grain_h, int32_t n_mat, const double* mat /* K rho Gc */,
                    const double* params, int32_t n_walls, const double* walls, int32_t n_cuts,
                    const int64_t* cuts, int32_t flags);
void pdref_destroy(pdref* s);
/* bonds, initial candidates, F^0 and a^0; returns 0 or -5 (unstable) */
int32_t pdref_build(pdref* s);
/* n velocity-Verlet steps; returns 0, or -5 when a step flagged an instability */
int32_t pdref_step(pdref* s, int64_t n);
void pdref_set_threads(int32_t n);

int64_t pdref_nnz(const pdref* s);
int64_t pdref_step_count(const pdref* s);
void pdref_get_bonds(const pdref* s, int64_t* row_ptr, int32_t* col, uint8_t* broken);
void pdref_get_state(const pdref* s, double* u, double* v, double* a, double* F);
void pdref_get_damage(const pdref* s, double* damage, int32_t* intact, int32_t* n0);
void pdref_get_walls(const pdref* s, double* force /* [n_walls][3] */, double* offset);
/* time integral of each wall's reaction: sum over completed steps of P_w dt */
void pdref_get_wall_impulse(const pdref* s, double* impulse /* [n_walls][3] */);
int64_t pdref_n_candidates(const pdref* s);
void pdref_get_candidates(const pdref* s, int64_t* row_ptr, int32_t* col);
/* energies: kinetic, elastic (bonds), contact, gravity potential */
void pdref_energy(const pdref* s, double* out4);
/* Break-decision margin of a bond: the minimum, over every evaluation of the
   bond (the one that breaks it included), of |s/s0 - 1| (with
   PDREF_ABS_STRETCH: ||s|/s0 - 1|).  A bond whose margin exceeds a tolerance
   took every break decision with that much room on either side.
   pdref_bond_margin fills [nnz] (aligned with the bond columns, +inf for a
   bond never evaluated); pdref_min_margin is the minimum over all bonds. */
double pdref_min_margin(const pdref* s);
void pdref_bond_margin(const pdref* s, double* out);
/* 1 when some node moved more than skin/2 since the last candidate rebuild
   (the guard pdref_step applies at each rebuild when contacts can exist, or
   before every evaluation with PDREF_ADAPTIVE_REBUILD, which rebuilds then) */
int32_t pdref_skin_exceeded(const pdref* s);
/* candidate rebuilds PDREF_ADAPTIVE_REBUILD added between the cadence ones */
int64_t pdref_early_rebuilds(const pdref* s);
/* overwrite u (tests compare lists on identical positions) and rebuild candidates */
void pdref_set_u(pdref* s, const double* u);
/* recompute the candidate list from the current u */
void pdref_rebuild_candidates(pdref* s);
/* per-node strain energy density W_i = 1/2 sum_j 1/2 c s^2 |xi| V_j at the current u */
void pdref_energy_density(const pdref* s, double* W);

#ifdef __cplusplus
}
#endif
#endif
