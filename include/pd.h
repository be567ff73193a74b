/*
 * pd.h -- C ABI of the MI355X peridynamic grain-aggregate library.
 *
 * One explicit-dynamics step of bond-based peridynamics for lattice-meshed
 * grains (arxiv 2506.05362):
 *   - bond force c s (xi+eta)/|xi+eta| over the horizon family of each node,
 *     with irreversible breaking when the stretch exceeds s0 and damage
 *     (Sec. 3.1 eq. (pmb), Sec. 3.1.1 eq. (peri-damage));
 *   - repulsive contact -K_n (R_c - |p_y - p_x|) e(y,x) from nodes of other
 *     grains (Sec. 3.2 eq. (repulsive-force)), found by a cell-list search;
 *   - rigid planar walls with the spherical-cap law (Sec. 4.1), several walls
 *     summed (Sec. 4.1.1); body force (Sec. 5.1 eq. (intra_particle));
 *   - velocity Verlet (Sec. 6.2).
 * The problem statement the calls follow is Sec. 2.1 (grains P_i, material
 * points x with displacement u, initial data u0, v0) and Sec. 5.1 (equation of
 * motion with F_int = F_intra + F_inter and F_ext = F_wall + b).
 *
 * Conventions shared by every call:
 *   - a "(3,N) field" is SoA FP64: x[0..N), y[N..2N), z[2N..3N);
 *   - nodes are grouped by grain; node n of grain g sits at
 *     X = origin[g] + h[g] * ijk[n] with grain-local lattice indices 0..1023;
 *   - the nodal volume is h[g]^3 (nodal quadrature, Sec. 6.1);
 *   - lengths in m, forces per volume in N/m^3, time in s.
 *
 * Ownership: every pointer passed in is caller-owned, read during the call
 * only and never retained.  The library owns its device buffers; it allocates
 * them through the caller's allocator callback (or hipMalloc when none is
 * given) and enqueues all work on the caller's HIP stream.
 *
 * Errors: every call returns a pd_status; no exception crosses the ABI.  A
 * per-context last-error string carries details.  Call order is
 * pd_init -> pd_build_bonds -> (pd_step | pd_get | pd_set_wall | state)*;
 * other orders return PD_ERR_STATE.  A context is single-threaded.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pd_status;
enum {
  PD_OK = 0,
  PD_ERR_INVALID = -1,     /* bad argument; details in pd_last_error */
  PD_ERR_STATE = -2,       /* call out of order */
  PD_ERR_OOM = -3,         /* allocation failed */
  PD_ERR_HIP = -4,         /* a HIP runtime call failed */
  PD_ERR_UNSTABLE = -5,    /* NaN/Inf force, wall penetration (d <= -R_c), Verlet skin
                              exceeded, or contact-candidate capacity exceeded */
  PD_ERR_UNSUPPORTED = -6, /* valid request the library does not implement */
  PD_ERR_CORRUPT = -7      /* checkpoint blob failed its size/magic/CRC check */
};

typedef struct pd_ctx pd_ctx;

/* Device allocator hooks (for example PyTorch's caching allocator).  alloc
   returns device memory of at least `bytes` bytes or NULL; free releases it. */
typedef void* (*pd_alloc_fn)(size_t bytes, void* user);
typedef void (*pd_free_fn)(void* ptr, void* user);

typedef struct {
  double bulk_modulus;    /* K [Pa]; Poisson ratio is 1/4 in bond-based PD (Sec. 3.1.1) */
  double density;         /* rho [kg/m^3] */
  double fracture_energy; /* G_c [J/m^2], sets the critical stretch (Sec. 3.1.1) */
} pd_material;

typedef struct {
  int32_t n_grains;
  const int64_t* node_begin; /* [n_grains+1]: grain g owns nodes [node_begin[g], node_begin[g+1]) */
  const int32_t* material;   /* [n_grains] index into the material table */
  const double* h;           /* [n_grains] lattice spacing > 0 */
  const double* origin;      /* (3, n_grains) SoA lattice origin */
} pd_grains;

typedef struct {
  int64_t n_nodes;
  const double* X;      /* (3,N) reference positions; must equal origin + h*ijk to 1e-9 h */
  const int32_t* ijk;   /* (3,N) grain-local lattice indices in [0, 1023] */
  const double* u0;     /* (3,N) initial displacement, or NULL for zero */
  const double* v0;     /* (3,N) initial velocity, or NULL for zero */
  const uint8_t* fixed; /* [N] nonzero = node keeps its displacement and has v = a = 0; or NULL */
} pd_mesh;

enum { PD_FLAG_TABLE_LITERAL = 1, /* use the printed 3-D table row for c and s0 */
       PD_FLAG_ABS_STRETCH = 2,   /* break on |s| > s0 instead of s > s0 */
       PD_FLAG_NO_GRAPH = 4,      /* launch every step's kernels directly instead of replaying
                                     a captured HIP graph of rebuild_every steps */
       PD_FLAG_CONIC = 8,         /* conic micromodulus c0 (1 - |xi|/delta) (the table's second row,
                                     Sec. 3.1.1): c0 = 90K/(pi delta^4), s0 = sqrt(2 G_c/(3 K delta)),
                                     the values for which a uniform stretch has energy 9Ks^2/2 and
                                     breaking the bonds across a unit area costs G_c; with
                                     PD_FLAG_TABLE_LITERAL the printed row */
       PD_FLAG_SELF_CONTACT = 16, /* self-contact (Sec. 5): nodes of one grain with no intact bond
                                     repel as nodes of different grains do (K_n (R_c - d) V_j with
                                     damping and friction).  The contact candidates then include the
                                     node's own grain; a pair whose bond is intact at the evaluation
                                     is skipped.  Requires contact_radius below every grain's
                                     lattice spacing (so no pair is shorter than R_c), else
                                     PD_ERR_INVALID; the skin guard then applies to a single grain
                                     too */
       PD_FLAG_WALL_CORNERS = 32, /* several walls (Sec. 4.1.1): a node touching two or three mutually
                                     orthogonal walls (a box edge or corner) gets the inclusion-exclusion
                                     sum F_l + F_l' - F_ll' (+ ...) of terms -K_n (R_c - |c_S - p|) |S| e_S
                                     over the parts S of its contact ball beyond the walls, volumes and
                                     centroids integrated numerically; each wall's reaction takes the
                                     corrections' components along its normal.  Damping and friction stay
                                     per wall; walls that are not orthogonal are summed.  A small pass
                                     before each evaluation finds the corner nodes; PD_LOOP_PERSISTENT
                                     is then refused (PD_ERR_UNSUPPORTED) */
       PD_FLAG_ADAPTIVE_REBUILD = 64 /* early candidate rebuilds (contact set, Sec. 3.2): before every
                                     evaluation between cadence rebuilds a pass checks every node's
                                     displacement since the last rebuild; once one exceeds skin/2
                                     that step is not taken, the candidates are rebuilt at those
                                     positions and pd_step goes on from the same step, so the skin
                                     error never arises and the result is that of a rebuild before
                                     every evaluation.  Costs one pass per step (56 bytes per node)
                                     and a status read after each captured run of steps;
                                     PD_LOOP_PERSISTENT is refused (PD_ERR_UNSUPPORTED) */ };

typedef struct {
  int32_t horizon_factor;  /* m: horizon delta = m h; bonds are same-grain pairs with
                              0 < |d ijk|^2 <= m^2 (1 <= m <= 6) */
  int32_t flags;           /* PD_FLAG_* */
  double contact_radius;   /* R_c [m] (Sec. 3.2) */
  double contact_horizon;  /* eps in K_n = 18 k / (pi eps^5) [m] */
  double skin;             /* Verlet skin [m]: candidates are other-grain nodes (with
                              PD_FLAG_SELF_CONTACT also same-grain nodes) within R_c + skin */
  int32_t rebuild_every;   /* candidate rebuild cadence in steps (>= 1) */
  int32_t candidate_capacity_per_node; /* candidate list capacity: N times this in total and
                                          twice this for any one node (0 = 16, or 48 with
                                          PD_FLAG_SELF_CONTACT); exceeding either raises
                                          PD_ERR_UNSTABLE */
  double dt;               /* time step [s] */
  double gravity[3];       /* body force per unit mass [m/s^2] */
  double contact_damping;  /* beta_d of the normal damping law (Sec. 3.4) [N s/m^7], >= 0;
                              0 disables it.  Between nodes of different grains within R_c
                              the force density on i is -beta_d (w . e) e V_j, w = velocity of
                              i relative to j, e the unit vector from i to j; against a wall
                              -beta_d (v . n - wall rate) |S| n.  Velocities are the mid-step
                              values v_n + dt/2 a_n (v_0 in the first evaluation). */
  double friction;         /* mu of the regularised stick-slip friction law (Sec. 3.3), >= 0;
                              0 disables it.  Per contact pair, with w_t the tangential part
                              of i's mid-step velocity relative to its partner (a wall moves
                              only along its normal), f_r the repulsive force density the
                              partner exerts on i (K_n (R_c - d) V_j, or K_n (R_c - |c - p|) |S|
                              for a wall) and rho i's density: slip, -mu f_r w_t/|w_t|, when
                              |w_t| > mu f_r dt / rho; stick, -(rho/dt) w_t, otherwise. */
} pd_params;

enum { PD_WALL_FIXED = 0, PD_WALL_VELOCITY = 1, PD_WALL_SERVO = 2 };

typedef struct {
  double normal[3];      /* unit normal pointing into the domain */
  double offset;         /* wall plane at t = 0: n . p = offset */
  double velocity;       /* PD_WALL_VELOCITY: offset(t) = offset + velocity * t */
  double lo[3], hi[3];   /* patch: node acted on only if lo <= p <= hi componentwise */
  int32_t mode;          /* PD_WALL_* */
  double target_stress;  /* PD_WALL_SERVO: target of sigma = -(P . n) / area [Pa] */
  double servo_gain;     /* PD_WALL_SERVO: d(offset)/dt = gain * (target - sigma) [m/s/Pa] */
  double area;           /* area that turns the reaction force into a stress [m^2] */
} pd_wall;

enum { PD_CUT_NOTCH = 0, PD_CUT_CAVITY_ENDPOINT = 1, PD_CUT_CAVITY_CHORD = 2 };

/* Bond removal (Sec. 6.3).  Coordinates are half-lattice integers of the grain:
   node ijk sits at (2i, 2j, 2k).  |lo|, |hi| >= 2^50 mean "unbounded".
   NOTCH: remove the bond P1->P2 when the plane a X + b Y + c Z + d = 0 cuts it
          at 0 < t < 1 and the crossing point lies in [lo, hi] (Sec. 6.3.1).
   CAVITY_ENDPOINT: remove when an endpoint is strictly inside the sphere (Sec. 6.3.2).
   CAVITY_CHORD: remove when the segment passes strictly inside the sphere. */
typedef struct {
  int32_t kind;
  int32_t grain;
  int64_t plane[4];
  int64_t lo[3], hi[3];
  int64_t center[3];
  int64_t radius2;
} pd_cut;

typedef enum {
  PD_DISPLACEMENT = 0,    /* (3,N) f64 u */
  PD_VELOCITY = 1,        /* (3,N) f64 v */
  PD_ACCEL = 2,           /* (3,N) f64 a = F/rho + g (0 on fixed nodes) */
  PD_FORCE_DENSITY = 3,   /* (3,N) f64 F = F_intra + F_inter + F_wall at the current u */
  PD_DAMAGE = 4,          /* [N] f64 1 - intact/initial (0 where initial = 0) */
  PD_INTACT_COUNT = 5,    /* [N] i32 intact bonds */
  PD_INITIAL_COUNT = 6,   /* [N] i32 bonds after cuts, before any breaking */
  PD_BOND_ROWPTR = 7,     /* [N+1] i64 CSR row pointer, rows in node order */
  PD_BOND_COL = 8,        /* [nnz] i32 CSR columns, ascending in each row */
  PD_BOND_BROKEN = 9,     /* [nnz] u8 1 = broken, aligned with PD_BOND_COL */
  PD_CONTACT_ROWPTR = 10, /* [N+1] i64 candidate rows of the last rebuild */
  PD_CONTACT_COL = 11,    /* [n_candidates] i32 candidate columns, ascending */
  PD_WALL_FORCE = 12,     /* [n_walls][3] f64 reaction P_w = -sum_i V_i F_wall,i (last evaluation) */
  PD_WALL_OFFSET = 13,    /* [n_walls] f64 wall offset used by the last evaluation */
  PD_ENERGY = 14,         /* [4] f64 kinetic, elastic (bonds), contact, gravity potential [J] */
  PD_STEP = 15,           /* [1] i64 completed steps */
  PD_WALL_IMPULSE = 16    /* [n_walls][3] f64 sum over completed steps of P_w dt: the
                             reaction averaged over steps a..b is (I_b - I_a) / ((b - a) dt) */
} pd_field;

/* Create a context: validates and copies the problem to the device.
   materials[n_mat]; walls[n_walls] (may be NULL when 0); stream = a hipStream_t
   that is not the legacy null stream (graph capture needs a real stream), or
   NULL for a stream the library creates and owns.
   alloc/free may be NULL (then hipMalloc/hipFree are used). */
pd_status pd_init(pd_ctx** out, const pd_grains* grains, const pd_mesh* mesh,
                  const pd_material* materials, int32_t n_mat, const pd_params* params,
                  const pd_wall* walls, int32_t n_walls, pd_alloc_fn alloc, pd_free_fn free_fn,
                  void* alloc_user, void* stream);

/* Build the bond family (Sec. 3.1, inclusive integer horizon shell) minus the cuts,
   the first contact candidate list and the initial force F^0 / acceleration a^0.
   cuts may be NULL when n_cuts == 0. */
pd_status pd_build_bonds(pd_ctx* ctx, const pd_cut* cuts, int32_t n_cuts);

/* Advance n_steps velocity-Verlet steps.  Enqueues on the context stream and
   waits for the device status word at the end.  PD_ERR_UNSTABLE reports a flag
   raised during these steps: the step that raised it completes, the steps
   after it change nothing, and the context is left at that step (PD_STEP and
   every field report it); the flag is cleared once reported.  Chunks of
   rebuild_every steps (doubled when odd) that start on a multiple of that
   length replay one captured HIP graph; the rest launch kernels directly.
   With PD_FLAG_ADAPTIVE_REBUILD the status is read after every such chunk
   (and every run of direct steps up to the next multiple), and an early
   rebuild is not an error. */
pd_status pd_step(pd_ctx* ctx, int64_t n_steps);

/* Bytes a field occupies (for sizing dst). */
pd_status pd_field_bytes(pd_ctx* ctx, pd_field field, int64_t* bytes);

/* Copy a field into dst (host memory, or device memory when dst_on_device != 0).
   dst_bytes smaller than the field gives PD_ERR_INVALID.  Synchronises the stream. */
pd_status pd_get(pd_ctx* ctx, pd_field field, void* dst, int64_t dst_bytes, int32_t dst_on_device);

/* The four energies of PD_ENERGY (kinetic, elastic, contact, gravity potential
   [J]) without allocating: for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   allocation).  Same kernels and summation order as pd_get(PD_ENERGY), so the
   values are the same; the per-workgroup partial sums go to a static device
   array of 4 MiB that the library holds on each GPU until the process ends
   (every context the library accepts, up to 2^25 nodes, fits; a larger one
   would be refused with PD_ERR_INVALID).  out4: 4 doubles in host memory, or
   device memory when out_on_device != 0.  Synchronises the stream.  All
   contexts on one GPU share that array and it keeps the last call's
   contents: calls that overlap on one GPU (contexts on different streams or
   threads) race. */
pd_status pd_energy_noalloc(pd_ctx* ctx, double* out4, int32_t out_on_device);

/* Replace wall w (for example to change a servo target between steps). */
pd_status pd_set_wall(pd_ctx* ctx, int32_t w, const pd_wall* wall);

/* Checkpoint: blob = header, u, v, a, broken bits, intact counts, walls, step
   counters, CRC32.  With blob == NULL, *bytes receives the size needed. */
pd_status pd_get_state(pd_ctx* ctx, void* blob, int64_t* bytes);
/* Restore a checkpoint taken from a context built from the same inputs. */
pd_status pd_set_state(pd_ctx* ctx, const void* blob, int64_t bytes);

/* Measurement hook: with enable != 0, pd_step launches every step directly
   (no graph replay) and brackets each launch of the fused step kernel with a
   pair of HIP events on the context stream.  pd_timing waits for the stream,
   returns the number of bracketed launches and their summed duration in
   milliseconds, and clears the record. */
pd_status pd_set_timing(pd_ctx* ctx, int32_t enable);
pd_status pd_timing(pd_ctx* ctx, int64_t* launches, double* total_ms);

/* Counts: n_nodes, nnz (real bonds), padded slots, candidates, steps. */
pd_status pd_info(pd_ctx* ctx, int64_t* out5);

/* The tiled bond loop's layout: the number of tiles (0 when the tiled loop is
   unavailable) and whether they cover one box over all grains (lattice mode:
   every grain on one lattice with one spacing, bond table and node order). */
pd_status pd_tile_info(pd_ctx* ctx, int64_t* n_tiles, int32_t* lattice);

/* How the steps of this context were launched so far: out6 = graph replays,
   steps run inside them, steps launched directly, persistent launches, steps
   run inside those (steps halted by a flag included), and early candidate
   rebuilds (PD_FLAG_ADAPTIVE_REBUILD). */
pd_status pd_loop_counts(pd_ctx* ctx, int64_t* out6);

/* How pd_step launches the step.  GRAPH, DIRECT and PERSISTENT, with any
   slices_per_block and xcd_remap, compute bitwise the same node state and wall
   reactions (same per-node order; wall reactions are reduced per slice and then
   in slice order).  PER_GRAIN computes bitwise the same node state when no wall
   is servo-controlled; its reactions agree to rounding (a slice holding nodes
   of two grains is reduced in two parts).
     PD_LOOP_GRAPH       all grains in one fused force+contact+walls+Verlet launch
                         per step; runs of rebuild_every steps (doubled when odd)
                         replay one captured HIP graph (default);
     PD_LOOP_DIRECT      the same launches, issued one by one;
     PD_LOOP_PERSISTENT  one cooperative launch per run of steps between candidate
                         rebuilds: workgroups stay resident, share out the
                         slices evenly (those of one XCD side by side), and meet
                         at one grid barrier per step, where the last to arrive
                         reduces the wall reactions;
     PD_LOOP_PER_GRAIN   unbatched reference: one launch per grain per step.
   slices_per_block: 64-node slices (wavefronts) per workgroup, 1, 2, 4 or 8
   (GRAPH and DIRECT; the others use 4).  xcd_remap: 1 maps consecutive
   workgroups to contiguous slice ranges per XCD, 0 keeps dispatch order.
   persistent_blocks: workgroups of the persistent launch, 0 = as many as can be
   resident.
   bond_path: how the bond sum (Sec. 3.1) reads its neighbours.
     PD_BONDS_SLICES  sliced-ELL rows of column words, neighbour u gathered from
                      HBM (default; every loop);
     PD_BONDS_TILES   workgroups over 8 x 4 x 16-cell tiles of each grain's
                      lattice (or of one box over all grains when they share a
                      lattice, see pd_tile_info) with u of the tile and a 3-cell
                      halo staged in LDS, the bond memory in per-node class masks.  Needs the bonds
                      built, horizon factor 3 and every grain's nodes in
                      lexicographic lattice order along some axis order
                      (PD_ERR_UNSUPPORTED otherwise), and the GRAPH or DIRECT
                      loop.  Node state is bitwise the same as with slices (the
                      same per-bond arithmetic in the same order); wall
                      reactions are reduced per tile wavefront and agree to
                      rounding, so with servo walls the node state does too.
   Switching the bond path hands the bond memory over; pd_get, pd_get_state
   and pd_set_state see the same bond state either way.  Setting a
   configuration drops the captured graph. */
enum { PD_LOOP_GRAPH = 0, PD_LOOP_DIRECT = 1, PD_LOOP_PERSISTENT = 2, PD_LOOP_PER_GRAIN = 3 };
enum { PD_BONDS_SLICES = 0, PD_BONDS_TILES = 1 };
typedef struct {
  int32_t loop;
  int32_t slices_per_block;
  int32_t xcd_remap;
  int32_t persistent_blocks;
  int32_t bond_path;
} pd_launch;
pd_status pd_set_launch(pd_ctx* ctx, const pd_launch* launch);
pd_status pd_get_launch(pd_ctx* ctx, pd_launch* launch);

void pd_destroy(pd_ctx* ctx);
const char* pd_last_error(const pd_ctx* ctx);
const char* pd_status_string(pd_status status);

#ifdef __cplusplus
}
#endif
#endif
