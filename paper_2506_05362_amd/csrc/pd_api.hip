// Host runtime of the peridynamic grain-aggregate library: validation, device
// buffers, the step sequence and the C ABI declared in pd.h.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "pd_internal.h"

using namespace pdk;

namespace {

// A roctx range over a host-side phase (enqueueing work, not its run time on
// the device), visible in rocprofv3 --marker-trace next to the kernels.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kMagic = 0x3130536b4450554dull;  // checkpoint magic
constexpr int64_t kUnboundedCut = ((int64_t)1) << 50;

// Scratch of the allocation-free energy call (pd_energy_noalloc): the energy
// kernel's per-workgroup partial sums, 4 doubles per 256 nodes (a context holds
// at most 2^25 nodes, so at most 2^17 workgroups), then the 4 reduced values.
// Each GPU holds its own copy; host code uses the address hipGetSymbolAddress
// returned for the device, never the array's name.
constexpr int64_t kNoAllocPartials = (int64_t)1 << 17;
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

static __device__ __align__(256) double scratch[4 * kNoAllocPartials + 4];

struct pd_ctx {
  // configuration
  int64_t n = 0;
  int32_t n_grains = 0, n_mat = 0, n_walls = 0;
  int32_t m = 3, flags = 0, rebuild_every = 1, cap_per_node = 16;
  double Rc = 0, eps = 0, skin = 0, dt = 0, g[3] = {0, 0, 0}, beta = 0, mu = 0;
  hipStream_t stream = nullptr;
  int own_stream = 0;
  pd_alloc_fn alloc = nullptr;
  pd_free_fn free_fn = nullptr;
  void* user = nullptr;
  std::string err;
  int built = 0;
  int64_t step = 0;
  int cur = 0;  // u4[cur] holds u_n, u4[cur^1] holds the drift to u_{n+1}
  // host copies needed by the bond build
  std::vector<int64_t> grain_begin;
  std::vector<int32_t> ijk_h;  // (3,N)
  std::vector<GrainC> grains_h;
  std::vector<WallDev> walls_h;
  std::vector<void*> owned;
  // device state
  double4* u4[2] = {nullptr, nullptr};
  double4* vh[2] = {nullptr, nullptr};  // mid-step velocities, indexed like u4 (beta or mu > 0)
  double *v = nullptr, *a = nullptr, *X = nullptr, *F = nullptr;
  double4* X4 = nullptr;
  uint8_t* fixed = nullptr;
  GrainC* grains = nullptr;
  StencilC* stencil = nullptr;
  int32_t n_stencil = 0, n_classes = 1, node_bits = 31;
  uint32_t sentinel_hi = 0;
  double* Kn = nullptr;
  WallDev* walls = nullptr;
  double* wall_partial = nullptr;
  double* wall_chunk = nullptr;
  int64_t* box_chunks = nullptr;
  int32_t n_box_chunks = 0;
  int64_t* step_d = nullptr;
  uint32_t* status = nullptr;
  uint32_t* halt = nullptr;  // status when the current step began: later steps do nothing once set
  // bonds
  int64_t nslices = 0, padded = 0, nnz = 0;
  int32_t* rowlen = nullptr;
  int64_t* slice_off = nullptr;
  uint32_t* colE = nullptr;
  uint32_t* colOrig = nullptr;
  int32_t* intact = nullptr;
  // contact
  uint32_t T = 0;
  int64_t capacity = 0;
  long long* cellkey = nullptr;
  int4* srec = nullptr;
  int32_t* cand_scratch = nullptr;
  int32_t scratch_w = 32;
  int32_t *bucket_count = nullptr, *bucket_start = nullptr, *bucket_fill = nullptr,
          *cand_ptr = nullptr, *cand = nullptr;
  uint32_t* cellh = nullptr;
  int64_t* grid = nullptr;  // [8] cell grid of the last rebuild
  double* u_build = nullptr;
  long long* gbox = nullptr;
  int32_t *gpair_count = nullptr, *gpair = nullptr;
  uint8_t* active = nullptr;
  int32_t* scan32 = nullptr;
  int64_t* scan64 = nullptr;
  double* energy_partial = nullptr;
  double* scratch_dev = nullptr;  // this context's GPU's copy of the allocation-free scratch
  double* energy_out = nullptr;
  // measurement hook
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  // launch configuration (pd_set_launch) and its per-grain tables
  pd_launch launch{PD_LOOP_GRAPH, kSlicesPerBlock, 1, 0, PD_BONDS_SLICES};
  std::vector<int64_t> pg_slice_lo, pg_slice_hi, pg_part_base;
  int64_t pg_cols = 0;  // wall-partial columns of the per-grain launches (shared slices twice)
  int64_t partial_cols = 0;  // columns allocated in wall_partial
  uint32_t* barrier = nullptr;  // [2]: arrival count, generation
  // tiled bond loop (PD_BONDS_TILES): available when the horizon factor is 3
  // and every grain's nodes are in lexicographic order of some axis order
  int tile_ok = 0;
  int tile_lattice = 0;  // the tiles cover one box over every grain
  int64_t n_tiles = 0;
  int4* tiles = nullptr;
  TileGrain* tgrain = nullptr;
  int32_t* tmap = nullptr;
  StencilC* ttab = nullptr;
  int16_t* ctob = nullptr;  // [6][n_stencil]: slice-path class -> mask bit per axis order
  double* corner_gl = nullptr;  // Gauss-Legendre nodes and weights on [0, pi] (wall corners)
  uint32_t* corner_w = nullptr;  // [N]
  double* corner_c = nullptr;    // [3N]
  uint64_t* lmask = nullptr;  // [n_tiles * kTS][kTileClasses] lane masks of intact bonds
  int32_t* slot = nullptr;    // [N] node -> (tile * kTS + wavefront) * 64 + lane
  std::vector<StencilC> stencil_h;  // host copy of the slice-path tables
  std::vector<int> sd_h;            // horizon offsets (dx, dy, dz) of the slice-path classes
  // captured step loop of graph_len steps
  int use_graph = 1;
  int64_t graph_len = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // how the steps of this context were launched: graph replays, steps in them,
  // directly launched steps, persistent launches and the steps in them, early
  // candidate rebuilds
  int64_t counts[6] = {0, 0, 0, 0, 0, 0};
};

namespace {

pd_status fail(pd_ctx* c, pd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((ctx), PD_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorName(e_),      \
                  __FILE__, __LINE__);                                                         \
  } while (0)

void* dev_alloc(pd_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->owned.push_back(p);
  return p;
}

void dev_free(pd_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->owned.begin(), c->owned.end(), p);
  if (it != c->owned.end()) c->owned.erase(it);
  if (c->free_fn)
    c->free_fn(p, c->user);
  else
    (void)hipFree(p);
}

template <typename T>
pd_status alloc_n(pd_ctx* c, T** out, int64_t count, const char* what) {
  *out = static_cast<T*>(dev_alloc(c, sizeof(T) * (size_t)(count > 0 ? count : 1)));
  if (!*out) return fail(c, PD_ERR_OOM, "device allocation of %s (%lld elements) failed", what, (long long)count);
  return PD_OK;
}

#define TRY(expr)                 \
  do {                            \
    pd_status s_ = (expr);        \
    if (s_ != PD_OK) return s_;   \
  } while (0)

// 3-D micromodulus constants (Sec. 3.1.1 and its table): c, or c0 of the conic
// form c0 (1 - |xi|/delta), and the critical stretch s0.
void micro_constants(double K, double Gc, double delta, int flags, double* c, double* s0) {
  const bool conic = (flags & PD_FLAG_CONIC) != 0;
  const double d4 = delta * delta * delta * delta;
  if (flags & PD_FLAG_TABLE_LITERAL) {
    const double nu = 0.25, E = 3.0 * K * (1.0 - 2.0 * nu);
    *c = (conic ? 60.0 : 12.0) * E / (kPi * d4 * (1.0 - nu));
    *s0 = sqrt((conic ? 7.0 : 5.0) * kPi * Gc / (12.0 * E * delta));
  } else if (conic) {
    // energy-consistent: pi c0 delta^4 / 20 = 9K/2 and pi c0 s0^2 delta^5 / 60 = G_c
    *c = 90.0 * K / (kPi * d4);
    *s0 = sqrt(2.0 * Gc / (3.0 * K * delta));
  } else {
    // energy-consistent: pi c delta^4 / 4 = 9K/2 and pi c s0^2 delta^5 / 10 = G_c
    *c = 18.0 * K / (kPi * d4);
    *s0 = sqrt(5.0 * Gc / (9.0 * K * delta));
  }
}

WallDev to_dev(const pd_wall& w, int64_t next_step, double dt) {
  WallDev d{};
  for (int q = 0; q < 3; ++q) {
    d.n[q] = w.normal[q];
    d.lo[q] = w.lo[q];
    d.hi[q] = w.hi[q];
  }
  d.vel = w.velocity;
  d.off = w.offset;
  d.off_used = w.offset;
  d.off0 = w.mode == PD_WALL_VELOCITY ? w.offset - w.velocity * ((double)next_step * dt) : w.offset;
  d.target = w.target_stress;
  d.gain = w.servo_gain;
  d.area = w.area;
  d.mode = w.mode;
  d.rate = d.rate_used = w.mode == PD_WALL_VELOCITY ? w.velocity : 0.0;
  return d;
}

pd_status check_wall(pd_ctx* c, const pd_wall& w, int k) {
  const double nn = w.normal[0] * w.normal[0] + w.normal[1] * w.normal[1] + w.normal[2] * w.normal[2];
  if (!(fabs(nn - 1.0) < 1e-12)) return fail(c, PD_ERR_INVALID, "wall %d: normal is not a unit vector", k);
  if (w.mode < 0 || w.mode > 2) return fail(c, PD_ERR_INVALID, "wall %d: mode %d", k, w.mode);
  if (!(w.area > 0)) return fail(c, PD_ERR_INVALID, "wall %d: area must be > 0", k);
  if (!isfinite(w.offset)) return fail(c, PD_ERR_INVALID, "wall %d: offset not finite", k);
  return PD_OK;
}

// Gauss-Legendre rule of n points mapped to [0, pi]: nodes then weights.  The
// roots of P_n by Newton's method from the usual cosine guesses.
std::vector<double> gauss_legendre_0_pi(int n) {
  std::vector<double> out((size_t)2 * n);
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    out[(size_t)i] = 0.5 * M_PI * (x + 1.0);
    out[(size_t)(n + i)] = 0.5 * M_PI * 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return out;
}

// the skin guard protects contact pairs; a single grain without self-contact
// has none to miss
int skin_guard(const pd_ctx* c) {
  return (c->n_grains > 1 || (c->flags & PD_FLAG_SELF_CONTACT)) ? 1 : 0;
}

// PD_FLAG_ADAPTIVE_REBUILD, where contact pairs can exist
bool early_rebuilds(const pd_ctx* c) {
  return (c->flags & PD_FLAG_ADAPTIVE_REBUILD) && skin_guard(c);
}

StepArgs step_args(pd_ctx* c) {
  StepArgs A{};
  A.ucur = c->u4[c->cur];
  A.unext = c->u4[c->cur ^ 1];
  A.v = c->v;
  A.a = c->a;
  A.Fout = c->F;
  A.vh_cur = c->vh[c->cur];
  A.vh_next = c->vh[c->cur ^ 1];
  A.beta = c->beta;
  A.mu = c->mu;
  A.slice_base = 0;
  A.slice_end = c->nslices;
  A.node_lo = 0;
  A.node_hi = c->n;
  A.partial_base = 0;
  A.partial_stride = c->nslices;
  A.xcd_remap = c->launch.xcd_remap;
  A.fixed = c->fixed;
  A.grains = c->grains;
  A.stencil = c->stencil;
  A.n_stencil = c->n_stencil;
  A.n_classes = c->n_classes;
  A.node_bits = c->node_bits;
  A.slice_off = c->slice_off;
  A.rowlen = c->rowlen;
  A.colE = c->colE;
  A.sentinel_hi = c->sentinel_hi;
  A.intact = c->intact;
  A.self_contact = (c->flags & PD_FLAG_SELF_CONTACT) ? 1 : 0;
  A.colOrig = c->colOrig;
  A.ctob = c->ctob;
  A.wall_corners = (c->flags & PD_FLAG_WALL_CORNERS) && c->n_walls > 1 ? 1 : 0;
  A.corner_gl = c->corner_gl;
  A.corner_ngl = kCornerGL;
  A.corner_w = c->corner_w;
  A.corner_c = c->corner_c;
  A.cand_ptr = c->cand_ptr;
  A.cand = c->cand;
  A.cand_capacity = c->capacity;
  A.X = c->X;
  A.X4 = c->X4;
  A.Kn = c->Kn;
  A.walls = c->walls;
  A.wall_partial = c->wall_partial;
  A.wall_chunk = c->wall_chunk;
  A.step = c->step_d;
  A.advance = 1;
  A.status = c->status;
  A.halt = c->halt;
  A.n = c->n;
  A.nslices = c->nslices;
  A.n_walls = c->n_walls;
  A.n_mat = c->n_mat;
  A.Rc = c->Rc;
  A.Rc2 = c->Rc * c->Rc;
  A.dt = c->dt;
  for (int q = 0; q < 3; ++q) A.g[q] = c->g[q];
  A.abs_stretch = (c->flags & PD_FLAG_ABS_STRETCH) ? 1 : 0;
  A.tiles = c->tiles;
  A.n_tiles = c->n_tiles;
  A.tgrain = c->tgrain;
  A.tmap = c->tmap;
  A.ttab = c->ttab;
  A.lmask = c->lmask;
  A.slot = c->slot;
  return A;
}

ContactArgs contact_args(pd_ctx* c, int buf) {
  ContactArgs C{};
  C.u = c->u4[buf];
  C.X = c->X;
  C.X4 = c->X4;
  C.cellkey = c->cellkey;
  C.srec = c->srec;
  C.cand_scratch = c->cand_scratch;
  C.scratch_w = c->scratch_w;
  C.cellh = c->cellh;
  C.bucket_count = c->bucket_count;
  C.bucket_start = c->bucket_start;
  C.bucket_fill = c->bucket_fill;
  C.cand_count = c->cand_ptr;
  C.cand = c->cand;
  C.u_build = c->u_build;
  C.scan_scratch = c->scan32;
  C.gbox = c->gbox;
  C.gpair_count = c->gpair_count;
  C.gpair = c->gpair;
  C.active = c->active;
  C.box_chunks = c->box_chunks;
  C.n_box_chunks = c->n_box_chunks;
  C.n_grains = c->n_grains;
  C.status = c->status;
  C.halt = c->halt;
  C.n = c->n;
  C.T = c->T;
  C.grid = c->grid;
  C.capacity = c->capacity;
  const double cut = c->Rc + c->skin;
  C.inv_cell = 1.0 / (cut * 1.01);
  C.cut2 = cut * cut;
  C.skin_half2 = 0.25 * c->skin * c->skin;
  C.self_contact = (c->flags & PD_FLAG_SELF_CONTACT) ? 1 : 0;
  return C;
}

// one step on the device: rebuild on cadence, force+Verlet, walls.
// ev0/ev1 (optional) bracket the step kernel.
pd_status enqueue_step_ev(pd_ctx* c, int64_t s, hipEvent_t ev0, hipEvent_t ev1) {
  Range r("pd step: enqueue one step");
  const int nxt = c->cur ^ 1;
  const bool watch = early_rebuilds(c);
  if (s % c->rebuild_every == 0) {
    Range rr("pd step: contact rebuild");
    ContactArgs C = contact_args(c, nxt);
    // with the watch every evaluation since the last rebuild was checked
    HIPCHK(c, launch_contact_rebuild(C, watch ? 0 : skin_guard(c), c->stream));
  } else if (watch) {
    HIPCHK(c, launch_skin_watch(contact_args(c, nxt), c->halt, c->stream));
  }
  c->cur = nxt;  // the drifted positions are the current ones now
  StepArgs A = step_args(c);
  HIPCHK(c, launch_wall_corners(A, 0, c->stream));
  // a single step launch records ev0/ev1 itself, tightly around the kernel
  if (c->launch.bond_path == PD_BONDS_TILES) {
    A.partial_stride = kTS * c->n_tiles;  // one wall-partial column per tile wavefront
    HIPCHK(c, launch_step_tile(A, c->stream, ev0, ev1));
  } else if (c->launch.loop == PD_LOOP_PER_GRAIN) {
    if (ev0) HIPCHK(c, hipEventRecord(ev0, c->stream));
    // one launch per grain over the slices that hold its nodes; a slice shared
    // by two grains is visited by both launches, each lane working for its own
    A.partial_stride = c->pg_cols;
    for (int32_t g = 0; g < c->n_grains; ++g) {
      StepArgs Ag = A;
      Ag.slice_base = c->pg_slice_lo[(size_t)g];
      Ag.slice_end = c->pg_slice_hi[(size_t)g];
      Ag.node_lo = c->grain_begin[(size_t)g];
      Ag.node_hi = c->grain_begin[(size_t)g + 1];
      Ag.partial_base = c->pg_part_base[(size_t)g];
      Ag.xcd_remap = 0;
      HIPCHK(c, launch_step_spb(Ag, kSlicesPerBlock, c->stream));
    }
    if (ev1) HIPCHK(c, hipEventRecord(ev1, c->stream));
  } else {
    HIPCHK(c, launch_step_spb(A, c->launch.slices_per_block, c->stream, ev0, ev1));
  }
  HIPCHK(c, launch_wall_finalize(A, c->stream));
  return PD_OK;
}

// PD_FLAG_ADAPTIVE_REBUILD: the watch halted step done + 1 before its
// evaluation; rebuild the list at the positions that evaluation uses (the ones
// the watch saw), clear the flags, and let pd_step go on from there
pd_status early_rebuild(pd_ctx* c) {
  Range r("pd step: early contact rebuild");
  int64_t done = 0;
  HIPCHK(c, hipMemcpyAsync(&done, c->step_d, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(uint32_t), c->stream));
  HIPCHK(c, hipMemsetAsync(c->halt, 0, sizeof(uint32_t), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = done;
  c->cur = (int)(done & 1);  // u4[step % 2] holds u_step, the other buffer the next positions
  ContactArgs C = contact_args(c, c->cur ^ 1);
  HIPCHK(c, launch_contact_rebuild(C, 0, c->stream));
  c->counts[5] += 1;
  return PD_OK;
}

// PD_LOOP_PERSISTENT: steps c->step+1 .. c->step+k in one launch, k chosen so
// that no candidate rebuild falls inside (a rebuild due at the first step runs
// before the launch).
pd_status enqueue_persistent(pd_ctx* c, int64_t left, int64_t* done, hipEvent_t ev0, hipEvent_t ev1) {
  Range r("pd step: persistent run");
  const int64_t s = c->step + 1;
  const int64_t R = c->rebuild_every;
  const int64_t k = std::min<int64_t>(left, (s / R + 1) * R - s);
  if (s % R == 0) {
    ContactArgs C = contact_args(c, c->cur ^ 1);
    HIPCHK(c, launch_contact_rebuild(C, skin_guard(c), c->stream));
  }
  if (!c->barrier) TRY(alloc_n(c, &c->barrier, 2, "grid barrier"));
  HIPCHK(c, launch_fill_i32(reinterpret_cast<int32_t*>(c->barrier), 0, 2, c->stream));
  // (occupancy depends on the kernel and its LDS only, not on the buffer parity)
  const int32_t maxb = persistent_max_blocks(step_args(c));
  if (maxb <= 0) return fail(c, PD_ERR_HIP, "no resident workgroups for the persistent step kernel");
  const int32_t nb = c->launch.persistent_blocks > 0 ? std::min(c->launch.persistent_blocks, maxb) : maxb;
  c->cur ^= 1;
  StepArgs A = step_args(c);
  BarrierArgs B{c->barrier, c->barrier + 1, 1u << 24};
  if (ev0) HIPCHK(c, hipEventRecord(ev0, c->stream));
  HIPCHK(c, launch_step_persistent(A, k, nb, B, c->stream));
  if (ev1) HIPCHK(c, hipEventRecord(ev1, c->stream));
  if ((k - 1) & 1) c->cur ^= 1;  // the kernel flipped the buffers k - 1 more times
  *done = k;
  return PD_OK;
}

// capture graph_len steps starting at a multiple of graph_len (buffer parity 0)
pd_status capture_graph(pd_ctx* c) {
  if (c->graph_exec) return PD_OK;
  Range r("pd step: capture the step graph");
  const int cur0 = c->cur;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  pd_status st = PD_OK;
  for (int64_t p = 1; p <= c->graph_len && st == PD_OK; ++p)
    st = enqueue_step_ev(c, p, nullptr, nullptr);  // p stands for any step congruent to it
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->stream, &g);
  c->cur = cur0;
  if (st != PD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess) return fail(c, PD_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorName(ec));
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
  return PD_OK;
}

pd_status drop_graphs(pd_ctx* c) {
  if (c->graph_exec) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGraphExecDestroy(c->graph_exec));
  }
  if (c->graph) HIPCHK(c, hipGraphDestroy(c->graph));
  c->graph_exec = nullptr;
  c->graph = nullptr;
  return PD_OK;
}

pd_status next_events(pd_ctx* c, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!c->timing) return PD_OK;
  while (c->ev_pool.size() < c->ev_used + 2) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  *e0 = c->ev_pool[c->ev_used];
  *e1 = c->ev_pool[c->ev_used + 1];
  c->ev_used += 2;
  return PD_OK;
}

pd_status enqueue_step(pd_ctx* c, int64_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    while (c->ev_pool.size() < c->ev_used + 2) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
    e0 = c->ev_pool[c->ev_used];
    e1 = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
  }
  return enqueue_step_ev(c, s, e0, e1);
}

pd_status read_status(pd_ctx* c, uint32_t* st) {
  HIPCHK(c, hipMemcpyAsync(st, c->status, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PD_OK;
}

// A flag raised by a step lets that step complete and halts the steps after
// it (their kernels change nothing): the context's step count and state are
// those of the step that raised it.  The flags are cleared once reported.
pd_status report_status(pd_ctx* c) {
  uint32_t st = 0;
  TRY(read_status(c, &st));
  if (!st) return PD_OK;
  int64_t done = 0;
  HIPCHK(c, hipMemcpyAsync(&done, c->step_d, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(uint32_t), c->stream));
  HIPCHK(c, hipMemsetAsync(c->halt, 0, sizeof(uint32_t), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = done;
  c->cur = (int)(done & 1);  // u4[step % 2] holds u_step
  std::string why;
  if (st & ST_NAN) why += " non-finite force;";
  if (st & ST_PENETRATION) why += " node at or beyond -R_c behind a wall;";
  if (st & ST_SKIN) why += " displacement since the last candidate rebuild exceeded skin/2;";
  if (st & ST_CAND_OVERFLOW) why += " contact candidate capacity exceeded;";
  if (st & ST_BARRIER) why += " a grid barrier of the persistent step loop timed out;";
  if (st & ST_REBUILD) why += " an early candidate rebuild was pending;";
  return fail(c, PD_ERR_UNSTABLE, "instability flagged:%s", why.c_str());
}

uint32_t crc32_update(uint32_t crc, const void* data, size_t n) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t r = i;
      for (int k = 0; k < 8; ++k) r = (r & 1) ? 0xEDB88320u ^ (r >> 1) : r >> 1;
      table[i] = r;
    }
    init = true;
  }
  const uint8_t* p = static_cast<const uint8_t*>(data);
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xff] ^ (crc >> 8);
  return ~crc;
}

bool any_servo(const pd_ctx* c) {
  for (const WallDev& w : c->walls_h)
    if (w.mode == PD_WALL_SERVO) return true;
  return false;
}

// The six axis orders (slowest first), as in the tile kernels.
constexpr int kAxisOrders[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Tiles of the bond loop: for every grain an axis order in which its node
// indices ascend lexicographically (the order of the slice path's sorted rows),
// its box on those axes, a cell -> node map, the 8 x 4 x 16-cell tiles that hold
// nodes, the bond table of each (stencil class, axis order) in tile class order
// and the class masks of the built bonds.  When every grain shares one
// lattice (equal spacing, origins a whole number of spacings apart), one bond
// table and one axis order, the tiles cover one box over all grains instead
// (lattice mode): a dense aggregate then fills its tiles, and bonds, which
// never join two grains, are told apart by the class masks.  Leaves tile_ok = 0
// when some grain has no such order or the horizon factor is not 3.
pd_status build_tiles(pd_ctx* c) {
  c->tile_ok = 0;
  c->tile_lattice = 0;
  if (c->m != kTileR || c->n_stencil != kTileClasses) return PD_OK;
  const int64_t N = c->n;
  const int32_t G = c->n_grains;
  std::vector<TileGrain> tg((size_t)G);
  std::vector<int4> tiles;
  int64_t map_total = 0;
  std::vector<int> table_of((size_t)6 * c->n_classes, -1);
  int n_tables = 0;
  auto table_for = [&](int perm, int cls) {
    int& tab = table_of[(size_t)perm * c->n_classes + cls];
    if (tab < 0) tab = n_tables++;
    return tab;
  };
  // each grain's axis order and lattice box
  std::vector<std::array<int, 3>> glo((size_t)G), ghi((size_t)G);
  for (int32_t g = 0; g < G; ++g) {
    const int64_t b = c->grain_begin[(size_t)g], e = c->grain_begin[(size_t)g + 1];
    int perm = -1;
    for (int p = 0; p < 6 && perm < 0; ++p) {
      const int* P = kAxisOrders[p];
      bool ok = true;
      int64_t prev = -1;
      for (int64_t i = b; i < e && ok; ++i) {
        const int64_t key = ((int64_t)c->ijk_h[P[0] * N + i] << 20) | ((int64_t)c->ijk_h[P[1] * N + i] << 10) |
                            (int64_t)c->ijk_h[P[2] * N + i];
        ok = key > prev;
        prev = key;
      }
      if (ok) perm = p;
    }
    if (perm < 0) return PD_OK;  // this grain's node order is not a lattice order
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {0, 0, 0};
    for (int64_t i = b; i < e; ++i)
      for (int q = 0; q < 3; ++q) {
        lo[q] = std::min(lo[q], c->ijk_h[q * N + i]);
        hi[q] = std::max(hi[q], c->ijk_h[q * N + i]);
      }
    if (e == b) lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0;
    for (int q = 0; q < 3; ++q) {
      glo[(size_t)g][(size_t)q] = lo[q];
      ghi[(size_t)g][(size_t)q] = hi[q];
    }
    tg[(size_t)g].perm = perm;
    tg[(size_t)g].box = g;
  }
  // lattice mode: one spacing, one bond table, one axis order, origins on one lattice
  bool lattice = G > 1;
  std::vector<std::array<int64_t, 3>> koff((size_t)G);
  for (int32_t g = 0; g < G && lattice; ++g) {
    const GrainC& a = c->grains_h[0];
    const GrainC& b = c->grains_h[(size_t)g];
    if (b.h != a.h || b.cls != a.cls || tg[(size_t)g].perm != tg[0].perm) lattice = false;
    for (int q = 0; q < 3 && lattice; ++q) {
      const double k = (b.origin[q] - a.origin[q]) / a.h;
      const double kr = nearbyint(k);
      if (!(fabs(k - kr) <= 1e-6) || fabs(kr) > (1 << 20)) lattice = false;
      koff[(size_t)g][(size_t)q] = (int64_t)kr;
    }
  }
  std::vector<int32_t> slot_h((size_t)N, -1);
  // the boxes to tile: each grain's, or the shared one
  struct Box {
    int perm, lo[3], hi[3];  // lo/hi on the x, y, z axes of the box's lattice
    int cls;
    std::vector<int32_t> grains;
  };
  std::vector<Box> boxes;
  if (lattice) {
    int64_t kmin[3] = {0, 0, 0};
    for (int32_t g = 0; g < G; ++g)
      for (int q = 0; q < 3; ++q) kmin[q] = std::min(kmin[q], koff[(size_t)g][(size_t)q]);
    Box B;
    B.perm = tg[0].perm;
    B.cls = c->grains_h[0].cls;
    for (int q = 0; q < 3; ++q) {
      B.lo[q] = 1 << 30;
      B.hi[q] = -(1 << 30);
    }
    for (int32_t g = 0; g < G; ++g) {
      for (int q = 0; q < 3; ++q) {
        const int64_t o = koff[(size_t)g][(size_t)q] - kmin[q];
        tg[(size_t)g].goff[q] = (int32_t)o;
        if (c->grain_begin[(size_t)g + 1] > c->grain_begin[(size_t)g]) {
          B.lo[q] = std::min<int64_t>(B.lo[q], glo[(size_t)g][(size_t)q] + o);
          B.hi[q] = std::max<int64_t>(B.hi[q], ghi[(size_t)g][(size_t)q] + o);
        }
      }
      tg[(size_t)g].box = G;
      B.grains.push_back(g);
    }
    if (B.lo[0] > B.hi[0]) B.lo[0] = B.lo[1] = B.lo[2] = B.hi[0] = B.hi[1] = B.hi[2] = 0;
    if ((int64_t)(B.hi[0] - B.lo[0] + 1) * (B.hi[1] - B.lo[1] + 1) * (B.hi[2] - B.lo[2] + 1) > ((int64_t)1 << 31))
      lattice = false;
    else
      boxes.push_back(B);
  }
  if (!lattice) {
    boxes.clear();
    for (int32_t g = 0; g < G; ++g) {
      Box B;
      B.perm = tg[(size_t)g].perm;
      B.cls = c->grains_h[(size_t)g].cls;
      for (int q = 0; q < 3; ++q) {
        B.lo[q] = glo[(size_t)g][(size_t)q];
        B.hi[q] = ghi[(size_t)g][(size_t)q];
        tg[(size_t)g].goff[q] = 0;
      }
      tg[(size_t)g].box = g;
      B.grains.push_back(g);
      boxes.push_back(B);
    }
  }
  // box records (appended after the grains in lattice mode), their maps and tiles
  std::vector<TileGrain> rec = tg;
  for (size_t bi = 0; bi < boxes.size(); ++bi) {
    const Box& B = boxes[bi];
    const int* P = kAxisOrders[B.perm];
    const int32_t r = lattice ? G : B.grains[0];
    if (lattice) rec.push_back(TileGrain{});
    TileGrain& T = rec[(size_t)r];
    T.perm = B.perm;
    T.box = r;
    T.lo_s = B.lo[P[0]];
    T.lo_m = B.lo[P[1]];
    T.lo_f = B.lo[P[2]];
    T.es = B.hi[P[0]] - B.lo[P[0]] + 1;
    T.em = B.hi[P[1]] - B.lo[P[1]] + 1;
    T.ef = B.hi[P[2]] - B.lo[P[2]] + 1;
    T.map_off = map_total;
    map_total += (int64_t)T.es * T.em * T.ef;
    T.table = table_for(B.perm, B.cls);
    for (int32_t g : B.grains) tg[(size_t)g].table = T.table;
    // tiles holding at least one node, in (s, m, f) tile order, and each node's
    // slot: (tile * kTS + its layer in the tile) * 64 + its lane
    const int nts = (T.es + kTS - 1) / kTS, ntm = (T.em + kTM - 1) / kTM, ntf = (T.ef + kTF - 1) / kTF;
    std::vector<int64_t> tid((size_t)nts * ntm * ntf, -1);
    auto node_cell = [&](int32_t g, int64_t i, int& cs, int& cm, int& cf) {
      int x[3];
      for (int q = 0; q < 3; ++q) x[q] = c->ijk_h[q * N + i] + tg[(size_t)g].goff[q];
      cs = x[P[0]] - T.lo_s;
      cm = x[P[1]] - T.lo_m;
      cf = x[P[2]] - T.lo_f;
    };
    for (int32_t g : B.grains)
      for (int64_t i = c->grain_begin[(size_t)g]; i < c->grain_begin[(size_t)g + 1]; ++i) {
        int cs, cm, cf;
        node_cell(g, i, cs, cm, cf);
        tid[((size_t)(cs / kTS) * ntm + cm / kTM) * ntf + cf / kTF] = 0;
      }
    for (int ts = 0; ts < nts; ++ts)
      for (int tm = 0; tm < ntm; ++tm)
        for (int tf = 0; tf < ntf; ++tf) {
          int64_t& id = tid[((size_t)ts * ntm + tm) * ntf + tf];
          if (id < 0) continue;
          id = (int64_t)tiles.size();
          tiles.push_back(make_int4(r, ts * kTS, tm * kTM, tf * kTF));
        }
    for (int32_t g : B.grains)
      for (int64_t i = c->grain_begin[(size_t)g]; i < c->grain_begin[(size_t)g + 1]; ++i) {
        int cs, cm, cf;
        node_cell(g, i, cs, cm, cf);
        const int64_t id = tid[((size_t)(cs / kTS) * ntm + cm / kTM) * ntf + cf / kTF];
        slot_h[(size_t)i] = (int32_t)((id * kTS + cs % kTS) * kWave + (cm % kTM) * kTF + cf % kTF);
      }
  }
  for (int32_t g = 0; g < G; ++g) {
    rec[(size_t)g].perm = tg[(size_t)g].perm;
    rec[(size_t)g].box = tg[(size_t)g].box;
    rec[(size_t)g].table = tg[(size_t)g].table;
    for (int q = 0; q < 3; ++q) rec[(size_t)g].goff[q] = tg[(size_t)g].goff[q];
  }
  // tile class K of axis order p is the offset (ds, dm, df) K-th in lexicographic
  // order; (dx, dy, dz) puts ds on axis P[0] and so on
  std::vector<int> cls_of_offset(15 * 15 * 15, -1);
  for (int k = 0; k < c->n_stencil; ++k)
    cls_of_offset[(size_t)(((c->sd_h[3 * k] + 7) * 15 + (c->sd_h[3 * k + 1] + 7)) * 15 + (c->sd_h[3 * k + 2] + 7))] = k;
  std::vector<int16_t> ctob((size_t)6 * c->n_stencil, -1);
  std::vector<std::vector<int>> btoc(6, std::vector<int>(kTileClasses, -1));
  for (int p = 0; p < 6; ++p) {
    const int* P = kAxisOrders[p];
    int K = 0;
    for (int a = -kTileR; a <= kTileR; ++a)
      for (int bb = -kTileR; bb <= kTileR; ++bb)
        for (int cc = -kTileR; cc <= kTileR; ++cc) {
          const int d2 = a * a + bb * bb + cc * cc;
          if (d2 == 0 || d2 > kTileR * kTileR) continue;
          int d[3];
          d[P[0]] = a;
          d[P[1]] = bb;
          d[P[2]] = cc;
          const int k = cls_of_offset[(size_t)(((d[0] + 7) * 15 + (d[1] + 7)) * 15 + (d[2] + 7))];
          if (k < 0) return fail(c, PD_ERR_HIP, "tile stencil: offset missing from the horizon stencil");
          btoc[(size_t)p][(size_t)K] = k;
          ctob[(size_t)p * c->n_stencil + k] = (int16_t)K;
          ++K;
        }
  }
  std::vector<StencilC> ttab((size_t)n_tables * kTileClasses);
  for (int p = 0; p < 6; ++p)
    for (int cl = 0; cl < c->n_classes; ++cl) {
      const int t = table_of[(size_t)p * c->n_classes + cl];
      if (t < 0) continue;
      for (int K = 0; K < kTileClasses; ++K)
        ttab[(size_t)t * kTileClasses + K] =
            c->stencil_h[(size_t)cl * (c->n_stencil + 1) + btoc[(size_t)p][(size_t)K]];
    }
  hipStream_t s = c->stream;
  c->n_tiles = (int64_t)tiles.size();
  TRY(alloc_n(c, &c->tiles, std::max<int64_t>(c->n_tiles, 1), "tiles"));
  TRY(alloc_n(c, &c->tgrain, std::max<int64_t>((int64_t)rec.size(), 1), "tile boxes"));
  TRY(alloc_n(c, &c->tmap, std::max<int64_t>(map_total, 1), "tile cell map"));
  TRY(alloc_n(c, &c->ttab, std::max<int64_t>((int64_t)ttab.size(), 1), "tile bond tables"));
  TRY(alloc_n(c, &c->ctob, std::max<int64_t>((int64_t)ctob.size(), 1), "class to mask bit"));
  if ((int64_t)tiles.size() * kTS * kWave >= ((int64_t)1 << 31))
    return fail(c, PD_ERR_UNSUPPORTED, "%lld tiles exceed the 31-bit node slots", (long long)tiles.size());
  TRY(alloc_n(c, &c->lmask, std::max<int64_t>((int64_t)tiles.size() * kTS * kTileClasses, 1), "lane masks"));
  TRY(alloc_n(c, &c->slot, std::max<int64_t>(N, 1), "node slots"));
  if (N) HIPCHK(c, hipMemcpyAsync(c->slot, slot_h.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
  if (c->n_tiles)
    HIPCHK(c, hipMemcpyAsync(c->tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->tgrain, rec.data(), sizeof(TileGrain) * rec.size(), hipMemcpyHostToDevice, s));
  if (!ttab.empty())
    HIPCHK(c, hipMemcpyAsync(c->ttab, ttab.data(), sizeof(StencilC) * ttab.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->ctob, ctob.data(), sizeof(int16_t) * ctob.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, launch_fill_i32(c->tmap, -1, map_total, s));
  StepArgs A = step_args(c);
  HIPCHK(c, launch_tile_map_fill(A, s));
  HIPCHK(c, launch_cols_to_mask(A, c->ctob, c->colOrig, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->tile_ok = 1;
  c->tile_lattice = lattice ? 1 : 0;
  return PD_OK;
}

// the tile path keeps the bond memory in class masks; bring the column words
// up to date before anything reads them
pd_status sync_columns(pd_ctx* c) {
  if (c->launch.bond_path != PD_BONDS_TILES) return PD_OK;
  StepArgs A = step_args(c);
  HIPCHK(c, launch_mask_to_cols(A, c->ctob, c->colOrig, c->stream));
  return PD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* pd_status_string(pd_status s) {
  switch (s) {
    case PD_OK: return "ok";
    case PD_ERR_INVALID: return "invalid argument";
    case PD_ERR_STATE: return "call out of order";
    case PD_ERR_OOM: return "out of device memory";
    case PD_ERR_HIP: return "HIP runtime error";
    case PD_ERR_UNSTABLE: return "instability flagged";
    case PD_ERR_UNSUPPORTED: return "unsupported";
    case PD_ERR_CORRUPT: return "corrupt checkpoint";
    default: return "unknown status";
  }
}

const char* pd_last_error(const pd_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pd_status pd_init(pd_ctx** out, const pd_grains* grains, const pd_mesh* mesh,
                  const pd_material* materials, int32_t n_mat, const pd_params* params,
                  const pd_wall* walls, int32_t n_walls, pd_alloc_fn alloc, pd_free_fn free_fn,
                  void* alloc_user, void* stream) {
  if (!out) return PD_ERR_INVALID;
  *out = nullptr;
  if (!grains || !mesh || !materials || !params) return PD_ERR_INVALID;
  if ((alloc == nullptr) != (free_fn == nullptr)) return PD_ERR_INVALID;
  pd_ctx* c = new (std::nothrow) pd_ctx();
  if (!c) return PD_ERR_OOM;
  *out = c;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = alloc_user;
  c->stream = static_cast<hipStream_t>(stream);
  if (!c->stream) {
    if (hipStreamCreate(&c->stream) != hipSuccess) return fail(c, PD_ERR_HIP, "hipStreamCreate failed");
    c->own_stream = 1;
  }
  {
    // the allocation-free scratch's address on this GPU, looked up once per device
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, PD_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
      void* p = nullptr;
      HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      g_scratch_dev[dev] = static_cast<double*>(p);
    }
    c->scratch_dev = g_scratch_dev[dev];
  }

  const int64_t N = mesh->n_nodes;
  const int32_t G = grains->n_grains;
  if (N < 0 || N > INT32_MAX - 64) return fail(c, PD_ERR_INVALID, "n_nodes %lld out of range", (long long)N);
  if (G < 1) return fail(c, PD_ERR_INVALID, "n_grains must be >= 1");
  if (!grains->node_begin || !grains->material || !grains->h || !grains->origin)
    return fail(c, PD_ERR_INVALID, "grain arrays must not be NULL");
  if (N > 0 && (!mesh->X || !mesh->ijk)) return fail(c, PD_ERR_INVALID, "mesh X/ijk must not be NULL");
  if (n_mat < 1) return fail(c, PD_ERR_INVALID, "n_mat must be >= 1");
  if (n_walls < 0 || n_walls > kMaxWalls) return fail(c, PD_ERR_INVALID, "n_walls must be in [0, %d]", kMaxWalls);
  if (n_walls > 0 && !walls) return fail(c, PD_ERR_INVALID, "walls must not be NULL");
  if (grains->node_begin[0] != 0 || grains->node_begin[G] != N)
    return fail(c, PD_ERR_INVALID, "node_begin must start at 0 and end at n_nodes");
  for (int32_t g = 0; g < G; ++g) {
    if (grains->node_begin[g + 1] < grains->node_begin[g])
      return fail(c, PD_ERR_INVALID, "node_begin not monotone at grain %d", g);
    if (!(grains->h[g] > 0)) return fail(c, PD_ERR_INVALID, "grain %d: h must be > 0", g);
    if (grains->material[g] < 0 || grains->material[g] >= n_mat)
      return fail(c, PD_ERR_INVALID, "grain %d: material %d out of range", g, grains->material[g]);
  }
  for (int32_t k = 0; k < n_mat; ++k) {
    const pd_material& mt = materials[k];
    if (!(mt.bulk_modulus > 0 && mt.density > 0 && mt.fracture_energy > 0))
      return fail(c, PD_ERR_INVALID, "material %d: K, rho and G_c must be > 0", k);
  }
  const pd_params& P = *params;
  if (P.horizon_factor < 1 || P.horizon_factor > kMaxHorizon)
    return fail(c, PD_ERR_INVALID, "horizon_factor must be in [1, %d]", kMaxHorizon);
  if (!(P.contact_radius > 0) || !(P.contact_horizon > 0) || !(P.skin >= 0))
    return fail(c, PD_ERR_INVALID, "contact radius/horizon must be > 0 and skin >= 0");
  if (!(P.dt > 0)) return fail(c, PD_ERR_INVALID, "dt must be > 0");
  if (P.rebuild_every < 1) return fail(c, PD_ERR_INVALID, "rebuild_every must be >= 1");
  if (!(P.contact_damping >= 0) || !isfinite(P.contact_damping))
    return fail(c, PD_ERR_INVALID, "contact_damping must be finite and >= 0");
  if (!(P.friction >= 0) || !isfinite(P.friction))
    return fail(c, PD_ERR_INVALID, "friction must be finite and >= 0");
  if (P.flags & ~(PD_FLAG_TABLE_LITERAL | PD_FLAG_ABS_STRETCH | PD_FLAG_NO_GRAPH | PD_FLAG_CONIC |
                  PD_FLAG_SELF_CONTACT | PD_FLAG_WALL_CORNERS | PD_FLAG_ADAPTIVE_REBUILD))
    return fail(c, PD_ERR_INVALID, "unknown flag bits 0x%x", P.flags);
  for (int32_t w = 0; w < n_walls; ++w) TRY(check_wall(c, walls[w], w));

  c->n = N;
  c->n_grains = G;
  c->n_mat = n_mat;
  c->n_walls = n_walls;
  c->m = P.horizon_factor;
  c->flags = P.flags;
  c->Rc = P.contact_radius;
  c->eps = P.contact_horizon;
  c->skin = P.skin;
  c->dt = P.dt;
  c->beta = P.contact_damping;
  c->mu = P.friction;
  c->rebuild_every = P.rebuild_every;
  c->use_graph = (P.flags & PD_FLAG_NO_GRAPH) ? 0 : 1;
  if (!c->use_graph) c->launch.loop = PD_LOOP_DIRECT;
  c->graph_len = (P.rebuild_every % 2 == 0) ? P.rebuild_every : 2 * (int64_t)P.rebuild_every;
  c->cap_per_node = P.candidate_capacity_per_node > 0 ? P.candidate_capacity_per_node
                                                      : ((P.flags & PD_FLAG_SELF_CONTACT) ? 48 : 16);
  for (int q = 0; q < 3; ++q) c->g[q] = P.gravity[q];
  c->grain_begin.assign(grains->node_begin, grains->node_begin + G + 1);

  // lattice indices and the X = origin + h ijk consistency the kernels rely on
  c->ijk_h.assign(mesh->ijk, mesh->ijk + 3 * N);
  for (int32_t g = 0; g < G; ++g) {
    const double h = grains->h[g];
    for (int64_t i = c->grain_begin[g]; i < c->grain_begin[g + 1]; ++i)
      for (int q = 0; q < 3; ++q) {
        const int32_t v = c->ijk_h[q * N + i];
        if (v < 0 || v > 1023) return fail(c, PD_ERR_INVALID, "node %lld: ijk out of [0, 1023]", (long long)i);
        const double x = grains->origin[q * G + g] + h * (double)v;
        if (!(fabs(mesh->X[q * N + i] - x) <= 1e-9 * h))
          return fail(c, PD_ERR_INVALID, "node %lld: X does not match origin + h*ijk", (long long)i);
      }
  }

  // per-grain constants; grains sharing (h, material) share a stencil table
  c->grains_h.resize(G);
  std::vector<std::pair<double, int32_t>> classes;
  for (int32_t g = 0; g < G; ++g) {
    const pd_material& mt = materials[grains->material[g]];
    const double h = grains->h[g], delta = P.horizon_factor * h;
    if ((P.flags & PD_FLAG_SELF_CONTACT) && !(P.contact_radius < h))
      return fail(c, PD_ERR_INVALID, "grain %d: self-contact needs the contact radius below the lattice spacing", g);
    double cc, s0;
    micro_constants(mt.bulk_modulus, mt.fracture_energy, delta, P.flags, &cc, &s0);
    GrainC& gc = c->grains_h[g];
    gc.V = h * h * h;
    gc.cVih = cc * gc.V / h;
    gc.conic_inv_delta = (P.flags & PD_FLAG_CONIC) ? 1.0 / delta : 0.0;
    // break tests on |y|^2 - |xi|^2 against |xi|^2 ((1 +- s0)^2 - 1), |xi|^2 = h^2 |d|^2
    gc.thr = h * h * s0 * (2.0 + s0);
    gc.abs_ratio = (2.0 - s0) / (2.0 + s0);
    gc.h = h;
    gc.rho = mt.density;
    for (int q = 0; q < 3; ++q) gc.origin[q] = grains->origin[q * G + g];
    gc.mat = grains->material[g];
    const std::pair<double, int32_t> key(h, gc.mat);
    auto it = std::find(classes.begin(), classes.end(), key);
    gc.cls = (int32_t)(it - classes.begin());
    if (it == classes.end()) classes.push_back(key);
  }
  std::vector<double> kn((size_t)n_mat * n_mat);
  for (int32_t a = 0; a < n_mat; ++a)
    for (int32_t b = 0; b < n_mat; ++b) {
      const double ka = materials[a].bulk_modulus, kb = materials[b].bulk_modulus;
      const double keff = 2.0 * ka * kb / (ka + kb);
      kn[(size_t)a * n_mat + b] = 18.0 * keff / (kPi * pow(P.contact_horizon, 5));
    }
  // horizon stencil 0 < |d|^2 <= m^2 in lexicographic order; its index rides in
  // the top bits of every column word
  std::vector<int> sd;
  for (int dx = -c->m; dx <= c->m; ++dx)
    for (int dy = -c->m; dy <= c->m; ++dy)
      for (int dz = -c->m; dz <= c->m; ++dz) {
        const int d2 = dx * dx + dy * dy + dz * dz;
        if (d2 == 0 || d2 > c->m * c->m) continue;
        sd.push_back(dx);
        sd.push_back(dy);
        sd.push_back(dz);
      }
  c->n_stencil = (int32_t)(sd.size() / 3);
  c->n_classes = (int32_t)classes.size();
  if ((int64_t)c->n_classes * (c->n_stencil + 1) * (int64_t)sizeof(StencilC) > kMaxLdsTables)
    return fail(c, PD_ERR_UNSUPPORTED, "%d distinct (h, material) classes exceed the stencil-table space",
                c->n_classes);
  std::vector<StencilC> st;
  for (int32_t cl = 0; cl < c->n_classes; ++cl) {
    const double h = classes[(size_t)cl].first;
    const pd_material& mt = materials[classes[(size_t)cl].second];
    double cc, s0;
    micro_constants(mt.bulk_modulus, mt.fracture_energy, P.horizon_factor * h, P.flags, &cc, &s0);
    const double cV = cc * h * h * h;
    for (int32_t k = 0; k < c->n_stencil; ++k) {
      const double d2 = (double)(sd[3 * k] * sd[3 * k] + sd[3 * k + 1] * sd[3 * k + 1] + sd[3 * k + 2] * sd[3 * k + 2]);
      const double l0 = h * sqrt(d2), l0sq = h * h * d2;
      // micromodulus weight: 1, or 1 - |xi|/delta for the conic form
      const double w = (P.flags & PD_FLAG_CONIC) ? 1.0 - l0 / (P.horizon_factor * h) : 1.0;
      st.push_back(StencilC{h * sd[3 * k], h * sd[3 * k + 1], h * sd[3 * k + 2], l0sq * s0 * (2.0 + s0),
                            1.0 / l0sq, cV * w / l0, l0, l0sq});
    }
    // zero-force class: xi = 0, x = 0, c V / |xi| = 0 (broken bonds, padding)
    st.push_back(StencilC{0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 1.0});
  }
  c->stencil_h = st;
  c->sd_h = sd;
  int sbits = 0;
  while ((1 << sbits) < c->n_stencil + 1) ++sbits;
  c->node_bits = 32 - sbits;
  c->sentinel_hi = (uint32_t)c->n_stencil << c->node_bits;
  if (N > ((int64_t)1 << c->node_bits))
    return fail(c, PD_ERR_UNSUPPORTED, "%lld nodes exceed the %d-bit node field of a column word at horizon factor %d",
                (long long)N, c->node_bits, c->m);
  c->walls_h.resize(n_walls);
  for (int32_t w = 0; w < n_walls; ++w) c->walls_h[w] = to_dev(walls[w], 0, P.dt);

  // device buffers
  TRY(alloc_n(c, &c->u4[0], N, "u"));
  TRY(alloc_n(c, &c->u4[1], N, "u'"));
  TRY(alloc_n(c, &c->v, 3 * N, "v"));
  TRY(alloc_n(c, &c->a, 3 * N, "a"));
  TRY(alloc_n(c, &c->X, 3 * N, "X"));
  TRY(alloc_n(c, &c->X4, std::max<int64_t>(N, 1), "X as double4"));
  TRY(alloc_n(c, &c->grains, G, "grain constants"));
  TRY(alloc_n(c, &c->stencil, (int64_t)st.size(), "stencil tables"));
  TRY(alloc_n(c, &c->Kn, (int64_t)n_mat * n_mat, "K_n"));
  TRY(alloc_n(c, &c->walls, kMaxWalls, "walls"));
  if (P.flags & PD_FLAG_WALL_CORNERS) {
    const std::vector<double> gl = gauss_legendre_0_pi(kCornerGL);
    TRY(alloc_n(c, &c->corner_gl, (int64_t)gl.size(), "corner quadrature"));
    TRY(alloc_n(c, &c->corner_w, std::max<int64_t>(N, 1), "corner walls"));
    TRY(alloc_n(c, &c->corner_c, std::max<int64_t>(3 * N, 1), "corner corrections"));
    HIPCHK(c, hipMemcpyAsync(c->corner_gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  TRY(alloc_n(c, &c->step_d, 1, "step"));
  TRY(alloc_n(c, &c->status, 1, "status"));
  TRY(alloc_n(c, &c->halt, 1, "halt"));
  if (mesh->fixed) TRY(alloc_n(c, &c->fixed, N, "fixed"));
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(c->X, mesh->X, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
  HIPCHK(c, launch_pack_x4(c->X, c->X4, N, s));
  HIPCHK(c, hipMemcpyAsync(c->grains, c->grains_h.data(), sizeof(GrainC) * G, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->stencil, st.data(), sizeof(StencilC) * st.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->Kn, kn.data(), sizeof(double) * kn.size(), hipMemcpyHostToDevice, s));
  if (n_walls)
    HIPCHK(c, hipMemcpyAsync(c->walls, c->walls_h.data(), sizeof(WallDev) * n_walls, hipMemcpyHostToDevice, s));
  if (mesh->fixed) HIPCHK(c, hipMemcpyAsync(c->fixed, mesh->fixed, (size_t)N, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemsetAsync(c->step_d, 0, sizeof(int64_t), s));
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(uint32_t), s));
  HIPCHK(c, hipMemsetAsync(c->halt, 0, sizeof(uint32_t), s));
  if (mesh->v0)
    HIPCHK(c, hipMemcpyAsync(c->v, mesh->v0, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
  else
    HIPCHK(c, hipMemsetAsync(c->v, 0, sizeof(double) * 3 * N, s));
  HIPCHK(c, hipMemsetAsync(c->a, 0, sizeof(double) * 3 * N, s));
  if (c->beta > 0 || c->mu > 0) {
    // the first evaluation's damping and friction see v_0 (zero on fixed nodes)
    TRY(alloc_n(c, &c->vh[0], N, "mid-step velocity"));
    TRY(alloc_n(c, &c->vh[1], N, "mid-step velocity'"));
    std::vector<double4> vh0((size_t)N, make_double4(0.0, 0.0, 0.0, 0.0));
    if (mesh->v0)
      for (int64_t i = 0; i < N; ++i)
        if (!(mesh->fixed && mesh->fixed[i]))
          vh0[(size_t)i] = make_double4(mesh->v0[i], mesh->v0[N + i], mesh->v0[2 * N + i], 0.0);
    HIPCHK(c, hipMemcpyAsync(c->vh[0], vh0.data(), sizeof(double4) * N, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->vh[1], vh0.data(), sizeof(double4) * N, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  // packed u buffers: (u0, ijk | grain << 32)
  {
    double* u0d;
    int32_t* ijkd;
    int64_t* gofd;
    TRY(alloc_n(c, &u0d, 3 * N, "u0 staging"));
    TRY(alloc_n(c, &ijkd, 3 * N, "ijk staging"));
    TRY(alloc_n(c, &gofd, N, "grain staging"));
    std::vector<int64_t> gof((size_t)N);
    for (int32_t g = 0; g < G; ++g)
      for (int64_t i = c->grain_begin[g]; i < c->grain_begin[g + 1]; ++i) gof[(size_t)i] = g;
    if (mesh->u0)
      HIPCHK(c, hipMemcpyAsync(u0d, mesh->u0, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
    else
      HIPCHK(c, hipMemsetAsync(u0d, 0, sizeof(double) * 3 * N, s));
    HIPCHK(c, hipMemcpyAsync(ijkd, mesh->ijk, sizeof(int32_t) * 3 * N, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(gofd, gof.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice, s));
    HIPCHK(c, launch_fill_u4(c->u4[0], u0d, ijkd, gofd, N, s));
    HIPCHK(c, hipMemcpyAsync(c->u4[1], c->u4[0], sizeof(double4) * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    dev_free(c, u0d);
    dev_free(c, ijkd);
    dev_free(c, gofd);
  }
  return PD_OK;
}

pd_status pd_build_bonds(pd_ctx* c, const pd_cut* cuts, int32_t n_cuts) {
  if (!c) return PD_ERR_INVALID;
  Range r("pd_build_bonds");
  if (c->built) return fail(c, PD_ERR_STATE, "bonds already built");
  if (c->grains_h.empty()) return fail(c, PD_ERR_STATE, "context not initialised");
  if (n_cuts < 0 || (n_cuts > 0 && !cuts)) return fail(c, PD_ERR_INVALID, "bad cut array");
  const int64_t N = c->n;
  const int32_t G = c->n_grains;
  hipStream_t s = c->stream;

  // cuts grouped by grain
  std::vector<CutDev> cd;
  std::vector<int32_t> cut_begin(G + 1, 0);
  for (int32_t k = 0; k < n_cuts; ++k) {
    if (cuts[k].kind < 0 || cuts[k].kind > 2) return fail(c, PD_ERR_INVALID, "cut %d: kind %d", k, cuts[k].kind);
    if (cuts[k].grain < 0 || cuts[k].grain >= G) return fail(c, PD_ERR_INVALID, "cut %d: grain out of range", k);
    if (cuts[k].kind != 0 && cuts[k].radius2 < 0) return fail(c, PD_ERR_INVALID, "cut %d: radius2 < 0", k);
    for (int q = 0; q < 3; ++q) {
      const bool lo_b = cuts[k].lo[q] > -kUnboundedCut, hi_b = cuts[k].hi[q] < kUnboundedCut;
      if ((lo_b && llabs(cuts[k].lo[q]) > (1 << 20)) || (hi_b && llabs(cuts[k].hi[q]) > (1 << 20)) ||
          llabs(cuts[k].center[q]) > (1 << 20))
        return fail(c, PD_ERR_INVALID, "cut %d: coordinates beyond +-2^20 half-cells", k);
    }
    for (int q = 0; q < 4; ++q)
      if (llabs(cuts[k].plane[q]) > (1 << 20)) return fail(c, PD_ERR_INVALID, "cut %d: plane coefficient too large", k);
    cut_begin[cuts[k].grain + 1]++;
  }
  for (int32_t g = 0; g < G; ++g) cut_begin[g + 1] += cut_begin[g];
  cd.resize(n_cuts);
  {
    std::vector<int32_t> fill(cut_begin.begin(), cut_begin.end() - 1);
    for (int32_t k = 0; k < n_cuts; ++k) {
      const pd_cut& u = cuts[k];
      CutDev& d = cd[fill[u.grain]++];
      d.kind = u.kind;
      d.grain = u.grain;
      for (int q = 0; q < 4; ++q) d.plane[q] = u.plane[q];
      for (int q = 0; q < 3; ++q) {
        d.lo[q] = u.lo[q];
        d.hi[q] = u.hi[q];
        d.c[q] = u.center[q];
      }
      d.r2 = u.radius2;
    }
  }

  // per-grain lattice maps over the bounding box of its indices
  std::vector<int64_t> gmap_off(G + 1, 0);
  std::vector<int32_t> gdim(3 * G, 1), glo(3 * G, 0);
  for (int32_t g = 0; g < G; ++g) {
    int32_t lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int64_t i = c->grain_begin[g]; i < c->grain_begin[g + 1]; ++i)
      for (int q = 0; q < 3; ++q) {
        lo[q] = std::min(lo[q], c->ijk_h[q * N + i]);
        hi[q] = std::max(hi[q], c->ijk_h[q * N + i]);
      }
    int64_t vol = 1;
    for (int q = 0; q < 3; ++q) {
      if (hi[q] < lo[q]) {
        lo[q] = 0;
        hi[q] = 0;
      }
      glo[3 * g + q] = lo[q];
      gdim[3 * g + q] = hi[q] - lo[q] + 1;
      vol *= gdim[3 * g + q];
    }
    gmap_off[g + 1] = gmap_off[g] + vol;
  }
  // lexicographic horizon stencil 0 < |d|^2 <= m^2
  std::vector<int32_t> stencil;
  for (int dx = -c->m; dx <= c->m; ++dx)
    for (int dy = -c->m; dy <= c->m; ++dy)
      for (int dz = -c->m; dz <= c->m; ++dz) {
        const int d2 = dx * dx + dy * dy + dz * dz;
        if (d2 == 0 || d2 > c->m * c->m) continue;
        stencil.push_back((dx + 8) | ((dy + 8) << 8) | ((dz + 8) << 16));
      }

  int64_t *gmap_off_d, *scan_scratch64;
  int32_t *gdim_d, *glo_d, *gmap_d, *cut_begin_d, *stencil_d;
  CutDev* cuts_d;
  TRY(alloc_n(c, &gmap_off_d, G + 1, "grain map offsets"));
  TRY(alloc_n(c, &gdim_d, 3 * G, "grain map dims"));
  TRY(alloc_n(c, &glo_d, 3 * G, "grain map origin"));
  TRY(alloc_n(c, &gmap_d, gmap_off[G], "grain maps"));
  TRY(alloc_n(c, &cut_begin_d, G + 1, "cut offsets"));
  TRY(alloc_n(c, &stencil_d, (int64_t)stencil.size(), "stencil"));
  TRY(alloc_n(c, &cuts_d, std::max<int64_t>(n_cuts, 1), "cuts"));
  c->nslices = (N + kWave - 1) / kWave;
  TRY(alloc_n(c, &c->rowlen, N, "row lengths"));
  TRY(alloc_n(c, &c->slice_off, c->nslices + 1, "slice offsets"));
  TRY(alloc_n(c, &c->intact, N, "intact counts"));
  TRY(alloc_n(c, &scan_scratch64, scan_scratch_elems(c->nslices + 1), "scan scratch"));
  HIPCHK(c, hipMemcpyAsync(gmap_off_d, gmap_off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(gdim_d, gdim.data(), sizeof(int32_t) * 3 * G, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(glo_d, glo.data(), sizeof(int32_t) * 3 * G, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(cut_begin_d, cut_begin.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(stencil_d, stencil.data(), sizeof(int32_t) * stencil.size(), hipMemcpyHostToDevice, s));
  if (n_cuts) HIPCHK(c, hipMemcpyAsync(cuts_d, cd.data(), sizeof(CutDev) * n_cuts, hipMemcpyHostToDevice, s));
  HIPCHK(c, launch_fill_i32(gmap_d, -1, gmap_off[G], s));

  BuildArgs B{};
  B.u = c->u4[0];
  B.gmap_off = gmap_off_d;
  B.gmap_dim = gdim_d;
  B.gmap_lo = glo_d;
  B.gmap = gmap_d;
  B.cuts = cuts_d;
  B.cut_begin = cut_begin_d;
  B.stencil = stencil_d;
  B.n_stencil = (int32_t)stencil.size();
  B.node_bits = c->node_bits;
  B.sentinel_hi = c->sentinel_hi;
  B.n = N;
  B.rowlen = c->rowlen;
  B.slice_off = c->slice_off;
  B.nslices = c->nslices;
  HIPCHK(c, launch_map_fill(B, s));
  HIPCHK(c, launch_bond_count(B, s));
  HIPCHK(c, launch_slice_width(B, s));
  HIPCHK(c, scan_i64(c->slice_off, c->slice_off, c->nslices, scan_scratch64, s));
  HIPCHK(c, hipMemcpyAsync(&c->padded, c->slice_off + c->nslices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  TRY(alloc_n(c, &c->colE, c->padded, "bond columns"));
  TRY(alloc_n(c, &c->colOrig, c->padded, "bond columns as built"));
  B.colE = c->colE;
  B.colOrig = c->colOrig;
  HIPCHK(c, launch_bond_fill(B, s));
  HIPCHK(c, hipMemcpyAsync(c->intact, c->rowlen, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, s));
  {
    std::vector<int32_t> rl((size_t)N);
    HIPCHK(c, hipMemcpyAsync(rl.data(), c->rowlen, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    int64_t nnz = 0;
    for (int32_t x : rl) nnz += x;
    c->nnz = nnz;
  }
  dev_free(c, gmap_off_d);
  dev_free(c, gdim_d);
  dev_free(c, glo_d);
  dev_free(c, gmap_d);
  dev_free(c, cut_begin_d);
  dev_free(c, stencil_d);
  dev_free(c, cuts_d);
  dev_free(c, scan_scratch64);

  // contact structures
  uint32_t T = 1024;
  while ((int64_t)T < 2 * N) T <<= 1;
  c->T = T;
  c->capacity = std::max<int64_t>((int64_t)c->cap_per_node * N, 1 << 16);
  c->scratch_w = 2 * c->cap_per_node;
  TRY(alloc_n(c, &c->cellkey, N, "cell keys"));
  TRY(alloc_n(c, &c->srec, N, "binned records"));
  TRY(alloc_n(c, &c->cand_scratch, (int64_t)c->scratch_w * N, "candidate scratch rows"));
  TRY(alloc_n(c, &c->cellh, N, "cell hashes"));
  TRY(alloc_n(c, &c->grid, 8, "cell grid"));
  TRY(alloc_n(c, &c->bucket_count, T, "bucket counts"));
  TRY(alloc_n(c, &c->bucket_start, (int64_t)T + 1, "bucket starts"));
  TRY(alloc_n(c, &c->bucket_fill, T, "bucket fill"));
  TRY(alloc_n(c, &c->cand_ptr, N + 1, "candidate rows"));
  TRY(alloc_n(c, &c->cand, c->capacity, "candidates"));
  TRY(alloc_n(c, &c->u_build, 3 * N, "positions at rebuild"));
  TRY(alloc_n(c, &c->scan32, scan_scratch_elems(std::max<int64_t>(T, N)), "scan scratch"));
  TRY(alloc_n(c, &c->gbox, 6 * (int64_t)G, "grain boxes"));
  TRY(alloc_n(c, &c->gpair_count, (int64_t)G + 1, "grain pair counts"));
  TRY(alloc_n(c, &c->gpair, (int64_t)G * G, "grain pairs"));
  TRY(alloc_n(c, &c->active, N, "active flags"));
  {
    // grain-box reduction work: chunks of at most 16384 nodes of one grain
    std::vector<int64_t> ch;
    for (int32_t g = 0; g < G; ++g)
      for (int64_t b = c->grain_begin[g]; b < c->grain_begin[g + 1]; b += 16384) {
        ch.push_back(g);
        ch.push_back(b);
        ch.push_back(std::min<int64_t>(b + 16384, c->grain_begin[g + 1]));
      }
    c->n_box_chunks = (int32_t)(ch.size() / 3);
    TRY(alloc_n(c, &c->box_chunks, (int64_t)ch.size(), "box chunks"));
    HIPCHK(c, hipMemcpyAsync(c->box_chunks, ch.data(), sizeof(int64_t) * ch.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  // per-grain launch geometry (PD_LOOP_PER_GRAIN) and wall partial columns for
  // the largest grid of any mode (one slice per workgroup, or the per-grain sum)
  c->pg_slice_lo.assign((size_t)G, 0);
  c->pg_slice_hi.assign((size_t)G, 0);
  c->pg_part_base.assign((size_t)G, 0);
  c->pg_cols = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t b = c->grain_begin[(size_t)g], e = c->grain_begin[(size_t)g + 1];
    c->pg_slice_lo[(size_t)g] = b / kWave;
    c->pg_slice_hi[(size_t)g] = e > b ? (e - 1) / kWave + 1 : b / kWave;
    c->pg_part_base[(size_t)g] = c->pg_cols;
    c->pg_cols += c->pg_slice_hi[(size_t)g] - c->pg_slice_lo[(size_t)g];
  }
  TRY(build_tiles(c));
  c->partial_cols = std::max<int64_t>(std::max<int64_t>(std::max<int64_t>(c->nslices, c->pg_cols), kTS * c->n_tiles), 1);
  TRY(alloc_n(c, &c->wall_partial, c->partial_cols * 3 * std::max(c->n_walls, 1), "wall partials"));
  TRY(alloc_n(c, &c->wall_chunk, ((c->partial_cols + kChunk - 1) / kChunk) * 3 * std::max(c->n_walls, 1),
              "wall chunk sums"));

  // first candidate list at u0, then F^0 and a^0 (velocity untouched)
  ContactArgs C = contact_args(c, c->cur);
  HIPCHK(c, launch_contact_rebuild(C, 0, s));
  StepArgs A = step_args(c);
  A.advance = 0;
  HIPCHK(c, launch_wall_corners(A, 0, s));
  HIPCHK(c, launch_step(A, MODE_FIRST, s));
  HIPCHK(c, launch_wall_finalize(A, s));
  c->built = 1;
  c->step = 0;
  return report_status(c);
}

pd_status pd_step(pd_ctx* c, int64_t n_steps) {
  if (!c) return PD_ERR_INVALID;
  Range r("pd_step");
  if (!c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  if (n_steps < 0) return fail(c, PD_ERR_INVALID, "n_steps < 0");
  int64_t left = n_steps;
  const int64_t step0 = c->step;
  const bool watch = early_rebuilds(c);
  // (a mesh without nodes has no workgroup to carry the walls through a
  // persistent launch: its steps take the launches below)
  while (left > 0 && c->launch.loop == PD_LOOP_PERSISTENT && c->nslices > 0) {
    hipEvent_t e0, e1;
    TRY(next_events(c, &e0, &e1));
    int64_t k = 0;
    TRY(enqueue_persistent(c, left, &k, e0, e1));
    c->step += k;
    left -= k;
    c->counts[3] += 1;
    c->counts[4] += k;
  }
  while (left > 0) {
    // timing brackets each step kernel with events, so it launches directly
    const bool aligned = c->use_graph && c->launch.loop == PD_LOOP_GRAPH && !c->timing &&
                         c->step % c->graph_len == 0 && left >= c->graph_len;
    if (aligned) {
      TRY(capture_graph(c));
      Range rg("pd step: graph replay");
      HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
      c->step += c->graph_len;
      left -= c->graph_len;
      c->counts[0] += 1;
      c->counts[1] += c->graph_len;
    } else {
      TRY(enqueue_step(c, c->step + 1));
      c->step += 1;
      left -= 1;
      c->counts[2] += 1;
    }
    // the watch's flag is read once per captured run (or run of direct steps
    // up to the next multiple of its length)
    if (watch && (aligned || c->step % c->graph_len == 0 || left == 0)) {
      uint32_t st = 0;
      TRY(read_status(c, &st));
      if (st == ST_REBUILD) {
        TRY(early_rebuild(c));
        left = n_steps - (c->step - step0);
      } else if (st) {
        break;
      }
    }
  }
  return report_status(c);
}

pd_status pd_set_launch(pd_ctx* c, const pd_launch* l) {
  if (!c || !l) return PD_ERR_INVALID;
  if (l->loop < PD_LOOP_GRAPH || l->loop > PD_LOOP_PER_GRAIN)
    return fail(c, PD_ERR_INVALID, "unknown step loop %d", l->loop);
  if (l->loop == PD_LOOP_PERSISTENT && (c->flags & PD_FLAG_WALL_CORNERS))
    return fail(c, PD_ERR_UNSUPPORTED, "wall corners need the per-evaluation corner pass: no persistent loop");
  if (l->loop == PD_LOOP_PERSISTENT && (c->flags & PD_FLAG_ADAPTIVE_REBUILD))
    return fail(c, PD_ERR_UNSUPPORTED, "early candidate rebuilds need a host decision between steps: no persistent loop");
  const int spb = l->slices_per_block;
  if (!(spb == 1 || spb == 2 || spb == 4 || spb == 8))
    return fail(c, PD_ERR_INVALID, "slices_per_block must be 1, 2, 4 or 8");
  if (l->xcd_remap != 0 && l->xcd_remap != 1) return fail(c, PD_ERR_INVALID, "xcd_remap must be 0 or 1");
  if (l->persistent_blocks < 0) return fail(c, PD_ERR_INVALID, "persistent_blocks must be >= 0");
  if (l->bond_path != PD_BONDS_SLICES && l->bond_path != PD_BONDS_TILES)
    return fail(c, PD_ERR_INVALID, "unknown bond path %d", l->bond_path);
  if (l->bond_path == PD_BONDS_TILES) {
    if (!c->built) return fail(c, PD_ERR_STATE, "the tiled bond loop needs the bonds built first");
    if (!c->tile_ok)
      return fail(c, PD_ERR_UNSUPPORTED,
                  "the tiled bond loop needs horizon factor 3 and every grain's nodes in lattice order");
    if (l->loop != PD_LOOP_GRAPH && l->loop != PD_LOOP_DIRECT)
      return fail(c, PD_ERR_INVALID, "the tiled bond loop runs with the graph or direct step loop only");
  }
  TRY(drop_graphs(c));
  if (c->built && l->bond_path != c->launch.bond_path) {
    // hand the bond memory over: column words <-> class masks
    StepArgs A = step_args(c);
    if (l->bond_path == PD_BONDS_TILES) HIPCHK(c, launch_cols_to_mask(A, c->ctob, c->colOrig, c->stream));
    else HIPCHK(c, launch_mask_to_cols(A, c->ctob, c->colOrig, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->launch = *l;
  return PD_OK;
}

pd_status pd_get_launch(pd_ctx* c, pd_launch* l) {
  if (!c || !l) return PD_ERR_INVALID;
  *l = c->launch;
  return PD_OK;
}

pd_status pd_set_timing(pd_ctx* c, int32_t enable) {
  if (!c) return PD_ERR_INVALID;
  c->timing = enable != 0;
  c->ev_used = 0;
  return PD_OK;
}

pd_status pd_timing(pd_ctx* c, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return PD_ERR_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  int64_t n = 0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
    tot += ms;
    ++n;
  }
  *launches = n;
  *total_ms = tot;
  c->ev_used = 0;
  return PD_OK;
}

pd_status pd_tile_info(pd_ctx* c, int64_t* n_tiles, int32_t* lattice) {
  if (!c || !n_tiles || !lattice) return PD_ERR_INVALID;
  if (!c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  *n_tiles = c->tile_ok ? c->n_tiles : 0;
  *lattice = c->tile_ok ? c->tile_lattice : 0;
  return PD_OK;
}

pd_status pd_loop_counts(pd_ctx* c, int64_t* out6) {
  if (!c || !out6) return PD_ERR_INVALID;
  for (int k = 0; k < 6; ++k) out6[k] = c->counts[k];
  return PD_OK;
}

pd_status pd_info(pd_ctx* c, int64_t* out5) {
  if (!c || !out5) return PD_ERR_INVALID;
  out5[0] = c->n;
  out5[1] = c->nnz;
  out5[2] = c->padded;
  out5[3] = 0;
  if (c->built) {
    int32_t nc = 0;
    HIPCHK(c, hipMemcpyAsync(&nc, c->cand_ptr + c->n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out5[3] = nc;
  }
  out5[4] = c->step;
  return PD_OK;
}

pd_status pd_field_bytes(pd_ctx* c, pd_field f, int64_t* bytes) {
  if (!c || !bytes) return PD_ERR_INVALID;
  const int64_t N = c->n;
  switch (f) {
    case PD_DISPLACEMENT: case PD_VELOCITY: case PD_ACCEL: case PD_FORCE_DENSITY:
      *bytes = 24 * N; return PD_OK;
    case PD_DAMAGE: *bytes = 8 * N; return PD_OK;
    case PD_INTACT_COUNT: case PD_INITIAL_COUNT: *bytes = 4 * N; return PD_OK;
    case PD_BOND_ROWPTR: case PD_CONTACT_ROWPTR: *bytes = 8 * (N + 1); return PD_OK;
    case PD_BOND_COL: *bytes = 4 * c->nnz; return PD_OK;
    case PD_BOND_BROKEN: *bytes = c->nnz; return PD_OK;
    case PD_CONTACT_COL: {
      int64_t info[5];
      TRY(pd_info(c, info));
      *bytes = 4 * std::min<int64_t>(info[3], c->capacity);
      return PD_OK;
    }
    case PD_WALL_FORCE: *bytes = 24 * c->n_walls; return PD_OK;
    case PD_WALL_OFFSET: *bytes = 8 * c->n_walls; return PD_OK;
    case PD_WALL_IMPULSE: *bytes = 24 * c->n_walls; return PD_OK;
    case PD_ENERGY: *bytes = 32; return PD_OK;
    case PD_STEP: *bytes = 8; return PD_OK;
  }
  return fail(c, PD_ERR_INVALID, "unknown field %d", (int)f);
}

pd_status pd_get(pd_ctx* c, pd_field f, void* dst, int64_t dst_bytes, int32_t dst_on_device) {
  if (!c || !dst) return PD_ERR_INVALID;
  const bool needs_build = !(f == PD_STEP || f == PD_WALL_OFFSET);
  if (needs_build && !c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  int64_t need = 0;
  TRY(pd_field_bytes(c, f, &need));
  if (dst_bytes < need) return fail(c, PD_ERR_INVALID, "dst too small: field needs %lld bytes", (long long)need);
  const int64_t N = c->n;
  hipStream_t s = c->stream;
  std::vector<uint8_t> host((size_t)need);
  auto deliver = [&](const void* src_host) -> pd_status {
    if (dst_on_device)
      HIPCHK(c, hipMemcpyAsync(dst, src_host, (size_t)need, hipMemcpyHostToDevice, s));
    else
      memcpy(dst, src_host, (size_t)need);
    HIPCHK(c, hipStreamSynchronize(s));
    return PD_OK;
  };
  auto soa_from_dev = [&](const double* d) -> pd_status {
    HIPCHK(c, hipMemcpyAsync(host.data(), d, (size_t)need, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return deliver(host.data());
  };
  switch (f) {
    case PD_DISPLACEMENT: {
      std::vector<double4> u4((size_t)N);
      HIPCHK(c, hipMemcpyAsync(u4.data(), c->u4[c->cur], sizeof(double4) * N, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      double* o = reinterpret_cast<double*>(host.data());
      for (int64_t i = 0; i < N; ++i) {
        o[i] = u4[i].x;
        o[N + i] = u4[i].y;
        o[2 * N + i] = u4[i].z;
      }
      return deliver(host.data());
    }
    case PD_VELOCITY: return soa_from_dev(c->v);
    case PD_ACCEL: return soa_from_dev(c->a);
    case PD_FORCE_DENSITY: {
      if (!c->F) TRY(alloc_n(c, &c->F, 3 * N, "force output"));
      TRY(sync_columns(c));  // the force-only pass reads the bond memory from the column words
      StepArgs A = step_args(c);
      HIPCHK(c, launch_wall_corners(A, 1, s));
      HIPCHK(c, launch_step(A, MODE_FORCE_ONLY, s));
      return soa_from_dev(c->F);
    }
    case PD_DAMAGE: case PD_INTACT_COUNT: case PD_INITIAL_COUNT: {
      std::vector<int32_t> it((size_t)N), n0((size_t)N);
      HIPCHK(c, hipMemcpyAsync(it.data(), c->intact, 4 * N, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipMemcpyAsync(n0.data(), c->rowlen, 4 * N, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (f == PD_INTACT_COUNT) return deliver(it.data());
      if (f == PD_INITIAL_COUNT) return deliver(n0.data());
      double* o = reinterpret_cast<double*>(host.data());
      for (int64_t i = 0; i < N; ++i) o[i] = n0[i] > 0 ? 1.0 - (double)it[i] / (double)n0[i] : 0.0;
      return deliver(host.data());
    }
    case PD_BOND_ROWPTR: case PD_BOND_COL: case PD_BOND_BROKEN: {
      TRY(sync_columns(c));
      std::vector<int32_t> rl((size_t)N);
      std::vector<uint32_t> col((size_t)c->padded);
      const uint32_t node_mask = (1u << c->node_bits) - 1u;
      std::vector<int64_t> so((size_t)c->nslices + 1);
      HIPCHK(c, hipMemcpyAsync(rl.data(), c->rowlen, 4 * N, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipMemcpyAsync(so.data(), c->slice_off, 8 * (c->nslices + 1), hipMemcpyDeviceToHost, s));
      if (f == PD_BOND_COL)
        HIPCHK(c, hipMemcpyAsync(col.data(), c->colOrig, 4 * c->padded, hipMemcpyDeviceToHost, s));
      if (f == PD_BOND_BROKEN)
        HIPCHK(c, hipMemcpyAsync(col.data(), c->colE, 4 * c->padded, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      int64_t e = 0;
      for (int64_t i = 0; i < N; ++i) {
        const int64_t sl = i / kWave, lane = i % kWave;
        if (f == PD_BOND_ROWPTR) reinterpret_cast<int64_t*>(host.data())[i] = e;
        for (int k = 0; k < rl[(size_t)i]; ++k, ++e) {
          const uint32_t w = col[(size_t)(so[(size_t)sl] + (int64_t)k * kWave + lane)];
          if (f == PD_BOND_COL) reinterpret_cast<int32_t*>(host.data())[e] = (int32_t)(w & node_mask);
          if (f == PD_BOND_BROKEN) host[(size_t)e] = (uint8_t)((w & ~node_mask) == c->sentinel_hi);
        }
      }
      if (f == PD_BOND_ROWPTR) reinterpret_cast<int64_t*>(host.data())[N] = e;
      return deliver(host.data());
    }
    case PD_CONTACT_ROWPTR: case PD_CONTACT_COL: {
      std::vector<int32_t> cp((size_t)N + 1);
      HIPCHK(c, hipMemcpyAsync(cp.data(), c->cand_ptr, 4 * (N + 1), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (f == PD_CONTACT_ROWPTR) {
        int64_t* o = reinterpret_cast<int64_t*>(host.data());
        for (int64_t i = 0; i <= N; ++i) o[i] = cp[(size_t)i];
        return deliver(host.data());
      }
      if (need > 0) {
        HIPCHK(c, hipMemcpyAsync(host.data(), c->cand, (size_t)need, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
      }
      return deliver(host.data());
    }
    case PD_WALL_FORCE: case PD_WALL_OFFSET: case PD_WALL_IMPULSE: {
      std::vector<WallDev> w((size_t)std::max(c->n_walls, 1));
      if (c->n_walls) {
        HIPCHK(c, hipMemcpyAsync(w.data(), c->walls, sizeof(WallDev) * c->n_walls, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
      }
      double* o = reinterpret_cast<double*>(host.data());
      for (int32_t k = 0; k < c->n_walls; ++k) {
        if (f == PD_WALL_FORCE)
          for (int q = 0; q < 3; ++q) o[3 * k + q] = w[(size_t)k].force[q];
        else if (f == PD_WALL_IMPULSE)
          for (int q = 0; q < 3; ++q) o[3 * k + q] = w[(size_t)k].impulse[q];
        else
          o[k] = c->built ? w[(size_t)k].off_used : w[(size_t)k].off;
      }
      return deliver(host.data());
    }
    case PD_ENERGY: {
      TRY(sync_columns(c));
      const int32_t nb = (int32_t)((N + kBlock - 1) / kBlock);
      if (!c->energy_partial) {
        TRY(alloc_n(c, &c->energy_partial, 4 * (int64_t)std::max(nb, 1), "energy partials"));
        TRY(alloc_n(c, &c->energy_out, 4, "energy"));
      }
      StepArgs A = step_args(c);
      HIPCHK(c, launch_energy(A, c->energy_partial, nb, s));
      HIPCHK(c, launch_reduce_energy(c->energy_partial, nb, c->energy_out, s));
      return soa_from_dev(c->energy_out);
    }
    case PD_STEP: {
      memcpy(host.data(), &c->step, 8);
      return deliver(host.data());
    }
  }
  return fail(c, PD_ERR_INVALID, "unknown field %d", (int)f);
}

pd_status pd_energy_noalloc(pd_ctx* c, double* out4, int32_t out_on_device) {
  if (!c || !out4) return PD_ERR_INVALID;
  if (!c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  const int64_t nb = (c->n + kBlock - 1) / kBlock;
  if (nb > kNoAllocPartials)
    return fail(c, PD_ERR_INVALID, "%lld nodes need %lld energy partials; the static scratch holds %lld",
                (long long)c->n, (long long)nb, (long long)kNoAllocPartials);
  if (!c->scratch_dev) return fail(c, PD_ERR_STATE, "no scratch address for this context's device");
  hipStream_t s = c->stream;
  TRY(sync_columns(c));  // the energy kernel reads the bond memory from the column words
  StepArgs A = step_args(c);
  double* red = c->scratch_dev + 4 * kNoAllocPartials;
  HIPCHK(c, launch_energy(A, c->scratch_dev, (int32_t)nb, s));
  HIPCHK(c, launch_reduce_energy(c->scratch_dev, (int32_t)nb, out_on_device ? out4 : red, s));
  if (!out_on_device) HIPCHK(c, hipMemcpyAsync(out4, red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return PD_OK;
}

pd_status pd_set_wall(pd_ctx* c, int32_t w, const pd_wall* wall) {
  if (!c || !wall) return PD_ERR_INVALID;
  if (w < 0 || w >= c->n_walls) return fail(c, PD_ERR_INVALID, "wall index %d out of range", w);
  TRY(check_wall(c, *wall, w));
  WallDev old;
  HIPCHK(c, hipMemcpyAsync(&old, c->walls + w, sizeof(WallDev), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  WallDev d = to_dev(*wall, c->built ? c->step + 1 : 0, c->dt);
  d.off_used = old.off_used;
  for (int q = 0; q < 3; ++q) {
    d.force[q] = old.force[q];
    d.impulse[q] = old.impulse[q];
  }
  HIPCHK(c, hipMemcpyAsync(c->walls + w, &d, sizeof(WallDev), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->walls_h[(size_t)w] = d;
  return PD_OK;
}

// checkpoint layout: header[8] (magic, n, padded, n_walls, step, cur, nnz, crc-less size),
// then u4[cur], u4[cur^1], v, a, live column words, intact, u_build, walls,
// [vh[cur], vh[cur^1] when damping or friction is on], crc32
pd_status pd_get_state(pd_ctx* c, void* blob, int64_t* bytes) {
  Range r("pd_get_state");
  if (!c || !bytes) return PD_ERR_INVALID;
  if (!c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  const int64_t N = c->n;
  const int64_t words = c->padded;
  const int64_t nvh = (c->beta > 0 || c->mu > 0) ? 2 * 32 * N : 0;
  const int64_t body = 8 * 8 + 2 * 32 * N + 2 * 24 * N + 4 * words + 4 * N + 24 * N +
                       (int64_t)sizeof(WallDev) * c->n_walls + nvh;
  const int64_t total = body + 4;
  if (!blob) {
    *bytes = total;
    return PD_OK;
  }
  if (*bytes < total) return fail(c, PD_ERR_INVALID, "checkpoint buffer needs %lld bytes", (long long)total);
  uint8_t* p = static_cast<uint8_t*>(blob);
  const int64_t hdr[8] = {(int64_t)kMagic, N, c->padded, c->n_walls, c->step, 0, c->nnz, body};
  memcpy(p, hdr, sizeof hdr);
  int64_t o = sizeof hdr;
  hipStream_t s = c->stream;
  auto grab = [&](const void* d, int64_t n) -> pd_status {
    if (n) HIPCHK(c, hipMemcpyAsync(p + o, d, (size_t)n, hipMemcpyDeviceToHost, s));
    o += n;
    return PD_OK;
  };
  TRY(grab(c->u4[c->cur], 32 * N));
  TRY(grab(c->u4[c->cur ^ 1], 32 * N));
  TRY(grab(c->v, 24 * N));
  TRY(grab(c->a, 24 * N));
  TRY(sync_columns(c));
  TRY(grab(c->colE, 4 * words));
  TRY(grab(c->intact, 4 * N));
  TRY(grab(c->u_build, 24 * N));
  TRY(grab(c->walls, (int64_t)sizeof(WallDev) * c->n_walls));
  if (nvh) {
    TRY(grab(c->vh[c->cur], 32 * N));
    TRY(grab(c->vh[c->cur ^ 1], 32 * N));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  const uint32_t crc = crc32_update(0, p, (size_t)body);
  memcpy(p + body, &crc, 4);
  *bytes = total;
  return PD_OK;
}

pd_status pd_set_state(pd_ctx* c, const void* blob, int64_t bytes) {
  Range r("pd_set_state");
  if (!c || !blob) return PD_ERR_INVALID;
  if (!c->built) return fail(c, PD_ERR_STATE, "pd_build_bonds must come first");
  const uint8_t* p = static_cast<const uint8_t*>(blob);
  if (bytes < 68) return fail(c, PD_ERR_CORRUPT, "checkpoint too short");
  int64_t hdr[8];
  memcpy(hdr, p, sizeof hdr);
  const int64_t N = c->n, words = c->padded;
  const int64_t nvh = (c->beta > 0 || c->mu > 0) ? 2 * 32 * N : 0;
  const int64_t body = 8 * 8 + 2 * 32 * N + 2 * 24 * N + 4 * words + 4 * N + 24 * N +
                       (int64_t)sizeof(WallDev) * c->n_walls + nvh;
  if (hdr[0] != (int64_t)kMagic || hdr[1] != N || hdr[2] != c->padded || hdr[3] != c->n_walls ||
      hdr[6] != c->nnz || hdr[7] != body || bytes != body + 4)
    return fail(c, PD_ERR_CORRUPT, "checkpoint does not match this context");
  uint32_t crc;
  memcpy(&crc, p + body, 4);
  if (crc32_update(0, p, (size_t)body) != crc) return fail(c, PD_ERR_CORRUPT, "checkpoint CRC mismatch");
  hipStream_t s = c->stream;
  int64_t o = sizeof hdr;
  auto put = [&](void* d, int64_t n) -> pd_status {
    if (n) HIPCHK(c, hipMemcpyAsync(d, p + o, (size_t)n, hipMemcpyHostToDevice, s));
    o += n;
    return PD_OK;
  };
  c->cur = (int)(hdr[4] & 1);  // u4[step % 2] holds u_step, the invariant captured graphs rely on
  TRY(put(c->u4[c->cur], 32 * N));
  TRY(put(c->u4[c->cur ^ 1], 32 * N));
  TRY(put(c->v, 24 * N));
  TRY(put(c->a, 24 * N));
  TRY(put(c->colE, 4 * words));
  TRY(put(c->intact, 4 * N));
  TRY(put(c->u_build, 24 * N));
  TRY(put(c->walls, (int64_t)sizeof(WallDev) * c->n_walls));
  if (nvh) {
    TRY(put(c->vh[c->cur], 32 * N));
    TRY(put(c->vh[c->cur ^ 1], 32 * N));
  }
  if (c->launch.bond_path == PD_BONDS_TILES) {
    StepArgs A = step_args(c);
    HIPCHK(c, launch_cols_to_mask(A, c->ctob, c->colOrig, s));
  }
  c->step = hdr[4];
  HIPCHK(c, hipMemcpyAsync(c->step_d, &c->step, 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  // the candidate list of the last rebuild, rebuilt from the positions it was made from
  {
    double4* tmp;
    TRY(alloc_n(c, &tmp, N, "rebuild staging"));
    ContactArgs C = contact_args(c, c->cur);
    std::vector<double4> ub((size_t)N);
    HIPCHK(c, hipMemcpyAsync(ub.data(), c->u4[c->cur], 32 * N, hipMemcpyDeviceToHost, s));
    std::vector<double> bld((size_t)(3 * N));
    HIPCHK(c, hipMemcpyAsync(bld.data(), c->u_build, 24 * N, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int64_t i = 0; i < N; ++i) {
      ub[(size_t)i].x = bld[(size_t)i];
      ub[(size_t)i].y = bld[(size_t)(N + i)];
      ub[(size_t)i].z = bld[(size_t)(2 * N + i)];
    }
    HIPCHK(c, hipMemcpyAsync(tmp, ub.data(), 32 * N, hipMemcpyHostToDevice, s));
    C.u = tmp;
    HIPCHK(c, launch_contact_rebuild(C, 0, s));
    HIPCHK(c, hipStreamSynchronize(s));
    dev_free(c, tmp);
  }
  return report_status(c);
}

void pd_destroy(pd_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  std::vector<void*> all = c->owned;
  for (void* p : all) dev_free(c, p);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
