// Internal declarations shared by the host runtime and the HIP kernels of the
// peridynamic grain-aggregate library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pd.h"

namespace pdk {

constexpr int kWave = 64;           // CDNA wavefront
constexpr int kBlock = 256;         // 4 waves = 4 SELL slices per workgroup
constexpr int kSlicesPerBlock = kBlock / kWave;
constexpr int kMaxWalls = 8;
constexpr int kMaxHorizon = 6;      // m <= 6 keeps |d|^2 <= 36 and rows <= 925
constexpr int kMaxD2 = kMaxHorizon * kMaxHorizon;
constexpr int kCellDirs = 27;
constexpr int kChunk = 1024;        // wall-partial columns reduced by one workgroup
#ifndef PD_CONTACT_BATCH
#define PD_CONTACT_BATCH 2
#endif
constexpr int kContactBatch = PD_CONTACT_BATCH;  // contact candidates whose gathers a lane issues together
#ifndef PD_BOND_UNROLL
#define PD_BOND_UNROLL 8
#endif
constexpr int kUnroll = PD_BOND_UNROLL;  // bond entries in flight per lane; slice widths are padded to it

// per-grain constants
struct GrainC {
  double cVih;    // c * V / h (micromodulus, or c0 of the conic form, times nodal volume, over h)
  double conic_inv_delta;  // 1/delta with the conic micromodulus c0 (1 - |xi|/delta), else 0
  double thr;     // h^2 s0 (2 + s0): bond breaks when |y|^2 - |xi|^2 > thr * |d|^2  (s > s0)
  double abs_ratio;  // (2 - s0) / (2 + s0): with the |s| reading a bond also breaks when
                     // |y|^2 - |xi|^2 < -abs_ratio * thr * |d|^2  (s < -s0)
  double h;
  double V;       // h^3
  double rho;
  double origin[3];
  int32_t mat;
  int32_t cls;    // index of the (h, material) stencil table
};

// One row per horizon-stencil offset d (lexicographic order) and per
// (h, material) class, with every constant of the bond law folded in:
// xi = h d, the break threshold on |y|^2 - |xi|^2, 1/|xi|^2, c V / |xi|,
// |xi| and |xi|^2.  The last row of each class is the zero-force class used by
// broken bonds and padding.
struct StencilC {
  double hx, hy, hz;  // xi
  double thr_d;       // |xi|^2 ((1 + s0)^2 - 1)
  double inv_l0sq;    // 1 / |xi|^2
  double civ;         // c V / |xi|
  double l0, l0sq;    // |xi|, |xi|^2
};
constexpr int kMaxLdsTables = 48 * 1024;  // bytes of stencil tables a workgroup may stage
constexpr int kMaxStencil = 1024;
constexpr int kCornerGL = 32;  // Gauss-Legendre points per piece of a wall-corner region integral

// ---- tiled bond loop (horizon factor 3): a workgroup owns a tile of
// kTS x kTM x kTF lattice cells of one grain, in the grain's node-ordering axes
// (s slowest, m, f fastest), and stages u of the tile plus a kTileR-cell halo in
// LDS.  The 122 horizon classes run in lexicographic (ds, dm, df) order, the
// order of ascending neighbour index.  The bond memory is one 64-bit lane mask
// per (wavefront of a tile, class): bit l says the bond of class K of the node
// in lane l is intact, so the kernel tests and updates it in scalar registers.
constexpr int kTileR = 3;
#ifndef PD_TILE_LAYERS
#define PD_TILE_LAYERS 8
#endif
#ifndef PD_TILE_M
#define PD_TILE_M 4
#endif
#ifndef PD_TILE_F
#define PD_TILE_F 16
#endif
constexpr int kTS = PD_TILE_LAYERS, kTM = PD_TILE_M, kTF = PD_TILE_F;  // one s-layer of kTM x kTF cells per wavefront
static_assert(kTM * kTF == kWave, "a wavefront holds one layer of a tile");
constexpr int kHS = kTS + 2 * kTileR, kHM = kTM + 2 * kTileR, kHF = kTF + 2 * kTileR;
constexpr int kHalo = kHS * kHM * kHF;      // 3080 cells, 73920 B of FP64 planes (8 layers)
constexpr int kTileClasses = 122;           // 0 < |d|^2 <= 9

// A tile box: a grain's own lattice box, or (lattice mode) one box over every
// grain when all of them share one lattice, spacing, bond table and node order.
// Entries 0..G-1 describe the grains; in lattice mode entry G is the shared box
// and each grain's box field points at it.
struct TileGrain {
  int64_t map_off;     // cell (s, m, f) of the box -> node at tmap[map_off + (s em + m) ef + f]
  int32_t es, em, ef;  // box extents in the node-ordering axes
  int32_t table;       // bond table: ttab[table * kTileClasses + class] (slice-path StencilC rows)
  int32_t perm;        // node-ordering axes (slowest first): index into the six axis orders
  int32_t lo_s, lo_m, lo_f;  // lattice index of the box corner on those axes
  int32_t box;         // the box this grain's nodes are tiled in (itself, or the shared box)
  int32_t goff[3];     // x, y, z offset of the grain's lattice indices in that box's lattice
};

struct WallDev {
  double n[3];
  double off0;      // offset at t = 0
  double off;       // offset used by the next force evaluation
  double off_used;  // offset used by the last force evaluation
  double vel;
  double lo[3], hi[3];
  double target, gain, area;
  double rate;      // d(offset)/dt over the step into the next evaluation
  double rate_used; // the same for the last evaluation
  double force[3];  // reaction of the last evaluation
  double impulse[3];  // sum over completed steps of force * dt
  int32_t mode;
  int32_t pad;
};

struct CutDev {
  int64_t kind, grain, plane[4], lo[3], hi[3], c[3], r2;
};

// status word bits
enum : uint32_t {
  ST_NAN = 1u,
  ST_PENETRATION = 2u,
  ST_SKIN = 4u,
  ST_CAND_OVERFLOW = 8u,
  ST_BARRIER = 16u,  // a grid-barrier wait of the persistent kernel gave up
  ST_REBUILD = 32u,  // early-rebuild watch: a node moved skin/2; the step was not taken
};

enum ForceMode { MODE_FIRST = 0, MODE_STEP = 1, MODE_FORCE_ONLY = 2 };

// everything the fused step kernel reads
struct StepArgs {
  const double4* ucur;  // (x,y,z, packed ijk | grain<<32)
  double4* unext;
  double* v;            // SoA
  double* a;            // SoA
  double* Fout;         // MODE_FORCE_ONLY output (SoA)
  const double4* vh_cur;  // mid-step velocity seen by damping and friction (beta or mu > 0)
  double4* vh_next;       // ... written for the next evaluation
  const uint8_t* fixed;
  const GrainC* grains;
  const StencilC* stencil;  // [n_classes][n_stencil + 1]
  int32_t n_stencil;
  int32_t n_classes;
  int32_t node_bits;        // column word = node | stencil_class << node_bits
  uint32_t sentinel_hi;     // zero-force class << node_bits (broken bonds and padding)
  const int64_t* slice_off;
  const int32_t* rowlen;
  uint32_t* colE;           // live column words; a broken bond becomes node_i | sentinel_hi
  int32_t* intact;
  const int32_t* cand_ptr;
  const int32_t* cand;
  int64_t cand_capacity;
  const double* X;      // SoA, contact path only
  const double4* X4;    // the same as (x, y, z, 0) per node: one load per contact candidate
  const double* Kn;     // [n_mat * n_mat]
  WallDev* walls;
  double* wall_partial;  // [n_walls][3][partial_stride]: one column per slice (component-major)
  double* wall_chunk;    // [n_walls][3][chunks]: sums of 1024-column chunks of wall_partial
  int64_t* step;         // device step counter
  int32_t advance;       // 1 when this evaluation completes a step, 0 for the initial one
  uint32_t* status;
  // status as it stood when the current step began (written by the last kernel
  // of each step): once nonzero, the kernels of later steps change nothing, so
  // the state stays at the step that raised the flag
  uint32_t* halt;
  int64_t n;
  int64_t nslices;
  int32_t n_walls;
  int32_t n_mat;
  double Rc, Rc2;
  double dt;
  double g[3];
  double beta;           // normal damping coefficient, 0 = off
  double mu;             // stick-slip friction coefficient, 0 = off
  int32_t abs_stretch;
  // launch geometry: the slices [slice_base, slice_end) of this launch, nodes
  // outside [node_lo, node_hi) idle (per-grain launches), and the column of
  // wall_partial that slice s writes (partial_base + s - slice_base of partial_stride)
  int64_t slice_base, slice_end;
  int64_t node_lo, node_hi;
  int64_t partial_base, partial_stride;
  int32_t xcd_remap;     // 1: workgroup -> XCD-contiguous slice ranges
  // tiled bond loop (launch_step_tile): tile records (grain, s0, m0, f0), the
  // per-grain boxes and cell maps, bond tables and per-node class masks
  // (lane masks); the tile kernel's wall partials use column kTS t + wave
  const int4* tiles;
  int64_t n_tiles;
  const TileGrain* tgrain;
  const int32_t* tmap;
  const StencilC* ttab;
  uint64_t* lmask;        // [n_tiles * kTS][kTileClasses] lane masks of intact bonds
  const int32_t* slot;    // [n]: node -> (tile * kTS + wavefront) * 64 + lane, or -1
  // self-contact inside a grain (Sec. 5): a same-grain candidate pair is
  // skipped while its bond is intact, found in the built column words (rows
  // sorted by neighbour) and, on the tiled path, the class masks through ctob
  // ([6][n_stencil] slice class -> mask bit per axis order)
  int32_t self_contact;
  const uint32_t* colOrig;
  const int16_t* ctob;
  // inclusion-exclusion of orthogonal walls at a corner (Sec. 4.1.1):
  // Gauss-Legendre nodes and weights on [0, pi] for the region integrals
  int32_t wall_corners;
  const double* corner_gl;  // [2][corner_ngl]
  int32_t corner_ngl;
  uint32_t* corner_w;       // [n] walls touched: count | indices << 8 (k + 1), 0 below two
  double* corner_c;         // [n][3] corrections of those walls' normal magnitudes
};

// grid barrier state of the persistent step kernel (zeroed before each launch)
struct BarrierArgs {
  uint32_t* count;
  uint32_t* gen;
  uint32_t spin_limit;  // iterations of a wait before it gives up and flags ST_BARRIER
};

struct BuildArgs {
  const double4* u;
  const int64_t* gmap_off;   // [G]
  const int32_t* gmap_dim;   // [3G]
  const int32_t* gmap_lo;    // [3G]
  int32_t* gmap;
  const CutDev* cuts;
  const int32_t* cut_begin;  // [G+1]
  const int32_t* stencil;    // [n_stencil] packed (dx+8) | (dy+8)<<8 | (dz+8)<<16, lexicographic
  int32_t n_stencil;
  int32_t node_bits;
  uint32_t sentinel_hi;
  int64_t n;
  int32_t* rowlen;
  int64_t* slice_off;
  uint32_t* colE;
  uint32_t* colOrig;         // column words as built (kept for output)
  int64_t nslices;
};

struct ContactArgs {
  const double4* u;
  const double* X;
  const double4* X4;  // (x, y, z, 0) per node: one load per candidate position
  long long* cellkey;    // [N] packed cell coordinates of each binned node
  uint32_t* cellh;       // [N]
  int32_t* bucket_count;  // [T]
  int32_t* bucket_start;  // [T+1]
  int32_t* bucket_fill;   // [T]
  int4* srec;             // [N] bucket-sorted (node, grain, cell key lo, hi)
  int32_t* cand_scratch;  // [N][scratch_w] unsorted candidates of each node
  int32_t scratch_w;
  int32_t* cand_count;    // [N+1] (scanned in place to cand_ptr)
  int32_t* cand;
  double* u_build;        // SoA
  int32_t* scan_scratch;  // >= scan_scratch_elems(max(T, N))
  long long* gbox;        // [G][6] order-preserving encodings of min xyz, max xyz of p
  int32_t* gpair_count;   // [G+1] (scanned in place)
  int32_t* gpair;         // [G*G] other grains whose boxes come within the cutoff
  uint8_t* active;        // [N] node within the cutoff of another grain's box
  const int64_t* box_chunks;  // [n_box_chunks][3]: grain, first node, end node (one grain each)
  int32_t n_box_chunks;
  int32_t n_grains;
  uint32_t* status;
  const uint32_t* halt;   // nonzero: an earlier step raised a flag; leave the positions at rebuild alone
  int64_t n;
  uint32_t T;             // power of two
  // cell grid of this rebuild (k_grid_setup): [0] 1 when the cells of the box
  // around all nodes fit in T buckets, which are then the cells themselves in
  // lexicographic order (neighbouring cells sit next to each other in memory);
  // otherwise cells are hashed into the T buckets.  [1..3] the box's first
  // cell, [4..6] its extent in cells.
  int64_t* grid;
  int64_t capacity;
  double inv_cell;
  double cut2;            // (R_c + skin)^2
  double skin_half2;
  // self-contact: nodes of the node's own grain are candidates too
  int32_t self_contact;
};

// ---- launchers (pd_kernels.hip) ----
hipError_t launch_map_fill(const BuildArgs& b, hipStream_t s);
hipError_t launch_bond_count(const BuildArgs& b, hipStream_t s);
hipError_t launch_slice_width(const BuildArgs& b, hipStream_t s);
hipError_t launch_bond_fill(const BuildArgs& b, hipStream_t s);
hipError_t launch_step(const StepArgs& a, int mode, hipStream_t s);
// corner corrections of this evaluation (before the step kernel)
hipError_t launch_wall_corners(const StepArgs& a, int force_only, hipStream_t s);
// MODE_STEP with slices_per_block in {1, 2, 4, 8}; e0/e1, when given, are
// recorded by the launch itself around the kernel
hipError_t launch_step_spb(const StepArgs& a, int slices_per_block, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
// nsteps steps with no rebuild in between, one cooperative launch of nblocks
// workgroups that share out the 4-slice blocks of every step and meet at one
// grid barrier per step
hipError_t launch_step_persistent(const StepArgs& a, int64_t nsteps, int32_t nblocks, const BarrierArgs& b,
                                  hipStream_t s);
// workgroups of the persistent kernel that fit on the device at once
int32_t persistent_max_blocks(const StepArgs& a);
int32_t step_blocks_spb(int64_t nslices, int slices_per_block);
// wall reactions, next wall offsets and the step counter after a step launch
hipError_t launch_wall_finalize(const StepArgs& a, hipStream_t s);

hipError_t launch_contact_rebuild(const ContactArgs& c, int check_skin, hipStream_t s);
hipError_t launch_skin_watch(const ContactArgs& c, uint32_t* halt, hipStream_t s);
hipError_t launch_energy(const StepArgs& a, double* partial4, int32_t nblocks, hipStream_t s);
hipError_t launch_reduce_energy(const double* partial4, int32_t nblocks, double* out4,
                                hipStream_t s);
hipError_t launch_fill_u4(double4* u4, const double* u, const int32_t* ijk, const int64_t* grain_of,
                          int64_t n, hipStream_t s);
// exclusive scans with a total in out[n]; scratch >= scan_scratch_elems(n) elements
int64_t scan_scratch_elems(int64_t n);
hipError_t scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s);
hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s);
int32_t step_grid_blocks(int64_t nslices);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// X4[i] = (X[i], X[n + i], X[2n + i], 0)
hipError_t launch_pack_x4(const double* X, double4* X4, int64_t n, hipStream_t s);
// tiled bond loop: MODE_STEP over all tiles (events as for launch_step_spb)
hipError_t launch_step_tile(const StepArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// per-node cell map of the tile grains: tmap[map_off + (s em + m) ef + f] = node
hipError_t launch_tile_map_fill(const StepArgs& a, hipStream_t s);
// bond state between the slice path's column words and the tile path's class
// masks; ctob[perm][slice class] = mask bit (or -1)
hipError_t launch_cols_to_mask(const StepArgs& a, const int16_t* ctob, const uint32_t* colOrig,
                               hipStream_t s);
hipError_t launch_mask_to_cols(const StepArgs& a, const int16_t* ctob, const uint32_t* colOrig,
                               hipStream_t s);

}  // namespace pdk
