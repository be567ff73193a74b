// HIP kernels (gfx950) of the peridynamic grain-aggregate step.
//
// Layout in HBM
//   u      : two buffers of double4 (x, y, z, w); w carries the node's packed
//            grain-local lattice index (10 bits per axis) in its low 32 bits
//            and its grain id in the high 32 bits, so one 32-byte gather per
//            bond brings both the neighbour displacement and its lattice offset.
//   v, a   : SoA FP64, touched only by the owning lane.
//   bonds  : sliced-ELL (SELL-64) CSR.  Slice s = nodes [64 s, 64 s + 64) (one
//            wavefront); entry k of lane l sits at colE[slice_off[s] + 64 k + l],
//            so the column loads of a wavefront are one coalesced 256-byte read.
//            A column word is node_j | class << node_bits, class = index of the
//            lattice offset in the horizon stencil.  Bond memory lives in the
//            word itself: a bond that breaks is rewritten to node_i with the
//            zero-force class, which is also what padding entries hold, so the
//            step kernel needs no separate broken-flag reads.
//
// Each lane owns one node and evaluates its row in order (gather formulation,
// Sec. 3.1 eq. (peri-damage) with nodal quadrature, Sec. 6.1): no atomics, so
// results are bitwise reproducible run to run.

#include <hip/hip_ext.h>

#include <algorithm>
#include <utility>

#include "pd_internal.h"

namespace pdk {

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; map them
// so each XCD walks one contiguous range of slices (its L2 then holds that
// range's neighbourhood instead of every eighth slice of the whole mesh).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// the halt word, read the same by every lane of the launch
__device__ __forceinline__ bool halted(const uint32_t* halt) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(halt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0u;
}

__device__ __forceinline__ int unpack_x(int p) { return p & 1023; }
__device__ __forceinline__ int unpack_y(int p) { return (p >> 10) & 1023; }
__device__ __forceinline__ int unpack_z(int p) { return (p >> 20) & 1023; }
__device__ __forceinline__ int packed_ijk(double w) { return (int)(__double_as_longlong(w) & 0xffffffffll); }
__device__ __forceinline__ int packed_grain(double w) { return (int)(__double_as_longlong(w) >> 32); }

// reference position origin + h*ijk evaluated exactly as the input lays it out
__device__ __forceinline__ double lattice_pos(double origin, double h, int idx) {
  return __dadd_rn(origin, __dmul_rn(h, (double)idx));
}

// 1/sqrt(x) to full double precision: hardware estimate refined by one
// Newton step with the cubic term, r (1 + e/2 + 3e^2/8), e = 1 - x r^2.
__device__ __forceinline__ double rsqrt_full(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double t = x * r;
  const double e = fma(-t, r, 1.0);
  return fma(r * e, fma(0.375, e, 0.5), r);
}

// 1/x to full double precision: hardware estimate refined by r (1 + e + e^2),
// e = 1 - x r.
__device__ __forceinline__ double rcp_full(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// ---------------------------------------------------------------------------
// bond family (Sec. 3.1) and bond removal (Sec. 6.3)
// ---------------------------------------------------------------------------

constexpr int64_t kUnbounded = ((int64_t)1) << 50;

// The notch plane cuts the segment A->B strictly inside (0 < t < 1) exactly
// when the plane function changes sign between the endpoints; the crossing
// point A + t (B - A), t = fA / (fA - fB), is tested against the bounds with
// everything multiplied by the positive denominator.
__device__ bool notch_cuts(const CutDev& c, const int64_t A[3], const int64_t B[3]) {
  const int64_t fa = c.plane[0] * A[0] + c.plane[1] * A[1] + c.plane[2] * A[2] + c.plane[3];
  const int64_t fb = c.plane[0] * B[0] + c.plane[1] * B[1] + c.plane[2] * B[2] + c.plane[3];
  if (fa == 0 || fb == 0 || ((fa < 0) == (fb < 0))) return false;
  int64_t num = fa, den = fa - fb;
  if (den < 0) {
    num = -num;
    den = -den;
  }
  for (int q = 0; q < 3; ++q) {
    const int64_t qs = A[q] * den + num * (B[q] - A[q]);
    if (c.lo[q] > -kUnbounded && qs < c.lo[q] * den) return false;
    if (c.hi[q] < kUnbounded && qs > c.hi[q] * den) return false;
  }
  return true;
}

__device__ __forceinline__ int64_t sq_dist(const int64_t A[3], const int64_t C[3]) {
  const int64_t a = A[0] - C[0], b = A[1] - C[1], d = A[2] - C[2];
  return a * a + b * b + d * d;
}

// closest point of segment A->B to the centre, all in integers
__device__ bool chord_cuts(const CutDev& c, const int64_t A[3], const int64_t B[3]) {
  int64_t D[3], W[3];
  for (int q = 0; q < 3; ++q) {
    D[q] = B[q] - A[q];
    W[q] = c.c[q] - A[q];
  }
  const int64_t dd = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
  const int64_t wd = W[0] * D[0] + W[1] * D[1] + W[2] * D[2];
  if (wd <= 0) return sq_dist(A, c.c) < c.r2;
  if (wd >= dd) return sq_dist(B, c.c) < c.r2;
  const int64_t ww = W[0] * W[0] + W[1] * W[1] + W[2] * W[2];
  return ww * dd - wd * wd < c.r2 * dd;
}

__device__ bool cut_between(const CutDev* cuts, const int32_t* cut_begin, int g, int pi, int pj) {
  const int c0 = cut_begin[g], c1 = cut_begin[g + 1];
  if (c0 == c1) return false;
  const int64_t A[3] = {2 * (int64_t)unpack_x(pi), 2 * (int64_t)unpack_y(pi), 2 * (int64_t)unpack_z(pi)};
  const int64_t B[3] = {2 * (int64_t)unpack_x(pj), 2 * (int64_t)unpack_y(pj), 2 * (int64_t)unpack_z(pj)};
  for (int k = c0; k < c1; ++k) {
    const CutDev& c = cuts[k];
    if (c.kind == 0 && notch_cuts(c, A, B)) return true;
    if (c.kind == 1 && (sq_dist(A, c.c) < c.r2 || sq_dist(B, c.c) < c.r2)) return true;
    if (c.kind == 2 && chord_cuts(c, A, B)) return true;
  }
  return false;
}

__device__ __forceinline__ bool bond_cut(const BuildArgs& b, int g, int pi, int pj) {
  return cut_between(b.cuts, b.cut_begin, g, pi, pj);
}

// node index at lattice point ijk + d of grain g, or -1
__device__ __forceinline__ int lookup(const BuildArgs& b, int g, int p, int s) {
  const int dx = (s & 255) - 8, dy = ((s >> 8) & 255) - 8, dz = ((s >> 16) & 255) - 8;
  const int lx = unpack_x(p) - b.gmap_lo[3 * g] + dx;
  const int ly = unpack_y(p) - b.gmap_lo[3 * g + 1] + dy;
  const int lz = unpack_z(p) - b.gmap_lo[3 * g + 2] + dz;
  const int ex = b.gmap_dim[3 * g], ey = b.gmap_dim[3 * g + 1], ez = b.gmap_dim[3 * g + 2];
  if (lx < 0 || ly < 0 || lz < 0 || lx >= ex || ly >= ey || lz >= ez) return -1;
  return b.gmap[b.gmap_off[g] + ((int64_t)lx * ey + ly) * ez + lz];
}

__global__ void k_map_fill(BuildArgs b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const double w = b.u[i].w;
  const int p = packed_ijk(w), g = packed_grain(w);
  const int lx = unpack_x(p) - b.gmap_lo[3 * g];
  const int ly = unpack_y(p) - b.gmap_lo[3 * g + 1];
  const int lz = unpack_z(p) - b.gmap_lo[3 * g + 2];
  const int ey = b.gmap_dim[3 * g + 1], ez = b.gmap_dim[3 * g + 2];
  b.gmap[b.gmap_off[g] + ((int64_t)lx * ey + ly) * ez + lz] = (int32_t)i;
}

__global__ void k_bond_count(BuildArgs b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const double w = b.u[i].w;
  const int p = packed_ijk(w), g = packed_grain(w);
  int cnt = 0;
  for (int k = 0; k < b.n_stencil; ++k) {
    const int j = lookup(b, g, p, b.stencil[k]);
    if (j < 0) continue;
    if (bond_cut(b, g, p, packed_ijk(b.u[j].w))) continue;
    ++cnt;
  }
  b.rowlen[i] = cnt;
}

// padded slot count (64 * widest row) of every slice
__global__ void k_slice_width(BuildArgs b) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.nslices) return;
  int w = 0;
  for (int l = 0; l < kWave; ++l) {
    const int64_t i = s * kWave + l;
    if (i < b.n) w = max(w, b.rowlen[i]);
  }
  w = (w + kUnroll - 1) / kUnroll * kUnroll;
  b.slice_off[s] = (int64_t)w * kWave;
}

// one wavefront per slice: write the row (stencil order), sort it ascending,
// pad it with the node itself and write the slice's padding masks
__global__ __launch_bounds__(kBlock) void k_bond_fill(BuildArgs b) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
  if (s >= b.nslices) return;  // whole wavefront leaves together
  const int64_t i = s * kWave + lane;
  const bool valid = i < b.n;
  const int64_t off = b.slice_off[s];
  const int W = (int)((b.slice_off[s + 1] - off) / kWave);
  uint32_t* col = b.colE + off + lane;
  uint32_t* orig = b.colOrig + off + lane;
  const uint32_t node_mask = (1u << b.node_bits) - 1u;
  int len = 0;
  if (valid) {
    const double w = b.u[i].w;
    const int p = packed_ijk(w), g = packed_grain(w);
    for (int k = 0; k < b.n_stencil; ++k) {
      const int j = lookup(b, g, p, b.stencil[k]);
      if (j < 0) continue;
      if (bond_cut(b, g, p, packed_ijk(b.u[j].w))) continue;
      col[(int64_t)len * kWave] = (uint32_t)j | ((uint32_t)k << b.node_bits);
      ++len;
    }
    // insertion sort on the node index (rows come out nearly sorted)
    for (int k = 1; k < len; ++k) {
      const uint32_t x = col[(int64_t)k * kWave];
      int q = k - 1;
      while (q >= 0 && (col[(int64_t)q * kWave] & node_mask) > (x & node_mask)) {
        col[(int64_t)(q + 1) * kWave] = col[(int64_t)q * kWave];
        --q;
      }
      col[(int64_t)(q + 1) * kWave] = x;
    }
    for (int k = len; k < W; ++k) col[(int64_t)k * kWave] = (uint32_t)i | b.sentinel_hi;
  } else {
    for (int k = 0; k < W; ++k) col[(int64_t)k * kWave] = b.sentinel_hi;
  }
  for (int k = 0; k < W; ++k) orig[(int64_t)k * kWave] = col[(int64_t)k * kWave];
}

// ---------------------------------------------------------------------------
// the fused step: bond force + break + damage, contact, walls, velocity Verlet
// ---------------------------------------------------------------------------

// contact distance exactly as p_j - p_i = (X_j - X_i) + (u_j - u_i), no contraction
__device__ __forceinline__ double contact_d2(double xj, double xi, double uj, double ui, double yj,
                                             double yi, double vj, double vi, double zj, double zi,
                                             double wj, double wi, double& dx, double& dy,
                                             double& dz) {
  dx = __dadd_rn(__dsub_rn(xj, xi), __dsub_rn(uj, ui));
  dy = __dadd_rn(__dsub_rn(yj, yi), __dsub_rn(vj, vi));
  dz = __dadd_rn(__dsub_rn(zj, zi), __dsub_rn(wj, wi));
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

#ifndef PD_STEP_WAVES_PER_EU
#define PD_STEP_WAVES_PER_EU 4
#endif

// 1 - (1 + x)^(-1/2) = x q(x).  For |x| <= kPolyRange q is a degree-8
// polynomial: the interpolant of q at the nine Chebyshev nodes of the interval
// (coefficients from csrc/bond_series.py), constant term exactly 1/2, relative
// error about 1e-18 with its coefficients in double.
constexpr double kPolyRange = 0.02;
// The eight non-trivial coefficients, highest degree first.  They may be held
// in registers (poly_in_registers), with the same arithmetic either way: as
// literals the compiler rebuilds each 64-bit constant with two moves per use.
struct PolyG {
  double c[8];
};
constexpr PolyG kPolyG{{0x1.7c2767adf6933p-3, -0x1.92832f94213d7p-3, 0x1.acfff9e68ffc4p-3, -0x1.cdfff99c37884p-3,
                        0x1.f80000002c6aep-3, -0x1.1800000017442p-2, 0x1.3fffffffffffdp-2, -0x1.7fffffffffffdp-2}};
__device__ __forceinline__ PolyG poly_in_registers() {
  PolyG P = kPolyG;
#pragma unroll
  for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(P.c[k]));
  return P;
}
__device__ __forceinline__ double one_minus_rsqrt1p_over_x(double x, const PolyG& P) {
  double p = fma(P.c[0], x, P.c[1]);
#pragma unroll
  for (int k = 2; k < 8; ++k) p = fma(p, x, P.c[k]);
  return fma(p, x, 0.5);
}
__device__ __forceinline__ double one_minus_rsqrt1p_over_x(double x) { return one_minus_rsqrt1p_over_x(x, kPolyG); }

// The fused step of one workgroup: SPB slices (one wavefront each) starting at
// slice slice_base + SPB * blk.  s_st holds the stencil tables in LDS.
// Regularised Coulomb friction (Sec. 3.3) added to f: t is the tangential
// velocity of the node relative to its partner, mu_fr = mu times the repulsive
// force density of the pair.  Slip when |t| exceeds the threshold mu_fr dt / rho:
// magnitude mu_fr against t; otherwise stick, -(rho / dt) t, which would stop t
// in one step.  The two branches agree at the threshold.
__device__ __forceinline__ void stick_slip(double mu_fr, double rho, double dt, double tx, double ty,
                                           double tz, double& fx, double& fy, double& fz) {
  const double vt = sqrt(tx * tx + ty * ty + tz * tz);
  const double k = vt > mu_fr * dt / rho ? mu_fr / vt : rho / dt;
  fx = fma(-k, tx, fx);
  fy = fma(-k, ty, fy);
  fz = fma(-k, tz, fz);
}

// ---- several walls at a corner (Sec. 4.1.1) ----
// Area and first moments (v, w) of {v > b, w > c, v^2 + w^2 < r^2}: for a
// given v the region spans w in (max(c, -s), s), s = sqrt(r^2 - v^2), which
// integrates in closed form over the pieces of the v axis where the lower end
// is c (|v| < e = sqrt(r^2 - c^2)) or -s.  Differences of squares are taken
// as (r - x)(r + x): with a fused multiply-add r*r - x*x at x = r leaves the
// rounding error of x*x, whose square root would enter at 1e-8 relative.
__device__ __forceinline__ double disk_f0(double r, double x) {
  const double q = fmax((r - x) * (r + x), 0.0);
  return 0.5 * (x * sqrt(q) + r * r * asin(fmin(1.0, fmax(-1.0, x / r))));
}
__device__ __forceinline__ double disk_f1(double r, double x) {
  const double q = fmax((r - x) * (r + x), 0.0);
  return -q * sqrt(q) * (1.0 / 3.0);
}
__device__ void disk_cut(double r, double b, double c, double& A, double& Mv, double& Mw) {
  A = Mv = Mw = 0.0;
  if (!(r > 0.0) || b >= r || c >= r) return;
  const double v0 = fmax(b, -r);
  const bool lower_c = c > -r;  // the bound w > c cuts the disk
  const double e = lower_c ? sqrt(fmax((r - c) * (r + c), 0.0)) : r;
  // piece |v| < e with lower end c (when the bound cuts), pieces e <= |v| < r with -s
  for (int k = 0; k < 3; ++k) {
    double x0, x1;
    bool with_c;
    if (!lower_c) {
      if (k != 1) continue;
      x0 = -r, x1 = r, with_c = false;
    } else if (k == 1) {
      x0 = -e, x1 = e, with_c = true;
    } else {
      if (c >= 0.0) continue;  // there -s > c: nothing outside |v| < e
      x0 = k == 0 ? -r : e, x1 = k == 0 ? -e : r, with_c = false;
    }
    x0 = fmax(x0, v0);
    if (!(x1 > x0)) continue;
    const double dA = disk_f0(r, x1) - disk_f0(r, x0), dM = disk_f1(r, x1) - disk_f1(r, x0);
    if (with_c) {
      A += dA - c * (x1 - x0);
      Mv += dM - 0.5 * c * ((x1 - x0) * (x1 + x0));
      Mw += 0.5 * ((r - c) * (r + c) * (x1 - x0) - (x1 * x1 * x1 - x0 * x0 * x0) * (1.0 / 3.0));
    } else {
      A += 2.0 * dA;
      Mv += 2.0 * dM;
    }
  }
}

// Volume and centroid (along u, v, w) of {|x| < R, u > a, v > b, w > c}
// (c = -inf: two planes).  Slices u = R cos(phi) are integrated over phi, split
// where a slice changes shape, each piece by Gauss-Legendre on a cosine map of
// the piece (gl: nodes and weights on [0, pi]), which makes the end-point
// power laws of the slice area smooth.
__device__ void corner_region(const double* gl, int ngl, double R, double a, double b, double c, double& V,
                              double& cu, double& cv, double& cw) {
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  const double u0 = fmax(a, -R);
  double cuts[8];
  int nc = 0;
  cuts[nc++] = u0;
  const double rr[3] = {fabs(b), fabs(c), sqrt(b * b + c * c)};
  for (int k = 0; k < 3; ++k) {
    if (!(rr[k] < R)) continue;
    const double uk = sqrt((R - rr[k]) * (R + rr[k]));
    if (uk > u0 && uk < R) cuts[nc++] = uk;
    if (-uk > u0 && -uk < R) cuts[nc++] = -uk;
  }
  cuts[nc++] = R;
  for (int i = 1; i < nc; ++i)
    for (int j = i; j > 0 && cuts[j] < cuts[j - 1]; --j) {
      const double t = cuts[j];
      cuts[j] = cuts[j - 1];
      cuts[j - 1] = t;
    }
  for (int k = 0; k + 1 < nc; ++k) {
    if (!(cuts[k + 1] > cuts[k])) continue;
    const double p0 = acos(fmin(1.0, fmax(-1.0, cuts[k + 1] / R)));
    const double p1 = acos(fmin(1.0, fmax(-1.0, cuts[k] / R)));
    const double mid = 0.5 * (p0 + p1), half = 0.5 * (p1 - p0);
    for (int q = 0; q < ngl; ++q) {
      const double th = gl[q], w = gl[ngl + q];
      const double ph = mid - half * cos(th);
      const double sp = sin(ph), u = R * cos(ph);
      const double jw = w * half * sin(th) * R * sp;
      double A, Mv, Mw;
      disk_cut(R * sp, b, c, A, Mv, Mw);
      acc0 += jw * A;
      acc1 += jw * u * A;
      acc2 += jw * Mv;
      acc3 += jw * Mw;
    }
  }
  V = acc0;
  const double inv = acc0 > 0.0 ? 1.0 / acc0 : 0.0;
  cu = acc1 * inv;
  cv = acc2 * inv;
  cw = acc3 * inv;
}

// Inclusion-exclusion over the walls the node touches (at most three taken,
// in wall order): pairs of orthogonal walls subtract, an orthogonal triple
// adds, each term -K_n (R_c - |c - p|) |S| (c - p)/|c - p| over the part S of
// the contact ball beyond all of its walls.  Wall l takes each term's
// component along its normal: corr[k] for the wall index hw[k].
__device__ void wall_corner_terms(const StepArgs& A, double Kn, const double* hd, const int* hw, int nh,
                                  double* corr) {
  bool orth[3][3];
  for (int x = 0; x < nh; ++x)
    for (int y = 0; y < nh; ++y) {
      const double* na = A.walls[hw[x]].n;
      const double* nb = A.walls[hw[y]].n;
      orth[x][y] = fabs(na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2]) < 1e-12;
    }
  // the three pairs (x, y) and, with three walls, the triple
  const int terms = nh == 3 ? 4 : 1;
  for (int t = 0; t < terms; ++t) {
    int m[3] = {0, 1, -1};
    if (t == 1) m[0] = 0, m[1] = 2;
    if (t == 2) m[0] = 1, m[1] = 2;
    if (t == 3) m[2] = 2;
    const bool triple = m[2] >= 0;
    if (!orth[m[0]][m[1]] || (triple && (!orth[m[0]][2] || !orth[m[1]][2]))) continue;
    double V, cu, cv, cw;
    corner_region(A.corner_gl, A.corner_ngl, A.Rc, hd[m[0]], hd[m[1]], triple ? hd[2] : -INFINITY, V, cu, cv, cw);
    if (!(V > 0.0)) continue;
    const double cen[3] = {cu, cv, cw};
    double cp[3] = {0.0, 0.0, 0.0};  // c - p along the outward directions -n_l
    for (int k = 0; k < (triple ? 3 : 2); ++k)
      for (int q = 0; q < 3; ++q) cp[q] -= cen[k] * A.walls[hw[m[k]]].n[q];
    const double ell = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
    if (!(ell > 0.0)) continue;
    const double f = (triple ? 1.0 : -1.0) * -Kn * (A.Rc - ell) * V / ell;
    for (int k = 0; k < (triple ? 3 : 2); ++k) {
      const double* nl = A.walls[hw[m[k]]].n;
      corr[m[k]] += f * (cp[0] * nl[0] + cp[1] * nl[1] + cp[2] * nl[2]);
    }
  }
}

// Corner corrections of every node for this evaluation: nodes touching two or
// three walls get corner_w = count | wall indices << 8 (k + 1) and their
// corrections in corner_c; the others 0.  force_only: walls at the offsets of
// the last evaluation.
__global__ void k_wall_corners(StepArgs A, int force_only) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n || (!force_only && halted(A.halt))) return;
  const double4 ui = A.ucur[i];
  const GrainC* G = A.grains + packed_grain(ui.w);
  const int p = packed_ijk(ui.w);
  const double px = lattice_pos(G->origin[0], G->h, unpack_x(p)) + ui.x;
  const double py = lattice_pos(G->origin[1], G->h, unpack_y(p)) + ui.y;
  const double pz = lattice_pos(G->origin[2], G->h, unpack_z(p)) + ui.z;
  int hw[3];
  double hd[3];
  int nh = 0;
  for (int w = 0; w < A.n_walls && nh < 3; ++w) {
    const WallDev* Wd = A.walls + w;
    const bool in = px >= Wd->lo[0] && px <= Wd->hi[0] && py >= Wd->lo[1] && py <= Wd->hi[1] &&
                    pz >= Wd->lo[2] && pz <= Wd->hi[2];
    const double o = force_only ? Wd->off_used : Wd->off;
    const double d = Wd->n[0] * px + Wd->n[1] * py + Wd->n[2] * pz - o;
    if (in && d < A.Rc && d > -A.Rc) {
      hw[nh] = w;
      hd[nh] = d;
      ++nh;
    }
  }
  uint32_t pw = 0u;
  if (nh >= 2) {
    double corr[3] = {0.0, 0.0, 0.0};
    wall_corner_terms(A, A.Kn[G->mat * A.n_mat + G->mat], hd, hw, nh, corr);
    pw = (uint32_t)nh;
    for (int k = 0; k < nh; ++k) {
      pw |= (uint32_t)hw[k] << (8 * (k + 1));
      A.corner_c[3 * i + k] = corr[k];
    }
  }
  A.corner_w[i] = pw;
}

// Everything after the bond sum for the node of this lane: contact with other
// grains, damping and friction (Secs. 3.2-3.4), rigid walls (Sec. 4.1) with the
// wavefront's reaction partial in wall_partial column col (written when col_ok),
// and velocity Verlet (Sec. 6.2).  Every lane of the wavefront takes part (the
// wall partials are wavefront sums); lanes without a node pass valid = false.
// The node's velocity and previous acceleration, read by the Verlet update.
struct NodeVA {
  double vx, vy, vz, ax, ay, az;
};
__device__ __forceinline__ NodeVA load_va(const StepArgs& A, int64_t i, bool valid) {
  NodeVA r{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (valid) {
    r.vx = A.v[i];
    r.vy = A.v[A.n + i];
    r.vz = A.v[2 * A.n + i];
    r.ax = A.a[i];
    r.ay = A.a[A.n + i];
    r.az = A.a[2 * A.n + i];
  }
  return r;
}

// Is the bond from node i to node j (same grain) intact after this evaluation's
// breaks?  The node's built entries are sorted by neighbour index, so a binary
// search finds j's entry; a pair with no entry (outside the horizon, or cut)
// has no bond.  The bond memory is the live column word on the slice path
// (perm < 0) and, on the tiled path, the node's lane bit in the lane mask of
// its class in the grain's axis order perm (the tile kernel stores a class's
// mask as soon as a bond of it breaks, before any node's tail).
__device__ __forceinline__ bool bond_intact(const StepArgs& A, int64_t i, int j, int perm) {
  const uint32_t node_mask = (1u << A.node_bits) - 1u;
  const int64_t base = A.slice_off[i >> 6] + (i & 63);
  int lo = 0, hi = A.rowlen[i] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int64_t at = base + ((int64_t)mid << 6);
    const uint32_t wo = A.colOrig[at];
    const int jm = (int)(wo & node_mask);
    if (jm < j) {
      lo = mid + 1;
    } else if (jm > j) {
      hi = mid - 1;
    } else {
      if (perm < 0) return A.colE[at] == wo;
      const int b = A.ctob[perm * A.n_stencil + (int)(wo >> A.node_bits)];
      const int32_t sl = A.slot[i];
      return ((A.lmask[(int64_t)(sl >> 6) * kTileClasses + b] >> (sl & 63)) & 1ull) != 0ull;
    }
  }
  return false;
}

// Repulsion of node j on node i when closer than R_c (Sec. 3.2), with normal
// damping (Sec. 3.4) and stick-slip friction (Sec. 3.3): between grains, and
// between nodes of one grain without an intact bond (Sec. 5, where c_w / R_c
// is the same K_n; self-contact needs R_c below the lattice spacing, so the
// repulsive-only bond of pairs shorter than R_c never arises).
// uj and Xj are the partner's displacement and reference position.
template <bool EXTRA>
__device__ __forceinline__ void contact_pair(const StepArgs& A, int64_t i, int j, const double4& uj,
                                             const double4& Xj, const double4& Xi, const double4& ui,
                                             const double4& vhi, int mi, double rho_i, bool damp, bool fric,
                                             int perm, double& fx, double& fy, double& fz) {
  double yx, yy, yz;
  const double d2 = contact_d2(Xj.x, Xi.x, uj.x, ui.x, Xj.y, Xi.y, uj.y, ui.y, Xj.z, Xi.z, uj.z, ui.z, yx, yy, yz);
  if (d2 < A.Rc2 && d2 > 0.0) {
    // a node of the same grain repels only while no intact bond joins the two
    if (EXTRA && A.self_contact && packed_grain(uj.w) == packed_grain(ui.w) && bond_intact(A, i, j, perm))
      return;
    const GrainC* Gj = A.grains + packed_grain(uj.w);
    const double d = sqrt(d2);
    const double rep = A.Kn[mi * A.n_mat + Gj->mat] * (A.Rc - d) * Gj->V;
    double coef = -rep / d;
    double4 vhj = make_double4(0.0, 0.0, 0.0, 0.0);
    if (damp || fric) vhj = A.vh_cur[j];
    const double wx = vhi.x - vhj.x, wy = vhi.y - vhj.y, wz = vhi.z - vhj.z;
    if (damp) {
      // -beta (w . e) e V_j, w = velocity of i relative to j, e = y / d
      const double w = wx * yx + wy * yy + wz * yz;
      coef -= A.beta * Gj->V * w / d2;
    }
    fx = fma(coef, yx, fx);
    fy = fma(coef, yy, fy);
    fz = fma(coef, yz, fz);
    if (fric) {
      // tangential part of w against the repulsive force density rep
      const double inv_d = 1.0 / d;
      const double ex = yx * inv_d, ey = yy * inv_d, ez = yz * inv_d;
      const double wn = wx * ex + wy * ey + wz * ez;
      stick_slip(A.mu * rep, rho_i, A.dt, wx - wn * ex, wy - wn * ey, wz - wn * ez, fx, fy, fz);
    }
  }
}

// EXTRA = false compiles out self-contact and the wall-corner corrections (the
// tiled kernel's variant for runs with neither).
template <int MODE, bool EXTRA = true>
__device__ __forceinline__ void node_tail(const StepArgs& A, int64_t i, bool valid, const double4& ui,
                                          const GrainC* G, int ix, int iy, int iz, double fx, double fy,
                                          double fz, int nbroke, bool col_ok, int64_t col, const NodeVA& va,
                                          int perm) {
  const int lane = threadIdx.x & 63;
  const double h = G->h;
  // mid-step velocity of this node for the normal damping (Sec. 3.4) and
  // stick-slip friction (Sec. 3.3) laws
  const bool damp = A.beta > 0.0, fric = A.mu > 0.0, vdep = damp || fric;
  double4 vhi = make_double4(0.0, 0.0, 0.0, 0.0);
  if (vdep && valid) vhi = A.vh_cur[i];
  const double rho_i = G->rho;

  // ---- repulsive contact with the candidates: nodes of other grains and, with
  // self-contact, of the same grain (Secs. 3.2, 5) ----
  if (valid && A.cand_ptr != nullptr) {
    // rows past the capacity were not stored (the rebuild flagged it)
    const int32_t c0 = (int32_t)min((int64_t)A.cand_ptr[i], A.cand_capacity);
    const int32_t c1 = (int32_t)min((int64_t)A.cand_ptr[i + 1], A.cand_capacity);
    if (c1 > c0) {
      // keep the candidate gathers here: hoisted above the bond loop they
      // would hold their registers through it
      asm volatile("" ::: "memory");
      const double4 Xi = A.X4[i];
      // kContactBatch candidates at a time: their indices, then their u and
      // reference positions, are all in flight before the first pair is
      // evaluated; the pairs are still added in row order
      for (int32_t e = c0; e < c1; e += kContactBatch) {
        int jj[kContactBatch];
        double4 uj[kContactBatch], Xj[kContactBatch];
#pragma unroll
        for (int k = 0; k < kContactBatch; ++k) jj[k] = e + k < c1 ? A.cand[e + k] : -1;
#pragma unroll
        for (int k = 0; k < kContactBatch; ++k) {
          if (jj[k] >= 0) {
            uj[k] = A.ucur[jj[k]];
            const double* xp = reinterpret_cast<const double*>(A.X4 + jj[k]);
            Xj[k] = make_double4(xp[0], xp[1], xp[2], 0.0);
          }
        }
#pragma unroll
        for (int k = 0; k < kContactBatch; ++k)
          if (jj[k] >= 0)
            contact_pair<EXTRA>(A, i, jj[k], uj[k], Xj[k], Xi, ui, vhi, G->mat, rho_i, damp, fric, perm, fx, fy,
                                fz);
      }
    }
  }

  // ---- several walls at a corner (Sec. 4.1.1): the corrections of the normal
  // magnitudes that k_wall_corners left for this node (at most three walls) ----
  const uint32_t corner_pw = (EXTRA && A.wall_corners && valid) ? A.corner_w[i] : 0u;

  // ---- rigid walls: spherical-cap law (Sec. 4.1), walls summed ----
  for (int w = 0; w < A.n_walls; ++w) {
    const WallDev* Wd = A.walls + w;
    bool hit = false;
    double mag = 0.0, ftx = 0.0, fty = 0.0, ftz = 0.0;  // normal magnitude, friction
    if (valid) {
      const double px = lattice_pos(G->origin[0], h, ix) + ui.x;
      const double py = lattice_pos(G->origin[1], h, iy) + ui.y;
      const double pz = lattice_pos(G->origin[2], h, iz) + ui.z;
      const bool in = px >= Wd->lo[0] && px <= Wd->hi[0] && py >= Wd->lo[1] && py <= Wd->hi[1] &&
                      pz >= Wd->lo[2] && pz <= Wd->hi[2];
      const double o = MODE == MODE_FORCE_ONLY ? Wd->off_used : Wd->off;
      const double d = Wd->n[0] * px + Wd->n[1] * py + Wd->n[2] * pz - o;
      if (in && d < A.Rc) {
        if (d <= -A.Rc) {
          if (MODE != MODE_FORCE_ONLY) atomicOr(A.status, ST_PENETRATION);
        } else {
          // cap of the contact ball beyond the wall: height Rc - d, volume
          // (pi/3)(Rc-d)^2(2Rc+d); its centroid lies 3(Rc+d)^2/(4(2Rc+d)) from p
          const double H = A.Rc - d, q = 2.0 * A.Rc + d;
          const double vol = (M_PI / 3.0) * H * H * q;
          const double ell = 0.75 * (A.Rc + d) * (A.Rc + d) / q;
          const double rep = A.Kn[G->mat * A.n_mat + G->mat] * (A.Rc - ell) * vol;
          mag = rep;
          if (EXTRA) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
              if ((int)(corner_pw & 3u) > k && (int)((corner_pw >> (8 * (k + 1))) & 255u) == w)
                mag += A.corner_c[3 * i + k];
          }
          const double rate = MODE == MODE_FORCE_ONLY ? Wd->rate_used : Wd->rate;
          if (damp) {
            // damping against the wall: relative normal velocity v . n - wall rate
            const double vn = Wd->n[0] * vhi.x + Wd->n[1] * vhi.y + Wd->n[2] * vhi.z;
            mag -= A.beta * (vn - rate) * vol;
          }
          if (fric) {
            // the wall moves along its normal only: friction sees v's tangential part
            const double wx = vhi.x - rate * Wd->n[0], wy = vhi.y - rate * Wd->n[1],
                         wz = vhi.z - rate * Wd->n[2];
            const double wn = wx * Wd->n[0] + wy * Wd->n[1] + wz * Wd->n[2];
            stick_slip(A.mu * rep, rho_i, A.dt, wx - wn * Wd->n[0], wy - wn * Wd->n[1],
                       wz - wn * Wd->n[2], ftx, fty, ftz);
          }
          hit = true;
        }
      }
    }
    if (hit) {
      fx = fma(mag, Wd->n[0], fx) + ftx;
      fy = fma(mag, Wd->n[1], fy) + fty;
      fz = fma(mag, Wd->n[2], fz) + ftz;
    }
    if (MODE != MODE_FORCE_ONLY) {
      const uint64_t any = __ballot(hit);
      double r0 = 0.0, r1 = 0.0, r2 = 0.0;
      if (any) {
        const double vm = hit ? G->V * mag : 0.0, vf = hit ? G->V : 0.0;
        r0 = wave_sum(fma(vf, ftx, vm * Wd->n[0]));
        r1 = wave_sum(fma(vf, fty, vm * Wd->n[1]));
        r2 = wave_sum(fma(vf, ftz, vm * Wd->n[2]));
      }
      // one partial per slice (wavefront), component-major: the finalize sums
      // them in slice order, whatever the workgroup size or launch split
      if (lane == 0 && col_ok) {
        A.wall_partial[(int64_t)(3 * w) * A.partial_stride + col] = r0;
        A.wall_partial[(int64_t)(3 * w + 1) * A.partial_stride + col] = r1;
        A.wall_partial[(int64_t)(3 * w + 2) * A.partial_stride + col] = r2;
      }
    }
  }

  // ---- velocity Verlet (Sec. 6.2) and stores ----
  if (valid) {
    if (MODE == MODE_FORCE_ONLY) {
      A.Fout[i] = fx;
      A.Fout[A.n + i] = fy;
      A.Fout[2 * A.n + i] = fz;
    } else {
      if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicOr(A.status, ST_NAN);
      const bool fixed = A.fixed != nullptr && A.fixed[i] != 0;
      const double rho = G->rho, dt = A.dt, hdt = 0.5 * dt, hdt2 = 0.5 * dt * dt;
      const double anx = fixed ? 0.0 : fx / rho + A.g[0];
      const double any = fixed ? 0.0 : fy / rho + A.g[1];
      const double anz = fixed ? 0.0 : fz / rho + A.g[2];
      double vx = va.vx, vy = va.vy, vz = va.vz;
      if (MODE == MODE_STEP) {
        vx = fixed ? 0.0 : fma(hdt, va.ax + anx, vx);
        vy = fixed ? 0.0 : fma(hdt, va.ay + any, vy);
        vz = fixed ? 0.0 : fma(hdt, va.az + anz, vz);
      } else if (fixed) {
        vx = vy = vz = 0.0;
      }
      A.v[i] = vx;
      A.v[A.n + i] = vy;
      A.v[2 * A.n + i] = vz;
      A.a[i] = anx;
      A.a[A.n + i] = any;
      A.a[2 * A.n + i] = anz;
      // positions of the next step: u + dt v + dt^2/2 a
      double4 un = ui;
      if (!fixed) {
        un.x = fma(hdt2, anx, fma(dt, vx, ui.x));
        un.y = fma(hdt2, any, fma(dt, vy, ui.y));
        un.z = fma(hdt2, anz, fma(dt, vz, ui.z));
      }
      A.unext[i] = un;
      if (vdep) {
        // the next evaluation's damping and friction see v_{n+1} + dt/2 a_{n+1}
        A.vh_next[i] = fixed ? make_double4(0.0, 0.0, 0.0, 0.0)
                             : make_double4(fma(hdt, anx, vx), fma(hdt, any, vy), fma(hdt, anz, vz), 0.0);
      }
      if (nbroke) A.intact[i] -= nbroke;
    }
  }
}

template <int MODE, bool ABS, int SPB>
__device__ __forceinline__ void step_body(const StepArgs& A, const StencilC* s_st, int64_t blk) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int64_t slice = A.slice_base + blk * SPB + wid;
  const bool slice_ok = slice < A.slice_end;
  const int64_t i = slice * kWave + lane;
  const bool valid = slice_ok && i >= A.node_lo && i < A.node_hi;

  double4 ui = make_double4(0.0, 0.0, 0.0, 0.0);
  if (valid) ui = A.ucur[i];
  const int pi = packed_ijk(ui.w);
  const int gi = valid ? packed_grain(ui.w) : 0;
  const GrainC* G = A.grains + gi;
  const double abs_ratio = G->abs_ratio;
  const int ix = unpack_x(pi), iy = unpack_y(pi), iz = unpack_z(pi);
  const uint32_t node_mask = (1u << A.node_bits) - 1u;
  const int node_bits = A.node_bits;

  double fx = 0.0, fy = 0.0, fz = 0.0;
  int nbroke = 0;

  // ---- peridynamic bonds with bond memory ----
  // Slice width W is a multiple of kUnroll: the column words of kUnroll entries
  // are loaded one iteration ahead, then their kUnroll neighbour gathers, so
  // each lane keeps several memory requests in flight.  Broken bonds and
  // padding carry the zero-force class and point at the node itself, so every
  // entry is evaluated the same way.
  //
  // Bond law (Sec. 3.1): the force on i is c s V_j y/|y|, y = xi + eta, and
  //   c V s / |y| = (c V / |xi|) g,   g = 1 - |xi|/|y| = 1 - (1 + x)^(-1/2),
  //   x = (|y|^2 - |xi|^2) / |xi|^2,   |y|^2 - |xi|^2 = eta . (2 xi + eta).
  // g comes from its polynomial when |x| <= kPolyRange (no square
  // root or division), else from g = (|y|^2 - |xi|^2) / (|y| (|y| + |xi|));
  // neither form subtracts nearly equal numbers.  The choice is made per lane,
  // so any grouping of bonds (the tiled path) computes the same values.
  int64_t off = 0;
  int W = 0;
  if (slice_ok) {
    off = A.slice_off[slice];
    W = (int)((A.slice_off[slice + 1] - off) >> 6);
  }
  uint32_t* cp = A.colE + off + lane;
  const char* ubase = reinterpret_cast<const char*>(A.ucur);
  const char* tbase = reinterpret_cast<const char*>(s_st) +
                      (uint32_t)G->cls * (uint32_t)(A.n_stencil + 1) * (uint32_t)sizeof(StencilC);
  const uint32_t mine = (uint32_t)(valid ? i : 0) | A.sentinel_hi;
  uint32_t cn[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) cn[u] = W > 0 ? cp[u * kWave] : mine;
  for (int k = 0; k < W; k += kUnroll) {
    uint32_t cw[kUnroll];
    double4 uj[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) cw[u] = cn[u];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      uj[u] = *reinterpret_cast<const double4*>(ubase + ((cw[u] & node_mask) << 5));
    if (k + kUnroll < W) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) cn[u] = cp[(k + kUnroll + u) * kWave];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const StencilC& S =
          *reinterpret_cast<const StencilC*>(tbase + (cw[u] >> node_bits) * (uint32_t)sizeof(StencilC));
      const double ex = uj[u].x - ui.x, ey = uj[u].y - ui.y, ez = uj[u].z - ui.z;
      const double yx = S.hx + ex, yy = S.hy + ey, yz = S.hz + ez;  // y = xi + eta
      // |y|^2 - |xi|^2 = eta . (2 xi + eta)
      const double d = fma(ex, yx + S.hx, fma(ey, yy + S.hy, ez * (yz + S.hz)));
      // s > s0  <=>  |y|^2 - |xi|^2 > |xi|^2 ((1 + s0)^2 - 1)
      bool over = d > S.thr_d;
      if (ABS) over = over || d < -abs_ratio * S.thr_d;
      const double x = d * S.inv_l0sq;
      double g = x * one_minus_rsqrt1p_over_x(x);
      if (!(fabs(x) <= kPolyRange)) {
        const double lsq = S.l0sq + d;
        const double l = lsq * rsqrt_full(lsq);
        g = d * rcp_full(fma(l, S.l0, lsq));
      }
      const double coef = over ? 0.0 : S.civ * g;
      fx = fma(coef, yx, fx);
      fy = fma(coef, yy, fy);
      fz = fma(coef, yz, fz);
      if (MODE != MODE_FORCE_ONLY && over && valid) {
        cp[(k + u) * kWave] = mine;  // the bond stays broken from now on
        ++nbroke;
      }
    }
  }

  node_tail<MODE>(A, i, valid, ui, G, ix, iy, iz, fx, fy, fz, nbroke, slice_ok,
                  A.partial_base + (slice - A.slice_base), load_va(A, i, valid), -1);
}

__device__ __forceinline__ void stage_stencil(const StepArgs& A, StencilC* s_st) {
  const int rows = A.n_classes * (A.n_stencil + 1);
  for (int k = threadIdx.x; k < rows; k += blockDim.x) s_st[k] = A.stencil[k];
  __syncthreads();
}

template <int MODE, bool ABS, int SPB>
__global__ __launch_bounds__(SPB * kWave) __attribute__((amdgpu_waves_per_eu(PD_STEP_WAVES_PER_EU)))
void k_step(StepArgs A) {
  extern __shared__ StencilC s_st[];
  if (MODE == MODE_STEP && halted(A.halt)) return;
  stage_stencil(A, s_st);
  const int64_t blk = A.xcd_remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  step_body<MODE, ABS, SPB>(A, s_st, blk);
}

// ---------------------------------------------------------------------------
// tiled bond loop: u of a tile and its halo in LDS, bond memory in class masks
// ---------------------------------------------------------------------------

// Offset, in the halo box, of the neighbour in horizon class k (lexicographic
// (ds, dm, df) with 0 < |d|^2 <= 9) from the lane's corner cell (its own cell
// minus kTileR on each axis); -1 past the last class.
constexpr int tile_class_off(int k) {
  int n = 0;
  for (int a = -kTileR; a <= kTileR; ++a)
    for (int b = -kTileR; b <= kTileR; ++b)
      for (int c = -kTileR; c <= kTileR; ++c) {
        const int d2 = a * a + b * b + c * c;
        if (d2 == 0 || d2 > kTileR * kTileR) continue;
        if (n == k) return ((a + kTileR) * kHM + (b + kTileR)) * kHF + (c + kTileR);
        ++n;
      }
  return -1;
}
static_assert(tile_class_off(kTileClasses - 1) >= 0 && tile_class_off(kTileClasses) < 0,
              "horizon factor 3 has 122 classes");
static_assert((kHalo + tile_class_off(kTileClasses - 1)) * sizeof(double) <= 65535,
              "plane and class offsets must fit the LDS immediate offset");

// bond tables read through the constant address space: the table of a tile is
// the same for the whole wavefront, so these become scalar loads
typedef const __attribute__((address_space(4))) StencilC* TileTab;

// Operands of one horizon class: the neighbour's u from LDS and the class's
// bond-law constants through scalar loads.  An opaque copy of the row address
// keeps each class's scalar loads where they are issued instead of all 122
// rows' being hoisted to the kernel entry.
struct TileIn {
  double ux, uy, uz;
  double hx, hy, hz, thr, inv, civ;
  uint64_t live;       // lanes whose bond of this class is intact
  uint64_t live_next;  // the same for the next class, loaded a class earlier still
  const StencilC* rowp;
};

typedef const __attribute__((address_space(4))) uint64_t* MaskTab;

template <int K>
__device__ __forceinline__ void tile_load(const double* L, const double* Lz, const StencilC* tabp,
                                          const uint64_t* mrow, TileIn& in) {
  constexpr int off = tile_class_off(K);
  const StencilC* rowp = tabp + K;
  asm volatile("" : "+s"(rowp));
  const TileTab row = (TileTab)rowp;
  in.ux = L[off];
  in.uy = L[kHalo + off];
  in.uz = Lz[off];
  in.hx = row->hx;
  in.hy = row->hy;
  in.hz = row->hz;
  in.thr = row->thr_d;
  in.inv = row->inv_l0sq;
  in.civ = row->civ;
  // lane masks travel two classes ahead: a wait for this class's operands then
  // never waits for the mask as well
  in.live = in.live_next;
  if constexpr (K + 1 < kTileClasses) {
    const uint64_t* mp = mrow + (K + 1);
    asm volatile("" : "+s"(mp));
    in.live_next = *(MaskTab)mp;
  }
  in.rowp = rowp;
}

// a lane's x where its bit of the scalar lane mask m is set, else +0.0
__device__ __forceinline__ double lanes_select(uint64_t m, double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
  asm("v_cndmask_b32_e64 %0, 0, %0, %1" : "+v"(lo) : "s"(m));
  asm("v_cndmask_b32_e64 %0, 0, %0, %1" : "+v"(hi) : "s"(m));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One horizon class of the lane's node: the same arithmetic, in the same order,
// as an entry of the slice path, so the two paths agree bitwise.  A class with
// no bond (outside the grain, another grain, cut, or broken) adds an exact
// zero.  The operands of class K arrived during class K - 1; once the first of
// them is used (which waits for all of them) class K + 1's loads are issued, so
// that they travel while class K computes.  The class's lane mask of intact
// bonds decides in scalar registers which lanes add a force, and loses the
// lanes whose bond breaks now; a wavefront in which one breaks stores the mask
// (lane 0) and counts the breaks per lane.
template <int K, bool ABS>
__device__ __forceinline__ void tile_bond(const double* L, const double* Lz, const StencilC* tabp,
                                          const uint64_t* mrow, uint64_t* mrow_w, TileIn& in, const PolyG& PG,
                                          double uix, double uiy, double uiz, double abs_ratio, int& nbroke,
                                          double& fx, double& fy, double& fz) {
  const double ex = in.ux - uix, ey = in.uy - uiy, ez = in.uz - uiz;
  const double hx = in.hx, hy = in.hy, hz = in.hz;
  const double yx = hx + ex, yy = hy + ey, yz = hz + ez;
  const double thr = in.thr, inv = in.inv, civ = in.civ;
  const uint64_t live = in.live;
  const TileTab row = (TileTab)in.rowp;
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (K + 1 < kTileClasses) tile_load<K + 1>(L, Lz, tabp, mrow, in);
  const double d = fma(ex, yx + hx, fma(ey, yy + hy, ez * (yz + hz)));
  bool over = d > thr;
  if (ABS) over = over || d < -abs_ratio * thr;
  const double x = d * inv;
  // the per-lane choice of the slice path (series, or the exact form past
  // kPolyRange), the exact form computed only when a lane with an intact bond
  // needs it
  double g = x * one_minus_rsqrt1p_over_x(x, PG);
  const bool exact = !(fabs(x) <= kPolyRange);
  if ((__ballot(exact) & live) != 0ull) {
    const double lsq = row->l0sq + d;
    const double l = lsq * rsqrt_full(lsq);
    const double ge = d * rcp_full(fma(l, row->l0, lsq));
    g = exact ? ge : g;
  }
  // an intact bond within its limit adds its force, the others an exact zero
  // (as in the slice path); a bond past its limit stays broken from now on
  const uint64_t ov = __ballot(over);
  const double coef = lanes_select(live & ~ov, civ * g);
  fx = fma(coef, yx, fx);
  fy = fma(coef, yy, fy);
  fz = fma(coef, yz, fz);
  const uint64_t brk = live & ov;
  if (brk != 0ull) {
    const int lane = __lane_id();
    if (lane == 0) mrow_w[K] = live & ~ov;
    nbroke += (int)((brk >> lane) & 1ull);
  }
  // materialise the running sums here: left alone, the compiler sinks every
  // class's accumulation to the end and keeps all 122 classes' terms live
  asm volatile("" : "+v"(fx), "+v"(fy), "+v"(fz));
}

template <bool ABS, int... K>
__device__ __forceinline__ void tile_bonds(std::integer_sequence<int, K...>, const double* L, const double* Lz,
                                           const StencilC* tab, const uint64_t* mrow, uint64_t* mrow_w,
                                           const PolyG& PG, double uix, double uiy, double uiz, double abs_ratio,
                                           int& nbroke, double& fx, double& fy, double& fz) {
  TileIn in;
  in.live_next = *(MaskTab)mrow;
  tile_load<0>(L, Lz, tab, mrow, in);
  (tile_bond<K, ABS>(L, Lz, tab, mrow, mrow_w, in, PG, uix, uiy, uiz, abs_ratio, nbroke, fx, fy, fz), ...);
}

__device__ __forceinline__ int64_t tile_cell(const TileGrain& TG, int s, int m, int f) {
  return TG.map_off + ((int64_t)s * TG.em + m) * TG.ef + f;
}

// One workgroup per tile: stage u of the tile and its halo (cells outside the
// grain hold zeros and have no bonds), evaluate the 122 horizon classes of each
// lane's cell from LDS, then the node tail of the slice path.  Lane l of
// wavefront w owns cell (s0 + w, m0 + l / 16, f0 + l % 16).
template <bool ABS, bool EXTRA>
__global__ __launch_bounds__(kTS * kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_step_tile(StepArgs A) {
  // x, y and z planes of the halo box
  __shared__ double s_u[3 * kHalo];
  constexpr int kNT = kTS * kWave;
  constexpr int kFill = (kHalo + kNT - 1) / kNT;  // halo cells per thread
  if (halted(A.halt)) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t t = A.xcd_remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int4 T = A.tiles[t];
  const TileGrain TG = A.tgrain[T.x];
  // the lane's own cell, then the halo: every map read is issued before the
  // first wait and every u read before the second, so the fill costs two
  // memory round trips rather than two per cell
  const int lm = lane / kTF, lf = lane % kTF;
  const int cs = T.y + wid, cm = T.z + lm, cf = T.w + lf;
  const bool own_in = cs < TG.es && cm < TG.em && cf < TG.ef;
  int64_t i = own_in ? (int64_t)A.tmap[tile_cell(TG, cs, cm, cf)] : -1;
  int j[kFill];
#pragma unroll
  for (int r = 0; r < kFill; ++r) {
    const int c = tid + r * kNT;
    const int hs = c / (kHM * kHF), rr = c - hs * (kHM * kHF);
    const int hm = rr / kHF, hf = rr - hm * kHF;
    const int ps = T.y - kTileR + hs, pm = T.z - kTileR + hm, pf = T.w - kTileR + hf;
    j[r] = -1;
    if (c < kHalo && ps >= 0 && ps < TG.es && pm >= 0 && pm < TG.em && pf >= 0 && pf < TG.ef)
      j[r] = A.tmap[tile_cell(TG, ps, pm, pf)];
  }
  const bool valid = i >= 0;
  double4 ui = make_double4(0.0, 0.0, 0.0, 0.0);
  if (valid) ui = A.ucur[i];
  // bring this wavefront's lane masks (122 x 8 B) into the L2 with the other
  // prologue loads, so that the class loop's scalar loads of them hit there
  const uint64_t* mrow_r = A.lmask + ((int64_t)t * kTS + wid) * kTileClasses;
  uint4 mpre = make_uint4(0u, 0u, 0u, 0u);
  if (lane < kTileClasses / 2) mpre = reinterpret_cast<const uint4*>(mrow_r)[lane];
  double hx_[kFill], hy_[kFill], hz_[kFill];
#pragma unroll
  for (int r = 0; r < kFill; ++r) {
    hx_[r] = hy_[r] = hz_[r] = 0.0;
    if (j[r] >= 0) {
      const double4 u = A.ucur[j[r]];
      hx_[r] = u.x;
      hy_[r] = u.y;
      hz_[r] = u.z;
    }
  }
#pragma unroll
  for (int r = 0; r < kFill; ++r) {
    const int c = tid + r * kNT;
    if (c < kHalo) {
      s_u[c] = hx_[r];
      s_u[kHalo + c] = hy_[r];
      s_u[2 * kHalo + c] = hz_[r];
    }
  }
  // the lane's own grain (in lattice mode a tile holds nodes of several grains)
  const GrainC* G = A.grains + (valid ? packed_grain(ui.w) : 0);
  const int pi = packed_ijk(ui.w);
  __syncthreads();

  const double* L = s_u + (wid * kHM + lm) * kHF + lf;
  const double* Lz = L + 2 * kHalo;  // own base: plane and class offsets must fit the 16-bit immediate
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const StencilC* tab = A.ttab + (int64_t)TG.table * kTileClasses;
  // this wavefront's lane masks, one per class
  uint64_t* mrow_w = A.lmask + ((int64_t)t * kTS + wid) * kTileClasses;
  const PolyG PG = poly_in_registers();
  int nbroke = 0;  // bonds of this lane's node broken in this step
  // a layer beyond the last nodes of the box (the far ends of a lattice-mode
  // box) has no bonds: its wavefront leaves the vector units to the others
  if (__ballot(valid) != 0ull)
    tile_bonds<ABS>(std::make_integer_sequence<int, kTileClasses>{}, L, Lz, tab, mrow_r, mrow_w, PG, ui.x, ui.y,
                    ui.z, G->abs_ratio, nbroke, fx, fy, fz);
  // the prefetch's data is not needed; consuming it keeps the load
  asm volatile("" ::"v"(mpre.x ^ mpre.y ^ mpre.z ^ mpre.w));
  node_tail<MODE_STEP, EXTRA>(A, i, valid, ui, G, unpack_x(pi), unpack_y(pi), unpack_z(pi), fx, fy, fz, nbroke,
                              true, (int64_t)kTS * t + wid, load_va(A, i, valid), TG.perm);
}

// the six orders of the lattice axes (slowest first)
__device__ __constant__ int kAxisPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// cell of node (packed grain-local ijk p) of grain g in its tile box B
__device__ __forceinline__ void tile_coords(const TileGrain& Gg, const TileGrain& B, int p, int& s, int& m, int& f) {
  const int q[3] = {unpack_x(p) + Gg.goff[0], unpack_y(p) + Gg.goff[1], unpack_z(p) + Gg.goff[2]};
  s = q[kAxisPerm[B.perm][0]] - B.lo_s;
  m = q[kAxisPerm[B.perm][1]] - B.lo_m;
  f = q[kAxisPerm[B.perm][2]] - B.lo_f;
}

__global__ void k_tile_map_fill(StepArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const double w = A.ucur[i].w;
  const TileGrain Gg = A.tgrain[packed_grain(w)];
  const TileGrain B = A.tgrain[Gg.box];
  int s, m, f;
  tile_coords(Gg, B, packed_ijk(w), s, m, f);
  const_cast<int32_t*>(A.tmap)[tile_cell(B, s, m, f)] = (int32_t)i;
}

// Lane masks from the column words: one wavefront per layer of a tile, lane l
// on the cell it owns in the step kernel.  Each lane gathers its node's live
// built bonds as tile-class bits (class ctob[perm][slice class]); a ballot per
// class forms the wavefront's mask.
__global__ __launch_bounds__(256) void k_cols_to_mask(StepArgs A, const int16_t* ctob, const uint32_t* colOrig) {
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (wv >= A.n_tiles * kTS) return;  // whole wavefronts leave together
  const int lane = threadIdx.x & 63;
  const int64_t t = wv / kTS;
  const int w = (int)(wv % kTS);
  const int4 T = A.tiles[t];
  const TileGrain TG = A.tgrain[T.x];
  const int cs = T.y + w, cm = T.z + lane / kTF, cf = T.w + lane % kTF;
  const int64_t i = (cs < TG.es && cm < TG.em && cf < TG.ef) ? (int64_t)A.tmap[tile_cell(TG, cs, cm, cf)] : -1;
  uint32_t m[4] = {0u, 0u, 0u, 0u};
  if (i >= 0) {
    const int64_t sc = i / kWave, sl = i % kWave;
    const int64_t off = A.slice_off[sc];
    const int W = (int)((A.slice_off[sc + 1] - off) / kWave);
    const int perm = A.tgrain[packed_grain(A.ucur[i].w)].perm;
    for (int e = 0; e < W; ++e) {
      const int64_t at = off + (int64_t)e * kWave + sl;
      const uint32_t wo = colOrig[at];
      const int cls = (int)(wo >> A.node_bits);
      if (cls >= A.n_stencil || A.colE[at] != wo) continue;
      const int b = ctob[perm * A.n_stencil + cls];
      m[b >> 5] |= 1u << (b & 31);
    }
  }
  uint64_t* row = A.lmask + wv * kTileClasses;
  for (int K = 0; K < kTileClasses; ++K) {
    const uint64_t bits = __ballot(((m[K >> 5] >> (K & 31)) & 1u) != 0u);
    if (lane == 0) row[K] = bits;
  }
}

// the inverse: an entry whose lane bit is clear becomes a broken column word
__global__ void k_mask_to_cols(StepArgs A, const int16_t* ctob, const uint32_t* colOrig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int32_t sl = A.slot[i];
  if (sl < 0) return;
  const int64_t sc = i / kWave, lane = i % kWave;
  const int64_t off = A.slice_off[sc];
  const int W = (int)((A.slice_off[sc + 1] - off) / kWave);
  const int perm = A.tgrain[packed_grain(A.ucur[i].w)].perm;
  const uint64_t* rowm = A.lmask + (int64_t)(sl >> 6) * kTileClasses;
  for (int e = 0; e < W; ++e) {
    const int64_t at = off + (int64_t)e * kWave + lane;
    const uint32_t wo = colOrig[at];
    const int cls = (int)(wo >> A.node_bits);
    if (cls >= A.n_stencil) continue;
    const uint64_t m = rowm[ctob[perm * A.n_stencil + cls]];
    A.colE[at] = ((m >> (sl & 63)) & 1ull) ? wo : ((uint32_t)i | A.sentinel_hi);
  }
}

// Wall reactions are reduced in a fixed order in two levels, the same in every
// step-loop mode: (1) chunk q of 1024 slice columns of a component is summed by
// one wavefront, lane l taking columns 1024 q + l + 64 k (k = 0..15) in turn,
// then across the lanes; (2) the chunk sums of a component are summed as by
// 1024 threads (virtual thread v takes chunks v, v + 1024, ...), across each
// virtual wave's lanes and over the 16 virtual waves in order.  With at most 64
// chunks only virtual wave 0 holds data and (2) is one wavefront's lane sum.
__device__ __forceinline__ double chunk_sum(const StepArgs& A, int c, int64_t q) {
  const int lane = threadIdx.x & 63;
  const int64_t n = A.partial_stride, b = q * kChunk + lane;
  const double* p = A.wall_partial + (int64_t)c * n;
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = b + 64 * k < n ? p[b + 64 * k] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  return wave_sum(s);
}

// Level (2) by one workgroup of NT threads from the chunk sums in wall_chunk,
// then the reactions and the wall positions of the next step: prescribed
// velocity or servo on the measured stress.
template <int NT>
__device__ __forceinline__ void finalize_level2(const StepArgs& A, double (*red)[1024 / kWave],
                                                double* tot, int64_t* s_step) {
  constexpr int VT = 1024 / NT;
  constexpr int CB = NT >= 1024 ? 8 : 2;  // components per batch (register budget)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nc = 3 * A.n_walls;
  const int64_t nq = (A.partial_stride + kChunk - 1) / kChunk;
  if (nq <= kWave) {
    if (wv == 0)
      for (int c = 0; c < nc; ++c) {
        const double t = wave_sum(lane < nq ? A.wall_chunk[(int64_t)c * nq + lane] : 0.0);
        if (lane == 0) tot[c] = t;
      }
  } else {
    for (int c0 = 0; c0 < nc; c0 += CB) {
      double acc[CB][VT];
#pragma unroll
      for (int cc = 0; cc < CB; ++cc)
#pragma unroll
        for (int k = 0; k < VT; ++k) acc[cc][k] = 0.0;
      for (int64_t b0 = 0; b0 < nq; b0 += 1024) {
#pragma unroll
        for (int k = 0; k < VT; ++k) {
          const int64_t b = b0 + tid + (int64_t)NT * k;  // virtual thread tid + NT k
#pragma unroll
          for (int cc = 0; cc < CB; ++cc) {
            const int c = c0 + cc;
            if (c < nc && b < nq) acc[cc][k] += A.wall_chunk[(int64_t)c * nq + b];
          }
        }
      }
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        if (c0 + cc < nc) {
#pragma unroll
          for (int k = 0; k < VT; ++k) {
            const double t = wave_sum(acc[cc][k]);
            if (lane == 0) red[c0 + cc][wv + (NT / kWave) * k] = t;
          }
        }
      }
    }
    __syncthreads();
    if (tid < nc) {
      double t = 0.0;
      for (int k = 0; k < 1024 / kWave; ++k) t += red[tid][k];
      tot[tid] = t;
    }
  }
  // a halted step changes neither the walls nor the step count
  if (A.advance && halted(A.halt)) return;
  if (tid == 0) *s_step = *A.step + A.advance;  // the step this evaluation belonged to
  __syncthreads();
  const int64_t s = *s_step;
  if (tid == 0) *A.step = s;
  // one thread per wall: its loads are independent of the other walls'
  if (tid < A.n_walls) {
    WallDev W = A.walls[tid];
    for (int q = 0; q < 3; ++q) {
      W.force[q] = -tot[3 * tid + q];
      if (A.advance) W.impulse[q] += W.force[q] * A.dt;
    }
    W.off_used = W.off;
    W.rate_used = W.rate;
    if (W.mode == PD_WALL_VELOCITY) {
      W.off = W.off0 + W.vel * ((double)(s + 1) * A.dt);
      W.rate = W.vel;
    } else if (W.mode == PD_WALL_SERVO) {
      const double sigma = -(W.force[0] * W.n[0] + W.force[1] * W.n[1] + W.force[2] * W.n[2]) / W.area;
      W.rate = W.gain * (W.target - sigma);
      W.off = W.off + A.dt * W.rate;
    }
    A.walls[tid] = W;
  }
}

// Level (1): one wavefront per (component, chunk) pair.  Level (2) and the
// wall update run in the next kernel, whose start sees every chunk sum (a
// kernel boundary instead of a device-scope fence per workgroup).
__global__ __launch_bounds__(kWave) void k_wall_chunks(StepArgs A) {
  const int nc = 3 * A.n_walls;
  const int64_t nq = (A.partial_stride + kChunk - 1) / kChunk;
  if ((int64_t)blockIdx.x >= (int64_t)nc * nq) return;
  const int c = (int)(blockIdx.x / nq);
  const int64_t q = blockIdx.x % nq;
  const double t = chunk_sum(A, c, q);
  if (threadIdx.x == 0) A.wall_chunk[(int64_t)c * nq + q] = t;
}

// 1024 threads: level (2) is written for 1024 virtual threads, so each takes
// one of them (the sums are the same for any workgroup size)
__global__ __launch_bounds__(1024) void k_wall_finalize(StepArgs A) {
  __shared__ double red[kMaxWalls * 3][1024 / kWave];
  __shared__ double tot[kMaxWalls * 3];
  __shared__ int64_t s_step;
  finalize_level2<1024>(A, red, tot, &s_step);
  if (threadIdx.x == 0) {
    // the last kernel of the step: the next step halts if this one raised a flag
    __hip_atomic_store(A.halt, __hip_atomic_load(A.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// persistent step loop: nsteps steps (no candidate rebuild among them) in one
// cooperative launch.  Workgroups walk their slice blocks of a step and meet at
// one grid barrier per step; the workgroup that arrives last reduces the wall
// reactions (in the order the launched wall kernels use, so the result is the
// same bit for bit) and writes the halt word before it releases the others,
// who then read the new wall state and the halt word.  Every wait has a spin
// limit, so each wave exits even if a barrier were never completed.
// ---------------------------------------------------------------------------

// Arrive at the grid barrier; returns (uniformly over the workgroup) whether
// this workgroup arrived last.  The last one must call grid_release after its
// serial work; the others have already waited for that release on return.
__device__ __forceinline__ bool grid_arrive(const BarrierArgs& B, uint32_t nblocks, uint32_t* status,
                                            uint32_t* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // release this workgroup's writes to every XCD
    const uint32_t g = __hip_atomic_load(B.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = atomicAdd(B.count, 1u) == nblocks - 1u;
    if (!last) {
      uint32_t spins = 0;
      while (__hip_atomic_load(B.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > B.spin_limit) {
          atomicOr(status, ST_BARRIER);
          break;
        }
      }
    }
    __threadfence();  // acquire the other workgroups' writes
    *s_flag = last ? 1u : 0u;
  }
  __syncthreads();
  return *s_flag != 0u;
}

__device__ __forceinline__ void grid_release(const BarrierArgs& B) {
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicExch(B.count, 0u);
    __threadfence();  // release the serial work before the generation moves
    atomicAdd(B.gen, 1u);
  }
  __syncthreads();
}

template <bool ABS>
__global__ __launch_bounds__(4 * kWave) __attribute__((amdgpu_waves_per_eu(kUnroll > 4 ? 3 : 4)))
void k_step_persistent(StepArgs A, int64_t nsteps, BarrierArgs B) {
  extern __shared__ StencilC s_st[];
  __shared__ double red[kMaxWalls * 3][1024 / kWave];
  __shared__ double tot[kMaxWalls * 3];
  __shared__ int64_t s_step;
  __shared__ uint32_t s_last;
  if (halted(A.halt)) return;
  stage_stencil(A, s_st);
  // the nv 4-slice blocks are cut evenly into rounds x gridDim runs (of 0 or
  // 1 blocks mostly).  In dispatch order workgroup b takes run q gridDim + b in
  // round q; in XCD order (gridDim a multiple of 8) the nx = gridDim / 8
  // workgroups of XCD x walk the x-th eighth of the runs side by side, so each
  // XCD's L2 serves one contiguous eighth of the mesh.  An even cut by blocks
  // measured faster than one by padded bond slots: the per-node work of a
  // slice (contact, walls, Verlet) does not scale with its bonds.
  const int64_t nv = (A.slice_end - A.slice_base + 3) / 4;
  const int64_t nb = gridDim.x, rounds = (nv + nb - 1) / nb, np = rounds * nb;
  int64_t p0 = blockIdx.x, pstep = nb;
  if (A.xcd_remap && (gridDim.x & 7u) == 0u) {
    const int64_t nx = nb >> 3;
    p0 = (int64_t)(blockIdx.x & 7u) * rounds * nx + (blockIdx.x >> 3);
    pstep = nx;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    for (int64_t q = 0; q < rounds; ++q) {
      const int64_t p = p0 + q * pstep;
      const int64_t vb1 = nv * (p + 1) / np;
      for (int64_t vb = nv * p / np; vb < vb1; ++vb) step_body<MODE_STEP, ABS, 4>(A, s_st, vb);
    }
    if (grid_arrive(B, gridDim.x, A.status, &s_last)) {
      // level (1) by this workgroup's wavefronts, then level (2)
      const int64_t nq = (A.partial_stride + kChunk - 1) / kChunk;
      for (int64_t pq = threadIdx.x >> 6; pq < (int64_t)(3 * A.n_walls) * nq; pq += 4) {
        const double t = chunk_sum(A, (int)(pq / nq), pq % nq);
        if ((threadIdx.x & 63) == 0) A.wall_chunk[pq] = t;
      }
      __threadfence_block();
      __syncthreads();
      finalize_level2<4 * kWave>(A, red, tot, &s_step);
      if (threadIdx.x == 0)
        __hip_atomic_store(A.halt, __hip_atomic_load(A.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      grid_release(B);
    }
    if (halted(A.halt)) break;
    // the drift just written is the next step's position; mid-step velocities likewise
    const double4* uc = A.ucur;
    A.ucur = A.unext;
    A.unext = const_cast<double4*>(uc);
    const double4* vc = A.vh_cur;
    A.vh_cur = A.vh_next;
    A.vh_next = const_cast<double4*>(vc);
  }
}

// ---------------------------------------------------------------------------
// energies (diagnostic): kinetic, elastic, contact, gravity potential
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_energy(StepArgs A, double* partial4) {
  __shared__ double red[4][kBlock];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kBlock + tid;
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < A.n) {
    const double4 ui = A.ucur[i];
    const GrainC* G = A.grains + packed_grain(ui.w);
    const int pi = packed_ijk(ui.w);
    const double V = G->V, rho = G->rho;
    const double vx = A.v[i], vy = A.v[A.n + i], vz = A.v[2 * A.n + i];
    e[0] = 0.5 * rho * V * (vx * vx + vy * vy + vz * vz);
    e[3] = -rho * V * (A.g[0] * ui.x + A.g[1] * ui.y + A.g[2] * ui.z);
    const int64_t s = i / kWave;
    const int lane = (int)(i % kWave);
    const int64_t off = A.slice_off[s];
    const int W = (int)((A.slice_off[s + 1] - off) / kWave);
    double w = 0.0;
    for (int k = 0; k < W; ++k) {
      const uint32_t cw = A.colE[off + (int64_t)k * kWave + lane];
      if ((cw & ~((1u << A.node_bits) - 1u)) == A.sentinel_hi) continue;  // broken or padding
      const int j = (int)(cw & ((1u << A.node_bits) - 1u));
      const double4 uj = A.ucur[j];
      const int pj = packed_ijk(uj.w);
      const int dx = unpack_x(pj) - unpack_x(pi), dy = unpack_y(pj) - unpack_y(pi),
                dz = unpack_z(pj) - unpack_z(pi);
      const double xx = G->h * dx, xy = G->h * dy, xz = G->h * dz;
      const double ex = uj.x - ui.x, ey = uj.y - ui.y, ez = uj.z - ui.z;
      const double yx = xx + ex, yy = xy + ey, yz = xz + ez;
      const double l0 = sqrt(xx * xx + xy * xy + xz * xz), l = sqrt(yx * yx + yy * yy + yz * yz);
      const double dd = ex * (2.0 * xx + ex) + ey * (2.0 * xy + ey) + ez * (2.0 * xz + ez);
      const double st = dd / (l0 * (l + l0));
      // micropotential 1/2 c w(|xi|) s^2 |xi| times V_j
      w += 0.5 * (G->cVih * G->h) * (1.0 - l0 * G->conic_inv_delta) * st * st * l0;
    }
    e[1] = 0.5 * V * w;
    if (A.cand_ptr != nullptr) {
      const int32_t c0 = (int32_t)min((int64_t)A.cand_ptr[i], A.cand_capacity);
      const int32_t c1 = (int32_t)min((int64_t)A.cand_ptr[i + 1], A.cand_capacity);
      for (int32_t c = c0; c < c1; ++c) {
        const int j = A.cand[c];
        const double4 uj = A.ucur[j];
        double yx, yy, yz;
        const double d2 = contact_d2(A.X[j], A.X[i], uj.x, ui.x, A.X[A.n + j], A.X[A.n + i], uj.y,
                                     ui.y, A.X[2 * A.n + j], A.X[2 * A.n + i], uj.z, ui.z, yx, yy, yz);
        if (!(d2 < A.Rc2)) continue;
        const GrainC* Gj = A.grains + packed_grain(uj.w);
        const double d = sqrt(d2);
        e[2] += 0.5 * V * 0.5 * A.Kn[G->mat * A.n_mat + Gj->mat] * (A.Rc - d) * (A.Rc - d) * Gj->V;
      }
    }
  }
  for (int q = 0; q < 4; ++q) red[q][tid] = e[q];
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (tid < o)
      for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + o];
    __syncthreads();
  }
  if (tid < 4) partial4[(int64_t)blockIdx.x * 4 + tid] = red[tid][0];
}

__global__ void k_reduce_energy(const double* partial4, int32_t nblocks, double* out4) {
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial4[(int64_t)b * 4 + threadIdx.x];
    out4[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// contact candidates: hashed uniform cell grid, counting sort, per-node rows
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t cell_hash(int cx, int cy, int cz, uint32_t T) {
  return (((uint32_t)cx * 73856093u) ^ ((uint32_t)cy * 19349663u) ^ ((uint32_t)cz * 83492791u)) &
         (T - 1u);
}

// cell coordinates are clamped to |c| < 2^20 - 1 so that a cell and its
// neighbours pack into one 63-bit key (21 bits per axis); nodes beyond the clamp
// share boundary cells and are still separated by the exact distance test
constexpr int kCellClamp = (1 << 20) - 2;

__device__ __forceinline__ int cell_coord(double p, double inv_cell) {
  double c = floor(p * inv_cell);
  c = fmin(fmax(c, -(double)kCellClamp), (double)kCellClamp);
  return (int)c;
}

__device__ __forceinline__ long long cell_key(int cx, int cy, int cz) {
  return ((long long)(cx + (1 << 20)) << 42) | ((long long)(cy + (1 << 20)) << 21) |
         (long long)(cz + (1 << 20));
}

// Grain-box culling.  A pair (i, j) of different grains closer than the
// cutoff needs p_i within the cutoff of grain(j)'s box and p_j within the
// cutoff of grain(i)'s box, so only nodes within the cutoff of another grain's
// box ("active" nodes) are binned and searched; the result is unchanged.

__device__ __forceinline__ long long ord_key(double x) {
  const long long b = __double_as_longlong(x);
  return b ^ ((b >> 63) & 0x7fffffffffffffffll);
}
__device__ __forceinline__ double ord_val(long long k) {
  return __longlong_as_double(k ^ ((k >> 63) & 0x7fffffffffffffffll));
}

__global__ void k_box_init(ContactArgs c) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)c.n_grains) return;
  c.gbox[t] = (t % 6) < 3 ? ord_key(INFINITY) : ord_key(-INFINITY);
}

__device__ __forceinline__ long long wave_min_ll(long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    const long long y = __shfl_xor(x, o, kWave);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ long long wave_max_ll(long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    const long long y = __shfl_xor(x, o, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// one workgroup per chunk of a single grain: LDS reduction, then 6 atomics
__global__ __launch_bounds__(256) void k_box(ContactArgs c) {
  __shared__ long long red[6][256];
  const int tid = threadIdx.x;
  const int64_t* ch = c.box_chunks + 3 * (int64_t)blockIdx.x;
  const int g = (int)ch[0];
  long long k[6] = {ord_key(INFINITY), ord_key(INFINITY), ord_key(INFINITY),
                    ord_key(-INFINITY), ord_key(-INFINITY), ord_key(-INFINITY)};
  for (int64_t i = ch[1] + tid; i < ch[2]; i += 256) {
    const double4 u = c.u[i];
    const long long x = ord_key(c.X[i] + u.x), y = ord_key(c.X[c.n + i] + u.y),
                    z = ord_key(c.X[2 * c.n + i] + u.z);
    k[0] = min(k[0], x);
    k[1] = min(k[1], y);
    k[2] = min(k[2], z);
    k[3] = max(k[3], x);
    k[4] = max(k[4], y);
    k[5] = max(k[5], z);
  }
  for (int q = 0; q < 6; ++q) red[q][tid] = k[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
      for (int q = 0; q < 6; ++q)
        red[q][tid] = q < 3 ? min(red[q][tid], red[q][tid + o]) : max(red[q][tid], red[q][tid + o]);
    __syncthreads();
  }
  if (tid < 3) atomicMin(c.gbox + 6 * g + tid, red[tid][0]);
  else if (tid < 6) atomicMax(c.gbox + 6 * g + tid, red[tid][0]);
}

// grain boxes closer than the cutoff: one wavefront per grain, the others
// tested 64 at a time; ballot prefix counts keep each list in ascending order
template <bool FILL>
__global__ __launch_bounds__(kWave) void k_box_pairs(ContactArgs c, double cut) {
  const int a = blockIdx.x, lane = threadIdx.x;
  double alo[3], ahi[3];
  for (int q = 0; q < 3; ++q) {
    alo[q] = ord_val(c.gbox[6 * a + q]) - cut;
    ahi[q] = ord_val(c.gbox[6 * a + 3 + q]) + cut;
  }
  int cnt = 0;
  const int base = FILL ? c.gpair_count[a] : 0;
  for (int b0 = 0; b0 < c.n_grains; b0 += kWave) {
    const int b = b0 + lane;
    bool ov = b < c.n_grains && b != a;
    if (ov)
      for (int q = 0; q < 3; ++q)
        ov = ov && ord_val(c.gbox[6 * b + q]) <= ahi[q] && ord_val(c.gbox[6 * b + 3 + q]) >= alo[q];
    const uint64_t m = __ballot(ov);
    if (FILL && ov) c.gpair[base + cnt + __popcll(m & ((1ull << lane) - 1ull))] = b;
    cnt += __popcll(m);
  }
  if (!FILL && lane == 0) c.gpair_count[a] = cnt;
}

__global__ void k_active(ContactArgs c, double cut) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const double4 u = c.u[i];
  const int g = packed_grain(u.w);
  const double p[3] = {c.X[i] + u.x, c.X[c.n + i] + u.y, c.X[2 * c.n + i] + u.z};
  // with self-contact every node can meet a node of its own grain
  uint8_t act = c.self_contact ? 1 : 0;
  for (int e = c.gpair_count[g]; e < c.gpair_count[g + 1] && !act; ++e) {
    const int b = c.gpair[e];
    bool in = true;
    for (int q = 0; q < 3; ++q)
      in = in && p[q] >= ord_val(c.gbox[6 * b + q]) - cut && p[q] <= ord_val(c.gbox[6 * b + 3 + q]) + cut;
    act = in ? 1 : 0;
  }
  c.active[i] = act;
}

// The cell grid of this rebuild: the box around every node's position (the
// union of the grain boxes), in cells; dense when its cell count fits the
// buckets.  One wavefront.
__global__ __launch_bounds__(kWave) void k_grid_setup(ContactArgs c) {
  const int lane = threadIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int g = lane; g < c.n_grains; g += kWave)
    for (int q = 0; q < 3; ++q) {
      const double a = ord_val(c.gbox[6 * g + q]), b = ord_val(c.gbox[6 * g + 3 + q]);
      if (a <= b) {  // grains without nodes keep an empty box
        lo[q] = fmin(lo[q], a);
        hi[q] = fmax(hi[q], b);
      }
    }
  for (int q = 0; q < 3; ++q)
    for (int o = 32; o > 0; o >>= 1) {
      lo[q] = fmin(lo[q], __shfl_xor(lo[q], o, kWave));
      hi[q] = fmax(hi[q], __shfl_xor(hi[q], o, kWave));
    }
  if (lane != 0) return;
  int64_t dense = 1, cells = 1, o[3], e[3];
  for (int q = 0; q < 3; ++q) {
    if (!(lo[q] <= hi[q])) dense = 0;
    o[q] = dense ? cell_coord(lo[q], c.inv_cell) : 0;
    e[q] = dense ? cell_coord(hi[q], c.inv_cell) - o[q] + 1 : 1;
    cells *= e[q];
  }
  if (cells > (int64_t)c.T) dense = 0;
  c.grid[0] = dense;
  for (int q = 0; q < 3; ++q) {
    c.grid[1 + q] = o[q];
    c.grid[4 + q] = e[q];
  }
}

// bucket of a cell: its lexicographic index in the dense grid, else its hash
__device__ __forceinline__ uint32_t cell_bucket(const ContactArgs& c, bool dense, int cx, int cy, int cz) {
  if (dense)
    return (uint32_t)(((int64_t)(cx - c.grid[1]) * c.grid[5] + (cy - c.grid[2])) * c.grid[6] + (cz - c.grid[3]));
  return cell_hash(cx, cy, cz, c.T);
}

__global__ void k_bin(ContactArgs c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n || !c.active[i]) return;
  const double4 u = c.u[i];
  const int cx = cell_coord(c.X[i] + u.x, c.inv_cell);
  const int cy = cell_coord(c.X[c.n + i] + u.y, c.inv_cell);
  const int cz = cell_coord(c.X[2 * c.n + i] + u.z, c.inv_cell);
  c.cellkey[i] = cell_key(cx, cy, cz);
  const uint32_t hsh = cell_bucket(c, c.grid[0] != 0, cx, cy, cz);
  c.cellh[i] = hsh;
  atomicAdd(c.bucket_count + hsh, 1);
}

__global__ void k_scatter(ContactArgs c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n || !c.active[i]) return;
  const uint32_t hsh = c.cellh[i];
  const int pos = c.bucket_start[hsh] + atomicAdd(c.bucket_fill + hsh, 1);
  const long long key = c.cellkey[i];
  c.srec[pos] = make_int4((int)i, packed_grain(c.u[i].w), (int)(key & 0xffffffffll), (int)(key >> 32));
}

// Search: every record of the 27 neighbouring cells' buckets is one 16-byte
// load (node, grain, cell key); records of other cells sharing the bucket and
// of the node's own grain are skipped before any position is read.  Threads
// walk the binned nodes in bucket order, so the nodes of one cell sit in
// neighbouring lanes and read the same buckets.  In a dense grid the three
// cells of a z-run are consecutive buckets, read as one range (and hold no
// other cells).  Hits go to a fixed-width scratch row; counts beyond the width
// raise the overflow flag.  Rows of nodes that were not binned stay at zero
// (cleared before the launch).
__device__ __forceinline__ void cand_consider(const ContactArgs& c, const int4& r, int64_t i, int gi, double Xx,
                                              double Xy, double Xz, const double4& ui, int32_t* row, int& cnt) {
  // with self-contact the node's own grain counts too (whether a pair is
  // bonded is decided at the force, from the bond memory)
  if (r.y == gi && (!c.self_contact || r.x == i)) return;
  const int j = r.x;
  const double4 uj = c.u[j];
  const double* xp = reinterpret_cast<const double*>(c.X4 + j);
  double yx, yy, yz;
  const double d2 = contact_d2(xp[0], Xx, uj.x, ui.x, xp[1], Xy, uj.y, ui.y, xp[2], Xz, uj.z, ui.z, yx, yy, yz);
  if (!(d2 < c.cut2)) return;
  if (cnt < c.scratch_w) row[cnt] = j;
  ++cnt;
}

__global__ __launch_bounds__(256) void k_cand_search(ContactArgs c) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e0 >= c.bucket_start[c.T]) return;
  const int4 me = c.srec[e0];
  const int64_t i = me.x;
  const int gi = me.y;
  const double4 ui = c.u[i];
  const long long key = ((long long)me.w << 32) | (long long)(uint32_t)me.z;
  const int cx = (int)((key >> 42) & 0x1fffff) - (1 << 20);
  const int cy = (int)((key >> 21) & 0x1fffff) - (1 << 20);
  const int cz = (int)(key & 0x1fffff) - (1 << 20);
  const double4 Xi = c.X4[i];
  const double Xx = Xi.x, Xy = Xi.y, Xz = Xi.z;
  int32_t* row = c.cand_scratch + i * (int64_t)c.scratch_w;
  int cnt = 0;
  if (c.grid[0]) {
    const int64_t ex = c.grid[4], ey = c.grid[5], ez = c.grid[6];
    const int64_t lx = cx - c.grid[1], ly = cy - c.grid[2], lz = cz - c.grid[3];
    const int64_t z0 = lz > 0 ? lz - 1 : 0, z1 = lz + 1 < ez ? lz + 1 : ez - 1;
    for (int d = 0; d < 9; ++d) {
      const int64_t nx = lx + d / 3 - 1, ny = ly + d % 3 - 1;
      if (nx < 0 || ny < 0 || nx >= ex || ny >= ey) continue;
      const int64_t b = (nx * ey + ny) * ez;
      const int e1 = c.bucket_start[b + z1 + 1];
      for (int e = c.bucket_start[b + z0]; e < e1; ++e) cand_consider(c, c.srec[e], i, gi, Xx, Xy, Xz, ui, row, cnt);
    }
  } else {
    for (int d = 0; d < kCellDirs; ++d) {
      const int nx = cx + d % 3 - 1, ny = cy + (d / 3) % 3 - 1, nz = cz + d / 9 - 1;
      const long long nkey = cell_key(nx, ny, nz);
      const int klo = (int)(nkey & 0xffffffffll), khi = (int)(nkey >> 32);
      const uint32_t hsh = cell_hash(nx, ny, nz, c.T);
      const int e1 = c.bucket_start[hsh + 1];
      for (int e = c.bucket_start[hsh]; e < e1; ++e) {
        const int4 r = c.srec[e];
        if (r.z != klo || r.w != khi) continue;  // another cell in the same bucket
        cand_consider(c, r, i, gi, Xx, Xy, Xz, ui, row, cnt);
      }
    }
  }
  if (cnt > c.scratch_w) {
    atomicOr(c.status, ST_CAND_OVERFLOW);
    cnt = c.scratch_w;
  }
  c.cand_count[i] = cnt;
}

// scratch row -> CSR row (ascending; rows past the total capacity are cut and flagged)
__global__ __launch_bounds__(256) void k_cand_compact(ContactArgs c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const int64_t base = c.cand_count[i];  // scanned row pointers
  const int cnt = (int)(c.cand_count[i + 1] - base);
  if (cnt == 0) return;
  const int32_t* row = c.cand_scratch + i * (int64_t)c.scratch_w;
  const int64_t end = base + cnt < c.capacity ? base + cnt : c.capacity;
  for (int64_t a = base; a < end; ++a) {
    const int32_t x = row[a - base];
    int64_t q = a - 1;
    while (q >= base && c.cand[q] > x) {
      c.cand[q + 1] = c.cand[q];
      --q;
    }
    c.cand[q + 1] = x;
  }
}

__global__ void k_cand_capacity(ContactArgs c) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && (int64_t)c.cand_count[c.n] > c.capacity)
    atomicOr(c.status, ST_CAND_OVERFLOW);
}

// displacement since the last rebuild beyond skin/2 invalidates the list
__global__ void k_skin(ContactArgs c, int check) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n || halted(c.halt)) return;
  const double4 u = c.u[i];
  if (check) {
    const double dx = u.x - c.u_build[i], dy = u.y - c.u_build[c.n + i], dz = u.z - c.u_build[2 * c.n + i];
    if (dx * dx + dy * dy + dz * dz > c.skin_half2) atomicOr(c.status, ST_SKIN);
  }
  c.u_build[i] = u.x;
  c.u_build[c.n + i] = u.y;
  c.u_build[2 * c.n + i] = u.z;
}

__global__ void k_fill_u4(double4* u4, const double* u, const int32_t* ijk, const int64_t* grain_of,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t w = (int64_t)(uint32_t)(ijk[i] | (ijk[n + i] << 10) | (ijk[2 * n + i] << 20)) |
                    (grain_of[i] << 32);
  u4[i] = make_double4(u[i], u[n + i], u[2 * n + i], __longlong_as_double(w));
}

// ---------------------------------------------------------------------------
// exclusive scans (3 passes: block-local, block sums, add)
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ T block_inclusive_scan(T x, T* s) {
  const int tid = threadIdx.x;
  s[tid] = x;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const T t = tid >= o ? s[tid - o] : T(0);
    __syncthreads();
    s[tid] += t;
    __syncthreads();
  }
  return s[tid];
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const T* in, T* out, int64_t n,
                                                             T* block_sums) {
  __shared__ T s[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T tot = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : T(0);
    tot += v[k];
  }
  const T inc = block_inclusive_scan(tot, s);
  T run = inc - tot;
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) block_sums[blockIdx.x] = inc;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_top(T* block_sums, int64_t nb, T* total) {
  __shared__ T s[kScanThreads];
  T carry = 0;
  for (int64_t c = 0; c < nb; c += kScanThreads) {
    const int64_t idx = c + threadIdx.x;
    const T x = idx < nb ? block_sums[idx] : T(0);
    const T inc = block_inclusive_scan(x, s);
    if (idx < nb) block_sums[idx] = carry + inc - x;
    const T chunk = s[kScanThreads - 1];
    __syncthreads();
    carry += chunk;
  }
  if (threadIdx.x == 0) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T* out, int64_t n, const T* block_sums) {
  const T add = block_sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] += add;
}

__global__ void k_pack_x4(const double* X, double4* X4, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X4[i] = make_double4(X[i], X[n + i], X[2 * n + i], 0.0);
}

__global__ void k_fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_pack_x4(const double* X, double4* X4, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_x4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, X4, n);
  return hipGetLastError();
}

template <typename T>
__global__ void k_set_value(T* p, T v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

int64_t scan_scratch_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename T>
static hipError_t scan_impl(const T* in, T* out, int64_t n, T* scratch, hipStream_t s) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_set_value<T>, dim3(1), dim3(64), 0, s, out, T(0));
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_local<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, scratch);
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kScanThreads), 0, s, scratch, nb, out + n);
  hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, n,
                     (const T*)scratch);
  return hipGetLastError();
}

hipError_t scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, scratch, s);
}
hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s) {
  return scan_impl<int32_t>(in, out, n, scratch, s);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned grid_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

hipError_t launch_map_fill(const BuildArgs& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_fill, dim3(grid_for(b.n, 256)), dim3(256), 0, s, b);
  return hipGetLastError();
}
hipError_t launch_bond_count(const BuildArgs& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bond_count, dim3(grid_for(b.n, 256)), dim3(256), 0, s, b);
  return hipGetLastError();
}
hipError_t launch_slice_width(const BuildArgs& b, hipStream_t s) {
  if (b.nslices == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_width, dim3(grid_for(b.nslices, 256)), dim3(256), 0, s, b);
  return hipGetLastError();
}
hipError_t launch_bond_fill(const BuildArgs& b, hipStream_t s) {
  if (b.nslices == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bond_fill, dim3(grid_for(b.nslices, kSlicesPerBlock)), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

int32_t step_blocks_spb(int64_t nslices, int slices_per_block) {
  return (int32_t)grid_for(nslices, slices_per_block);
}
int32_t step_grid_blocks(int64_t nslices) { return step_blocks_spb(nslices, kSlicesPerBlock); }

hipError_t launch_wall_finalize(const StepArgs& a, hipStream_t s) {
  const int64_t nq = (a.partial_stride + kChunk - 1) / kChunk;
  const int64_t pairs = (int64_t)(3 * a.n_walls) * nq;
  if (pairs > 0) hipLaunchKernelGGL(k_wall_chunks, dim3((unsigned)pairs), dim3(kWave), 0, s, a);
  hipLaunchKernelGGL(k_wall_finalize, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

static size_t step_lds(const StepArgs& a) {
  return sizeof(StencilC) * (size_t)(a.n_stencil + 1) * (size_t)a.n_classes;
}

template <int MODE, int SPB>
static void launch_step_t(const StepArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const int32_t nb = step_blocks_spb(a.slice_end - a.slice_base, SPB);
  if (nb == 0) return;
  // with events, the launch itself records them around the kernel
  if (e0 || e1) {
    if (a.abs_stretch)
      hipExtLaunchKernelGGL((k_step<MODE, true, SPB>), dim3(nb), dim3(SPB * kWave), step_lds(a), s, e0, e1, 0, a);
    else
      hipExtLaunchKernelGGL((k_step<MODE, false, SPB>), dim3(nb), dim3(SPB * kWave), step_lds(a), s, e0, e1, 0, a);
  } else if (a.abs_stretch) {
    hipLaunchKernelGGL((k_step<MODE, true, SPB>), dim3(nb), dim3(SPB * kWave), step_lds(a), s, a);
  } else {
    hipLaunchKernelGGL((k_step<MODE, false, SPB>), dim3(nb), dim3(SPB * kWave), step_lds(a), s, a);
  }
}

hipError_t launch_step(const StepArgs& a, int mode, hipStream_t s) {
  if (mode == MODE_FIRST) launch_step_t<MODE_FIRST, kSlicesPerBlock>(a, s);
  else if (mode == MODE_STEP) launch_step_t<MODE_STEP, kSlicesPerBlock>(a, s);
  else launch_step_t<MODE_FORCE_ONLY, kSlicesPerBlock>(a, s);
  return hipGetLastError();
}

hipError_t launch_step_spb(const StepArgs& a, int slices_per_block, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (slices_per_block) {
    case 1: launch_step_t<MODE_STEP, 1>(a, s, e0, e1); break;
    case 2: launch_step_t<MODE_STEP, 2>(a, s, e0, e1); break;
    case 4: launch_step_t<MODE_STEP, 4>(a, s, e0, e1); break;
    case 8: launch_step_t<MODE_STEP, 8>(a, s, e0, e1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int32_t persistent_max_blocks(const StepArgs& a) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = a.abs_stretch ? reinterpret_cast<const void*>(&k_step_persistent<true>)
                                 : reinterpret_cast<const void*>(&k_step_persistent<false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 4 * kWave, step_lds(a)) != hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t launch_step_persistent(const StepArgs& a, int64_t nsteps, int32_t nblocks, const BarrierArgs& b,
                                  hipStream_t s) {
  if (nsteps <= 0) return hipSuccess;
  if (step_blocks_spb(a.slice_end - a.slice_base, 4) == 0) return hipSuccess;
  StepArgs aa = a;
  BarrierArgs bb = b;
  void* args[] = {&aa, &nsteps, &bb};
  const void* fn = a.abs_stretch ? reinterpret_cast<const void*>(&k_step_persistent<true>)
                                 : reinterpret_cast<const void*>(&k_step_persistent<false>);
  // a cooperative launch fails rather than start more workgroups than can be
  // resident at once, which the grid barrier relies on
  return hipLaunchCooperativeKernel(fn, dim3((unsigned)nblocks), dim3(4 * kWave), args,
                                    (unsigned)step_lds(a), s);
}

// early-rebuild watch, before an evaluation between cadence rebuilds: a node
// beyond skin/2 of where the list was built may have a partner within R_c
// that the list lacks.  The flag halts this step and the ones after it (the
// step kernel and the wall pass see the halt word), so the host can rebuild
// the list at these positions and go on from the same step.
__global__ void k_skin_watch(ContactArgs c, uint32_t* halt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n || halted(c.halt)) return;
  const double4 u = c.u[i];
  const double dx = u.x - c.u_build[i], dy = u.y - c.u_build[c.n + i], dz = u.z - c.u_build[2 * c.n + i];
  if (dx * dx + dy * dy + dz * dz > c.skin_half2) {
    atomicOr(c.status, ST_REBUILD);
    atomicOr(halt, ST_REBUILD);
  }
}

hipError_t launch_skin_watch(const ContactArgs& c, uint32_t* halt, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_skin_watch, dim3(grid_for(c.n, 256)), dim3(256), 0, s, c, halt);
  return hipGetLastError();
}

hipError_t launch_contact_rebuild(const ContactArgs& c, int check_skin, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const unsigned g = grid_for(c.n, 256);
  const double cut = sqrt(c.cut2) * (1.0 + 1e-9) + 1e-300;  // boxes inflated by the cutoff
  hipError_t e;
  // clears by kernel (not memset nodes) so the sequence can live in a captured graph
  if ((e = launch_fill_i32(c.bucket_count, 0, (int64_t)c.T, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(c.bucket_fill, 0, (int64_t)c.T, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_skin, dim3(g), dim3(256), 0, s, c, check_skin);
  hipLaunchKernelGGL(k_box_init, dim3(grid_for(6 * (int64_t)c.n_grains, 256)), dim3(256), 0, s, c);
  hipLaunchKernelGGL(k_box, dim3((unsigned)c.n_box_chunks), dim3(256), 0, s, c);
  const unsigned gg = (unsigned)c.n_grains;
  hipLaunchKernelGGL(k_box_pairs<false>, dim3(gg), dim3(kWave), 0, s, c, cut);
  if ((e = scan_i32(c.gpair_count, c.gpair_count, c.n_grains, c.scan_scratch, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_box_pairs<true>, dim3(gg), dim3(kWave), 0, s, c, cut);
  hipLaunchKernelGGL(k_active, dim3(g), dim3(256), 0, s, c, cut);
  hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(kWave), 0, s, c);
  hipLaunchKernelGGL(k_bin, dim3(g), dim3(256), 0, s, c);
  if ((e = scan_i32(c.bucket_count, c.bucket_start, (int64_t)c.T, c.scan_scratch, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, c);
  if ((e = launch_fill_i32(c.cand_count, 0, c.n, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cand_search, dim3(g), dim3(256), 0, s, c);
  if ((e = scan_i32(c.cand_count, c.cand_count, c.n, c.scan_scratch, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cand_capacity, dim3(1), dim3(64), 0, s, c);
  hipLaunchKernelGGL(k_cand_compact, dim3(g), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_energy(const StepArgs& a, double* partial4, int32_t nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_energy, dim3(nblocks), dim3(kBlock), 0, s, a, partial4);
  return hipGetLastError();
}

hipError_t launch_reduce_energy(const double* partial4, int32_t nblocks, double* out4,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(64), 0, s, partial4, nblocks, out4);
  return hipGetLastError();
}

template <bool ABS, bool EXTRA>
void launch_tile_variant(const StepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)a.n_tiles), block(kTS * kWave);
  void (*kern)(StepArgs) = k_step_tile<ABS, EXTRA>;
  if (e0 || e1) hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, a);
  else hipLaunchKernelGGL(kern, grid, block, 0, s, a);
}

hipError_t launch_step_tile(const StepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.n_tiles == 0) return hipSuccess;
  const bool extra = a.self_contact || a.wall_corners;
  if (a.abs_stretch) {
    if (extra) launch_tile_variant<true, true>(a, s, e0, e1);
    else launch_tile_variant<true, false>(a, s, e0, e1);
  } else {
    if (extra) launch_tile_variant<false, true>(a, s, e0, e1);
    else launch_tile_variant<false, false>(a, s, e0, e1);
  }
  return hipGetLastError();
}

hipError_t launch_tile_map_fill(const StepArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_map_fill, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cols_to_mask(const StepArgs& a, const int16_t* ctob, const uint32_t* colOrig, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cols_to_mask, dim3(grid_for(a.n_tiles * kTS * kWave, 256)), dim3(256), 0, s, a, ctob, colOrig);
  return hipGetLastError();
}

hipError_t launch_mask_to_cols(const StepArgs& a, const int16_t* ctob, const uint32_t* colOrig, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_to_cols, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a, ctob, colOrig);
  return hipGetLastError();
}

hipError_t launch_wall_corners(const StepArgs& a, int force_only, hipStream_t s) {
  if (a.n == 0 || !a.wall_corners) return hipSuccess;
  hipLaunchKernelGGL(k_wall_corners, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a, force_only);
  return hipGetLastError();
}

hipError_t launch_fill_u4(double4* u4, const double* u, const int32_t* ijk, const int64_t* grain_of,
                          int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u4, dim3(grid_for(n, 256)), dim3(256), 0, s, u4, u, ijk, grain_of, n);
  return hipGetLastError();
}

}  // namespace pdk
