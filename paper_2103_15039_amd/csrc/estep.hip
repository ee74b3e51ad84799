// The LSG-CPD E step on gfx950 (Sec. 3.1 Eq. 5, Sec. 3.4 Eq. 9-10).
//
// For every (target m, source n) pair the kernels evaluate
//   e_mn = K_mn / rho_n = 2^( l_m - c d_mn ),   c = log2(e) / (2 sigma^2),
//   d_mn = |r|^2 + (a_m . r)^2,  r = g(x_n) - y_m,  a_m = sqrt(alpha_m) n_m,
// i.e. sigma^2 times the Mahalanobis form of Eq. 2, and accumulate for each
// source the unnormalised sums  T_n[c] = sum_m e_mn f_m[c]  of 11 target
// features f_m = [1, alpha n n^T, M_m y_m, y_m^T M_m y_m]  (M_m = I + alpha n n^T).
// The normaliser of Eq. 9 is per source (a column of P), so one pass over the
// pairs suffices: P_mn = rho_n e_mn / (rho_n T_n[0] + gamma), and every
// P-weighted sum is rho_n T_n[c] / (rho_n T_n[0] + gamma).  The M x N posterior
// is never stored.
//
// Arithmetic per pair (gfx950 runs FP64 FMA at the FP32 rate, and packed FP32
// is not used): with the source pre-scaled, s_n = sqrt(c) g(x_n),
//   r = s_n - sqrt(c) y_m          3 FP64 FMA
//   q = l_m - |r|^2                 3 FP64 FMA
//   p = a_m . r                     3 FP64
//   z = q - p^2                     1 FP64 FMA   (= l_m - c d_mn)
//   e = exp2((float) z)             cvt + v_exp_f32 + cvt
//   T += e f_m                      11 FP64 add/FMA
// so residual and exponent are FP64 and only the exponential is float32
// (relative error of e about 2e-6 over the range that matters); features are
// exact FP64 functions of the float32 inputs and all sums are FP64.
//
// Back ends (same pair arithmetic, different data movement):
//  * estep_pairs_items (default): all lanes of a wave take the same target
//    at the same time, so the target record is wave-uniform and is read
//    through the scalar data cache straight into SGPR operands; each lane keeps
//    2 sources in registers (one of each half of a 128-source group).  Target tiles that provably hold only exact-zero
//    exponentials for a source group are dropped, and the rest is cut into
//    balanced work items.
//  * estep_pairs_lds<S>: the block stages tiles of target records in LDS and
//    every wave reads them back with broadcast LDS loads.
//  * estep_mfma: V_MFMA_F64_16X16X4 multiplies 16 (sources) x 4 (targets)
//    exponentials by 4 x 16 features.  On gfx950 matrix and vector
//    instructions of a SIMD do not execute concurrently and the FP64 matrix
//    rate equals the FP64 vector rate, so this is kept only for comparison.
// Work items (scalar) or target chunks (LDS, MFMA) give enough blocks for
// small N; their partial sums are combined in a fixed order by the
// finalisation (mstep.hip), so results are bitwise reproducible.
#include <math.h>
#include <string.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kTwoPi = 6.283185307179586477;
constexpr int kBlock = 256;
constexpr int kTile = 64;            // targets per LDS tile (LDS back end)

// sqrt(c) with c = log2(e) / (2 sigma^2)
__device__ __forceinline__ double sqrt_c_of(const DevState *s) {
  return sqrt(kLog2e / (2.0 * s->sigma2));
}

struct Src {
  double x0, x1, x2;  // sqrt(c) * g(x_n)
};

// Source n (zeros past the end, n >= N).  The load itself is unconditional,
// from an index clamped to the cloud (N >= 1 wherever a block runs), so that
// it issues as soon as the address is known.
__device__ __forceinline__ Src load_src(const float *__restrict__ X, int n, int N,
                                        const double *R, const double *t, double sc) {
  const int k = n < N ? n : N - 1;
  const float fx = X[3 * k], fy = X[3 * k + 1], fz = X[3 * k + 2];
  const double x = n < N ? (double)fx : 0.0, y = n < N ? (double)fy : 0.0,
               z = n < N ? (double)fz : 0.0;
  Src o;
  o.x0 = sc * fma(R[0], x, fma(R[1], y, fma(R[2], z, t[0])));
  o.x1 = sc * fma(R[3], x, fma(R[4], y, fma(R[5], z, t[1])));
  o.x2 = sc * fma(R[6], x, fma(R[7], y, fma(R[8], z, t[2])));
  return o;
}

// Exponent z = log2(e_mn) = l_m - c d_mn of one pair; negsc = -sqrt(c).
// Every operation is written out so that every kernel (and the P dump)
// produces the same value.
__device__ __forceinline__ double pair_z(const Src &s, double y0, double y1, double y2,
                                         double a0, double a1, double a2, double l,
                                         double negsc) {
  const double r0 = fma(negsc, y0, s.x0);
  const double r1 = fma(negsc, y1, s.x1);
  const double r2 = fma(negsc, y2, s.x2);
  double q = fma(-r0, r0, l);
  q = fma(-r1, r1, q);
  q = fma(-r2, r2, q);
  double p = a0 * r0;
  p = fma(a1, r1, p);
  p = fma(a2, r2, p);
  return fma(-p, p, q);
}

// e = K_mn / rho_n = 2^z, the only float32 step
__device__ __forceinline__ double exp2_of(double z) {
  return (double)__builtin_amdgcn_exp2f((float)z);
}

__device__ __forceinline__ double rec_z(const Src &s, const TRec &t, double negsc) {
  return pair_z(s, t.y[0], t.y[1], t.y[2], t.a[0], t.a[1], t.a[2], t.l, negsc);
}

__device__ __forceinline__ double rec_exp(const Src &s, const TRec &t, double negsc) {
  return exp2_of(rec_z(s, t, negsc));
}

// Below this exponent the float32 exp2 is exactly +0 (2^-160 is far below the
// smallest denormal, 2^-149), so such pairs add exact zeros to every sum.
constexpr double kZeroExponent = -160.0;

// Adds one target's contribution to the S sources of this lane.
template <int S>
__device__ __forceinline__ void accumulate(const Src (&x)[S], const TRec &t, double negsc,
                                           double (&acc)[S][kFeatUsed]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double e = rec_exp(x[s], t, negsc);
    acc[s][0] += e;
#pragma unroll
    for (int c = 1; c < kFeatUsed; ++c) acc[s][c] = fma(e, t.f[c - 1], acc[s][c]);
  }
}

// Adds one target's contribution to one source of this lane.
__device__ __forceinline__ void accumulate1(const Src &x, const TRec &t, double negsc,
                                            double (&acc)[kFeatUsed]) {
  const double e = rec_exp(x, t, negsc);
  acc[0] += e;
#pragma unroll
  for (int c = 1; c < kFeatUsed; ++c) acc[c] = fma(e, t.f[c - 1], acc[c]);
}

// The same exponent with both points taken relative to a centre o of the
// source group (scaled coordinates): u = s_n - o, v = sqrt(c) y_m - o,
//   z = l_m - |u - v|^2 - (a_m . (u - v))^2
//     = (l_m - |v|^2) - |u|^2 + u . (2 v) - (a_m . u - a_m . v)^2.
// Per target the pair kernel stages T = [2 v, l_m - |v|^2, -a_m . v] once
// per tile; per source it keeps u and |u|^2, so that a pair costs 8 FP64
// operations for the exponent instead of 10, on values of the size of the
// group's neighbourhood rather than of the clouds' coordinates.
struct SrcRel {
  double u0, u1, u2, uu;
};

__device__ __forceinline__ double rel_z(const SrcRel &x, const double *T, const double *a) {
  const double q = fma(x.u0, T[0], fma(x.u1, T[1], fma(x.u2, T[2], T[3] - x.uu)));
  const double p = fma(a[0], x.u0, fma(a[1], x.u1, fma(a[2], x.u2, T[4])));
  return fma(-p, p, q);
}

template <int S>
__device__ __forceinline__ void accumulate_rel(const SrcRel (&x)[S], const double *T,
                                               const TRec &t, double (&acc)[S][kFeatUsed]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double e = exp2_of(rel_z(x[s], T, t.a));
    acc[s][0] += e;
#pragma unroll
    for (int c = 1; c < kFeatUsed; ++c) acc[s][c] = fma(e, t.f[c - 1], acc[s][c]);
  }
}

__device__ __forceinline__ void accumulate1_rel(const SrcRel &x, const double *T, const TRec &t,
                                                double (&acc)[kFeatUsed]) {
  const double e = exp2_of(rel_z(x, T, t.a));
  acc[0] += e;
#pragma unroll
  for (int c = 1; c < kFeatUsed; ++c) acc[c] = fma(e, t.f[c - 1], acc[c]);
}

// Exact culling.  For sources whose scaled positions lie in the box
// [blo, bhi] and targets whose positions lie in [lo, hi] with log-priors
// <= lmax, every pair has |r|^2 >= d2 = sum_a gap_a^2 (gap_a = distance between
// the two intervals on axis a after scaling the targets by sqrt(c)), and since
// the plane term is non-negative, z = l - |r|^2 - p^2 <= lmax - d2.  If that
// bound is below kZeroExponent every such exponential is an exact zero and
// the pairs can be skipped without changing any sum by a single bit.  A
// single target is the box lo = hi = y_m, lmax = l_m.
__device__ __forceinline__ bool box_live(const double *lo, const double *hi, double lmax,
                                         const double (&blo)[3], const double (&bhi)[3],
                                         double sc) {
  double d2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double g = fmax(0.0, fmax(sc * lo[a] - bhi[a], blo[a] - sc * hi[a]));
    d2 = fma(g, g, d2);
  }
  return lmax - d2 >= kZeroExponent;
}

// ------------------------------------------------------- pair kernel (VALU)
// Scalar-cache back end with exact tile culling and balanced work items.
//
// Sources form groups of kGroup = 128 consecutive points (2 per lane of a
// wave); targets form tiles of kCullTile = 64 consecutive records.  Once per
// E step
//  * cull_groups (one block per group) takes the group's bounding box in
//    scaled coordinates and lists, in increasing order, the tiles that
//    box_live cannot rule out (with culling off: every tile);
//  * cull_items (one block per problem) cuts every group's list into items
//    of L tiles, with L chosen so that there are at most about `target` items
//    in all, and writes one descriptor per item (group, first tile, tile
//    count, and whether the group kept every tile);
//  * estep_pairs_items runs one block per item: the 4 waves hold the same 128
//    sources and take every 4th tile of the item (in a split item: every
//    tile, and of its targets every 4th).  Per tile, one lane per target
//    tests the target against the group box (not in an item whose group kept
//    every tile), stages its centred terms in the wave's LDS, and the wave
//    walks the set bits of the resulting 64-bit mask.  The 4 waves' sums are
//    added through LDS in a fixed order and the block writes one partial per
//    source and feature.
// Groups near much of the target cloud get many items and isolated ones few,
// so the blocks carry about equal work whatever the culling removes.  All
// counts are integers and every sum runs in a fixed order, so results are
// bitwise reproducible.
// 2 sources per lane measured faster than 4 (tighter group boxes, twice the
// groups to balance, more waves per SIMD) and than 1 on both benchmark pairs
constexpr int kSrcPerLane = 2;
static_assert(kGroup == 64 * kSrcPerLane, "a group is the two sources of each lane of a wave");
// the per-half culling (two half boxes per group, slot s of a lane = half s)
// is written for exactly two sources per lane
static_assert(kSrcPerLane == 2, "per-half culling assumes two sources per lane");
// Per source group: the boxes of its two halves of 64 sources (the sources
// of slot 0 and slot 1 of the pair kernel's lanes), lo and hi each.
constexpr int kGBox = 16;
// Per-target terms of the pair kernel's centred exponent (2 v, l - |v|^2,
// -a . v, and a pad to keep rows 16-byte aligned).
constexpr int kRelT = 6;
// A work item: its source group g and its tiles, positions k0 .. k0 + kn - 1
// of the group's live-tile list (one 16-byte load for the pair kernels).
// full: no tile of the target cloud was ruled out for the group (large
// sigma^2); the FP64 pair kernel then takes every target of the item's tiles
// without its per-target test.  That is exact either way: a target the test
// would have dropped only adds exponentials that are exact zeros.
struct __align__(16) Item {
  int g, k0, kn, full;
};
static_assert(sizeof(CullHdr) == 16, "the plan header is read as one 16-byte load");

// The plan header of problem p, read as one 16-byte vector: its item count
// decides whether a block has work, its other fields the block's item.
__device__ __forceinline__ CullHdr load_hdr(const CullHdr *h, int p) {
  const int4 v = reinterpret_cast<const int4 *>(h)[p];
  return CullHdr{v.x, v.y, v.z, v.w};
}
// BF16 matrix-core pair kernel (estep_pairs_f3, below): operand types, the
// feature count of its accumulation, and its exponent error bound: |dz| <=
// kF3Kappa (1 + alpha_m) (|u| + |v|)^2 (3 products of BF16 halves, each off
// by 2^-16 of its size, plus FP32 sums of 32 terms), admitted while it is at
// most kF3MaxDz for pairs within scaled distance 2 of a source half
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kF3Feat = 16;  // features 0 (the constant 1), 1..10, 11..15 zero
constexpr double kF3Kappa = 3.0 / 65536.0 + 64.0 / 16777216.0;
constexpr double kF3MaxDz = 1.0 / 32.0;

// Block order of one problem's work items: block i runs on XCD i mod 8
// (blocks are handed to the XCDs in turn), so each XCD gets a contiguous run
// of items -- neighbouring source groups, whose target tiles its own L2 then
// holds.  When every group has the same number c of items (no tile dropped,
// as in the dense first E steps, where each group streams all target
// records), the run is further taken chunk-major: segments of S groups (S c
// about one XCD's run), and within a segment every group's first item, then
// every group's second, ..., so that the blocks resident on an XCD at one
// time read the same target tiles.  A bijection on the item numbers: only the
// order of execution changes, not any sum.
__host__ __device__ __forceinline__ int item_order(int i, int nitems, int c) {
  const int x = i % 8, q = nitems / 8, r = nitems % 8;
  int t = x * q + (x < r ? x : r) + i / 8;
  if (c > 1) {
    const int ng = nitems / c;
    int S = q / c;
    S = S < 1 ? 1 : S;
    const int seg = t / (S * c), g0 = seg * S;
    const int Ss = ng - g0 < S ? ng - g0 : S;
    const int k = t - seg * S * c;
    t = (g0 + k % Ss) * c + k / Ss;
  }
  return t;
}

// Whether the BF16 matrix-core kernel takes a work item (group box gbox, its
// tiles tl[0 .. kn) among the problem's tile boxes bx): its exponent error
// bound must hold for every pair within scaled distance 2 of either half of
// the group, kF3Kappa (1 + A) (2 h + 2)^2 <= kF3MaxDz, with h the larger
// scaled half-diagonal of the two halves' boxes and A the largest alpha of
// the item's tiles (the `pad` of their boxes).  Evaluated per wave; both pair
// kernels take the same decision from the same data.
__device__ bool item_is_f3(const double *gbox, const TBox *bx, const int *tl, int kn) {
  double h = 0.0;
  for (int half = 0; half < 2; ++half) {
    const double *hb = gbox + 6 * half;
    if (hb[0] <= hb[3]) {  // a half without sources has an empty box
      const double e0 = hb[3] - hb[0], e1 = hb[4] - hb[1], e2 = hb[5] - hb[2];
      h = fmax(h, 0.5 * sqrt(e0 * e0 + e1 * e1 + e2 * e2));
    }
  }
  double a = 0.0;
  for (int q = threadIdx.x & 63; q < kn; q += 64) a = fmax(a, bx[tl[q]].pad);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, 64));
  const double r = 2.0 * h + 2.0;
  return kF3Kappa * (1.0 + a) * r * r <= kF3MaxDz;
}

// Scaled-coordinate bounding box of each source group (kept for the pair
// kernel), then the live tiles in increasing order.  One block per group of
// every problem of the batch.
__global__ __launch_bounds__(kBlock) void cull_groups(int single, const Slot *__restrict__ slots,
                                                      const int *__restrict__ grp_slot,
                                                      const DevState *__restrict__ states,
                                                      const TBox *__restrict__ boxes,
                                                      int *__restrict__ counts,
                                                      double *__restrict__ gbox,
                                                      int *__restrict__ list) {
  const int b = blockIdx.x;
  const int p = single ? 0 : grp_slot[b];  // one problem: no table lookup
  const DevState *st = states + p;
  // the slot and sigma^2 load with the done flag: every load here is issued
  // before any arithmetic on its value
  const Slot &sl = slots[p];
  const int done = st->done;
  const int g_off = sl.g_off, N = sl.N, ntiles = sl.ntiles, t_off = sl.t_off;
  const float *X = sl.X;
  const int64_t list_off = sl.list_off;
  const double s2 = st->sigma2;
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::"s"(done), "s"(g_off), "s"(N), "s"(ntiles), "s"(t_off), "s"(X),
               "s"(list_off), "s"(s2));
  if (done) return;
  const int g = b - g_off;
  const int n = g * kGroup + threadIdx.x;
  const bool mine = threadIdx.x < kGroup && n < N;
  // the source (index clamped to the cloud, N >= 1) and the pose, together
  const int nc = n < N ? n : N - 1;
  const float fx = X[3 * nc], fy = X[3 * nc + 1], fz = X[3 * nc + 2];
  const TBox *bx_t = boxes + t_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt(kLog2e / (2.0 * s2));  // sqrt_c_of
  const double x0 = fx, x1 = fy, x2 = fz;
  const double c0 = sc * fma(R[0], x0, fma(R[1], x1, fma(R[2], x2, t[0])));
  const double c1 = sc * fma(R[3], x0, fma(R[4], x1, fma(R[5], x2, t[1])));
  const double c2 = sc * fma(R[6], x0, fma(R[7], x1, fma(R[8], x2, t[2])));
  double lo[3] = {mine ? c0 : INFINITY, mine ? c1 : INFINITY, mine ? c2 : INFINITY};
  double hi[3] = {mine ? c0 : -INFINITY, mine ? c1 : -INFINITY, mine ? c2 : -INFINITY};
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, 64));
    }
  __shared__ double bx[4][6];
  __shared__ int wc[4];
  if (lane == 0)
    for (int a = 0; a < 3; ++a) {
      bx[wave][a] = lo[a];
      bx[wave][3 + a] = hi[a];
    }
  __syncthreads();
  // waves 0 and 1 hold the two halves (waves 2 and 3 hold no sources); a
  // half without sources has an empty box, which no tile or target passes
  double lo0[3], hi0[3], lo1[3], hi1[3];
  for (int a = 0; a < 3; ++a) {
    lo0[a] = bx[0][a];
    hi0[a] = bx[0][3 + a];
    lo1[a] = bx[1][a];
    hi1[a] = bx[1][3 + a];
  }
  if (threadIdx.x < 12) {
    const int h = threadIdx.x / 6, c = threadIdx.x % 6;
    gbox[(int64_t)b * kGBox + threadIdx.x] = bx[h][c];
  }
  int *out = list + list_off + (int64_t)g * ntiles;
  int base = 0;
  for (int t0 = 0; t0 < ntiles; t0 += kBlock) {
    const int ti = t0 + threadIdx.x;
    const bool live = ti < ntiles && (box_live(bx_t[ti].lo, bx_t[ti].hi, bx_t[ti].lmax, lo0, hi0, sc) ||
                                      box_live(bx_t[ti].lo, bx_t[ti].hi, bx_t[ti].lmax, lo1, hi1, sc));
    const uint64_t bal = __ballot(live);
    if (lane == 0) wc[wave] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wave; ++w) off += wc[w];
    if (live) out[off + __popcll(bal & ((1ull << lane) - 1ull))] = ti;
    base += wc[0] + wc[1] + wc[2] + wc[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[b] = base;
}

// Items of one problem (one block per problem): L tiles each (a multiple of
// 4, or any L >= 1 when the items are split), about `target` in all.  Without
// culling every group lists all tiles.  Also clears the problem's counters of
// evaluated pairs (evcounts[p], and evcounts[npairs + p] for the BF16
// matrix-core kernel).  Offsets: group g of problem p has its items at
// off[g_off + p + g] .. off[g_off + p + g + 1] - 1 (local to the problem's item
// range); item i of the problem is items[item_off + i].
template <bool CULL>
__global__ __launch_bounds__(kBlock) void cull_items(const Slot *__restrict__ slots,
                                                     const DevState *__restrict__ states,
                                                     const int *__restrict__ counts,
                                                     CullHdr *__restrict__ hdrs,
                                                     int *__restrict__ offs,
                                                     Item *__restrict__ items,
                                                     unsigned long long *__restrict__ evcounts) {
  const int p = blockIdx.x, npairs = gridDim.x;
  // the slot loads with the done flag
  const Slot &sl = slots[p];
  const int done = states[p].done;
  const int ngroups = sl.ngroups, ntiles = sl.ntiles, target = sl.target, cap = sl.item_cap,
            g_off = sl.g_off, item_off = sl.item_off, M = sl.M;
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::"s"(done), "s"(ngroups), "s"(ntiles), "s"(target), "s"(cap), "s"(g_off),
               "s"(item_off), "s"(M));
  if (done) return;
  const int *cnts = CULL ? counts + g_off : nullptr;
  int *off = offs + g_off + p;
  Item *its = items + item_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ int64_t red[4];
  __shared__ int wsum[4];
  int64_t tiles = 0;
  if (CULL) {
    for (int g0 = 0; g0 < ngroups; g0 += 4 * kBlock) {  // 4 loads in flight
      int c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = g0 + u * kBlock + (int)threadIdx.x;
        c[u] = g < ngroups ? cnts[g] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) tiles += c[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tiles += __shfl_xor(tiles, o, 64);
    if (lane == 0) red[wave] = tiles;
    __syncthreads();
    tiles = red[0] + red[1] + red[2] + red[3];
  } else {
    tiles = (int64_t)ngroups * ntiles;
  }
  // Each wave takes every 4th tile of its item (L a multiple of 4 keeps the
  // waves even), or, in a split item, the block's 4 waves share each tile
  // target by target (wave w takes targets w, w + 4, ...).  Split, for a
  // single problem: when its records outgrow an XCD's 4 MB L2 (the waves of
  // a block then stream one tile instead of four), and where items of 4
  // tiles would leave fewer than 512 blocks (two per CU).
  int64_t L = (tiles + target - 1) / target;
  const bool big = npairs == 1 && (int64_t)M * (int64_t)sizeof(TRec) > ((int64_t)4 << 20);
  const bool few = npairs == 1 && (tiles + 3) / 4 < 512 && L <= 2;
  const bool split = big || few;
  L = split ? (L < 1 ? 1 : L) : L < 4 ? 4 : (L + 3) / 4 * 4;
  const int Li = (int)L;
  int run = 0;
  int vmin = 0x7fffffff, vmax = 0;  // items per group
  for (int g0 = 0; g0 < ngroups; g0 += kBlock) {
    const int g = g0 + threadIdx.x;
    const int cnt = g < ngroups ? (CULL ? cnts[g] : ntiles) : 0;
    const int v = (cnt + Li - 1) / Li;
    if (g < ngroups) {
      vmin = v < vmin ? v : vmin;
      vmax = v > vmax ? v : vmax;
    }
    // exclusive prefix of v over the block: within the wave by shuffles,
    // then the totals of the waves before
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      incl += lane >= d ? y : 0;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int first = run + incl - v;
    for (int w = 0; w < wave; ++w) first += wsum[w];
    if (g < ngroups) {
      off[g] = first;
      for (int k = 0; k < v && first + k < cap; ++k) {
        const int k0 = k * Li;
        its[first + k] = Item{g, k0, cnt - k0 < Li ? cnt - k0 : Li, CULL && cnt == ntiles};
      }
    }
    run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int a = __shfl_xor(vmin, o, 64), b = __shfl_xor(vmax, o, 64);
    vmin = a < vmin ? a : vmin;
    vmax = b > vmax ? b : vmax;
  }
  __shared__ int mm[2][4];
  if (lane == 0) {
    mm[0][wave] = vmin;
    mm[1][wave] = vmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      vmin = mm[0][w] < vmin ? mm[0][w] : vmin;
      vmax = mm[1][w] > vmax ? mm[1][w] : vmax;
    }
    off[ngroups] = run;
    hdrs[p].items = run < cap ? run : cap;
    hdrs[p].tiles_per_item = Li;
    hdrs[p].uniform = vmin == vmax && run <= cap ? vmax : 0;
    hdrs[p].split = split ? 1 : 0;
    evcounts[p] = 0ull;           // pairs evaluated
    evcounts[npairs + p] = 0ull;  // of which by the BF16 matrix-core kernel
  }
}

// A lane's target of a tile: position, log-prior and plane vector (zeros
// past the end of the cloud).
struct TIn {
  double y[3], l, a[3];
};

__device__ __forceinline__ TIn load_tin(const TPt *pts, const TRec *rec, int ti, int Mi) {
  const int m = ti * kCullTile + (int)(threadIdx.x & 63);
  TIn t = {};
  if (m < Mi) {
    const TPt &p = pts[m];
    for (int a = 0; a < 3; ++a) {
      t.y[a] = p.y[a];
      t.a[a] = rec[m].a[a];
    }
    t.l = p.l;
  }
  return t;
}

// Lane j < n1 (its target's values in q) stages target j of a tile:
// T = [2 v, l - |v|^2, -a . v] with v = sqrt(c) y - o.  Made visible to the
// rest of the wave before return.
__device__ __forceinline__ void stage_tile(double (*T)[kRelT], const TIn &q, int n1, double sc,
                                           const double (&o)[3]) {
  const int lane = threadIdx.x & 63;
  // the walk over the previous tile's rows is done before they are replaced
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < n1) {
    const double v0 = fma(sc, q.y[0], -o[0]), v1 = fma(sc, q.y[1], -o[1]),
                 v2 = fma(sc, q.y[2], -o[2]);
    T[lane][0] = 2.0 * v0;
    T[lane][1] = 2.0 * v1;
    T[lane][2] = 2.0 * v2;
    T[lane][3] = fma(-v0, v0, fma(-v1, v1, fma(-v2, v2, q.l)));
    T[lane][4] = -fma(q.a[0], v0, fma(q.a[1], v1, q.a[2] * v2));
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool CULL>
// 5 waves per SIMD (at most 96 VGPRs; the LDS holds 5 blocks per CU) hide
// the scalar-load and FP64 latencies
__global__ __launch_bounds__(kBlock, 5) void estep_pairs_items(
    int single, const Slot *__restrict__ slots, const int *__restrict__ item_slot,
    const DevState *__restrict__ states, const CullHdr *__restrict__ hdrs,
    const Item *__restrict__ items, const TRec *__restrict__ recs,
    const TPt *__restrict__ ptss, const int *__restrict__ list,
    const double *__restrict__ gboxes, const TBox *__restrict__ boxes, int f3,
    unsigned long long *__restrict__ evcounts, double *__restrict__ partial) {
  constexpr int S = kSrcPerLane;
  // one problem (single): p = 0 without a table lookup, and the blocks take
  // the items in XCD order.  The done flag, the slot and the plan header are
  // independent loads; the exit test needs all three.  (The arguments the
  // first loads need come first, where the dispatch can preload them.)
  const int p = single ? 0 : item_slot[blockIdx.x];
  const DevState *st = states + p;
  const Slot &sl = slots[p];
  const int stopped = st->done;
  const CullHdr hd = load_hdr(hdrs, p);
  const int item_off = sl.item_off, N = sl.N, ntiles = sl.ntiles, g_off = sl.g_off,
            t_off = sl.t_off;
  const int64_t M = sl.M, y_off = sl.y_off, list_off = sl.list_off;
  // every load above is issued before any arithmetic on its value (see ready_s)
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::"s"(stopped), "s"(item_off), "s"(hd.items), "s"(hd.uniform),
               "s"(hd.split), "s"(N), "s"(ntiles), "s"(g_off), "s"(t_off), "s"(M), "s"(y_off),
               "s"(list_off));
  int item = blockIdx.x - item_off;
  const float *X = sl.X;
  const TRec *rec = recs + y_off + p;  // the problem's records, sentinel at rec[M]
  const TPt *pts = ptss + y_off;
  if ((stopped != 0) | (item >= hd.items)) return;
  if (single) item = item_order(item, hd.items, hd.uniform);
  const Item wi = items[item_off + item];
  const int b = item_off + item;
  // the wave index is wave-uniform; readfirstlane tells the compiler so, which
  // keeps the tile loop (and so the record loads) scalar
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wi.g, k0 = wi.k0, kn = wi.kn;
  const int *tl = list + list_off + (int64_t)g * ntiles + k0;
  const double *gbox = gboxes + (int64_t)(g_off + g) * kGBox;
  const bool split = hd.split != 0;
  const int nt = split ? kn : kn > wave ? (kn - wave + 3) / 4 : 0;
  // Everything the item needs next loads in one round trip: the lane's
  // sources (index clamped to the cloud), the group's two half boxes, the
  // pose and the first 64 of the wave's tiles; the scalar values are made
  // ready before the BF16 kernel's exit test.
  float xf[S][3];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int n = g * kGroup + s * 64 + lane, k = n < N ? n : N - 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) xf[s][c] = X[3 * k + c];
  }
  double gb[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) gb[k] = CULL ? gbox[k] : 0.0;
  double R[9], t[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double s2 = st->sigma2;
  int tv = 0;  // tile indices of the wave, 64 at a time, one per lane
  if (CULL) {
    const int jl = split ? lane : wave + 4 * lane;
    tv = jl < kn ? tl[jl] : 0;
  }
  asm volatile("" ::"s"(gb[0]), "s"(gb[1]), "s"(gb[2]), "s"(gb[3]), "s"(gb[4]), "s"(gb[5]),
               "s"(gb[6]), "s"(gb[7]), "s"(gb[8]), "s"(gb[9]), "s"(gb[10]), "s"(gb[11]));
  asm volatile("" ::"s"(R[0]), "s"(R[1]), "s"(R[2]), "s"(R[3]), "s"(R[4]), "s"(R[5]), "s"(R[6]),
               "s"(R[7]), "s"(R[8]), "s"(t[0]), "s"(t[1]), "s"(t[2]), "s"(s2));
  // an item the BF16 matrix-core kernel takes
  if (CULL && f3 && item_is_f3(gbox, boxes + t_off, tl, kn)) return;
  const double sc = sqrt(kLog2e / (2.0 * s2));  // sqrt_c_of
  Src x[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int n = g * kGroup + s * 64 + lane;
    const double x0 = n < N ? (double)xf[s][0] : 0.0, x1 = n < N ? (double)xf[s][1] : 0.0,
                 x2 = n < N ? (double)xf[s][2] : 0.0;
    x[s].x0 = sc * fma(R[0], x0, fma(R[1], x1, fma(R[2], x2, t[0])));
    x[s].x1 = sc * fma(R[3], x0, fma(R[4], x1, fma(R[5], x2, t[1])));
    x[s].x2 = sc * fma(R[6], x0, fma(R[7], x1, fma(R[8], x2, t[2])));
  }
  // the centre: that of the group's box (culled), else the group's first
  // source (any point of the group bounds |u| by the group's extent)
  double o[3];
  if constexpr (CULL) {
    const bool two = gb[6] <= gb[9];  // an empty half has an empty box
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double lo = two ? fmin(gb[a], gb[6 + a]) : gb[a];
      const double hi = two ? fmax(gb[3 + a], gb[9 + a]) : gb[3 + a];
      o[a] = 0.5 * (lo + hi);
    }
  } else {
    o[0] = __shfl(x[0].x0, 0, 64);
    o[1] = __shfl(x[0].x1, 0, 64);
    o[2] = __shfl(x[0].x2, 0, 64);
  }
  SrcRel xr[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    xr[s].u0 = x[s].x0 - o[0];
    xr[s].u1 = x[s].x1 - o[1];
    xr[s].u2 = x[s].x2 - o[2];
    xr[s].uu = fma(xr[s].u0, xr[s].u0, fma(xr[s].u1, xr[s].u1, xr[s].u2 * xr[s].u2));
  }
  // the current tile's target terms, one row of kRelT per target (wave-private)
  __shared__ __align__(16) double trel[4][kCullTile][kRelT];
  double acc[S][kFeatUsed];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) acc[s][c] = 0.0;
  const bool full = CULL && wi.full != 0;
  const bool two1 = gb[6] <= gb[9];  // the group's second half holds sources
  double blo0[3], bhi0[3], blo1[3], bhi1[3];
  if constexpr (CULL)
    for (int a = 0; a < 3; ++a) {
      blo0[a] = gb[a];
      bhi0[a] = gb[3 + a];
      blo1[a] = gb[6 + a];
      bhi1[a] = gb[9 + a];
    }
  const int Mi = (int)M;  // M < 2^27: 32-bit scalar loop arithmetic
  // the wave's tiles are j = wave, wave + 4, ... (split items: every tile,
  // and of its targets those with index = wave mod 4); their indices are
  // fetched 64 at a time, one per lane, and read back with readlane
  const uint64_t sel = split ? 0x1111111111111111ull << wave : ~0ull;
  int done = 0;   // targets this wave evaluated (for every source of the group)
  int done0 = 0, done1 = 0;  // the same for each half of the group (culled)
  if constexpr (CULL) {
    for (int q = 0; q < nt; ++q) {
      if ((q & 63) == 0 && q > 0) {
        const int jl = split ? q + lane : wave + 4 * (q + lane);
        tv = jl < kn ? tl[jl] : 0;
      }
      const int ti = __builtin_amdgcn_readlane(tv, q & 63);
      const int n1 = Mi - ti * kCullTile < kCullTile ? Mi - ti * kCullTile : kCullTile;
      // the tile's targets that the boxes of the group's two halves cannot
      // rule out: one lane per target tests it against both, and the two
      // ballots are (wave-uniform) masks; each half of the lanes' sources
      // takes only its own targets
      const TIn cur = load_tin(pts, rec, ti, Mi);
      bool on0 = false, on1 = false;
      if (lane < n1) {
        if (full) {  // every target (half 1 only if it holds sources)
          on0 = true;
          on1 = two1;
        } else {
          on0 = box_live(cur.y, cur.y, cur.l, blo0, bhi0, sc);
          on1 = box_live(cur.y, cur.y, cur.l, blo1, bhi1, sc);
        }
      }
      const uint64_t m0 = __ballot(on0) & sel, m1 = __ballot(on1) & sel;
      done0 += __popcll(m0);
      done1 += __popcll(m1);
      if ((m0 | m1) == 0) continue;
      const TRec *tr = rec + (int64_t)ti * kCullTile;
      stage_tile(trel[wave], cur, n1, sc, o);
      // targets live for both halves go through the interleaved two-source
      // path (its independent chains keep the FP64 pipeline full), the others
      // through one source each
      for (uint64_t mk = m0 & m1; mk; mk &= mk - 1) {
        const int j = __builtin_ctzll(mk);
        accumulate_rel<S>(xr, trel[wave][j], tr[j], acc);
      }
      for (uint64_t mk = m0 & ~m1; mk; mk &= mk - 1) {
        const int j = __builtin_ctzll(mk);
        accumulate1_rel(xr[0], trel[wave][j], tr[j], acc[0]);
      }
      for (uint64_t mk = m1 & ~m0; mk; mk &= mk - 1) {
        const int j = __builtin_ctzll(mk);
        accumulate1_rel(xr[1], trel[wave][j], tr[j], acc[1]);
      }
    }
  } else {
    for (int q = 0; q < nt; ++q) {
      if ((q & 63) == 0) tv = split ? k0 + q + lane : k0 + wave + 4 * (q + lane);
      const int ti = __builtin_amdgcn_readlane(tv, q & 63);
      const TRec *tr = rec + (int64_t)ti * kCullTile;
      const int n1 = Mi - ti * kCullTile < kCullTile ? Mi - ti * kCullTile : kCullTile;
      // targets m0, m0 + dm, ... of the tile; a do-while keeps one set of
      // accumulators
      const int m0 = split ? wave : 0, dm = split ? 4 : 1;
      if (m0 < n1) {
        stage_tile(trel[wave], load_tin(pts, rec, ti, Mi), n1, sc, o);
        done += (n1 - m0 + dm - 1) / dm;
        int m = m0;
        do {
          accumulate_rel<S>(xr, trel[wave][m], tr[m], acc);
        } while ((m += dm) < n1);
      }
    }
  }
  __shared__ int wdone[3][4];
  if (lane == 0) {
    wdone[0][wave] = done;
    wdone[1][wave] = done0;
    wdone[2][wave] = done1;
  }
  __shared__ double red[3][kFeatUsed][64];
  double *dst = partial + (size_t)b * kFeatUsed * kGroup;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (wave > 0)
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c) red[wave - 1][c][lane] = acc[s][c];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c)
        dst[c * kGroup + s * 64 + lane] =
            ((acc[s][c] + red[0][c][lane]) + red[1][c][lane]) + red[2][c][lane];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int rest = N - g * kGroup;  // sources of the group: halves of nv0 and nv1
    const unsigned long long nv = (unsigned long long)(rest < kGroup ? rest : kGroup);
    const unsigned long long nv0 = (unsigned long long)(rest < 64 ? rest : 64);
    const unsigned long long nv1 = (unsigned long long)(rest <= 64 ? 0 : rest < kGroup ? rest - 64 : 64);
    const unsigned long long ev =
        CULL ? nv0 * (unsigned long long)(wdone[1][0] + wdone[1][1] + wdone[1][2] + wdone[1][3]) +
                   nv1 * (unsigned long long)(wdone[2][0] + wdone[2][1] + wdone[2][2] + wdone[2][3])
             : nv * (unsigned long long)(wdone[0][0] + wdone[0][1] + wdone[0][2] + wdone[0][3]);
    atomicAdd(evcounts + p, ev);
  }
}

// ------------------------------------------- pair kernel (BF16 matrix cores)
// The exponent as a bilinear form of lifted features (Sec. 3.4, Eq. 10: the
// paper's own recast of the Mahalanobis term is this product).  With every
// coordinate scaled by sqrt(c) and taken relative to a centre o,
// u = s_n - o, v = sqrt(c) y_m - o and M_m = I + a_m a_m^T,
//   c d_mn = (u - v)^T M_m (u - v) = Phi_m . Psi_n,
//   Psi_n = [u0^2, u1^2, u2^2, 2u0u1, 2u0u2, 2u1u2, u0, u1, u2, 1],
//   Phi_m = [M00, M11, M22, M01, M02, M12, -2 M v, v^T M v],
// a K = 10 contraction.  Each value is split into BF16 high and low parts
// (v = hi + lo + O(2^-16 v)) and the K = 32 product
//   [Phi_hi, Phi_hi, Phi_lo, 0, 0] . [Psi_hi, Psi_lo, Psi_hi, 0, 0]
// runs as one V_MFMA_F32_16X16X32_BF16 per 16 targets x 16 sources, FP32
// accumulation; the exponential is float32 on the vector unit; the
// accumulation T_n += e_mn [1, f_m] is a second contraction over the targets,
//   [e_hi, e_hi, e_lo] x [F_hi, F_lo, F_hi]  (3 MFMAs per 32 targets),
// whose FP32 sums are moved into FP64 every second tile.
// Error: each product carries about 3 * 2^-16 of its own size, and the
// terms cancel for nearby pairs, so |dz| <= kF3Kappa (1 + alpha_m)
// (|u| + |v|)^2 up to the FP32 sums; the centre is the box centre of the
// wave's 64 sources (|u| <= h, its scaled half-diagonal).  A work item runs
// here (item_is_f3) only if kF3Kappa (1 + alpha_max) (2 h + 2)^2 <= kF3MaxDz
// for both source halves of its group and the largest alpha of its tiles,
// i.e. the bound holds for every pair within scaled distance 2 (e at least
// 2^-4 of its largest possible value) -- the early, large-sigma^2
// iterations; the FP64 kernel takes the other items.  Same items, partial
// layout and finalisation as the FP64 kernel; not a parity path (errors
// ~1e-4 in z).

__device__ __forceinline__ void split_bf16(double v, __bf16 &hi, __bf16 &lo) {
  const float f = (float)v;
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}

// Accumulation features of tile t (targets t*64 ..), BF16 high/low parts in
// the order the MFMA B operand reads them: [t][hi, lo][feature][target];
// and the tile's largest alpha (= |a_m|^2) in box[t].pad.  One wave per tile.
__global__ void f3_tables(const TRec *__restrict__ rec, int64_t M, __bf16 *__restrict__ ftab,
                          TBox *__restrict__ box) {
  const int64_t t = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t ntiles = (M + kCullTile - 1) / kCullTile;
  if (t >= ntiles) return;  // wave-uniform
  const int64_t m = t * kCullTile + lane;
  const bool valid = m < M;
  double f[kF3Feat];
  double a2 = 0.0;
#pragma unroll
  for (int c = 0; c < kF3Feat; ++c) f[c] = 0.0;
  if (valid) {
    const TRec &r = rec[m];
    f[0] = 1.0;
#pragma unroll
    for (int c = 0; c < 10; ++c) f[1 + c] = r.f[c];
    a2 = r.a[0] * r.a[0] + r.a[1] * r.a[1] + r.a[2] * r.a[2];
  }
  __bf16 *o = ftab + t * (2 * kF3Feat * kCullTile);
#pragma unroll
  for (int c = 0; c < kF3Feat; ++c) {
    __bf16 hi, lo;
    split_bf16(f[c], hi, lo);
    o[c * kCullTile + lane] = hi;
    o[(kF3Feat + c) * kCullTile + lane] = lo;
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) a2 = fmax(a2, __shfl_xor(a2, s, 64));
  if (lane == 0) box[t].pad = a2;
}

// Picks entries 8 q .. 8 q + 7 of a 32-vector held in registers (q = lane / 16).
__device__ __forceinline__ bf16x8 pick8(const __bf16 (&v)[32], int q) {
  bf16x8 o;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    o[j] = q == 0 ? v[j] : q == 1 ? v[8 + j] : q == 2 ? v[16 + j] : v[24 + j];
  return o;
}

// The K = 32 operand of a lifted 10-vector w: [hi, hi, lo] (targets, `first`)
// or [hi, lo, hi] (sources), zero-padded.
__device__ __forceinline__ void lifted32(const double (&w)[10], bool target, __bf16 (&v)[32]) {
  __bf16 hi[10], lo[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) split_bf16(w[k], hi[k], lo[k]);
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    v[k] = hi[k];
    v[10 + k] = target ? hi[k] : lo[k];
    v[20 + k] = target ? lo[k] : hi[k];
  }
  v[30] = v[31] = (__bf16)0.0f;
}

// One block of 4 waves per work item (the FP64 kernel's items).  Wave w takes
// the 64 sources of half w & 1 of the group (4 blocks of 16, lanes l & 15) and
// every second tile of the item (starting at w >> 1); the two waves of a half
// add their sums through LDS in a fixed order.
__global__ __launch_bounds__(kBlock, 2) void estep_pairs_f3(
    int single, const Slot *__restrict__ slots, const int *__restrict__ item_slot,
    const DevState *__restrict__ states, const CullHdr *__restrict__ hdrs,
    const Item *__restrict__ items, const TRec *__restrict__ recs,
    const __bf16 *__restrict__ ftabs, const int *__restrict__ list,
    const double *__restrict__ gboxes, const TBox *__restrict__ boxes,
    unsigned long long *__restrict__ evcounts, unsigned long long *__restrict__ f3counts,
    double *__restrict__ partial) {
  // the same item as the FP64 kernel's block of this index
  const int p = single ? 0 : item_slot[blockIdx.x];
  const DevState *st = states + p;
  const Slot &sl = slots[p];
  const CullHdr hd = load_hdr(hdrs, p);
  const int stopped = st->done;
  int item = blockIdx.x - sl.item_off;
  ready_s(hd.uniform);
  ready_s(hd.split);
  if ((stopped != 0) | (item >= hd.items)) return;
  if (single) item = item_order(item, hd.items, hd.uniform);
  const Item wi = items[sl.item_off + item];
  const int b = sl.item_off + item;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = wave & 1, par = wave >> 1;
  const int lq = lane >> 4, lc = lane & 15;
  const int N = sl.N, ntiles = sl.ntiles, Mi = sl.M;
  const TRec *rec = recs + sl.y_off + p;
  const __bf16 *ftab = ftabs + (int64_t)sl.t_off * (2 * kF3Feat * kCullTile);
  const int g = wi.g, k0 = wi.k0, kn = wi.kn;
  const int *tl = list + sl.list_off + (int64_t)g * ntiles + k0;
  if (!item_is_f3(gboxes + (int64_t)(sl.g_off + g) * kGBox, boxes + sl.t_off, tl, kn)) return;
  const double *hb = gboxes + (int64_t)(sl.g_off + g) * kGBox + 6 * half;
  const int rest = N - g * kGroup - half * 64;
  const int nv = rest < 0 ? 0 : rest < 64 ? rest : 64;  // sources of this half
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  double o[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = nv > 0 ? 0.5 * (hb[a] + hb[3 + a]) : 0.0;
  // B operands of the exponent: Psi of the lane's 4 sources
  bf16x8 psi[4];
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int j = 16 * sb + lc;
    const int n = g * kGroup + half * 64 + j;
    double w[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) w[k] = 0.0;
    if (j < nv) {
      const Src x = load_src(sl.X, n, N, R, t, sc);
      const double u0 = x.x0 - o[0], u1 = x.x1 - o[1], u2 = x.x2 - o[2];
      w[0] = u0 * u0;
      w[1] = u1 * u1;
      w[2] = u2 * u2;
      w[3] = 2.0 * u0 * u1;
      w[4] = 2.0 * u0 * u2;
      w[5] = 2.0 * u1 * u2;
      w[6] = u0;
      w[7] = u1;
      w[8] = u2;
      w[9] = 1.0;
    }
    __bf16 v[32];
    lifted32(w, false, v);
    psi[sb] = pick8(v, lq);
  }
  __shared__ bf16x8 phis[4][kCullTile][4];  // per wave: each target's 32-vector
  __shared__ float ls[4][kCullTile];
  f32x4 acc[4];
  double tot[4][4];
#pragma unroll
  for (int sb = 0; sb < 4; ++sb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[sb][i] = 0.0f;
      tot[sb][i] = 0.0;
    }
  int done = 0;  // targets evaluated (against each of the nv sources)
  int since = 0;
  for (int q = par; nv > 0 && q < kn; q += 2) {
    const int ti = tl[q];
    const int base = ti * kCullTile;
    const int n1 = Mi - base < kCullTile ? Mi - base : kCullTile;
    done += n1;
    {  // A operands of the exponent: Phi of the tile's targets (lane = target)
      double w[10];
      float l = -INFINITY;
#pragma unroll
      for (int k = 0; k < 10; ++k) w[k] = 0.0;
      if (lane < n1) {
        const TRec &r = rec[base + lane];
        const double v0 = fma(sc, r.y[0], -o[0]), v1 = fma(sc, r.y[1], -o[1]),
                     v2 = fma(sc, r.y[2], -o[2]);
        const double av = r.a[0] * v0 + r.a[1] * v1 + r.a[2] * v2;
        const double m0 = fma(r.a[0], av, v0), m1 = fma(r.a[1], av, v1), m2 = fma(r.a[2], av, v2);
        w[0] = fma(r.a[0], r.a[0], 1.0);
        w[1] = fma(r.a[1], r.a[1], 1.0);
        w[2] = fma(r.a[2], r.a[2], 1.0);
        w[3] = r.a[0] * r.a[1];
        w[4] = r.a[0] * r.a[2];
        w[5] = r.a[1] * r.a[2];
        w[6] = -2.0 * m0;
        w[7] = -2.0 * m1;
        w[8] = -2.0 * m2;
        w[9] = v0 * m0 + v1 * m1 + v2 * m2;
        l = (float)r.l;
      }
      __bf16 v[32];
      lifted32(w, true, v);
#pragma unroll
      for (int k = 0; k < 4; ++k) phis[wave][lane][k] = pick8(v, k);
      ls[wave][lane] = l;
    }
    __builtin_amdgcn_wave_barrier();
    const __bf16 *ft = ftab + (int64_t)ti * (2 * kF3Feat * kCullTile);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      // B operands of the accumulation: features lc of targets
      // 32 kc + 4 lq + (0..3) and 32 kc + 16 + 4 lq + (0..3), high and low
      bf16x8 fh, fl;
      {
        const __bf16 *ph = ft + lc * kCullTile + 32 * kc + 4 * lq;
        const __bf16 *pl = ph + kF3Feat * kCullTile;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          fh[j] = ph[j];
          fh[4 + j] = ph[16 + j];
          fl[j] = pl[j];
          fl[4 + j] = pl[16 + j];
        }
      }
      const bf16x8 a0 = phis[wave][32 * kc + lc][lq];
      const bf16x8 a1 = phis[wave][32 * kc + 16 + lc][lq];
      float lr[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        lr[i] = ls[wave][32 * kc + 4 * lq + i];
        lr[4 + i] = ls[wave][32 * kc + 16 + 4 * lq + i];
      }
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
        const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, psi[sb], zero, 0, 0, 0);
        const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, psi[sb], zero, 0, 0, 0);
        bf16x8 eh, el;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float e = __builtin_amdgcn_exp2f(lr[i] - (i < 4 ? d0[i] : d1[i - 4]));
          const __bf16 h = (__bf16)e;
          eh[i] = h;
          el[i] = (__bf16)(e - (float)h);
        }
        acc[sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh, fh, acc[sb], 0, 0, 0);
        acc[sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh, fl, acc[sb], 0, 0, 0);
        acc[sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(el, fh, acc[sb], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (++since == 2) {  // FP32 sums of at most 128 targets, then FP64
      since = 0;
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          tot[sb][i] += (double)acc[sb][i];
          acc[sb][i] = 0.0f;
        }
    }
  }
#pragma unroll
  for (int sb = 0; sb < 4; ++sb)
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[sb][i] += (double)acc[sb][i];
  // lane (lq, lc) holds T[source 16 sb + 4 lq + i of the half][feature lc]
  __shared__ double red[2][4][4][64];
  if (par == 1)
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[half][sb][i][lane] = tot[sb][i];
  __syncthreads();
  if (par == 0 && lc < kFeatUsed) {
    double *dst = partial + (size_t)b * kFeatUsed * kGroup + (size_t)lc * kGroup + half * 64;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[16 * sb + 4 * lq + i] = tot[sb][i] + red[half][sb][i][lane];
  }
  if (lane == 0 && nv > 0 && done > 0) {
    atomicAdd(evcounts + p, (unsigned long long)nv * (unsigned long long)done);
    atomicAdd(f3counts + p, (unsigned long long)nv * (unsigned long long)done);
  }
}

// LDS back end: the block stages tiles of target records in LDS and every
// wave reads them back with broadcast loads; a block owns 256*S sources.
template <int S>
__global__ __launch_bounds__(kBlock) void estep_pairs_lds(const float *__restrict__ X, int N,
                                                          const TRec *__restrict__ rec, int64_t M,
                                                          const DevState *__restrict__ st,
                                                          int64_t mchunk, int nsplit,
                                                          double *__restrict__ partial) {
  if (st->done) return;
  const int split = blockIdx.x % nsplit;
  const int sb = blockIdx.x / nsplit;
  const int64_t m0 = (int64_t)split * mchunk;
  const int64_t m1 = m0 + mchunk < M ? m0 + mchunk : M;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  const double negsc = -sc;
  Src x[S];
  int nidx[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    nidx[s] = sb * kBlock * S + s * kBlock + threadIdx.x;
    x[s] = load_src(X, nidx[s], N, R, t, sc);
  }
  double acc[S][kFeatUsed];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < kFeatUsed; ++c) acc[s][c] = 0.0;
  __shared__ TRec tile[kTile];
  for (int64_t mt = m0; mt < m1; mt += kTile) {
    const int cnt = (int)(m1 - mt < kTile ? m1 - mt : kTile);
    __syncthreads();
    const double *src = (const double *)(rec + mt);
    double *dst = (double *)tile;
    for (int i = threadIdx.x; i < cnt * kRecDoubles; i += kBlock) dst[i] = src[i];
    __syncthreads();
    for (int j = 0; j < cnt; ++j) accumulate<S>(x, tile[j], negsc, acc);
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (nidx[s] < N) {
#pragma unroll
      for (int c = 0; c < kFeatUsed; ++c)
        partial[((size_t)split * kFeatUsed + c) * N + nidx[s]] = acc[s][c];
    }
  }
}

// ------------------------------------------------------- pair kernel (MFMA)
// Wave layout: lane l, r = l % 16 (row in a 16-source group), kq = l / 16
// (target slot).  Each wave owns 64 sources (4 groups of 16).  Per step of 4
// targets, lane l computes e(source 16j + r, target 4s + kq) for j = 0..3 --
// the A operand (16 x 4) element it supplies -- and feature r of target
// 4s + kq is its B operand (4 x 16) element.
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void estep_mfma(const float *__restrict__ X, int N,
                                                    const TRec *__restrict__ rec, int64_t M,
                                                    const DevState *__restrict__ st,
                                                    int64_t mchunk, int nsplit,
                                                    double *__restrict__ partial) {
  if (st->done) return;
  const int split = blockIdx.x % nsplit;
  const int sb = blockIdx.x / nsplit;
  const int64_t m0 = (int64_t)split * mchunk;
  const int64_t m1 = m0 + mchunk < M ? m0 + mchunk : M;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15;
  const int kq = lane >> 4;
  const int wbase = sb * kBlock + wave * 64;
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  const double negsc = -sc;
  Src x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = load_src(X, wbase + 16 * j + r, N, R, t, sc);
  d4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int64_t mt = m0; mt < m1; mt += 4) {
    const int64_t m = mt + kq;
    const bool ok = m < m1;
    const TRec &tr = rec[ok ? m : m0];
    const double b = !ok ? 0.0 : (r == 0 ? 1.0 : (r < kFeatUsed ? tr.f[r - 1] : 0.0));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double a = ok ? rec_exp(x[j], tr, negsc) : 0.0;
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    }
  }
  // lane holds rows kq + 4q (q = 0..3) of each 16 x 16 block, column r
  if (r < kFeatUsed) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = wbase + 16 * j + kq + 4 * q;
        if (n < N) partial[((size_t)split * kFeatUsed + r) * N + n] = acc[j][q];
      }
  }
}

__global__ void dump_P(const float *__restrict__ X, int N, const TRec *__restrict__ rec,
                       int64_t M, const float *__restrict__ w, const DevState *__restrict__ st,
                       const double *__restrict__ colS, float *__restrict__ P) {
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = st->R[i];
  for (int i = 0; i < 3; ++i) t[i] = st->t[i];
  const double sc = sqrt_c_of(st);
  const double gam = gamma_of(st);
  const int64_t total = M * (int64_t)N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = idx / N;
    const int n = (int)(idx - m * N);
    const Src x = load_src(X, n, N, R, t, sc);
    const double e = rec_exp(x, rec[m], -sc);
    const double wn = w ? (double)w[n] : st->w0;
    const double rho = (1.0 - wn) / wn;
    P[idx] = (float)(rho * e / (rho * colS[n] + gam));
  }
}

// ----------------------------------------------------------- target records
__global__ void prep_targets(const float *__restrict__ Y, const float *__restrict__ nrm,
                             const float *__restrict__ alpha, const float *__restrict__ pi,
                             const double *__restrict__ pi_sum,
                             const uint32_t *__restrict__ perm, int64_t M, int exact,
                             TRec *__restrict__ rec, TPt *__restrict__ pts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int64_t m = perm ? (int64_t)perm[i] : i;  // record i describes target m
  const double y0 = Y[3 * m], y1 = Y[3 * m + 1], y2 = Y[3 * m + 2];
  const double n0 = nrm[3 * m], n1 = nrm[3 * m + 1], n2 = nrm[3 * m + 2];
  const double al = alpha[m];
  const double pm = !pi ? 1.0 / (double)M : pi_sum ? (double)pi[m] / *pi_sum : (double)pi[m];
  double l = log2(pm);
  if (exact) l += 0.5 * log2(1.0 + al);
  const double sa = sqrt(al);
  const double s = y0 * n0 + y1 * n1 + y2 * n2;
  TRec r;
  r.y[0] = y0;
  r.y[1] = y1;
  r.y[2] = y2;
  r.a[0] = sa * n0;
  r.a[1] = sa * n1;
  r.a[2] = sa * n2;
  r.l = l;
  r.f[0] = al * n0 * n0;
  r.f[1] = al * n0 * n1;
  r.f[2] = al * n0 * n2;
  r.f[3] = al * n1 * n1;
  r.f[4] = al * n1 * n2;
  r.f[5] = al * n2 * n2;
  r.f[6] = y0 + al * s * n0;
  r.f[7] = y1 + al * s * n1;
  r.f[8] = y2 + al * s * n2;
  r.f[9] = y0 * y0 + y1 * y1 + y2 * y2 + al * s * s;
  r.pad = 0.0;
  rec[i] = r;
  if (i == 0) {  // sentinel rec[M]: exponent -inf, no features
    TRec z = {};
    z.l = -INFINITY;
    rec[M] = z;
  }
  TPt q;
  for (int a = 0; a < 3; ++a) q.y[a] = r.y[a];
  q.l = r.l;
  pts[i] = q;
}

// Bounding box and largest log-prior of every tile of kCullTile records.
// One wave per tile, one lane per target.
__global__ void tile_boxes(const TPt *__restrict__ pts, int64_t M, TBox *__restrict__ box) {
  const int64_t t = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t ntiles = (M + kCullTile - 1) / kCullTile;
  if (t >= ntiles) return;  // wave-uniform
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double lmax = -INFINITY;
  const int64_t m = t * kCullTile + lane;
  if (lane < kCullTile && m < M) {
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = pts[m].y[a];
    lmax = pts[m].l;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, 64));
    }
    lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  }
  if (lane == 0) {
    TBox b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = lo[a];
      b.hi[a] = hi[a];
    }
    b.lmax = lmax;
    b.pad = 0.0;
    box[t] = b;
  }
}

// ---------------------------------------------------------------- moments
__global__ __launch_bounds__(256) void moments_partial(const float *__restrict__ P, int n,
                                                       const DevState *__restrict__ pose,
                                                       double *__restrict__ part) {
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0, 0, 0};
  if (pose) {
    for (int i = 0; i < 9; ++i) R[i] = pose->R[i];
    for (int i = 0; i < 3; ++i) t[i] = pose->t[i];
  }
  double v[10] = {0, 0, 0, 0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double x = P[3 * i], y = P[3 * i + 1], z = P[3 * i + 2];
    const double p0 = fma(R[0], x, fma(R[1], y, fma(R[2], z, t[0])));
    const double p1 = fma(R[3], x, fma(R[4], y, fma(R[5], z, t[1])));
    const double p2 = fma(R[6], x, fma(R[7], y, fma(R[8], z, t[2])));
    v[0] += p0;
    v[1] += p1;
    v[2] += p2;
    v[3] += p0 * p0 + p1 * p1 + p2 * p2;
    v[4] = fmin(v[4], p0);
    v[5] = fmin(v[5], p1);
    v[6] = fmin(v[6], p2);
    v[7] = fmax(v[7], p0);
    v[8] = fmax(v[8], p1);
    v[9] = fmax(v[9], p2);
  }
  __shared__ double red[4][10];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    double a = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b = __shfl_xor(a, o, 64);
      a = k < 4 ? a + b : (k < 7 ? fmin(a, b) : fmax(a, b));
    }
    if (lane == 0) red[wave][k] = a;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int k = threadIdx.x;
    double a = red[0][k];
    for (int wv = 1; wv < 4; ++wv) {
      const double b = red[wv][k];
      a = k < 4 ? a + b : (k < 7 ? fmin(a, b) : fmax(a, b));
    }
    part[blockIdx.x * 10 + k] = a;
  }
}

// nblk <= 512 block partials: thread t combines partials t and t + 256, then a
// fixed tree combines the threads (sums for 0-3, min for 4-6, max for 7-9).
__global__ __launch_bounds__(256) void moments_final(const double *__restrict__ part, int nblk,
                                                     double *__restrict__ out) {
  const int t = threadIdx.x;
  __shared__ double r[10][256];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    double a = k < 4 ? 0.0 : (k < 7 ? INFINITY : -INFINITY);
    for (int b = t; b < nblk; b += 256) {
      const double c = part[b * 10 + k];
      a = k < 4 ? a + c : (k < 7 ? fmin(a, c) : fmax(a, c));
    }
    r[k][t] = a;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o)
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        const double a = r[k][t], c = r[k][t + o];
        r[k][t] = k < 4 ? a + c : (k < 7 ? fmin(a, c) : fmax(a, c));
      }
    __syncthreads();
  }
  if (t < 10) out[t] = r[t][0];
}

}  // namespace

// ----------------------------------------------------------------- launchers

BatchPlan batch_plan(int npairs, const int64_t *N, const int64_t *M, int backend, int cull,
                     int target_items) {
  BatchPlan pl;
  pl.backend = backend;
  pl.npairs = npairs;
  pl.slots.resize(npairs);
  double work = 0.0;
  for (int p = 0; p < npairs; ++p) work += (double)N[p] * (double)M[p];
  const int target = target_items >= 64 ? target_items : 8192;
  for (int p = 0; p < npairs; ++p) {
    Slot &sl = pl.slots[p];
    sl = Slot{};
    sl.N = (int32_t)N[p];
    sl.M = (int32_t)M[p];
    sl.x_off = pl.sources;
    sl.y_off = pl.targets;
    pl.sources += N[p];
    pl.targets += M[p];
    sl.ngroups = (int32_t)((N[p] + kGroup - 1) / kGroup);
    sl.ntiles = (int32_t)((M[p] + kCullTile - 1) / kCullTile);
    sl.g_off = (int32_t)pl.groups;
    sl.t_off = (int32_t)pl.tiles;
    sl.list_off = pl.list_ints;
    pl.groups += sl.ngroups;
    pl.tiles += sl.ntiles;
    pl.list_ints += (int64_t)sl.ngroups * sl.ntiles;
    // the problem's share of the work items, in proportion to M N;
    // sum_g ceil(count_g / L) < tiles / L + ngroups <= target + ngroups
    int64_t tp = (int64_t)((double)target * ((double)N[p] * (double)M[p]) / work + 0.5);
    sl.target = (int32_t)(tp < 16 ? 16 : tp);
    sl.item_cap = sl.target + sl.ngroups;
    sl.item_off = (int32_t)pl.items;
    pl.items += sl.item_cap;
    sl.nfin = (int32_t)((N[p] + kFinBlock - 1) / kFinBlock);
    sl.fin_off = (int32_t)pl.fins;
    pl.fins += sl.nfin;
  }
  // the live-tile lists take 4 bytes per (group, tile); beyond 2^28 of
  // them (1 GiB) every pair is evaluated
  pl.cull = backend == kBackendScalar && cull && pl.list_ints <= ((int64_t)1 << 28);
  if (!pl.cull)
    for (Slot &sl : pl.slots) sl.list_off = 0;
  if (!pl.cull) pl.list_ints = 0;
  pl.grp_slot.resize(pl.groups);
  pl.item_slot.resize(backend == kBackendScalar ? pl.items : 0);
  pl.fin_slot.resize(pl.fins);
  for (int p = 0; p < npairs; ++p) {
    const Slot &sl = pl.slots[p];
    for (int g = 0; g < sl.ngroups; ++g) pl.grp_slot[sl.g_off + g] = p;
    if (backend == kBackendScalar)
      for (int i = 0; i < sl.item_cap; ++i) pl.item_slot[sl.item_off + i] = p;
    for (int f = 0; f < sl.nfin; ++f) pl.fin_slot[sl.fin_off + f] = p;
  }
  if (backend != kBackendScalar) {
    // LDS and MFMA back ends (one problem): sources per block, target chunks
    const int64_t n = N[0], m = M[0];
    const int64_t per_block = backend == kBackendLds ? (int64_t)kBlock * kPairS : (int64_t)kBlock;
    pl.nsrc_blocks = (int)((n + per_block - 1) / per_block);
    // about 1024 blocks (4096 waves) fill the 256 CUs; every split adds one
    // FP64 partial per source and feature, so no more splits than that
    const int64_t want = 1024;
    int64_t ns = (want + pl.nsrc_blocks - 1) / pl.nsrc_blocks;
    const int64_t maxs = (m + 127) / 128;
    if (ns > maxs) ns = maxs;
    if (ns > 64) ns = 64;
    if (ns < 1) ns = 1;
    int64_t chunk = (m + ns - 1) / ns;
    chunk = (chunk + 3) / 4 * 4;
    ns = (m + chunk - 1) / chunk;
    pl.nsplit = (int)ns;
    pl.mchunk = chunk;
  }
  return pl;
}

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

size_t batch_tables_bytes(const BatchPlan &pl) {
  return align256(pl.slots.size() * sizeof(Slot)) + align256(pl.grp_slot.size() * sizeof(int)) +
         align256(pl.item_slot.size() * sizeof(int)) + align256(pl.fin_slot.size() * sizeof(int));
}

void batch_tables_pack(const BatchPlan &pl, std::vector<char> &host) {
  host.assign(batch_tables_bytes(pl), 0);
  char *p = host.data();
  memcpy(p, pl.slots.data(), pl.slots.size() * sizeof(Slot));
  p += align256(pl.slots.size() * sizeof(Slot));
  memcpy(p, pl.grp_slot.data(), pl.grp_slot.size() * sizeof(int));
  p += align256(pl.grp_slot.size() * sizeof(int));
  if (!pl.item_slot.empty()) memcpy(p, pl.item_slot.data(), pl.item_slot.size() * sizeof(int));
  p += align256(pl.item_slot.size() * sizeof(int));
  memcpy(p, pl.fin_slot.data(), pl.fin_slot.size() * sizeof(int));
}

BatchDev batch_tables_view(const BatchPlan &pl, const void *dev) {
  const char *p = (const char *)dev;
  BatchDev d;
  d.slots = (const Slot *)p;
  p += align256(pl.slots.size() * sizeof(Slot));
  d.grp_slot = (const int *)p;
  p += align256(pl.grp_slot.size() * sizeof(int));
  d.item_slot = (const int *)p;
  p += align256(pl.item_slot.size() * sizeof(int));
  d.fin_slot = (const int *)p;
  return d;
}

size_t estep_partial_bytes(const BatchPlan &pl) {
  if (pl.backend == kBackendScalar) return (size_t)pl.items * kFeatUsed * kGroup * sizeof(double);
  return (size_t)pl.nsplit * kFeatUsed * (size_t)pl.slots[0].N * sizeof(double);
}

// Work-item plan layout: CullHdr[npairs], evaluated-pair counters[2 npairs],
// counts[groups], off[groups + npairs], Item[items], gbox[groups][kGBox],
// list[list_ints].
namespace {
struct PlanPtrs {
  CullHdr *hdr;
  unsigned long long *evcount;
  int *counts, *off, *list;
  Item *items;
  double *gbox;
};
PlanPtrs plan_ptrs(const BatchPlan &pl, void *ws) {
  char *p = (char *)ws;
  PlanPtrs q;
  q.hdr = (CullHdr *)p;
  p += align256((size_t)pl.npairs * sizeof(CullHdr));
  q.evcount = (unsigned long long *)p;
  p += align256((size_t)2 * pl.npairs * sizeof(unsigned long long));
  q.counts = (int *)p;
  p += align256((size_t)pl.groups * sizeof(int));
  q.off = (int *)p;
  p += align256((size_t)(pl.groups + pl.npairs) * sizeof(int));
  q.items = (Item *)p;
  p += align256((size_t)pl.items * sizeof(Item));
  q.gbox = (double *)p;
  p += align256((size_t)pl.groups * kGBox * sizeof(double));
  q.list = (int *)p;
  return q;
}
}  // namespace

const int *estep_plan_offsets(const BatchPlan &pl, const void *plan_ws) {
  return pl.backend == kBackendScalar ? plan_ptrs(pl, (void *)plan_ws).off : nullptr;
}

size_t estep_plan_bytes(const BatchPlan &pl) {
  if (pl.backend != kBackendScalar) return 256;
  return align256((size_t)pl.npairs * sizeof(CullHdr)) +
         align256((size_t)2 * pl.npairs * sizeof(unsigned long long)) +
         align256((size_t)pl.groups * sizeof(int)) +
         align256((size_t)(pl.groups + pl.npairs) * sizeof(int)) +
         align256((size_t)pl.items * sizeof(Item)) +
         align256((size_t)pl.groups * kGBox * sizeof(double)) + (size_t)pl.list_ints * sizeof(int);
}

unsigned long long *estep_plan_counter(const BatchPlan &pl, void *plan_ws) {
  return pl.backend == kBackendScalar ? plan_ptrs(pl, plan_ws).evcount : nullptr;
}

hipError_t launch_estep_plan(const BatchPlan &pl, const BatchDev &bd, const TBox *boxes,
                             DevState *s, void *plan_ws, hipStream_t st) {
  if (pl.backend != kBackendScalar) return hipSuccess;
  const PlanPtrs q = plan_ptrs(pl, plan_ws);
  if (pl.cull) {
    hipLaunchKernelGGL(cull_groups, dim3((unsigned)pl.groups), dim3(kBlock), 0, st,
                       pl.npairs == 1 ? 1 : 0, bd.slots, bd.grp_slot, s, boxes, q.counts, q.gbox,
                       q.list);
    hipLaunchKernelGGL(cull_items<true>, dim3((unsigned)pl.npairs), dim3(kBlock), 0, st, bd.slots,
                       s, q.counts, q.hdr, q.off, q.items, q.evcount);
  } else {
    hipLaunchKernelGGL(cull_items<false>, dim3((unsigned)pl.npairs), dim3(kBlock), 0, st,
                       bd.slots, s, q.counts, q.hdr, q.off, q.items, q.evcount);
  }
  return hipGetLastError();
}

hipError_t launch_estep_pairs(const BatchPlan &pl, const BatchDev &bd, const TRec *rec,
                              const TPt *pts, const TBox *boxes, const void *ftab, DevState *s,
                              void *plan_ws, double *partial, hipStream_t st) {
  if (pl.backend == kBackendScalar) {
    const PlanPtrs q = plan_ptrs(pl, plan_ws);
    const int single = pl.npairs == 1 ? 1 : 0;
    if (pl.cull) {
      const int f3 = pl.f3 ? 1 : 0;
      hipLaunchKernelGGL(estep_pairs_items<true>, dim3((unsigned)pl.items), dim3(kBlock), 0, st,
                         single, bd.slots, bd.item_slot, s, q.hdr, q.items, rec, pts, q.list,
                         q.gbox, boxes, f3, q.evcount, partial);
      if (f3)
        hipLaunchKernelGGL(estep_pairs_f3, dim3((unsigned)pl.items), dim3(kBlock), 0, st, single,
                           bd.slots, bd.item_slot, s, q.hdr, q.items, rec, (const __bf16 *)ftab,
                           q.list, q.gbox, boxes, q.evcount, q.evcount + pl.npairs, partial);
    } else
      hipLaunchKernelGGL(estep_pairs_items<false>, dim3((unsigned)pl.items), dim3(kBlock), 0, st,
                         single, bd.slots, bd.item_slot, s, q.hdr, q.items, rec, pts, q.list,
                         q.gbox, boxes, 0, q.evcount, partial);
    return hipGetLastError();
  }
  // one problem: its records start at rec + 0
  const Slot &sl = pl.slots[0];
  dim3 grid((unsigned)(pl.nsrc_blocks * pl.nsplit));
  if (pl.backend == kBackendMfma)
    hipLaunchKernelGGL(estep_mfma, grid, dim3(kBlock), 0, st, sl.X, sl.N, rec, (int64_t)sl.M, s,
                       pl.mchunk, pl.nsplit, partial);
  else
    hipLaunchKernelGGL(estep_pairs_lds<kPairS>, grid, dim3(kBlock), 0, st, sl.X, sl.N, rec,
                       (int64_t)sl.M, s, pl.mchunk, pl.nsplit, partial);
  return hipGetLastError();
}

hipError_t launch_dump_P(const float *X, int64_t N, const TRec *rec, int64_t M, const float *w,
                         const DevState *s, const double *colS, float *P, hipStream_t st) {
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(dump_P, dim3((unsigned)blocks), dim3(256), 0, st, X, (int)N, rec, M, w, s,
                     colS, P);
  return hipGetLastError();
}

hipError_t launch_prep_targets(const float *Y, const float *normals, const float *alpha,
                               const float *pi, const double *pi_sum, const uint32_t *perm,
                               int64_t M, int exact, TRec *rec, TPt *pts, TBox *boxes,
                               void *ftab, hipStream_t st) {
  hipLaunchKernelGGL(prep_targets, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, Y,
                     normals, alpha, pi, pi_sum, perm, M, exact, rec, pts);
  const int64_t ntiles = (M + kCullTile - 1) / kCullTile;
  hipLaunchKernelGGL(tile_boxes, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, pts, M,
                     boxes);
  if (ftab)
    hipLaunchKernelGGL(f3_tables, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, rec, M,
                       (__bf16 *)ftab, boxes);
  return hipGetLastError();
}

size_t f3_table_bytes(int64_t tiles) {
  return (size_t)tiles * 2 * kF3Feat * kCullTile * sizeof(__bf16);
}

int moments_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 512) b = 512;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_moments(const float *P, int64_t n, const DevState *pose, double *partials,
                          int nblk, double *out, hipStream_t st) {
  hipLaunchKernelGGL(moments_partial, dim3((unsigned)nblk), dim3(256), 0, st, P, (int)n, pose,
                     partials);
  hipLaunchKernelGGL(moments_final, dim3(1), dim3(256), 0, st, partials, nblk, out);
  return hipGetLastError();
}

}  // namespace lsg
