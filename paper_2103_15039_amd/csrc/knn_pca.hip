// Target geometry on the GPU (Sec. 3.1 and Eq. 3 of LSG-CPD): exact k
// nearest neighbours, FP64 3x3 PCA of each neighbourhood, surface variation
// kappa and the penalty alpha.
//
// The caller puts the cloud in Hilbert order (order.hip) and passes the sorted
// copy Ys (x, y, z, original index).  Pass 1a (knn_seed): one wave per tile
// of 64 sorted queries scans the own tile and the two next to it, which gives
// every query a first list of its k best (distance, original index) keys and
// a bound on its k-th distance.  Pass 1b (knn_tiles): S waves per query tile
// skip every other tile whose box lies farther from the box of the wave's
// queries than their largest bound, which cannot change any answer (with a
// relative margin of 1e-5 for the float32 rounding of the distances), and
// share the remaining tiles; knn_merge combines their lists.  Isolated
// queries, whose k-th distance would widen the search of the whole wave, are
// instead answered by pass 2 (knn_hard), one wave per query over the tiles
// that their pass-1 list cannot rule out.
// Distances are float32 ((dx*dx + dy*dy) + dz*dz), no contraction, so that
// the neighbour set is decided exactly as the float32 definition says; keys
// are ordered by (distance bits, original index), i.e. by distance with ties
// to the lower index, so the result does not depend on the order of the scan.
// Pass 3 (knn_pca): one thread per query forms the neighbourhood covariance
// about its mean in FP64, diagonalises it by cyclic Jacobi rotations and
// writes the results at the query's original index.
#include <math.h>

#include <stdlib.h>

#include "lsgcpd_internal.h"

namespace lsg {

namespace {

constexpr int kKnnBlock = 256;
constexpr int kKnnTileW = 64;  // sorted points per tile (one wave of queries)
constexpr uint32_t kNoIndex = 0xffffffffu;

struct TBoxF {
  float lo[3], hi[3];
  float pad[2];
};

__device__ __forceinline__ float dist2_f32(float ax, float ay, float az, float bx, float by,
                                           float bz) {
#pragma clang fp contract(off)
  const float dx = ax - bx;
  const float dy = ay - by;
  const float dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ uint64_t make_key(float d, uint32_t i) {
  return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)i;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_index(uint64_t k) { return (uint32_t)k; }

// The KM smallest keys seen so far, sorted, in registers (all indices are
// compile-time constants, so nothing spills).  The caller uses the first
// k <= KM entries; `worst` is the k-th key, the bound a new key must beat.
template <int KM>
struct TopK {
  uint64_t key[KM];
  uint64_t worst;
  int k;

  __device__ __forceinline__ void init(int k_, uint64_t fill) {
    k = k_;
#pragma unroll
    for (int j = 0; j < KM; ++j) key[j] = fill;
    worst = fill;
  }

  // one bubbling pass: the new key moves past every smaller key
  __device__ __forceinline__ void insert(uint64_t kn) {
    uint64_t c = kn;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      const uint64_t o = key[j];
      const bool lt = c < o;
      key[j] = lt ? c : o;
      c = lt ? o : c;
    }
    uint64_t w = key[0];
#pragma unroll
    for (int j = 1; j < KM; ++j) w = (j == k - 1) ? key[j] : w;
    worst = w;
  }

  __device__ __forceinline__ void offer(uint64_t kn) {
    if (kn < worst) insert(kn);
  }
};

// Lower bound of the float32 squared distance between points of two boxes:
// the gap per axis in FP64, shrunk by a relative 1e-5 (far above the rounding
// of the float32 distance) and an absolute 1e-30 (float32 underflow).
__device__ __forceinline__ double box_gap2(const TBoxF &a, const TBoxF &b) {
  double d2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double g = fmax(0.0, fmax((double)a.lo[i] - (double)b.hi[i],
                                    (double)b.lo[i] - (double)a.hi[i]));
    d2 = fma(g, g, d2);
  }
  return d2 * (1.0 - 1e-5) - 1e-30;
}

__device__ __forceinline__ float lanef(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// Tile u as one vector load (lane j holds point j; zeros past the end).
__device__ __forceinline__ float4 load_tile(const float4 *__restrict__ Ys, int M, int u) {
  const int lane = threadIdx.x & 63;
  const int j = u * kKnnTileW + lane;
  return j < M ? Ys[j] : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Offers the n points of a loaded tile to every lane's list, reading them back
// with readlane.
template <int KM>
__device__ __forceinline__ void scan_loaded(const float4 &p, int n, float qx, float qy, float qz,
                                            TopK<KM> &top) {
  for (int j = 0; j < n; ++j) {
    const float d = dist2_f32(qx, qy, qz, lanef(p.x, j), lanef(p.y, j), lanef(p.z, j));
    // cheap float test first; the exact key order decides inside
    if (d <= key_dist(top.worst))
      top.offer(make_key(d, (uint32_t)__builtin_amdgcn_readlane(__float_as_int(p.w), j)));
  }
}

__device__ __forceinline__ int tile_count(int M, int u) {
  return M - u * kKnnTileW < kKnnTileW ? M - u * kKnnTileW : kKnnTileW;
}

// Pass 1a, one wave per query tile t.  The own tile and its two Hilbert-order
// neighbours give every query a first list and its current k-th distance
// tau; the list is written as list 0.  Queries whose tau is far above the
// wave's 75th percentile (isolated points such as outliers) are "hard": they
// are listed for pass 2 and left out of the culling, so that they do not
// widen the search of the whole wave; if the other queries would still need
// more than kLiveCap * S tiles, the queries with the largest tau are moved to
// the hard list, 4 at a time.  The box of the remaining ("easy") queries, the
// largest tau among them (r20) and the mask of easy lanes are kept for pass 1b.
constexpr int kLiveCap = 32;

struct TileMeta {
  TBoxF own;       // box of the easy queries
  double r20;      // largest current k-th distance of the easy queries
  uint64_t easy;   // lane mask of the easy queries
};

template <int KM>
__global__ __launch_bounds__(kKnnBlock) void knn_seed(const float4 *__restrict__ Ys, int M,
                                                      int k, const TBoxF *__restrict__ boxes,
                                                      int ntiles, int S,
                                                      uint64_t *__restrict__ out,
                                                      TileMeta *__restrict__ meta,
                                                      float *__restrict__ taus,
                                                      uint32_t *__restrict__ hard,
                                                      unsigned int *__restrict__ nhard) {
  const int lane = threadIdx.x & 63;
  const int t =
      __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kKnnBlock / 64) + (threadIdx.x >> 6)));
  if (t >= ntiles) return;  // wave-uniform
  const int q = t * kKnnTileW + lane;
  const bool valid = q < M;
  float qx = 0.f, qy = 0.f, qz = 0.f;
  if (valid) {
    const float4 p = Ys[q];
    qx = p.x;
    qy = p.y;
    qz = p.z;
  }
  TopK<KM> top;
  top.init(k, make_key(INFINITY, kNoIndex));
  {
    const float4 p0 = load_tile(Ys, M, t);
    const float4 pm = t > 0 ? load_tile(Ys, M, t - 1) : p0;
    const float4 pp = t + 1 < ntiles ? load_tile(Ys, M, t + 1) : p0;
    scan_loaded<KM>(p0, tile_count(M, t), qx, qy, qz, top);
    if (t > 0) scan_loaded<KM>(pm, kKnnTileW, qx, qy, qz, top);
    if (t + 1 < ntiles) scan_loaded<KM>(pp, tile_count(M, t + 1), qx, qy, qz, top);
  }
  // rank of tau among the valid lanes (ties by lane), the 75th percentile
  const float tau = key_dist(top.worst);
  int rank = 0;
  const int nvalid = tile_count(M, t);
  for (int l = 0; l < nvalid; ++l) {
    const float o = lanef(tau, l);
    rank += (o < tau || (o == tau && l < lane)) ? 1 : 0;
  }
  const uint64_t at = __ballot(valid && rank == (3 * nvalid) / 4);
  const float p75 = at ? lanef(tau, (int)__builtin_ctzll(at)) : INFINITY;
  // easy lanes: rank < h
  int h = __popcll(__ballot(valid && !(tau > 16.0f * p75)));
  TBoxF own;
  for (int rep = 0;; ++rep) {
    const bool easy = valid && rank < h;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (easy) {
      lo[0] = hi[0] = qx;
      lo[1] = hi[1] = qy;
      lo[2] = hi[2] = qz;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
        hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
      }
    for (int a = 0; a < 3; ++a) {
      own.lo[a] = lo[a];
      own.hi[a] = hi[a];
    }
    if (rep == 8 || h <= nvalid / 2) break;
    double r2 = easy ? (double)tau : -INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
    int live = 0;
    for (int c0 = 0; c0 < ntiles; c0 += 64) {
      const int u = c0 + lane;
      live += __popcll(__ballot(u < ntiles && !(box_gap2(own, boxes[u]) > r2)));
    }
    if (live <= kLiveCap * S) break;
    h -= 4;
  }
  const bool easy = valid && rank < h;
  double r20 = easy ? (double)tau : -INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r20 = fmax(r20, __shfl_xor(r20, o, 64));
  const uint64_t em = __ballot(easy);
  if (valid) {
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) out[(size_t)j * M + q] = top.key[j];
    taus[q] = tau;
  }
  if (lane == 0) {
    TileMeta mt;
    mt.own = own;
    mt.own.pad[0] = mt.own.pad[1] = 0.f;
    mt.r20 = r20;
    mt.easy = em;
    meta[t] = mt;
  }
  if (valid && !easy) hard[atomicAdd(nhard, 1u)] = (uint32_t)q;
}

// Pass 1b, wave (query tile t, split s of S): every tile other than the first
// three whose box does not lie farther from the box of the wave's easy queries
// than their largest tau after pass 1a (r20, shared by all S waves, so that
// the S waves agree on which tiles are live and which wave owns which) is
// scanned by one of the S waves, every S-th in turn; a wave also skips an
// owned tile beyond the largest current k-th distance of its own lists
// (those are never below the merged ones, so this is exact too).  Split 0
// continues the list of pass 1a; the other S - 1 start from sentinels at tau
// (no query's answer has a key above (tau, any index)), so that every
// candidate enters exactly one of the S lists.  Split s writes list s.
template <int KM>
__global__ __launch_bounds__(kKnnBlock) void knn_tiles(const float4 *__restrict__ Ys, int M,
                                                       int k, const TBoxF *__restrict__ boxes,
                                                       int ntiles, int S,
                                                       const TileMeta *__restrict__ meta,
                                                       const float *__restrict__ taus,
                                                       uint64_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int t =
      __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kKnnBlock / 64) + (threadIdx.x >> 6)));
  const int split = blockIdx.y;
  if (t >= ntiles) return;  // wave-uniform
  const int q = t * kKnnTileW + lane;
  const bool valid = q < M;
  const TileMeta mt = meta[t];
  const TBoxF own = mt.own;
  const double r20 = mt.r20;
  const bool easy = valid && ((mt.easy >> lane) & 1ull);
  float qx = 0.f, qy = 0.f, qz = 0.f;
  TopK<KM> top;
  top.init(k, make_key(INFINITY, kNoIndex));
  if (valid) {
    const float4 p = Ys[q];
    qx = p.x;
    qy = p.y;
    qz = p.z;
    if (split == 0) {
      uint64_t v[KM];
#pragma unroll
      for (int j = 0; j < KM; ++j) v[j] = j < k ? out[(size_t)j * M + q] : make_key(INFINITY, kNoIndex);
#pragma unroll
      for (int j = 0; j < KM; ++j) top.key[j] = v[j];
      top.worst = v[0];
#pragma unroll
      for (int j = 1; j < KM; ++j) top.worst = (j == k - 1) ? v[j] : top.worst;
    } else {
      top.init(k, make_key(taus[q], kNoIndex));
    }
  }
  int ord = 0;
  for (int c0 = 0; c0 < ntiles; c0 += 64) {
    double r2 = easy ? (double)key_dist(top.worst) : -INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
    const int u = c0 + lane;
    bool live = u < ntiles && (u < t - 1 || u > t + 1);
    double gap = 0.0;
    if (live) {
      gap = box_gap2(own, boxes[u]);
      live = !(gap > r20);
    }
    const uint64_t lm = __ballot(live);
    const int mine = ord + __popcll(lm & ((1ull << lane) - 1ull));
    uint64_t mk = __ballot(live && mine % S == split && !(gap > r2));
    ord += __popcll(lm);
    // walk the tiles, loading the next one while the current one is scanned
    if (mk) {
      int b = __builtin_ctzll(mk);
      mk &= mk - 1;
      float4 cur = load_tile(Ys, M, c0 + b);
      for (;;) {
        const int n = tile_count(M, c0 + b);
        const bool more = mk != 0;
        int bn = b;
        float4 nxt = cur;
        if (more) {
          bn = __builtin_ctzll(mk);
          mk &= mk - 1;
          nxt = load_tile(Ys, M, c0 + bn);
        }
        scan_loaded<KM>(cur, n, qx, qy, qz, top);
        if (!more) break;
        cur = nxt;
        b = bn;
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) out[((size_t)split * k + j) * M + q] = top.key[j];
  }
}

// Merge of the S partial lists of every query into list 0.  Four lanes per
// query: lane j keeps the k smallest keys of lists j, j + 4, ..., then k
// rounds of a minimum over the four lanes pop the answer in order.  Every real
// candidate is in one list only, and list 0 holds k real keys below every
// sentinel of the others, so the k keys popped are real and distinct (one
// lane pops per round).
constexpr int kMergeLanes = 4;

template <int KM>
__global__ __launch_bounds__(256) void knn_merge(int M, int k, int S,
                                                 uint64_t *__restrict__ keys) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = gid / kMergeLanes, part = gid % kMergeLanes;  // a query's lanes share a wave
  const bool valid = q < M;
  TopK<KM> top;
  top.init(k, ~(uint64_t)0);
  if (valid)
    for (int s = part; s < S; s += kMergeLanes) {
      // the whole list at once (k loads in flight)
      uint64_t v[KM];
#pragma unroll
      for (int j = 0; j < KM; ++j) v[j] = j < k ? keys[((size_t)s * k + j) * M + q] : ~(uint64_t)0;
#pragma unroll
      for (int j = 0; j < KM; ++j)
        if (j < k && v[j] < top.worst) top.insert(v[j]);
    }
  for (int r = 0; r < k; ++r) {
    uint64_t m = top.key[0];
#pragma unroll
    for (int o = 1; o < kMergeLanes; o <<= 1) {
      const uint32_t mh = (uint32_t)__shfl_xor((int)(uint32_t)(m >> 32), o, 64);
      const uint32_t ml = (uint32_t)__shfl_xor((int)(uint32_t)m, o, 64);
      const uint64_t v = ((uint64_t)mh << 32) | ml;
      m = v < m ? v : m;
    }
    if (valid && part == 0) keys[(size_t)r * M + q] = m;
    if (top.key[0] == m) {  // pop the head
#pragma unroll
      for (int j = 0; j + 1 < KM; ++j) top.key[j] = top.key[j + 1];
      top.key[KM - 1] = ~(uint64_t)0;
    }
  }
}

// Pass 2: one wave per hard query.  Its merged list from pass 1 holds k real
// candidates, so its k-th key bounds the answer: tiles whose box lies farther
// from the query than that distance (the same conservative FP64 gap as pass
// 1) hold no answer and are skipped, 64 tile boxes tested at a time.  Lane l
// takes point l of every other tile into a list of its own that starts from
// sentinels at the bound; k rounds of a wave minimum then merge the 64 lists
// (keys are unique, so exactly one lane pops per round).  Hard queries are
// taken in list order by a grid-stride loop that every wave leaves.  Writes
// list 0.
template <int KM>
__global__ __launch_bounds__(kKnnBlock) void knn_hard(const float4 *__restrict__ Ys, int M,
                                                      int k, const TBoxF *__restrict__ boxes,
                                                      int ntiles, const uint32_t *__restrict__ hard,
                                                      const unsigned int *__restrict__ nhard,
                                                      uint64_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int w0 = blockIdx.x * (kKnnBlock / 64) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (kKnnBlock / 64);
  const int nh = (int)*nhard;
  for (int h = w0; h < nh; h += nw) {
    const int q = (int)hard[h];
    const float4 qp = Ys[q];
    const float bound = key_dist(out[(size_t)(k - 1) * M + q]);
    TBoxF qb;
    qb.lo[0] = qb.hi[0] = qp.x;
    qb.lo[1] = qb.hi[1] = qp.y;
    qb.lo[2] = qb.hi[2] = qp.z;
    TopK<KM> top;
    top.init(k, make_key(bound, kNoIndex));
    for (int c0 = 0; c0 < ntiles; c0 += 64) {
      const int u = c0 + lane;
      uint64_t mk = __ballot(u < ntiles && !(box_gap2(qb, boxes[u]) > (double)bound));
      // walk the live tiles, loading the next point while the current one is used
      if (mk) {
        int b = __builtin_ctzll(mk);
        mk &= mk - 1;
        const int j0 = (c0 + b) * kKnnTileW + lane;
        float4 cur = j0 < M ? Ys[j0] : make_float4(NAN, NAN, NAN, 0.f);
        for (;;) {
          const bool more = mk != 0;
          float4 nxt = cur;
          if (more) {
            const int bn = __builtin_ctzll(mk);
            mk &= mk - 1;
            const int j1 = (c0 + bn) * kKnnTileW + lane;
            nxt = j1 < M ? Ys[j1] : make_float4(NAN, NAN, NAN, 0.f);
          }
          const float d = dist2_f32(qp.x, qp.y, qp.z, cur.x, cur.y, cur.z);
          if (d <= key_dist(top.worst)) top.offer(make_key(d, __float_as_uint(cur.w)));
          if (!more) break;
          cur = nxt;
        }
      }
    }
    for (int r = 0; r < k; ++r) {
      uint64_t m = top.key[0];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint32_t mh = (uint32_t)__shfl_xor((int)(uint32_t)(m >> 32), o, 64);
        const uint32_t ml = (uint32_t)__shfl_xor((int)(uint32_t)m, o, 64);
        const uint64_t v = ((uint64_t)mh << 32) | ml;
        m = v < m ? v : m;
      }
      if (lane == 0) out[(size_t)r * M + q] = m;
      if (top.key[0] == m) {  // pop the head
#pragma unroll
        for (int j = 0; j + 1 < KM; ++j) top.key[j] = top.key[j + 1];
        top.key[KM - 1] = make_key(INFINITY, kNoIndex);
      }
    }
  }
}

// Bounding box of every tile of kKnnTileW sorted points (one wave per tile).
// Also clears the counter of hard queries.
__global__ void knn_boxes(const float4 *__restrict__ Ys, int M, int ntiles,
                          TBoxF *__restrict__ boxes, unsigned int *__restrict__ nhard) {
  const int t = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t == 0 && lane == 0) *nhard = 0u;
  if (t >= ntiles) return;  // wave-uniform
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int q = t * kKnnTileW + lane;
  if (q < M) {
    const float4 p = Ys[q];
    lo[0] = hi[0] = p.x;
    lo[1] = hi[1] = p.y;
    lo[2] = hi[2] = p.z;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
  if (lane == 0) {
    TBoxF b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = lo[a];
      b.hi[a] = hi[a];
    }
    b.pad[0] = b.pad[1] = 0.f;
    boxes[t] = b;
  }
}

// Query q (sorted position) is target qorig[q] of the caller's order; keys
// hold original indices into Y.
template <int KM>
__global__ __launch_bounds__(256) void knn_pca(const float *__restrict__ Y, int M, int k,
                                               const uint64_t *__restrict__ keys,
                                               const uint32_t *__restrict__ qorig,
                                               double alpha_max, double lambda,
                                               float *__restrict__ normals,
                                               float *__restrict__ kappa,
                                               float *__restrict__ alpha) {
  const int qs = blockIdx.x * blockDim.x + threadIdx.x;
  if (qs >= M) return;
  const int q = (int)qorig[qs];
  // every slot holds a valid index unless the inputs were not finite; such
  // slots fall back to the query point itself
  int idx[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    const uint32_t i = j < k ? key_index(keys[(size_t)j * M + qs]) : kNoIndex;
    idx[j] = i < (uint32_t)M ? (int)i : q;
  }
  double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j < k) {
      mx += (double)Y[3 * idx[j]];
      my += (double)Y[3 * idx[j] + 1];
      mz += (double)Y[3 * idx[j] + 2];
    }
  }
  const double invk = 1.0 / (double)k;
  mx *= invk;
  my *= invk;
  mz *= invk;
  double c00 = 0, c01 = 0, c02 = 0, c11 = 0, c12 = 0, c22 = 0;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j < k) {
      const double dx = (double)Y[3 * idx[j]] - mx;
      const double dy = (double)Y[3 * idx[j] + 1] - my;
      const double dz = (double)Y[3 * idx[j] + 2] - mz;
      c00 += dx * dx;
      c01 += dx * dy;
      c02 += dx * dz;
      c11 += dy * dy;
      c12 += dy * dz;
      c22 += dz * dz;
    }
  }
  double a[3][3] = {{c00 * invk, c01 * invk, c02 * invk},
                    {c01 * invk, c11 * invk, c12 * invk},
                    {c02 * invk, c12 * invk, c22 * invk}};
  const double tr = a[0][0] + a[1][1] + a[2][2];
  double nx = 0.0, ny = 0.0, nz = 1.0, kap = 1.0 / 3.0;
  if (tr > 0.0) {
    double v[3][3];
    jacobi3(a, v);
    int imin = 0;
    if (a[1][1] < a[imin][imin]) imin = 1;
    if (a[2][2] < a[imin][imin]) imin = 2;
    nx = v[0][imin];
    ny = v[1][imin];
    nz = v[2][imin];
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nn;
    ny /= nn;
    nz /= nn;
    kap = fmin(fmax(a[imin][imin] / tr, 0.0), 1.0 / 3.0);
  }
  double al;
  if (kap <= 0.0) {
    al = alpha_max;
  } else {
    const double u = exp(lambda * (3.0 - 1.0 / kap));
    al = fmax((1.0 - u) / (1.0 + u) * alpha_max, 0.0);
  }
  normals[3 * q] = (float)nx;
  normals[3 * q + 1] = (float)ny;
  normals[3 * q + 2] = (float)nz;
  if (kappa) kappa[q] = (float)kap;
  alpha[q] = (float)al;
}

}  // namespace

// Target splits of pass 1: about 4096 waves in all, at most 256 / k lists.
int knn_splits(int64_t M, int k) {
  const int64_t ntiles = (M + kKnnTileW - 1) / kKnnTileW;
  // about 16384 waves in pass 1b (measured best on the 20k and 100k clouds;
  // keys take S k M 8 bytes, so large clouds get few splits)
  int64_t S = (16384 + ntiles - 1) / ntiles;
  // LSGCPD_KNN_SPLITS fixes S (1..16) for tuning sweeps
  if (const char *e = getenv("LSGCPD_KNN_SPLITS")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 16) return v;
  }
  const int64_t cap = 256 / (k > 8 ? k : 8);
  if (S > cap) S = cap;
  if (S > 16) S = 16;
  if (S < 1) S = 1;
  return (int)S;
}

// Workspace: keys[S][k][M], tile metadata, tile boxes, tau[M], hard list[M],
// hard counter.
size_t knn_workspace_bytes(int64_t M, int k) {
  const size_t ntiles = (size_t)((M + kKnnTileW - 1) / kKnnTileW);
  return (size_t)knn_splits(M, k) * k * (size_t)M * sizeof(uint64_t) +
         ntiles * sizeof(TileMeta) + ntiles * sizeof(TBoxF) + (size_t)M * sizeof(float) +
         (size_t)M * sizeof(uint32_t) + 256;
}

hipError_t launch_normals(const float *Y, int64_t M, const float4 *Ys, const uint32_t *perm,
                          int k, double alpha_max, double lambda, float *normals, float *kappa,
                          float *alpha, void *work, size_t work_bytes, hipStream_t st) {
  if (knn_workspace_bytes(M, k) > work_bytes) return hipErrorInvalidValue;
  const int Mi = (int)M;
  const int ntiles = (int)((M + kKnnTileW - 1) / kKnnTileW);
  const int S = knn_splits(M, k);
  uint64_t *keys = (uint64_t *)work;
  TileMeta *meta = (TileMeta *)(keys + (size_t)S * k * M);
  TBoxF *boxes = (TBoxF *)(meta + ntiles);
  float *taus = (float *)(boxes + ntiles);
  uint32_t *hard = (uint32_t *)(taus + M);
  unsigned int *nhard = (unsigned int *)(hard + M);
  hipLaunchKernelGGL(knn_boxes, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, Ys, Mi,
                     ntiles, boxes, nhard);
  const dim3 g0((unsigned)((ntiles + kKnnBlock / 64 - 1) / (kKnnBlock / 64)));
  const dim3 g1((unsigned)((ntiles + kKnnBlock / 64 - 1) / (kKnnBlock / 64)), (unsigned)S);
  const dim3 gh(512);
  const dim3 g2((unsigned)((M + 255) / 256));
  const dim3 gm((unsigned)((M * kMergeLanes + 255) / 256));
#define LSG_KNN(KM_)                                                                            \
  do {                                                                                          \
    hipLaunchKernelGGL(knn_seed<KM_>, g0, dim3(kKnnBlock), 0, st, Ys, Mi, k, boxes, ntiles, S,  \
                       keys, meta, taus, hard, nhard);                                          \
    hipLaunchKernelGGL(knn_tiles<KM_>, g1, dim3(kKnnBlock), 0, st, Ys, Mi, k, boxes, ntiles, S, \
                       meta, taus, keys);                                                       \
    if (S > 1)                                                                                  \
      hipLaunchKernelGGL(knn_merge<KM_>, gm, dim3(256), 0, st, Mi, k, S, keys);                 \
    hipLaunchKernelGGL(knn_hard<KM_>, gh, dim3(kKnnBlock), 0, st, Ys, Mi, k, boxes, ntiles,    \
                       hard, nhard, keys);                                                      \
    hipLaunchKernelGGL(knn_pca<KM_>, g2, dim3(256), 0, st, Y, Mi, k, keys, perm, alpha_max,     \
                       lambda, normals, kappa, alpha);                                          \
  } while (0)
  if (k <= 8) LSG_KNN(8);
  else if (k <= 16) LSG_KNN(16);
  else if (k <= 20) LSG_KNN(20);
  else LSG_KNN(32);
#undef LSG_KNN
  return hipGetLastError();
}

}  // namespace lsg
