// Tile binning: one instance per (record, covered tile), a stable LSD radix
// sort by (global tile, depth), and per-tile ranges of the sorted list.
//
// Radix sort (hand-written, stable, 8-bit digits, 256-thread blocks of 4096
// keys), one kernel per pass in the onesweep style (Adinets & Merrill 2022):
// a single histogram kernel reads the keys once and counts the digits of
// every pass; each pass kernel takes a block id from an atomic counter (so
// every lower id is already running), ranks its keys inside each wave64 with
// 8 ballots per key (lanes hold consecutive keys, so ranks are stable),
// publishes its per-digit counts, and finds its global offsets by looking
// back over the published counts of the blocks before it (decoupled
// look-back).  The look-back spin is bounded: it never hangs, it flags an
// error word instead.  Keys are staged in LDS in digit order so that
// consecutive lanes write consecutive addresses.
//
// Two orders of work give the same sorted list (by tile, then depth, then
// record index):
//   mode 0: 64-bit keys (tile << 32 | depth bits), written per record in
//           record order, sorted over 32 + tile bits;
//   mode 1: the M records are first sorted by depth (32-bit keys); the
//           instances are expanded in that order with 32-bit tile keys (load
//           balanced: one block per 2048 instances, not one thread per
//           record), then sorted over the tile bits only.  Stability keeps
//           depth order and index order inside a tile.  Far fewer bytes move.
#include <algorithm>

#include "sgs_dev.h"

namespace sgs {

sgs_status launch_scan_blocks(const uint32_t* in, uint32_t* out, int64_t nb, hipStream_t s);

constexpr int RS_T = 256;          // threads per block
constexpr int RS_IPT = 16;         // keys per thread
constexpr int RS_TILE = RS_T * RS_IPT;
constexpr int RS_MAX_PASSES = 8;
constexpr uint64_t ST_AGG = 1ull << 32;    // status: block's own digit count
constexpr uint64_t ST_INC = 2ull << 32;    // status: inclusive prefix over blocks
constexpr uint32_t SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint32_t count_of(const uint32_t* n_dev, uint32_t n_host, uint32_t cap) {
  const uint32_t n = n_dev ? *n_dev : n_host;
  return n < cap ? n : cap;
}

// Lanes holding the same digit as this lane (only lanes with valid set).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int nbits) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

// Exclusive scan over the 256 threads of a block of x (one value per thread).
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* ws4) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) ws4[w] = inc;
  __syncthreads();
  uint32_t e = inc - x;
  for (int k = 0; k < w; ++k) e += ws4[k];
  __syncthreads();
  return e;
}

// Digit histograms of every pass in one read of the keys.
template <typename K>
__global__ void __launch_bounds__(RS_T) k_os_hist(const K* __restrict__ keys, const uint32_t* n_dev,
                                                  uint32_t n_host, uint32_t cap, int bits,
                                                  uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[RS_MAX_PASSES][256];
  const int t = threadIdx.x;
  const int passes = (bits + 7) / 8;
  for (int k = t; k < RS_MAX_PASSES * 256; k += RS_T) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint32_t n = count_of(n_dev, n_host, cap);
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  for (int i = 0; i < RS_IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * RS_T + t;
    if (idx < n) {
      const K key = keys[idx];
      for (int p = 0; p < passes; ++p) atomicAdd(&h[p][digit_of<K>(key, 8 * p, 0xffu)], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][t]) atomicAdd(&ghist[p * 256 + t], h[p][t]);
}

template <typename K>
__global__ void __launch_bounds__(RS_T) k_os_pass(const K* __restrict__ kin,
                                                  const uint32_t* __restrict__ vin,
                                                  K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                  const uint32_t* n_dev, uint32_t n_host,
                                                  uint32_t cap, int shift, int nbits,
                                                  const uint32_t* __restrict__ ghist,
                                                  uint64_t* status, uint32_t* counter,
                                                  uint32_t* err) {
  __shared__ uint32_t wc[4][256];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t ws[4];
  __shared__ uint32_t s_bid;
  __shared__ K skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  if (t == 0) s_bid = atomicAdd(counter, 1u);
  for (int k = t; k < 1024; k += RS_T) (&wc[0][0])[k] = 0;
  __syncthreads();
  const uint32_t b = s_bid;
  const uint32_t n = count_of(n_dev, n_host, cap);
  const uint64_t bbase = (uint64_t)b * RS_TILE;
  if (bbase >= n) return;   // ids past the data: no later block waits on them
  const uint32_t mask = (1u << nbits) - 1u;
  const uint64_t base = bbase + (uint64_t)w * (RS_IPT * 64) + lane;
  const uint64_t lt = lanemask_lt();
  K key[RS_IPT];
  uint32_t val[RS_IPT];
  uint32_t rank[RS_IPT];
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * 64;
    const bool valid = idx < n;
    key[i] = valid ? kin[idx] : (K)0;
    val[i] = valid ? vin[idx] : 0u;
    const uint32_t d = digit_of<K>(key[i], shift, mask);
    const uint64_t peers = match_digit(d, valid, nbits);
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    const uint32_t c = wc[w][d];
    rank[i] = c + r;
    if (valid && r == 0) wc[w][d] = c + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  const uint32_t c0 = wc[0][t], c1 = wc[1][t], c2 = wc[2][t], c3 = wc[3][t];
  const uint32_t tot = c0 + c1 + c2 + c3;
  const uint32_t ls = block_excl_scan256(tot, ws);
  const uint32_t ds = block_excl_scan256(ghist[t], ws);   // start of digit t in the output
  lstart[t] = ls;
  wc[0][t] = ls;
  wc[1][t] = ls + c0;
  wc[2][t] = ls + c0 + c1;
  wc[3][t] = ls + c0 + c1 + c2;
  // publish this block's count of digit t, then look back for the prefix
  uint64_t* st = status + (uint64_t)b * 256 + t;
  if (b == 0) {
    __hip_atomic_store(st, ST_INC | (uint64_t)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    goff[t] = ds;
  } else {
    __hip_atomic_store(st, ST_AGG | (uint64_t)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0, spins = 0;
    uint32_t bp = b - 1;
    for (;;) {
      const uint64_t s = __hip_atomic_load(status + (uint64_t)bp * 256 + t, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t f = s & ~0xffffffffull;
      if (f == 0) {
        if (++spins > SPIN_LIMIT) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += (uint32_t)s;
      if (f == ST_INC || bp == 0) break;
      --bp;
    }
    __hip_atomic_store(st, ST_INC | (uint64_t)(excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    goff[t] = ds + excl;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * 64;
    if (idx < n) {
      const uint32_t d = digit_of<K>(key[i], shift, mask);
      const uint32_t pos = wc[w][d] + rank[i];
      skey[pos] = key[i];
      sval[pos] = val[i];
    }
  }
  __syncthreads();
  const uint32_t cnt = (uint32_t)min((uint64_t)RS_TILE, (uint64_t)n - bbase);
  for (uint32_t j = t; j < cnt; j += RS_T) {
    const K k = skey[j];
    const uint32_t d = digit_of<K>(k, shift, mask);
    const uint32_t g = goff[d] + (j - lstart[d]);
    if (g < n) {
      kout[g] = k;
      vout[g] = sval[j];
    }
  }
}

// ------------------------------------------------------------- duplicate
struct DupArgs {
  const float4* rec0;    // record planes: (mu_x, mu_y, a, b), (c, beta, d), (..., log_thr)
  const float4* rec1;
  const float4* rec2;
  float alpha_min;
  int32_t tile_w, tile_h;
  const uint32_t* rect;
  const uint32_t* tiles;
  const float* depth;
  const uint32_t* block_off;
  const sgs_camera* cams;
  int64_t n;
  int32_t nbx;
  int32_t nb_total;
  uint32_t cap;
  uint64_t* keys64;      // mode 0
  uint32_t* keys32;      // mode 1
  uint32_t* vals;
  uint32_t* n_inst;
  const uint32_t* order; // mode 1: records in depth order
  const uint32_t* offs;  // mode 1: exclusive instance offset of order[j]
  int64_t m;
};

// Skew cut of a record from its stored plane 1 (beta, opacity factor d):
// the same value the preprocess used when it counted the record's tiles.
__device__ __forceinline__ float record_zcut(const DupArgs& a, float4 q1) {
  if (q1.y == 0.0f && q1.z == 0.0f) return -1e30f;
  return skew_zcut(a.alpha_min, q1.w);
}

// Mode 0: records in index order; block (bx, v) covers records v*N + bx*256 + t.
__global__ void __launch_bounds__(256) k_duplicate64(DupArgs a) {
  __shared__ uint32_t ws[4];
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t m = (int64_t)v * a.n + i;
  const uint32_t cnt = i < a.n ? a.tiles[m] : 0u;
  const uint32_t off = a.block_off[(int64_t)v * a.nbx + blockIdx.x] + block_excl_scan256(cnt, ws);
  if (v == 0 && blockIdx.x == 0 && threadIdx.x == 0) *a.n_inst = a.block_off[a.nb_total];
  if (cnt == 0) return;
  const uint2 r = reinterpret_cast<const uint2*>(a.rect)[m];
  const int x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
  const sgs_camera& cam = a.cams[v];
  const uint64_t lo = (uint64_t)__float_as_uint(a.depth[m]);
  const float4 q0 = a.rec0[m], q1 = a.rec1[m], q2 = a.rec2[m];
  const float zc = record_zcut(a, q1);
  uint32_t k = off;
  for (int y = y0; y < y1; ++y) {
    int c0, c1;
    row_span(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, zc, y, a.tile_w, a.tile_h, x0, x1, c0, c1);
    for (int x = c0; x < c1 && k < off + cnt; ++x, ++k)
      if (k < a.cap) {
        const uint64_t tile = (uint64_t)(cam.tile_base + y * cam.tiles_x + x);
        a.keys64[k] = (tile << 32) | lo;
        a.vals[k] = (uint32_t)m;
      }
  }
}

// Mode 1, step 1: depth keys of all records (culled ones sort last).
__global__ void __launch_bounds__(256) k_depth_keys(const float* __restrict__ depth,
                                                    const uint32_t* __restrict__ tiles, int64_t m,
                                                    uint32_t* __restrict__ k, uint32_t* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  k[i] = tiles[i] ? __float_as_uint(depth[i]) : 0xffffffffu;
  v[i] = (uint32_t)i;
}

// Mode 1, step 2: per-block sums of tile counts in depth order.
__global__ void __launch_bounds__(256) k_sorted_block_sums(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ tiles,
                                                           int64_t m, uint32_t* __restrict__ sums) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t o = j < m ? order[j] : 0u;
  uint32_t c = (j < m && o < (uint64_t)m) ? tiles[o] : 0u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  __shared__ uint32_t ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Mode 1, step 3: exclusive instance offset of every record in depth order.
__global__ void __launch_bounds__(256) k_sorted_offsets(const uint32_t* __restrict__ order,
                                                        const uint32_t* __restrict__ tiles, int64_t m,
                                                        const uint32_t* __restrict__ block_off,
                                                        int64_t nb, uint32_t* __restrict__ offs,
                                                        uint32_t* __restrict__ n_inst) {
  __shared__ uint32_t ws[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t o = j < m ? order[j] : 0u;
  const uint32_t c = (j < m && o < (uint64_t)m) ? tiles[o] : 0u;
  const uint32_t e = block_excl_scan256(c, ws);
  if (j < m) offs[j] = block_off[blockIdx.x] + e;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_inst = block_off[nb];
}

// Mode 1, step 4: load-balanced expansion.  Block b writes instances
// [b*EX_TILE, (b+1)*EX_TILE).  Records in depth order with at least one tile
// come first (culled ones sort last), so the records that own this range are
// at most EX_TILE + 1 consecutive entries starting at the last record whose
// offset is <= the first instance; their offsets and ids are staged in LDS
// and each thread walks its EX_PT consecutive instances.
constexpr int EX_PT = 8;
constexpr int EX_TILE = 256 * EX_PT;

__global__ void __launch_bounds__(256) k_expand32(DupArgs a) {
  __shared__ uint32_t s_off[EX_TILE + 1];
  __shared__ uint32_t s_rec[EX_TILE + 1];
  __shared__ uint32_t s_j0, s_w;
  const uint32_t total = *a.n_inst;
  const uint32_t n = total < a.cap ? total : a.cap;
  const uint64_t o0 = (uint64_t)blockIdx.x * EX_TILE;
  if (o0 >= n) return;
  const int t = threadIdx.x;
  if (t == 0) {
    // last j with offs[j] <= o0 (offs is non-decreasing, offs[0] = 0)
    uint64_t lo = 0, hi = (uint64_t)a.m;   // offs[lo] <= o0, answer in [lo, hi)
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (a.offs[mid] <= o0) lo = mid; else hi = mid;
    }
    s_j0 = (uint32_t)lo;
    s_w = (uint32_t)min((uint64_t)(EX_TILE + 1), (uint64_t)a.m - lo);
  }
  __syncthreads();
  const uint32_t j0 = s_j0, W = s_w;
  for (uint32_t k = t; k < W; k += 256) {
    s_off[k] = a.offs[j0 + k];
    s_rec[k] = a.order[j0 + k];
  }
  __syncthreads();
  uint64_t o = o0 + (uint64_t)t * EX_PT;
  if (o >= n) return;
  // first record of this thread: last k with s_off[k] <= o
  uint32_t lo = 0, hi = W;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s_off[mid] <= o) lo = mid; else hi = mid;
  }
  uint32_t k = lo;
  uint32_t rec = 0xffffffffu, tb = 0, tx = 0, cum = 0;
  int x0 = 0, x1 = 0, y1 = 0, row = 0, c0 = 0, c1 = 0;
  float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
  float zc = -1e30f;
  for (int e = 0; e < EX_PT; ++e, ++o) {
    if (o >= n) break;
    while (k + 1 < W && s_off[k + 1] <= o) ++k;
    if (s_rec[k] != rec) {
      rec = s_rec[k];
      const uint64_t rm = rec < (uint64_t)a.m ? rec : 0;
      const uint2 r = reinterpret_cast<const uint2*>(a.rect)[rm];
      x0 = r.x & 0xffffu;
      x1 = r.y & 0xffffu;
      row = r.x >> 16;
      y1 = r.y >> 16;
      q0 = a.rec0[rm];
      q1 = a.rec1[rm];
      q2 = a.rec2[rm];
      const sgs_camera& cam = a.cams[rm / (uint64_t)a.n];
      tb = (uint32_t)cam.tile_base;
      tx = (uint32_t)cam.tiles_x;
      cum = 0;
      zc = record_zcut(a, q1);
      row_span(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, zc, row, a.tile_w, a.tile_h, x0, x1, c0, c1);
    }
    // instance q of this record: walk the rows of its rect until q falls in one
    const uint32_t q = (uint32_t)(o - s_off[k]);
    while (q >= cum + (uint32_t)(c1 - c0) && row + 1 < y1) {
      cum += (uint32_t)(c1 - c0);
      ++row;
      row_span(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, zc, row, a.tile_w, a.tile_h, x0, x1, c0, c1);
    }
    const uint32_t x = min((uint32_t)(c0 + (q - cum)), (uint32_t)max(x1 - 1, 0));
    a.keys32[o] = tb + (uint32_t)row * tx + x;
    a.vals[o] = rec;
  }
}

// 64-bit keys from sorted tile keys and the record depths (mode 1, optional).
__global__ void __launch_bounds__(256) k_make_keys64(const uint32_t* __restrict__ tk,
                                                     const uint32_t* __restrict__ vals,
                                                     const float* __restrict__ depth, uint64_t m,
                                                     const uint32_t* n_dev, uint32_t cap,
                                                     uint64_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count_of(n_dev, 0, cap)) return;
  const uint32_t v = vals[i];
  out[i] = ((uint64_t)tk[i] << 32) | (v < m ? (uint64_t)__float_as_uint(depth[v]) : 0ull);
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename K>
__global__ void __launch_bounds__(256) k_tile_ranges(const K* __restrict__ keys, int shift,
                                                     const uint32_t* n_dev, uint32_t cap,
                                                     uint32_t total_tiles,
                                                     uint32_t* __restrict__ ranges) {
  // each boundary between two different tiles ends one range and starts the next
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t n = count_of(n_dev, 0, cap);
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> shift);
  if (i == 0 && t < total_tiles) ranges[2 * (uint64_t)t] = 0u;
  const uint32_t tn = i + 1 < n ? (uint32_t)(keys[i + 1] >> shift) : 0xffffffffu;
  if (tn != t) {
    if (t < total_tiles) ranges[2 * (uint64_t)t + 1] = (uint32_t)(i + 1);
    if (tn < total_tiles) ranges[2 * (uint64_t)tn] = (uint32_t)(i + 1);
  }
}

// Keys that order tiles by decreasing list length (16 bits, saturating).
__global__ void __launch_bounds__(256) k_tile_len_keys(const uint32_t* __restrict__ ranges,
                                                       uint32_t total_tiles,
                                                       uint32_t* __restrict__ k,
                                                       uint32_t* __restrict__ v) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= total_tiles) return;
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  k[t] = 0xffffu - min(len, 0xffffu);
  v[t] = t;
}

// ------------------------------------------------------------------ host side
static inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
static int rs_passes(int bits) { return (bits + 7) / 8; }
static uint64_t rs_blocks(uint64_t cap) { return std::max<uint64_t>(1, cdiv(cap, RS_TILE)); }

// Scratch of one sort of up to `cap` keys, laid out contiguously so that one
// fill zeroes it: digit histograms [8][256] u32, look-back status words
// [8][blocks][256] u64, then block counters [8] and an error word.
static size_t rs_hist_words() { return (size_t)RS_MAX_PASSES * 256; }
static size_t rs_status_words(uint64_t cap) { return (size_t)RS_MAX_PASSES * rs_blocks(cap) * 256 * 2; }
static size_t rs_scratch_bytes(uint64_t cap) {
  return (rs_hist_words() + rs_status_words(cap) + 64) * 4;
}

struct RsScratch {
  uint32_t* ghist;
  uint64_t* status;
  uint32_t* counters;   // [RS_MAX_PASSES] block counters, error word at [RS_MAX_PASSES]
};

static RsScratch rs_carve(char* p, uint64_t cap) {
  RsScratch s;
  s.ghist = reinterpret_cast<uint32_t*>(p);
  s.status = reinterpret_cast<uint64_t*>(p + rs_hist_words() * 4);
  s.counters = reinterpret_cast<uint32_t*>(p + (rs_hist_words() + rs_status_words(cap)) * 4);
  return s;
}

// Sorts (k[src], v[src]) by bits [0, bits), one kernel per 8-bit pass,
// alternating buffers; the result is in buffer (src + passes) % 2.
template <typename K>
static sgs_status radix_sort(K* kb[2], uint32_t* vb[2], int src, const uint32_t* n_dev,
                             uint32_t n_host, uint64_t cap, int bits, RsScratch sc, hipStream_t s) {
  const uint64_t blocks = rs_blocks(cap);
  const int passes = rs_passes(bits);
  // zero the histograms and the status words of the passes used
  const uint64_t zw = rs_hist_words() + (uint64_t)passes * blocks * 256 * 2;
  k_fill_u32<<<(unsigned)cdiv(zw, 256), 256, 0, s>>>(sc.ghist, zw, 0u);
  SGS_LAUNCH_CHECK();
  k_fill_u32<<<1, 256, 0, s>>>(sc.counters, 64, 0u);
  SGS_LAUNCH_CHECK();
  k_os_hist<K><<<(unsigned)blocks, RS_T, 0, s>>>(kb[src], n_dev, n_host, (uint32_t)cap, bits, sc.ghist);
  SGS_LAUNCH_CHECK();
  int cur = src;
  for (int p = 0; p < passes; ++p) {
    const int nb = std::min(8, bits - 8 * p);
    k_os_pass<K><<<(unsigned)blocks, RS_T, 0, s>>>(
        kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n_dev, n_host, (uint32_t)cap, 8 * p, nb,
        sc.ghist + p * 256, sc.status + (size_t)p * blocks * 256, sc.counters + p,
        sc.counters + RS_MAX_PASSES);
    SGS_LAUNCH_CHECK();
    cur ^= 1;
  }
  return SGS_OK;
}

static int tile_bits(int64_t total_tiles) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) < total_tiles) ++b;
  return std::max(b, 1);
}

static uint64_t rs_capacity(int64_t m, int64_t cap, int64_t total_tiles, int mode) {
  return std::max<uint64_t>(std::max<uint64_t>((uint64_t)cap, mode == 1 ? (uint64_t)m : 0),
                            (uint64_t)total_tiles);
}

size_t bin_sort_scratch_bytes(int64_t m, int64_t cap, int64_t total_tiles, int mode) {
  const uint64_t rs_cap = rs_capacity(m, cap, total_tiles, mode);
  size_t bytes = align_up(rs_scratch_bytes(rs_cap));
  bytes += 3 * align_up((size_t)total_tiles * 4);            // tile-order keys x2, vals alt
  if (mode == 0) {
    bytes += align_up((size_t)cap * 8) + align_up((size_t)cap * 4);
  } else {
    bytes += 4 * align_up((size_t)m * 4);                    // depth keys/vals x2
    bytes += align_up((cdiv(m, 256) + 1) * 4);               // sorted block offsets
    bytes += align_up((size_t)m * 4);                        // per-record offsets
    bytes += 2 * align_up((size_t)cap * 4) + align_up((size_t)cap * 4);  // tile keys x2, vals alt
  }
  return bytes + 256;
}

sgs_status launch_bin_sort(const sgs_geom* g, int64_t m, int64_t n, const sgs_camera* cams_dev,
                           int32_t n_views, int64_t total_tiles, const sgs_options* opt,
                           int64_t cap, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           uint32_t* n_inst, uint32_t* tile_order, void* scratch, hipStream_t s) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(scratch) + 255) & ~(uintptr_t)255);
  auto take = [&](size_t bytes) { char* r = p; p += align_up(bytes); return r; };
  const int mode = opt->sort_mode;
  const uint64_t rs_cap = rs_capacity(m, cap, total_tiles, mode);
  RsScratch sc = rs_carve(take(rs_scratch_bytes(rs_cap)), rs_cap);
  uint32_t* ok[2] = {reinterpret_cast<uint32_t*>(take((size_t)total_tiles * 4)),
                     reinterpret_cast<uint32_t*>(take((size_t)total_tiles * 4))};
  uint32_t* ov[2] = {tile_order, reinterpret_cast<uint32_t*>(take((size_t)total_tiles * 4))};
  // tiles by decreasing list length (after the ranges are known)
  auto order_tiles = [&]() -> sgs_status {
    if (!tile_order) return SGS_OK;
    k_tile_len_keys<<<(unsigned)cdiv(total_tiles, 256), 256, 0, s>>>(ranges, (uint32_t)total_tiles, ok[0], ov[0]);
    SGS_LAUNCH_CHECK();
    return radix_sort<uint32_t>(ok, ov, 0, nullptr, (uint32_t)total_tiles, (uint64_t)total_tiles, 16, sc, s);
  };
  const int tb = tile_bits(total_tiles);
  k_fill_u32<<<(unsigned)cdiv(2 * total_tiles, 256), 256, 0, s>>>(ranges, 2 * (uint64_t)total_tiles, 0u);
  SGS_LAUNCH_CHECK();
  DupArgs a = {};
  const uint64_t mm = (uint64_t)m;
  a.rec0 = reinterpret_cast<const float4*>(g->rec);
  a.rec1 = a.rec0 + mm;
  a.rec2 = a.rec0 + 2 * mm;
  a.tile_w = opt->tile_w;
  a.tile_h = opt->tile_h;
  a.alpha_min = opt->alpha_min;
  a.rect = g->rect;
  a.tiles = g->tiles;
  a.depth = g->depth;
  a.cams = cams_dev;
  a.n = n;
  a.nbx = (int32_t)cdiv(n, 256);
  a.cap = (uint32_t)cap;
  a.vals = vals;
  a.n_inst = n_inst;
  a.m = m;
  if (mode == 0) {
    const int bits = 32 + tb;
    const int passes = rs_passes(bits);
    uint64_t* kalt = reinterpret_cast<uint64_t*>(take((size_t)cap * 8));
    uint32_t* valt = reinterpret_cast<uint32_t*>(take((size_t)cap * 4));
    uint64_t* kb[2] = {keys, kalt};
    uint32_t* vb[2] = {vals, valt};
    const int src = passes & 1;             // so that the result lands in buffer 0
    a.block_off = g->block_off;
    a.nb_total = a.nbx * n_views;
    a.keys64 = kb[src];
    a.vals = vb[src];
    if (n > 0) {
      k_duplicate64<<<dim3(a.nbx, n_views), 256, 0, s>>>(a);
      SGS_LAUNCH_CHECK();
    } else {
      k_fill_u32<<<1, 256, 0, s>>>(n_inst, 1, 0u);
      SGS_LAUNCH_CHECK();
    }
    if (cap > 0) {
      sgs_status st = radix_sort<uint64_t>(kb, vb, src, n_inst, 0, (uint64_t)cap, bits, sc, s);
      if (st != SGS_OK) return st;
      k_tile_ranges<uint64_t><<<(unsigned)cdiv(cap, 256), 256, 0, s>>>(keys, 32, n_inst, (uint32_t)cap,
                                                                      (uint32_t)total_tiles, ranges);
      SGS_LAUNCH_CHECK();
    }
    return order_tiles();
  }
  // mode 1
  uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(take((size_t)m * 4)), reinterpret_cast<uint32_t*>(take((size_t)m * 4))};
  uint32_t* dv[2] = {reinterpret_cast<uint32_t*>(take((size_t)m * 4)), reinterpret_cast<uint32_t*>(take((size_t)m * 4))};
  const uint64_t nbs = cdiv(m, 256);
  uint32_t* sbo = reinterpret_cast<uint32_t*>(take((nbs + 1) * 4));
  uint32_t* offs = reinterpret_cast<uint32_t*>(take((size_t)m * 4));
  uint32_t* tk[2] = {reinterpret_cast<uint32_t*>(take((size_t)cap * 4)), reinterpret_cast<uint32_t*>(take((size_t)cap * 4))};
  uint32_t* valt = reinterpret_cast<uint32_t*>(take((size_t)cap * 4));
  if (m == 0) {
    k_fill_u32<<<1, 256, 0, s>>>(n_inst, 1, 0u);
    SGS_LAUNCH_CHECK();
    return order_tiles();
  }
  k_depth_keys<<<(unsigned)nbs, 256, 0, s>>>(g->depth, g->tiles, m, dk[0], dv[0]);
  SGS_LAUNCH_CHECK();
  sgs_status st = radix_sort<uint32_t>(dk, dv, 0, nullptr, (uint32_t)m, (uint64_t)m, 32, sc, s);
  if (st != SGS_OK) return st;
  const uint32_t* order = dv[rs_passes(32) & 1];
  k_sorted_block_sums<<<(unsigned)nbs, 256, 0, s>>>(order, g->tiles, m, sbo);
  SGS_LAUNCH_CHECK();
  st = launch_scan_blocks(sbo, sbo, (int64_t)nbs, s);
  if (st != SGS_OK) return st;
  k_sorted_offsets<<<(unsigned)nbs, 256, 0, s>>>(order, g->tiles, m, sbo, (int64_t)nbs, offs, n_inst);
  SGS_LAUNCH_CHECK();
  const int passes = rs_passes(tb);
  const int src = passes & 1;
  uint32_t* vb[2] = {vals, valt};
  a.order = order;
  a.offs = offs;
  a.keys32 = tk[src];
  a.vals = vb[src];
  if (cap > 0) {
    k_expand32<<<(unsigned)cdiv(cap, EX_TILE), 256, 0, s>>>(a);
    SGS_LAUNCH_CHECK();
    st = radix_sort<uint32_t>(tk, vb, src, n_inst, 0, (uint64_t)cap, tb, sc, s);
    if (st != SGS_OK) return st;
    k_tile_ranges<uint32_t><<<(unsigned)cdiv(cap, 256), 256, 0, s>>>(tk[0], 0, n_inst, (uint32_t)cap,
                                                                      (uint32_t)total_tiles, ranges);
    SGS_LAUNCH_CHECK();
    if (keys) {
      k_make_keys64<<<(unsigned)cdiv(cap, 256), 256, 0, s>>>(tk[0], vals, g->depth, (uint64_t)m, n_inst,
                                                              (uint32_t)cap, keys);
      SGS_LAUNCH_CHECK();
    }
  }
  return order_tiles();
}

}  // namespace sgs
