// Tile binning: one instance per (record, covered tile), a stable LSD radix
// sort by (global tile, depth), and per-tile ranges of the sorted list.
//
// Radix sort (hand-written, stable, 8-bit digits, 256-thread blocks of
// 4096 keys): per pass an upsweep writes each block's digit histogram, three
// small kernels turn the [blocks][256] histograms into exclusive scatter
// offsets, and a downsweep ranks keys inside each wave with 8 ballots per
// key (wave64 multisplit; lanes of one wave hold consecutive keys, so the
// rank is stable), stages the block's keys in digit order in LDS and writes
// them out so consecutive lanes write consecutive addresses.
//
// Two orders of work give the same sorted list (by tile, then depth, then
// record index):
//   mode 0: 64-bit keys (tile << 32 | depth bits) sorted over 32 + tile bits;
//   mode 1: the M records are first sorted by depth (32-bit keys), instances
//           are written in that order with 32-bit tile keys, which are then
//           sorted over the tile bits only (stable, so depth order and index
//           order within a tile survive).  Far fewer bytes move.
#include <algorithm>

#include "sgs_dev.h"

namespace sgs {

sgs_status launch_scan_blocks(const uint32_t* in, uint32_t* out, int64_t nb, hipStream_t s);

constexpr int RS_T = 256;          // threads per block
constexpr int RS_IPT = 16;         // keys per thread
constexpr int RS_TILE = RS_T * RS_IPT;

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

template <typename K>
__global__ void __launch_bounds__(RS_T) k_rs_upsweep(const K* __restrict__ keys,
                                                     const uint32_t* n_dev, uint32_t n_host,
                                                     uint32_t cap, int shift, uint32_t mask,
                                                     int nbits, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int k = t; k < 1024; k += RS_T) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint32_t n = count_of(n_dev, n_host, cap);
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)w * (RS_IPT * 64) + lane;
  const uint64_t lt = lanemask_lt();
  for (int i = 0; i < RS_IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * 64;
    const bool valid = idx < n;
    const uint32_t d = valid ? digit_of<K>(keys[idx], shift, mask) : 0u;
    const uint64_t peers = match_digit(d, valid, nbits);
    if (valid && (peers & lt) == 0) h[w][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  hist[(uint64_t)blockIdx.x * 256 + t] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

// Column sums of `group` histogram rows per group -> part[g][256].
__global__ void __launch_bounds__(256) k_rs_scan_a(const uint32_t* __restrict__ hist, uint32_t rows,
                                                   uint32_t group, uint32_t* __restrict__ part) {
  const uint32_t g = blockIdx.x, d = threadIdx.x;
  const uint32_t r0 = g * group, r1 = min(rows, r0 + group);
  uint32_t s = 0;
  for (uint32_t r = r0; r < r1; ++r) s += hist[(uint64_t)r * 256 + d];
  part[(uint64_t)g * 256 + d] = s;
}

// part[g][d] -> digit start + exclusive prefix over groups.
__global__ void __launch_bounds__(256) k_rs_scan_b(uint32_t* __restrict__ part, uint32_t groups) {
  __shared__ uint32_t ws[4];
  const uint32_t d = threadIdx.x, lane = d & 63, w = d >> 6;
  uint32_t run = 0;
  for (uint32_t g = 0; g < groups; ++g) {
    const uint32_t x = part[(uint64_t)g * 256 + d];
    part[(uint64_t)g * 256 + d] = run;
    run += x;
  }
  uint32_t inc = run;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off);
    if ((int)lane >= off) inc += y;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t start = inc - run;
  for (uint32_t k = 0; k < w; ++k) start += ws[k];
  for (uint32_t g = 0; g < groups; ++g) part[(uint64_t)g * 256 + d] += start;
}

// In place: hist[r][d] -> exclusive global scatter offset of digit d, block r.
__global__ void __launch_bounds__(256) k_rs_scan_c(uint32_t* __restrict__ hist, uint32_t rows,
                                                   uint32_t group, const uint32_t* __restrict__ part) {
  const uint32_t g = blockIdx.x, d = threadIdx.x;
  const uint32_t r0 = g * group, r1 = min(rows, r0 + group);
  uint32_t run = part[(uint64_t)g * 256 + d];
  for (uint32_t r = r0; r < r1; ++r) {
    const uint32_t x = hist[(uint64_t)r * 256 + d];
    hist[(uint64_t)r * 256 + d] = run;
    run += x;
  }
}

template <typename K>
__global__ void __launch_bounds__(RS_T) k_rs_downsweep(const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       const uint32_t* n_dev, uint32_t n_host,
                                                       uint32_t cap, int shift, uint32_t mask,
                                                       int nbits, const uint32_t* __restrict__ offs) {
  __shared__ uint32_t wc[4][256];
  __shared__ uint32_t lstart[256];
  __shared__ uint32_t wsum[4];
  __shared__ K skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  const uint32_t n = count_of(n_dev, n_host, cap);
  const uint64_t bbase = (uint64_t)blockIdx.x * RS_TILE;
  if (bbase >= n) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int k = t; k < 1024; k += RS_T) (&wc[0][0])[k] = 0;
  __syncthreads();
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
  {
    const uint32_t c0 = wc[0][t], c1 = wc[1][t], c2 = wc[2][t], c3 = wc[3][t];
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t inc = tot;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t ls = inc - tot;
    for (int k = 0; k < w; ++k) ls += wsum[k];
    lstart[t] = ls;
    wc[0][t] = ls;
    wc[1][t] = ls + c0;
    wc[2][t] = ls + c0 + c1;
    wc[3][t] = ls + c0 + c1 + c2;
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
  const uint32_t* ob = offs + (uint64_t)blockIdx.x * 256;
  for (uint32_t j = t; j < cnt; j += RS_T) {
    const K k = skey[j];
    const uint32_t d = digit_of<K>(k, shift, mask);
    const uint32_t g = ob[d] + (j - lstart[d]);
    if (g < n) {
      kout[g] = k;
      vout[g] = sval[j];
    }
  }
}

// ------------------------------------------------------------- duplicate
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
  return e;
}

struct DupArgs {
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
  int64_t m;
};

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
  const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
  const sgs_camera& cam = a.cams[v];
  const uint64_t lo = (uint64_t)__float_as_uint(a.depth[m]);
  uint32_t k = off;
  for (uint32_t y = y0; y < y1; ++y)
    for (uint32_t x = x0; x < x1; ++x, ++k)
      if (k < a.cap) {
        const uint64_t tile = (uint64_t)(cam.tile_base + y * cam.tiles_x + x);
        a.keys64[k] = (tile << 32) | lo;
        a.vals[k] = (uint32_t)m;
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
  uint32_t c = j < m ? tiles[order[j]] : 0u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  __shared__ uint32_t ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Mode 1, step 3: instances in depth order with 32-bit tile keys.
__global__ void __launch_bounds__(256) k_duplicate32(DupArgs a) {
  __shared__ uint32_t ws[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t mrec = j < a.m ? a.order[j] : 0u;
  if (mrec >= (uint64_t)a.m) mrec = 0u;
  const uint32_t cnt = j < a.m ? a.tiles[mrec] : 0u;
  const uint32_t off = a.block_off[blockIdx.x] + block_excl_scan256(cnt, ws);
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_inst = a.block_off[a.nb_total];
  if (cnt == 0) return;
  const int v = (int)(mrec / (uint64_t)a.n);
  const uint2 r = reinterpret_cast<const uint2*>(a.rect)[mrec];
  const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
  const sgs_camera& cam = a.cams[v];
  uint32_t k = off;
  for (uint32_t y = y0; y < y1; ++y)
    for (uint32_t x = x0; x < x1; ++x, ++k)
      if (k < a.cap) {
        a.keys32[k] = (uint32_t)(cam.tile_base + y * cam.tiles_x + x);
        a.vals[k] = mrec;
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
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t n = count_of(n_dev, 0, cap);
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> shift);
  if (t >= total_tiles) return;
  if (i == 0 || (uint32_t)(keys[i - 1] >> shift) != t) ranges[2 * (uint64_t)t] = (uint32_t)i;
  if (i + 1 == n || (uint32_t)(keys[i + 1] >> shift) != t) ranges[2 * (uint64_t)t + 1] = (uint32_t)(i + 1);
}

// ------------------------------------------------------------------ host side
static inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct RsScratch {
  uint32_t* hist;
  uint32_t* part;
};

static uint32_t rs_groups(uint64_t rows, uint32_t* group) {
  uint32_t g = (uint32_t)std::max<uint64_t>(64, cdiv(rows, 512));
  *group = g;
  return (uint32_t)std::max<uint64_t>(1, cdiv(rows, g));
}

static size_t rs_hist_entries(uint64_t cap) { return std::max<uint64_t>(1, cdiv(cap, RS_TILE)) * 256; }
// rs_groups never returns more than 512 groups (group >= rows/512), so the
// partials buffer has a fixed size.
static size_t rs_part_entries(uint64_t) { return (size_t)512 * 256; }

static int rs_passes(int bits) { return (bits + 7) / 8; }

// Sorts (k[src], v[src]) by bits [0, bits) in rs_passes(bits) passes,
// alternating buffers; the result is in buffer (src + passes) % 2.
template <typename K>
static sgs_status radix_sort(K* kb[2], uint32_t* vb[2], int src, const uint32_t* n_dev,
                             uint32_t n_host, uint64_t cap, int bits, RsScratch sc, hipStream_t s) {
  const uint64_t rows = std::max<uint64_t>(1, cdiv(cap, RS_TILE));
  uint32_t group;
  const uint32_t groups = rs_groups(rows, &group);
  int cur = src;
  for (int shift = 0; shift < bits; shift += 8) {
    const int nb = std::min(8, bits - shift);
    const uint32_t mask = (1u << nb) - 1u;
    k_rs_upsweep<K><<<(unsigned)rows, RS_T, 0, s>>>(kb[cur], n_dev, n_host, (uint32_t)cap, shift, mask, nb, sc.hist);
    SGS_LAUNCH_CHECK();
    k_rs_scan_a<<<groups, 256, 0, s>>>(sc.hist, (uint32_t)rows, group, sc.part);
    SGS_LAUNCH_CHECK();
    k_rs_scan_b<<<1, 256, 0, s>>>(sc.part, groups);
    SGS_LAUNCH_CHECK();
    k_rs_scan_c<<<groups, 256, 0, s>>>(sc.hist, (uint32_t)rows, group, sc.part);
    SGS_LAUNCH_CHECK();
    k_rs_downsweep<K><<<(unsigned)rows, RS_T, 0, s>>>(kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n_dev,
                                                      n_host, (uint32_t)cap, shift, mask, nb, sc.hist);
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

size_t bin_sort_scratch_bytes(int64_t m, int64_t cap, int64_t total_tiles, int mode) {
  size_t bytes = 0;
  const uint64_t rs_cap = std::max<uint64_t>((uint64_t)cap, mode == 1 ? (uint64_t)m : 0);
  bytes += align_up(rs_hist_entries(rs_cap) * 4) + align_up(rs_part_entries(rs_cap) * 4);
  if (mode == 0) {
    bytes += align_up((size_t)cap * 8) + align_up((size_t)cap * 4);
  } else {
    bytes += 4 * align_up((size_t)m * 4);                    // depth keys/vals x2
    bytes += align_up((cdiv(m, 256) + 1) * 4);               // sorted block offsets
    bytes += 2 * align_up((size_t)cap * 4) + align_up((size_t)cap * 4);  // tile keys x2, vals alt
  }
  return bytes + 256;
}

sgs_status launch_bin_sort(const sgs_geom* g, int64_t m, int64_t n, const sgs_camera* cams_dev,
                           int32_t n_views, int64_t total_tiles, const sgs_options* opt,
                           int64_t cap, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           uint32_t* n_inst, void* scratch, hipStream_t s) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(scratch) + 255) & ~(uintptr_t)255);
  auto take = [&](size_t bytes) { char* r = p; p += align_up(bytes); return r; };
  const int mode = opt->sort_mode;
  const uint64_t rs_cap = std::max<uint64_t>((uint64_t)cap, mode == 1 ? (uint64_t)m : 0);
  RsScratch sc;
  sc.hist = reinterpret_cast<uint32_t*>(take(rs_hist_entries(rs_cap) * 4));
  sc.part = reinterpret_cast<uint32_t*>(take(rs_part_entries(rs_cap) * 4));
  const int tb = tile_bits(total_tiles);
  // ranges start empty
  k_fill_u32<<<(unsigned)cdiv(2 * total_tiles, 256), 256, 0, s>>>(ranges, 2 * (uint64_t)total_tiles, 0u);
  SGS_LAUNCH_CHECK();
  DupArgs a;
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
    return SGS_OK;
  }
  // mode 1
  uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(take((size_t)m * 4)), reinterpret_cast<uint32_t*>(take((size_t)m * 4))};
  uint32_t* dv[2] = {reinterpret_cast<uint32_t*>(take((size_t)m * 4)), reinterpret_cast<uint32_t*>(take((size_t)m * 4))};
  const uint64_t nbs = cdiv(m, 256);
  uint32_t* sbo = reinterpret_cast<uint32_t*>(take((nbs + 1) * 4));
  uint32_t* tk[2] = {reinterpret_cast<uint32_t*>(take((size_t)cap * 4)), reinterpret_cast<uint32_t*>(take((size_t)cap * 4))};
  uint32_t* valt = reinterpret_cast<uint32_t*>(take((size_t)cap * 4));
  if (m == 0) {
    k_fill_u32<<<1, 256, 0, s>>>(n_inst, 1, 0u);
    SGS_LAUNCH_CHECK();
    return SGS_OK;
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
  const int passes = rs_passes(tb);
  const int src = passes & 1;
  uint32_t* vb[2] = {vals, valt};
  a.order = order;
  a.block_off = sbo;
  a.nb_total = (int32_t)nbs;
  a.keys32 = tk[src];
  a.vals = vb[src];
  k_duplicate32<<<(unsigned)nbs, 256, 0, s>>>(a);
  SGS_LAUNCH_CHECK();
  if (cap > 0) {
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
  return SGS_OK;
}

}  // namespace sgs
