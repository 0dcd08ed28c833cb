// Tile binning: one instance per (record, covered tile), a stable LSD radix
// sort by (global tile, depth), and per-tile ranges of the sorted list.
//
// Radix sort (hand-written, stable, digits of at most 8 bits spread evenly
// over the passes, 256-thread blocks of 4096 keys), one kernel per pass in
// the onesweep style (Adinets & Merrill 2022):
// a single histogram kernel reads the keys once and counts the digits of
// every pass; each pass kernel takes a block id from an atomic counter (so
// every lower id is already running), ranks its keys inside each wave64 with
// one ballot per digit bit (lanes hold consecutive keys, so ranks are stable),
// publishes its per-digit counts, and finds its global offsets by looking
// back over the published counts of the blocks before it (decoupled
// look-back, eight predecessors read at once).  The look-back spin is
// bounded: it never hangs; it flags an error word and marks the instance
// count invalid (0xffffffff) instead.  Keys are staged in LDS in digit order
// so that consecutive lanes write consecutive addresses.  All look-back
// state, histograms and block counters of one bin_sort call are zeroed by a
// single fill kernel at its start.
//
// Two orders of work give the same sorted list (by tile, then depth, then
// record index):
//   mode 0: 64-bit keys (tile << 32 | depth bits), written per record in
//           record order, sorted over 32 + tile bits;
//   mode 1: the M records are first sorted by depth (32-bit keys: the depth
//           buffer's own bits, all-ones for records without tiles, so those
//           sort last); a single-pass scan (decoupled look-back) gives each
//           record its instance offset in that order; the instances are
//           expanded in that order with 32-bit tile keys (load balanced: one
//           block per 2048 instances, not one thread per record), then
//           sorted over the tile bits only.  Stability keeps depth order and
//           index order inside a tile.  Far fewer bytes move.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sgs_dev.h"

namespace sgs {

constexpr int RS_T = 256;          // threads per block
// keys per thread (a template parameter of the kernels).  16 measured best
// from 0.3M to 50M keys: fewer, longer blocks keep look-back chains short
// (4 doubled the time of a pass over 1M keys).
constexpr int RS_IPT = 16;
// Instances per expansion block: EX_TILE for large capacities (one pass
// block's worth, measured best at 52M instances against 1024 and 2048),
// EX_TILE_S up to EX_SMALL_CAP, where fewer, longer blocks would leave most
// of the chip idle.  A block spans at most its tile + 1 records.
constexpr int EX_TILE = 4096;
constexpr int EX_TILE_S = 1024;
constexpr uint64_t EX_SMALL_CAP = (uint64_t)EX_TILE * EX_TILE;
static inline int ex_shift_for(uint64_t cap) { return cap <= EX_SMALL_CAP ? 10 : 12; }
static_assert((1 << 10) == EX_TILE_S && (1 << 12) == EX_TILE, "expansion tile shifts");
constexpr int EC = 64;             // expansion blocks per chunk of the count scan
// pass blocks: 1024 threads for sorts of at most this many blocks (their
// time is one block's latency), 512 for larger ones (measured: 256 threads
// ran 5% slower at 52M keys, 1024 slower still)
constexpr uint64_t RS_WIDE_MAX_BLOCKS = 4096;
constexpr int RS_MAX_PASSES = 8;
// pass grids: workgroups resident at once on 256 CUs (1024 threads: 2 per
// CU; 512 threads: 3 per CU, by LDS)
constexpr uint64_t RS_GRID_1024 = 512;
constexpr uint64_t RS_GRID_512 = 768;
constexpr uint64_t ST_AGG = 1ull << 32;    // status: block's own digit count
constexpr uint64_t ST_INC = 2ull << 32;    // status: inclusive prefix over blocks
constexpr uint32_t SPIN_LIMIT = 1u << 22;
// look-back: predecessor statuses read at once (a template parameter of the
// pass kernel; 8 measured best: 32 slowed both small and large sorts)
constexpr int LB_W = 8;
constexpr int HC = 64;             // copies of the digit histograms (atomic contention)
constexpr uint64_t HC_MIN_BLOCKS = 1024;   // fewer blocks: one copy, no final sum
constexpr uint32_t N_INVALID = 0xffffffffu;   // instance count after a failed look-back

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
  const uint32_t inc = wave_incl_scan(x);
  if (lane == 63) ws4[w] = inc;
  __syncthreads();
  uint32_t e = inc - x;
  for (int k = 0; k < w; ++k) e += ws4[k];
  __syncthreads();
  return e;
}

// Optional transform of the 32-bit keys the first pass (and the histogram)
// read, for depth keys: the depth buffer's bits of a positive float (a
// record with tiles, depth > near > 0) become key - base (base = the bits of
// the nearest near plane), clamped below lim; all-ones bits (records without
// tiles) become lim, so they still sort last.  The order of the keys is kept
// (the clamp only ties depths more than 2^127 times the nearest near plane
// distance, which do not occur), and they fit in 30 bits.  on = false: the
// identity.
struct KeyXf {
  uint32_t base, lim;
  bool on;
};

template <typename K>
__device__ __forceinline__ K xf_key(K k, const KeyXf& x) {
  if constexpr (sizeof(K) == 4) {
    if (x.on) {
      const uint32_t u = (uint32_t)k;
      return (K)(u == 0xffffffffu ? x.lim : min(u - x.base, x.lim - 1u));
    }
  }
  return k;
}

// Digit histograms of every pass in one read of the keys, added into copy
// (block % ncopies) of the partial histograms [ncopies][passes][DB]: many
// blocks adding into one set of DB words serialise on those addresses
// (ncopies = 1 adds straight into the final histograms).  DB: bins per
// digit (256, or 1024 for the wide digits of small depth sorts).
template <typename K, int RS_IPT, int DB = 256>
__global__ void __launch_bounds__(RS_T) k_os_hist(const K* __restrict__ keys, const uint32_t* n_dev,
                                                  uint32_t n_host, uint32_t cap, int passes,
                                                  int width, uint32_t* __restrict__ hpart,
                                                  int ncopies, KeyXf xf) {
  constexpr int MP = DB == 256 ? RS_MAX_PASSES : 4;
  __shared__ uint32_t h[MP][DB];
  const int t = threadIdx.x;
  const uint32_t dmask = (1u << width) - 1u;
  for (int k = t; k < MP * DB; k += RS_T) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint32_t n = count_of(n_dev, n_host, cap);
  constexpr int RS_TILE = RS_T * RS_IPT;
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  // all loads first (in flight together), then the LDS counts
  K key[RS_IPT];
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * RS_T + t;
    key[i] = idx < n ? xf_key<K>(keys[idx], xf) : (K)0;
  }
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    if (base + (uint64_t)i * RS_T + t < n)
      for (int p = 0; p < passes; ++p) atomicAdd(&h[p][digit_of<K>(key[i], width * p, dmask)], 1u);
  }
  __syncthreads();
  uint32_t* dst = hpart + (size_t)(blockIdx.x % (unsigned)ncopies) * passes * DB;
  for (int p = 0; p < passes; ++p)
    for (int d = t; d < DB; d += RS_T)
      if (h[p][d]) atomicAdd(&dst[p * DB + d], h[p][d]);
}

// Per-block digit counts cnt[e][256] of the expansion blocks, scanned in two
// levels: k_chunk_scan turns each chunk of EC consecutive blocks into
// exclusive prefixes within the chunk (one workgroup per chunk, one thread
// per digit) and stores the chunk totals; k_chunk_totals scans those.  The
// keys of digit d before block e number cnt[e][d] + tot[e / EC][d].  Only
// the blocks that hold keys (min(*count_p, cap) keys in blocks of 2^shift)
// have counts: the rest of the capacity's blocks are neither read nor
// written (no pass block reads them).
__global__ void __launch_bounds__(256) k_chunk_scan(uint32_t* __restrict__ cnt, uint32_t n,
                                                    uint32_t* __restrict__ tot,
                                                    const uint32_t* __restrict__ count_p, uint32_t cap,
                                                    int shift) {
  const uint32_t t = threadIdx.x, e0 = blockIdx.x * EC;
  const uint32_t c = *count_p;
  const uint64_t keys = c < cap ? c : cap;
  n = (uint32_t)min((uint64_t)n, (keys + (1ull << shift) - 1) >> shift);
  uint32_t x[EC];
#pragma unroll
  for (int i = 0; i < EC; ++i) x[i] = e0 + i < n ? cnt[(uint64_t)(e0 + i) * 256 + t] : 0u;
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < EC; ++i) {
    if (e0 + i < n) cnt[(uint64_t)(e0 + i) * 256 + t] = run;
    run += x[i];
  }
  tot[(uint64_t)blockIdx.x * 256 + t] = run;
}

// One workgroup per digit; thread t takes CT consecutive chunks of each
// group of 256 * CT.
constexpr int CT = 8;

__global__ void __launch_bounds__(256) k_chunk_totals(uint32_t* __restrict__ tot, uint32_t nch) {
  __shared__ uint32_t ws[4];
  const uint32_t d = blockIdx.x, t = threadIdx.x;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nch; base += 256 * CT) {
    const uint32_t c0 = base + t * CT;
    uint32_t x[CT], sum = 0;
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      x[i] = c0 + i < nch ? tot[(uint64_t)(c0 + i) * 256 + d] : 0u;
      sum += x[i];
    }
    uint32_t run = carry + block_excl_scan256(sum, ws);
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      if (c0 + i < nch) tot[(uint64_t)(c0 + i) * 256 + d] = run;
      run += x[i];
    }
    // the last thread's running value is the carry into the next group
    if (t == 255) ws[0] = run;
    __syncthreads();
    carry = ws[0];
    __syncthreads();
  }
}

// Sums the HC partial copies of the digit histograms: ghist[p][d], DB bins
// per pass (blockIdx.x = pass, blockIdx.y = group of 256 bins).
__global__ void __launch_bounds__(256) k_hist_final(const uint32_t* __restrict__ hpart, int passes,
                                                    int db, uint32_t* __restrict__ ghist) {
  const int p = blockIdx.x, d = blockIdx.y * 256 + threadIdx.x;
  uint32_t sum = 0;
  for (int c = 0; c < HC; ++c) sum += hpart[((size_t)c * passes + p) * db + d];
  ghist[p * db + d] = sum;
}

// vin == nullptr: the values are the input positions (0, 1, 2, ...).
// On a look-back that does not finish in bounded time: err |= 1 and, when
// n_fold is given, *n_fold = N_INVALID.
// ranges != nullptr (last pass over tile keys): every run of equal keys in
// the block's output lowers ranges[2 key] to its first position and raises
// ranges[2 key + 1] to its end (ranges start as [0xffffffff, 0)).
// pre != nullptr: no look-back; the keys of digit d before this block are
// counted by the scanned per-block counts of the expansion blocks that wrote
// the input (k_chunk_scan; the first pass of sort mode 1).
// One pass over RS_TILE keys per block of NT threads (NT / 64 waves, each
// ranking RS_TILE / NT keys per lane): 512 threads for large sorts, 1024 for
// small ones, where a block's latency (mostly the per-wave ranking rounds)
// is the pass time.
// DB: bins per digit; thread t < DB handles digit t (DB <= NT).  xf: the key
// transform applied where the first pass reads its keys (see KeyXf).
// LOOP: the grid is smaller than the block count and its workgroups loop
// over the block ids (without it each workgroup takes one id and the loop
// compiles away).
template <typename K, int NT, int LB_W, int DB = 256, bool LOOP = false>
__global__ void __launch_bounds__(NT) k_os_pass(const K* __restrict__ kin,
                                                const uint32_t* __restrict__ vin,
                                                K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                const uint32_t* n_dev, uint32_t n_host,
                                                uint32_t cap, int shift, int nbits,
                                                const uint32_t* __restrict__ ghist,
                                                uint64_t* status, uint32_t* counter,
                                                uint32_t* err, uint32_t* n_fold,
                                                uint32_t* ranges, uint32_t n_tiles,
                                                const uint32_t* __restrict__ pre,
                                                const uint32_t* __restrict__ pre_tot, KeyXf xf) {
  static_assert(DB <= NT && DB % 64 == 0, "one thread per digit bin");
  constexpr int NW = NT / 64;
  constexpr int RS_TILE = RS_T * RS_IPT;
  constexpr int IPT = RS_TILE / NT;
  __shared__ uint32_t wc[NW][DB];
  __shared__ uint32_t lstart[DB];
  __shared__ uint32_t lend[DB];
  __shared__ uint32_t goff[DB];
  __shared__ uint32_t ws[2 * (DB / 64)];
  __shared__ uint32_t s_bid;
  __shared__ K skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint32_t n = count_of(n_dev, n_host, cap);
  // the workgroups take block ids in order until the data ends (a grid
  // smaller than the block count loops; every id waited on is held by a
  // running workgroup)
  for (;;) {
  if (t == 0) s_bid = atomicAdd(counter, 1u);
  for (int k = t; k < NW * DB; k += NT) (&wc[0][0])[k] = 0;
  __syncthreads();
  const uint32_t b = s_bid;
  const uint64_t bbase = (uint64_t)b * RS_TILE;
  if (bbase >= n) break;   // ids past the data: no later block waits on them
  const uint32_t mask = (1u << nbits) - 1u;
  const uint64_t base = bbase + (uint64_t)w * (IPT * 64) + lane;
  const uint64_t lt = lanemask_lt();
  // this lane's keys are base + 64 i for i < nv (the valid ones)
  const int nv = base < n ? (int)min((uint64_t)IPT, (n - base + 63) / 64) : 0;
  const uint32_t gh = t < DB ? ghist[t] : 0u;   // keys of digit t in the whole input
  K key[IPT];
  uint32_t val[IPT];
  uint32_t rank[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint64_t idx = base + (uint64_t)i * 64;
    key[i] = i < nv ? xf_key<K>(kin[idx], xf) : (K)0;
    val[i] = i < nv ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
  }
  // rank inside the wave: the lowest lane of each digit's peers reserves
  // their slots with one LDS atomic (the atomics of the IPT rounds are in
  // flight together), then every lane fetches its leader's base
  // (rank holds the rank among the peers in its low 8 bits and the
  // leader's lane above them until the bases are fetched)
  uint32_t lead_base[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const bool valid = i < nv;
    const uint32_t d = digit_of<K>(key[i], shift, mask);
    const uint64_t peers = match_digit(d, valid, nbits);
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    rank[i] = r | ((uint32_t)(peers ? __builtin_ctzll(peers) : lane) << 8);
    lead_base[i] = 0;
    if (valid && r == 0) lead_base[i] = atomicAdd(&wc[w][d], (uint32_t)__popcll(peers));
  }
#pragma unroll
  for (int i = 0; i < IPT; ++i) rank[i] = (rank[i] & 255u) + __shfl(lead_base[i], (int)(rank[i] >> 8));
  __syncthreads();
  // digit t (threads 0..DB-1, the first DB/64 waves): block total, start in
  // the block, per-wave starts, and start in the output (scan of ghist)
  constexpr int DW = DB / 64;
  uint32_t cw[NW];
  uint32_t tot = 0, ls = 0, ds = 0;
  if (t < DB) {
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      cw[v] = wc[v][t];
      tot += cw[v];
    }
    const uint32_t il = wave_incl_scan(tot), ig = wave_incl_scan(gh);
    if (lane == 63) {
      ws[w] = il;
      ws[DW + w] = ig;
    }
    ls = il - tot;
    ds = ig - gh;
  }
  __syncthreads();
  const bool has_digit = t < (1 << nbits);   // (nbits <= log2 DB: implies t < DB)
  uint64_t* st = status + (uint64_t)b * DB + t;
  if (t < DB) {
    for (int k = 0; k < w; ++k) {
      ls += ws[k];
      ds += ws[DW + k];
    }
    lstart[t] = ls;
    lend[t] = ls + tot;
    uint32_t run = ls;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      wc[v][t] = run;
      run += cw[v];
    }
    // publish this block's count of digit t as early as possible (later
    // blocks' look-backs wait for it); threads past the last digit idle, and
    // a pass with precomputed offsets has no look-backs
    if (has_digit && !pre)
      __hip_atomic_store(st, (b == 0 ? ST_INC : ST_AGG) | (uint64_t)tot, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  // stage the block's keys in digit order (local ranks only)
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (i < nv) {
      const uint32_t d = digit_of<K>(key[i], shift, mask);
      const uint32_t pos = wc[w][d] + rank[i];
      skey[pos] = key[i];
      sval[pos] = val[i];
    }
  }
  // look back for the prefix over the blocks before this one
  if (t < DB && pre) {
    // offsets of this block's keys within each digit were scanned beforehand
    // (256-bin digits only)
    static_assert(RS_TILE % EX_TILE == 0, "a pass block covers whole expansion blocks");
    const uint64_t e = (uint64_t)b * (RS_TILE / EX_TILE);
    goff[t] = ds + pre[e * 256 + t] + pre_tot[(e / EC) * 256 + t];
  } else if (t < DB && (b == 0 || !has_digit)) {
    goff[t] = ds;
  } else if (t < DB) {
    // walk back LB_W predecessors at a time (their loads are in flight
    // together), summing published counts until an inclusive prefix
    uint32_t excl = 0, spins = 0;
    int64_t q0 = (int64_t)b - 1;
    bool done = false;
    while (!done) {
      uint64_t sw[LB_W];
#pragma unroll
      for (int k = 0; k < LB_W; ++k) {
        const int64_t q = q0 - k;
        sw[k] = q >= 0 ? __hip_atomic_load(status + (uint64_t)q * DB + t, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)
                       : ST_INC;   // block 0 publishes an inclusive prefix: never reached
      }
      int adv = 0;
      bool stop = false;
#pragma unroll
      for (int k = 0; k < LB_W; ++k) {
        if (!stop) {
          const uint64_t f = sw[k] & ~0xffffffffull;
          if (f == 0) {
            stop = true;             // not yet published: reload from here
          } else {
            excl += (uint32_t)sw[k];
            ++adv;
            if (f == ST_INC) stop = done = true;
          }
        }
      }
      q0 -= adv;
      if (!done && adv == 0) {
        if (++spins > SPIN_LIMIT) {
          atomicOr(err, 1u);
          if (n_fold) atomicExch(n_fold, N_INVALID);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(st, ST_INC | (uint64_t)(excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    goff[t] = ds + excl;
  }
  __syncthreads();
  const uint32_t cnt = (uint32_t)min((uint64_t)RS_TILE, (uint64_t)n - bbase);
  for (uint32_t j = t; j < cnt; j += NT) {
    const K k = skey[j];
    const uint32_t d = digit_of<K>(k, shift, mask);
    const uint32_t g = goff[d] + (j - lstart[d]);
    if (g < n) {
      kout[g] = k;
      vout[g] = sval[j];
      if (ranges && (uint64_t)k < n_tiles) {
        const uint32_t tile = (uint32_t)k;
        if (j == lstart[d] || skey[j - 1] != k) atomicMin(&ranges[2 * (uint64_t)tile], g);
        if (j + 1 == lend[d] || skey[j + 1] != k) atomicMax(&ranges[2 * (uint64_t)tile + 1], g + 1);
      }
    }
  }
  // a grid that covers every data block in its first round of ids takes no
  // second id (that would cost one more atomic round trip)
  if (!LOOP || (uint64_t)gridDim.x * RS_TILE >= n) break;
  __syncthreads();   // (LDS reused by the next block id)
  }
}

// ------------------------------------------------------------- duplicate
struct DupArgs {
  const float4* rec;     // [M][4] record slots: (mu_x, mu_y, a, b), (c, beta, d), (..., log_thr), ...
  float alpha_min;
  int32_t tile_w, tile_h;
  const uint32_t* rect;
  const uint32_t* tiles;
  const uint32_t* rows;  // mode 2: non-empty tile rows per record
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
  const uint32_t* bstart;  // mode 1: record owning the first instance of each expansion block
  uint32_t* hpart;       // mode 1: partial digit histograms [HC][hpasses][256] of the tile keys
  uint32_t* cnt0;        // mode 1: per-block counts of the first digit [gridDim][256]
  int32_t hpasses;       //         digits of hwidth bits, hcopies copies
  int32_t hwidth;
  int32_t hcopies;
  int32_t enhanced;      // 0: each record's rect is in its slot 3 (one line per record)
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
  const float4* rp = a.rec + 4 * (uint64_t)m;
  const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2];
  Span sp;
  span_setup(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, record_zcut(a, q1), sp);
  uint32_t k = off;
  for (int y = y0; y < y1; ++y) {
    int c0, c1;
    span_row(sp, y, a.tile_w, a.tile_h, x0, x1, c0, c1);
    for (int x = c0; x < c1 && k < off + cnt; ++x, ++k)
      if (k < a.cap) {
        const uint64_t tile = (uint64_t)(cam.tile_base + y * cam.tiles_x + x);
        a.keys64[k] = (tile << 32) | lo;
        a.vals[k] = (uint32_t)m;
      }
  }
}


// Modes 1 and 2, step 2: exclusive offset of every record in depth order of
// its count (mode 1: tiles, the instance offsets; mode 2: non-empty tile
// rows, the row-item offsets), one pass: each block of SO_TILE entries scans
// its counts, publishes its total and looks back over the published totals
// of the blocks before it, 64 at a time (one per lane of wave 0).  The block
// that takes the last id writes the total to *n_out (N_INVALID after a failed
// look-back, here or in the depth sort; saturated at 2^32 - 2); with
// inst_total (mode 2) it also writes *n_inst = *inst_total (the preprocess's
// instance count) under the same rule.  Each record also marks the expansion
// blocks whose first entry it owns: bstart[b] = its position.
constexpr int SO_IPT = 8;
constexpr int SO_TILE = 256 * SO_IPT;

__global__ void __launch_bounds__(256) k_sorted_offsets(const uint32_t* __restrict__ order,
                                                        const uint32_t* __restrict__ tiles,
                                                        int64_t m, uint32_t* __restrict__ offs,
                                                        uint32_t* __restrict__ n_out,
                                                        uint64_t* status, uint32_t* counter,
                                                        uint32_t* err, uint32_t* __restrict__ bstart,
                                                        uint32_t n_bstart, int ex_shift,
                                                        const uint32_t* __restrict__ inst_total,
                                                        uint32_t* __restrict__ n_inst) {
  constexpr uint64_t VMASK = (1ull << 62) - 1;   // 62-bit running totals, 2 flag bits
  constexpr uint64_t F_AGG = 1ull << 62, F_INC = 2ull << 62;
  __shared__ uint32_t ws[4];
  __shared__ uint32_t s_bid, s_tot;
  __shared__ uint64_t s_excl;
  const int t = threadIdx.x, lane = t & 63;
  if (t == 0) s_bid = atomicAdd(counter, 1u);
  __syncthreads();
  const uint32_t b = s_bid;
  const int64_t j0 = (int64_t)b * SO_TILE + (int64_t)t * SO_IPT;
  uint32_t c[SO_IPT];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SO_IPT; ++k) {
    const int64_t j = j0 + k;
    const uint32_t o = j < m ? order[j] : 0xffffffffu;
    c[k] = o < (uint64_t)m ? tiles[o] : 0u;
    sum += c[k];
  }
  const uint32_t e = block_excl_scan256(sum, ws);
  if (t == 255) s_tot = e + sum;
  __syncthreads();
  const uint64_t tot = s_tot;
  if (t < 64) {
    uint64_t excl = 0;
    uint64_t* st = status + b;
    if (b == 0) {
      if (t == 0) __hip_atomic_store(st, F_INC | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (t == 0) __hip_atomic_store(st, F_AGG | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int64_t q0 = (int64_t)b - 1;
      uint32_t spins = 0;
      for (;;) {
        const int64_t q = q0 - lane;
        const uint64_t sv = q >= 0 ? __hip_atomic_load(status + q, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                                   : F_INC;
        const uint64_t f = sv & ~VMASK;
        const uint64_t ready = __ballot(f != 0);
        const uint64_t inc = __ballot(f == F_INC);
        const int nr = ready == ~0ull ? 64 : __builtin_ctzll(~ready);   // ready prefix
        const int fi = inc ? __builtin_ctzll(inc) : 64;                  // first inclusive
        const int take = fi < nr ? fi + 1 : nr;
        uint64_t v = lane < take ? (sv & VMASK) : 0ull;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        excl += v;
        if (fi < nr) break;
        q0 -= take;
        if (take == 0) {
          if (++spins > SPIN_LIMIT) {
            if (lane == 0) {
              atomicOr(err, 1u);
              atomicExch(n_out, N_INVALID);
              if (inst_total) atomicExch(n_inst, N_INVALID);
            }
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (t == 0)
        __hip_atomic_store(st, F_INC | ((excl + tot) & VMASK), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (t == 0) s_excl = excl;
  }
  __syncthreads();
  uint64_t run = s_excl + e;
#pragma unroll
  for (int k = 0; k < SO_IPT; ++k) {
    const int64_t j = j0 + k;
    if (j < m) {
      offs[j] = (uint32_t)run;
      const uint64_t ext = 1ull << ex_shift;
      for (uint64_t bb = (run + ext - 1) >> ex_shift; (bb << ex_shift) < run + c[k] && bb < n_bstart; ++bb)
        bstart[bb] = (uint32_t)j;
    }
    run += c[k];
  }
  if (b == gridDim.x - 1 && t == 0) {
    const uint64_t total = s_excl + tot;
    const bool bad = *err != 0u;
    atomicMax(n_out, bad ? N_INVALID : (total < N_INVALID ? (uint32_t)total : N_INVALID - 1u));
    if (inst_total) atomicMax(n_inst, bad ? N_INVALID : min(*inst_total, N_INVALID - 1u));
  }
}

// Exclusive scan of one value per thread; *tot receives the block total.
__device__ __forceinline__ uint32_t block_scan256_total(uint32_t x, uint32_t* ws4, uint32_t* tot) {
  const uint32_t e = block_excl_scan256(x, ws4);
  if (threadIdx.x == 255) *tot = e + x;
  __syncthreads();
  return e;
}

// Mode 1, step 3: load-balanced expansion.  Block b writes instances
// [o0, o1) = [b*EXT, (b+1)*EXT).  Records in depth order with at least
// one tile come first (culled ones sort last), so the records that own this
// range are at most EXT + 1 consecutive entries starting at the record
// j0 that owns instance o0 (bstart[b], from the offsets kernel).  They are
// taken in chunks of 256: each thread gathers one record and sets up its
// span once, into LDS; then the chunk's (record, tile row) items are
// enumerated in order, 256 at a time, without global loads: each thread
// evaluates one row's span, a block scan turns the row counts into instance
// offsets (a running sum from offs[j0]: records' instances are their rows'
// in order), and each thread writes the instances of its row that fall in
// [o0, o1).
// The digit histograms of the tile-key sort are counted here as well: a
// row's instances have consecutive tile keys, so the low digit is counted
// per instance and every higher digit once per run of equal high bits.

template <int EXT>
__global__ void __launch_bounds__(256) k_expand32(DupArgs a) {
  constexpr int NSP = 13;                 // Span words per record
  __shared__ float s_sp[NSP][256];        // the chunk's records' spans (set up once each)
  __shared__ uint32_t s_r0[256], s_r1[256];   // rect corners (tx | ty << 16)
  __shared__ uint32_t s_rec[256];
  __shared__ uint32_t s_tb[256], s_tx[256];   // view's tile base and tiles per row
  __shared__ uint32_t s_rows[257];        // exclusive prefix of the chunk's records' rows
  __shared__ uint32_t s_e[256], s_k0[256], s_irec[256];   // items: output offset, first key, record
  __shared__ uint16_t s_map[EXT];         // item of each output of a round (block-relative)
  __shared__ uint32_t s_mark[256];        // owner marks of the current item round
  __shared__ uint32_t s_wmax[4];          // their per-wave maxima
  __shared__ uint32_t hist[4][256];
  __shared__ uint32_t ws[4];
  __shared__ uint32_t s_tot, s_j0, s_w;
  const uint32_t total = *a.n_inst;
  const uint32_t n = total < a.cap ? total : a.cap;
  const uint64_t o0 = (uint64_t)blockIdx.x * EXT;
  if (o0 >= n) return;   // no instances (and no counts: the scan stops before this block)
  const uint64_t o1 = min(o0 + (uint64_t)EXT, (uint64_t)n);
  const int t = threadIdx.x;
  const uint32_t dmask = (1u << a.hwidth) - 1u;
  for (int k = t; k < 4 * 256; k += 256) (&hist[0][0])[k] = 0u;
  if (t == 0) {
    // the record that owns instance o0 (marked by the offsets kernel)
    const uint64_t jlo = min((uint64_t)a.bstart[blockIdx.x], (uint64_t)a.m - 1);
    s_j0 = (uint32_t)jlo;
    s_w = (uint32_t)min((uint64_t)EXT + 1, (uint64_t)a.m - jlo);
  }
  __syncthreads();
  const uint32_t j0 = s_j0, W = s_w;
  uint64_t run = a.offs[j0];    // instance offset of the next item
  // records in chunks of 256: each thread sets up one record's span (its
  // loads are the chunk's only dependent gathers), then the chunk's (record,
  // tile row) items are enumerated from LDS, 256 at a time.  A record has
  // tiles when the next offset in depth order is larger than its own (the
  // last record's count is read directly), and its rect sits in its own
  // 64-byte line unless the records carry enhanced opacity: one gathered
  // line per record.
  for (uint32_t c = 0; c < W && run < o1; c += 256) {
    const uint32_t k = c + t;
    uint32_t rows = 0;
    if (k < W) {
      const uint64_t j = (uint64_t)j0 + k;
      const uint32_t rec = a.order[j];
      s_rec[t] = rec;
      const uint32_t off = a.offs[j];
      bool has = false;
      if ((k == 0 || off < o1) && rec < (uint64_t)a.m)
        has = j + 1 < (uint64_t)a.m ? a.offs[j + 1] > off : a.tiles[rec] > 0;
      if (has) {
        const float4* rp = a.rec + 4 * (uint64_t)rec;
        const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2];
        uint2 r;
        if (a.enhanced) {
          r = reinterpret_cast<const uint2*>(a.rect)[rec];
        } else {
          const float4 q3 = rp[3];
          r = make_uint2(__float_as_uint(q3.x), __float_as_uint(q3.y));
        }
        rows = (r.y >> 16) - min(r.x >> 16, r.y >> 16);
        s_r0[t] = r.x;
        s_r1[t] = r.y;
        Span sp;
        span_setup(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, record_zcut(a, q1), sp);
        s_sp[0][t] = sp.mx;  s_sp[1][t] = sp.my;  s_sp[2][t] = sp.b;   s_sp[3][t] = sp.det;
        s_sp[4][t] = sp.ia;  s_sp[5][t] = sp.aR2; s_sp[6][t] = sp.ey;  s_sp[7][t] = sp.ex;
        s_sp[8][t] = sp.yx;  s_sp[9][t] = sp.bx;  s_sp[10][t] = sp.by; s_sp[11][t] = sp.need;
        s_sp[12][t] = __uint_as_float((sp.ok ? 1u : 0u) | (sp.cut ? 2u : 0u));
        const sgs_camera& cam = a.cams[rec / (uint64_t)a.n];
        s_tb[t] = (uint32_t)cam.tile_base;
        s_tx[t] = (uint32_t)cam.tiles_x;
      }
    }
    const uint32_t e = block_scan256_total(rows, ws, &s_tot);
    s_rows[t] = e;
    if (t == 255) s_rows[256] = e + rows;
    __syncthreads();
    const uint32_t R = s_rows[256];
    for (uint32_t base = 0; base < R && run < o1; base += 256) {
      const uint32_t i = base + t;
      // record of item i: the last record of the chunk starting at or
      // before it; each record overlapping [base, base + 256) marks its
      // first item there (distinct positions), a block max-scan spreads them
      s_mark[t] = 0u;
      __syncthreads();
      if (rows > 0 && e < base + 256 && e + rows > base) s_mark[(e > base ? e : base) - base] = (uint32_t)t + 1u;
      __syncthreads();
      const uint32_t wm = wave_incl_max(s_mark[t]);
      if ((t & 63) == 63) s_wmax[t >> 6] = wm;
      __syncthreads();
      uint32_t own = wm;
      for (int q = 0; q < (t >> 6); ++q) own = max(own, s_wmax[q]);
      uint32_t cnt = 0, rec = 0, tk = 0;
      int c0 = 0;
      if (i < R) {
        const uint32_t lo = own - 1u;
        rec = s_rec[lo];
        Span sp;
        sp.mx = s_sp[0][lo];  sp.my = s_sp[1][lo];  sp.b = s_sp[2][lo];   sp.det = s_sp[3][lo];
        sp.ia = s_sp[4][lo];  sp.aR2 = s_sp[5][lo]; sp.ey = s_sp[6][lo];  sp.ex = s_sp[7][lo];
        sp.yx = s_sp[8][lo];  sp.bx = s_sp[9][lo];  sp.by = s_sp[10][lo]; sp.need = s_sp[11][lo];
        const uint32_t fl = __float_as_uint(s_sp[12][lo]);
        sp.ok = (fl & 1u) != 0u;
        sp.cut = (fl & 2u) != 0u;
        const uint32_t r0 = s_r0[lo];
        const int x0 = r0 & 0xffffu, x1 = s_r1[lo] & 0xffffu;
        const int row = (int)(r0 >> 16) + (int)(i - s_rows[lo]);
        int c1;
        span_row(sp, row, a.tile_w, a.tile_h, x0, x1, c0, c1);
        cnt = (uint32_t)(c1 - c0);
        tk = s_tb[lo] + (uint32_t)row * s_tx[lo];
      }
      const uint32_t e2 = block_scan256_total(cnt, ws, &s_tot);
      s_e[t] = e2;
      s_k0[t] = tk + (uint32_t)c0;
      s_irec[t] = rec;
      // the items' instances are one contiguous output range; its part in
      // [o0, o1) is [blo, bhi): each item marks its outputs there with its
      // index, then thread t writes every 256th output (coalesced)
      const uint64_t blo = max(run, o0), bhi = min(run + s_tot, o1);
      const uint64_t start = run + e2;
      const uint64_t lo2 = max(start, o0), hi2 = min(start + cnt, o1);
      if (hi2 > lo2)   // (blo <= lo2 < hi2 <= bhi, bhi - blo <= EXT)
        for (uint32_t r = (uint32_t)(lo2 - blo), rend = (uint32_t)(hi2 - blo); r < rend; ++r)
          s_map[r] = (uint16_t)t;
      __syncthreads();
      const uint32_t nout = bhi > blo ? (uint32_t)(bhi - blo) : 0u, rbase = (uint32_t)(blo - run);
      uint32_t* __restrict__ kb = a.keys32 + blo;
      uint32_t* __restrict__ vb = a.vals + blo;
      for (uint32_t r = t; r < nout; r += 256) {
        const uint32_t it = s_map[r];
        const uint32_t key = s_k0[it] + (rbase + r - s_e[it]);
        kb[r] = key;
        vb[r] = s_irec[it];
        atomicAdd(&hist[0][key & dmask], 1u);
      }
      // the higher digits once per run of equal high bits of each row
      const uint32_t tlo = tk + (uint32_t)c0 + (uint32_t)(lo2 - start);
      if (a.hpasses > 1 && hi2 > lo2) {
        const uint32_t thi = tlo + (uint32_t)(hi2 - lo2);
        for (uint32_t seg = tlo; seg < thi;) {
          const uint32_t end = min(thi, (seg | dmask) + 1u);
          for (int p = 1; p < a.hpasses; ++p)
            atomicAdd(&hist[p][(seg >> (a.hwidth * p)) & dmask], end - seg);
          seg = end;
        }
      }
      run += s_tot;
      __syncthreads();
    }
  }
  if (a.cnt0) a.cnt0[(uint64_t)blockIdx.x * 256 + t] = hist[0][t];
  uint32_t* hdst = a.hpart + (size_t)(blockIdx.x % (unsigned)a.hcopies) * a.hpasses * 256;
  for (int p = 0; p < a.hpasses; ++p)
    if (hist[p][t]) atomicAdd(&hdst[p * 256 + t], hist[p][t]);
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

// Fills up to ZL_MAX regions (words), one grid row per region: even words
// get ev[region], odd words 0 (ev = 0: plain zeroing).
constexpr int ZL_MAX = 8;
struct ZeroList {
  uint32_t* p[ZL_MAX];
  uint64_t n[ZL_MAX];
  uint32_t ev[ZL_MAX];
};

__global__ void __launch_bounds__(256) k_zero(ZeroList z) {
  uint32_t* p = z.p[blockIdx.y];
  const uint64_t n = z.n[blockIdx.y];
  const uint32_t ev = z.ev[blockIdx.y];
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    p[i] = (i & 1) ? 0u : ev;
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

// Tile order for the blend, longest lists first: one workgroup buckets the
// tiles by list length on a quarter-octave scale (bucket 0: empty) and
// writes them bucket by bucket, longest bucket first.  Inside a bucket the
// order is whatever the LDS atomics give: it only schedules work, every
// tile's pixels are computed the same way in any order.
constexpr int OT_BUCKETS = 128;

__device__ __forceinline__ int len_bucket(uint32_t len) {
  if (len == 0) return 0;
  const int lg = 31 - __clz((int)len);                          // floor(log2 len)
  const int frac = lg >= 2 ? (int)((len >> (lg - 2)) & 3u) : (int)((len << (2 - lg)) & 3u);
  return min(OT_BUCKETS - 1, 1 + 4 * lg + frac);
}

// Also rewrites empty ranges (start >= end, as the fused range writer leaves
// tiles without instances) to [0, 0).  order == nullptr: normalising only.
__global__ void __launch_bounds__(1024) k_order_tiles(uint32_t* __restrict__ ranges,
                                                      uint32_t total_tiles,
                                                      uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[OT_BUCKETS];
  __shared__ uint32_t pos[OT_BUCKETS];
  const uint32_t t = threadIdx.x;
  if (t < OT_BUCKETS) cnt[t] = 0;
  __syncthreads();
  for (uint32_t i = t; i < total_tiles; i += 1024) {
    const uint32_t a = ranges[2 * i], b = ranges[2 * i + 1];
    if (a >= b && (a | b) != 0u) {
      ranges[2 * i] = 0u;
      ranges[2 * i + 1] = 0u;
    }
    if (order) atomicAdd(&cnt[len_bucket(b > a ? b - a : 0u)], 1u);
  }
  if (!order) return;
  __syncthreads();
  // pos[k] = tiles in buckets above k (longest first): the first two waves
  // take one bucket per lane in descending order and scan; wave 1 adds
  // wave 0's total
  static_assert(OT_BUCKETS == 128, "two full waves scan the buckets");
  __shared__ uint32_t s_w0;
  uint32_t c = 0, inc = 0;
  if (t < OT_BUCKETS) {
    c = cnt[OT_BUCKETS - 1 - t];
    inc = wave_incl_scan(c);
    if (t == 63) s_w0 = inc;
  }
  __syncthreads();
  if (t < OT_BUCKETS) pos[OT_BUCKETS - 1 - t] = inc - c + (t >= 64 ? s_w0 : 0u);
  __syncthreads();
  for (uint32_t i = t; i < total_tiles; i += 1024) {
    const uint32_t a = ranges[2 * i], b = ranges[2 * i + 1];
    const uint32_t p = atomicAdd(&pos[len_bucket(b > a ? b - a : 0u)], 1u);
    if (p < total_tiles) order[p] = i;
  }
}

// ------------------------------------------------------ row binning (mode 2)
// Sort mode 2 moves row items instead of instances.  Each non-empty tile row
// of a record's rect becomes one item (global tile row, first column,
// width; record), emitted in the records' depth order; a stable radix sort
// by the row (one or two passes over at most 10 bits) groups the items by
// row with depth order kept inside a row; then each row's items, in pieces,
// place their record into the row's tiles.  Per tile the record list is the
// one the tile-key sort of mode 1 produces (depth order, record index among
// equal depths), in the same global positions.  At 1M Gaussians a record
// covers about 6.6 tiles per row, so about 7 times fewer entries are sorted.
//
// Item key: row | first column << 16 | (width - 1) << 24 (tiles_x <= 256 per
// view, at most 1024 rows per launch, at most 64 views: the host falls back
// to mode 1 otherwise).  Global rows number the views' tile rows view by
// view, so row order is tile order.
constexpr int RB_MAX_VIEWS = 64;
constexpr int RB_MAX_ROWS = 1024;
constexpr int RB_MAX_GRID = 2048;  // grid-stride blocks of the piece kernels
constexpr int RB_STG = 2048;       // staged placements per group of 256 items

__device__ __forceinline__ uint32_t item_row(uint32_t k) { return k & 0xffffu; }
__device__ __forceinline__ uint32_t item_x0(uint32_t k) { return (k >> 16) & 0xffu; }
__device__ __forceinline__ uint32_t item_w(uint32_t k) { return (k >> 24) + 1u; }

// Items per piece: 2^nb_shift, from the capacity (the per-piece column
// counts are sized by it: at most about 2048 pieces per 2^22 capacity,
// plus one partial piece per row).
static inline int nb_shift_for(uint64_t cap) {
  int sh = 8;
  while (sh < 11 && (cap >> sh) > 2048) ++sh;
  return sh;
}

// Mode 2, step 3: row items.  Block b owns items [b*EXT, (b+1)*EXT) of the
// depth-ordered item list (grid-stride over such emission blocks).  Its
// records, from the one owning item b*EXT on, go to the block's waves in
// chunks of 64 (wave w takes chunks w, w + 4, ...): a chunk's items are one
// contiguous output range starting at its first record's item offset, so a
// wave enumerates its chunk's (record, rect row) pairs 64 at a time on its
// own (each record's span in LDS, found by a max-scan of marks), and a pair
// whose row has tiles becomes one item at that offset plus the count of
// such pairs before it (a DPP scan).  Counts the row digits for the row
// sort (per block for the first pass) and the items of each row (row_cnt,
// R rows).
template <int EXT>
__global__ void __launch_bounds__(256) k_emit_rows(DupArgs a, const uint32_t* __restrict__ n_items_p,
                                                   uint32_t* __restrict__ row_cnt, int n_rows, int n_views,
                                                   uint32_t n_eblocks) {
  constexpr int NSP = 13;
  __shared__ float s_sp[NSP][256];        // per wave and lane: its record's span
  __shared__ uint32_t s_r0[256], s_r1[256];
  __shared__ uint32_t s_rec[256];
  __shared__ uint32_t s_grow[256];        // global row of the record's first rect row
  __shared__ uint32_t s_first[256];       // the record's first pair in its wave's chunk
  __shared__ uint32_t s_mark[4][64];
  __shared__ uint32_t s_vrb[RB_MAX_VIEWS];   // first global row of each view
  __shared__ uint32_t hist[2][256];
  __shared__ uint32_t s_rc[RB_MAX_ROWS];     // items per row
  __shared__ uint32_t s_j0, s_w;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t total = *n_items_p;
  const uint32_t n = total < a.cap ? total : a.cap;
  const uint32_t dmask = (1u << a.hwidth) - 1u;
  for (int k = t; k < n_rows; k += 256) s_rc[k] = 0u;
  for (int k = t; k < 2 * 256; k += 256) (&hist[0][0])[k] = 0u;
  if (t < 64) {
    const uint32_t ty = t < n_views ? (uint32_t)a.cams[t].tiles_y : 0u;
    s_vrb[t] = wave_incl_scan(ty) - ty;
  }
  // emission blocks eb = blockIdx.x, + gridDim.x, ...
  for (uint32_t eb = blockIdx.x; eb < n_eblocks; eb += gridDim.x) {
    const uint64_t o0 = (uint64_t)eb * EXT;
    if (o0 >= n) continue;   // no items (and no counts: the scan stops before this block)
    const uint64_t o1 = min(o0 + (uint64_t)EXT, (uint64_t)n);
    if (t == 0) {
      const uint64_t jlo = min((uint64_t)a.bstart[eb], (uint64_t)a.m - 1);
      s_j0 = (uint32_t)jlo;
      s_w = (uint32_t)min((uint64_t)EXT + 1, (uint64_t)a.m - jlo);
    }
    __syncthreads();
    const uint32_t j0 = s_j0, W = s_w;
    for (uint32_t c = 64u * (uint32_t)w; c < W; c += 256) {
      const uint32_t k = c + (uint32_t)lane;
      const uint64_t j = (uint64_t)j0 + k;
      uint32_t rows = 0, rec = 0, off = 0;
      bool has = false;
      if (k < W) {
        rec = a.order[j];
        off = a.offs[j];
        if ((k == 0 || off < o1) && rec < (uint64_t)a.m)
          has = j + 1 < (uint64_t)a.m ? a.offs[j + 1] > off : a.rows[rec] > 0;
      }
      // the chunk's first item offset (lane 0's record: k = c < W)
      uint64_t run = (uint32_t)__builtin_amdgcn_readfirstlane((int)off);
      if (run >= o1) break;   // this and every later chunk start past the block
      if (has) {
        const float4* rp = a.rec + 4 * (uint64_t)rec;
        const float4 q0 = rp[0], q1 = rp[1], q2 = rp[2];
        uint2 r;
        if (a.enhanced) {
          r = reinterpret_cast<const uint2*>(a.rect)[rec];
        } else {
          const float4 q3 = rp[3];
          r = make_uint2(__float_as_uint(q3.x), __float_as_uint(q3.y));
        }
        rows = (r.y >> 16) - min(r.x >> 16, r.y >> 16);
        s_r0[t] = r.x;
        s_r1[t] = r.y;
        Span sp;
        span_setup(q0.x, q0.y, q0.z, q0.w, q1.x, q2.w, q1.y, q1.z, record_zcut(a, q1), sp);
        s_sp[0][t] = sp.mx;  s_sp[1][t] = sp.my;  s_sp[2][t] = sp.b;   s_sp[3][t] = sp.det;
        s_sp[4][t] = sp.ia;  s_sp[5][t] = sp.aR2; s_sp[6][t] = sp.ey;  s_sp[7][t] = sp.ex;
        s_sp[8][t] = sp.yx;  s_sp[9][t] = sp.bx;  s_sp[10][t] = sp.by; s_sp[11][t] = sp.need;
        s_sp[12][t] = __uint_as_float((sp.ok ? 1u : 0u) | (sp.cut ? 2u : 0u));
        const uint32_t v = rec / (uint32_t)a.n;
        s_grow[t] = (v < RB_MAX_VIEWS ? s_vrb[v] : 0u) + (r.x >> 16);
      }
      s_rec[t] = rec;
      const uint32_t incl = wave_incl_scan(rows);
      const uint32_t first = incl - rows;
      s_first[t] = first;
      const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      __builtin_amdgcn_wave_barrier();
      for (uint32_t base = 0; base < R && run < o1; base += 64) {
        const uint32_t i = base + (uint32_t)lane;
        // the pair's record: the last of the chunk starting at or before it
        // (each record overlapping [base, base + 64) marks its first pair
        // there, at distinct positions)
        s_mark[w][lane] = 0u;
        __builtin_amdgcn_wave_barrier();
        if (rows > 0 && first < base + 64 && incl > base) s_mark[w][(first > base ? first : base) - base] = (uint32_t)lane + 1u;
        __builtin_amdgcn_wave_barrier();
        const uint32_t own = wave_incl_max(s_mark[w][lane]);
        __builtin_amdgcn_wave_barrier();
        uint32_t ne = 0, item = 0, irec = 0;
        if (i < R) {
          const uint32_t lo = 64u * (uint32_t)w + own - 1u;
          irec = s_rec[lo];
          Span sp;
          sp.mx = s_sp[0][lo];  sp.my = s_sp[1][lo];  sp.b = s_sp[2][lo];   sp.det = s_sp[3][lo];
          sp.ia = s_sp[4][lo];  sp.aR2 = s_sp[5][lo]; sp.ey = s_sp[6][lo];  sp.ex = s_sp[7][lo];
          sp.yx = s_sp[8][lo];  sp.bx = s_sp[9][lo];  sp.by = s_sp[10][lo]; sp.need = s_sp[11][lo];
          const uint32_t fl = __float_as_uint(s_sp[12][lo]);
          sp.ok = (fl & 1u) != 0u;
          sp.cut = (fl & 2u) != 0u;
          const uint32_t r0 = s_r0[lo];
          const int x0 = r0 & 0xffffu, x1 = s_r1[lo] & 0xffffu;
          const uint32_t dy = i - s_first[lo];
          int c0, c1;
          span_row(sp, (int)(r0 >> 16) + (int)dy, a.tile_w, a.tile_h, x0, x1, c0, c1);
          if (c1 > c0) {
            ne = 1;
            item = ((s_grow[lo] + dy) & 0xffffu) | ((uint32_t)c0 << 16) | ((uint32_t)(c1 - c0 - 1) << 24);
          }
        }
        const uint32_t inc2 = wave_incl_scan(ne);
        const uint64_t pos = run + (inc2 - ne);
        if (ne && pos >= o0 && pos < o1) {
          a.keys32[pos] = item;
          a.vals[pos] = irec;
          const uint32_t row = item_row(item);
          atomicAdd(&hist[0][row & dmask], 1u);
          if (a.hpasses > 1) atomicAdd(&hist[1][(row >> a.hwidth) & dmask], 1u);
          if (row < (uint32_t)n_rows) atomicAdd(&s_rc[row], 1u);
        }
        run += (uint32_t)__builtin_amdgcn_readlane((int)inc2, 63);
      }
      // (the wave's record slots are rewritten by its next chunk)
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (a.cnt0) a.cnt0[(uint64_t)eb * 256 + t] = hist[0][t];
    uint32_t* hdst = a.hpart + (size_t)(eb % (unsigned)a.hcopies) * a.hpasses * 256;
    for (int p = 0; p < a.hpasses; ++p) {
      if (hist[p][t]) atomicAdd(&hdst[p * 256 + t], hist[p][t]);
      hist[p][t] = 0u;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int k = t; k < n_rows; k += 256)
    if (s_rc[k]) atomicAdd(&row_cnt[k], s_rc[k]);
}

// The views' first global rows, tiles per row and first tiles, in LDS
// (wave 0 of the block loads them; n_views <= RB_MAX_VIEWS); the caller
// synchronises before use.
struct ViewTable {
  uint32_t rb[RB_MAX_VIEWS + 1], tx[RB_MAX_VIEWS], tb[RB_MAX_VIEWS];
};

__device__ __forceinline__ void load_views(const sgs_camera* cams, int n_views, ViewTable& vt) {
  const int t = threadIdx.x;
  if (t < 64) {
    const bool on = t < n_views;
    const uint32_t ty = on ? (uint32_t)cams[t].tiles_y : 0u;
    const uint32_t inc = wave_incl_scan(ty);
    vt.rb[t] = inc - ty;
    vt.tx[t] = on ? (uint32_t)cams[t].tiles_x : 0u;
    vt.tb[t] = on ? (uint32_t)cams[t].tile_base : 0u;
    if (t == 63) vt.rb[RB_MAX_VIEWS] = inc;
  }
}

// First tile of a global tile row and its view's tiles_x.
__device__ __forceinline__ void row_view(const ViewTable& vt, int n_views, uint32_t row, uint32_t& tile0,
                                         uint32_t& tx) {
  int lo = 0, hi = n_views;   // rb[lo] <= row < rb[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (vt.rb[mid] <= row) lo = mid; else hi = mid;
  }
  tx = vt.tx[lo];
  tile0 = vt.tb[lo] + (row - vt.rb[lo]) * tx;
}

// Pieces: each row's sorted items in runs of at most 2^nb_shift (rows
// without items have none).  ptab = [pp[0..R], rs[0..R]]: pp[r] the first
// piece of row r, rs[r] its first item (exclusive scans of the per-row
// piece and item counts); pp[R] pieces in all.  Built in LDS by every block
// of the counting kernel from the per-row item counts (R <= RB_MAX_ROWS).

__device__ __forceinline__ void piece_table(const uint32_t* __restrict__ row_cnt, int R, int nb_shift,
                                            uint32_t* pp, uint32_t* rs, uint32_t* ws4) {
  const int t = threadIdx.x;
  uint32_t ci[4], cp[4], si = 0, sp = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = t * 4 + k;
    ci[k] = r < R ? row_cnt[r] : 0u;
    cp[k] = (ci[k] + (1u << nb_shift) - 1) >> nb_shift;
    si += ci[k];
    sp += cp[k];
  }
  uint32_t ei = block_excl_scan256(si, ws4);
  uint32_t ep = block_excl_scan256(sp, ws4);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = t * 4 + k;
    if (r <= R) {
      pp[r] = ep;
      rs[r] = ei;
    }
    ep += cp[k];
    ei += ci[k];
  }
  if (t == 255 && R == RB_MAX_ROWS) {
    pp[R] = ep;
    rs[R] = ei;
  }
}

// Largest r <= R - 1 with pp[r] <= p (rows without pieces are skipped).
__device__ __forceinline__ uint32_t piece_row(const uint32_t* pp, int R, uint32_t p) {
  uint32_t lo = 0, hi = (uint32_t)R;   // pp[lo] <= p < pp[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pp[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Mode 2, step 5: per piece, the count of its items covering each of the
// 256 columns (LDS difference array over the columns, then a block scan);
// block 0 also stores the piece table for the next steps.
__global__ void __launch_bounds__(256) k_piece_count(const uint32_t* __restrict__ ik,
                                                     const uint32_t* __restrict__ row_cnt, int R, int nb_shift,
                                                     uint32_t* __restrict__ cntp, uint32_t* __restrict__ ptab) {
  __shared__ uint32_t pp[RB_MAX_ROWS + 1], rs[RB_MAX_ROWS + 1];
  __shared__ uint32_t D[257];
  __shared__ uint32_t ws[4];
  const int t = threadIdx.x;
  piece_table(row_cnt, R, nb_shift, pp, rs, ws);
  __syncthreads();
  if (blockIdx.x == 0)
    for (int r = t; r <= R; r += 256) {
      ptab[r] = pp[r];
      ptab[R + 1 + r] = rs[r];
    }
  const uint32_t P = pp[R];
  for (uint32_t p = blockIdx.x; p < P; p += gridDim.x) {
    const uint32_t r = piece_row(pp, R, p);
    const uint32_t s = rs[r] + ((p - pp[r]) << nb_shift);
    const uint32_t e = min(s + (1u << nb_shift), rs[r + 1]);
    D[t] = 0u;
    if (t == 0) D[256] = 0u;
    __syncthreads();
    for (uint32_t i = s + t; i < e; i += 256) {
      const uint32_t key = ik[i];
      const uint32_t x0 = item_x0(key), x1 = x0 + item_w(key);
      atomicAdd(&D[x0], 1u);
      atomicAdd(&D[min(x1, 256u)], 0xffffffffu);   // (-1; column 256 is never read)
    }
    __syncthreads();
    const uint32_t d = D[t];
    cntp[(uint64_t)p * 256 + t] = block_excl_scan256(d, ws) + d;
  }
}

// Mode 2, step 6: per (row, column), the counts of the row's pieces before
// each piece (pre_col) and the row's total (the tile's instance count).
// One block per row, one thread per column.
__global__ void __launch_bounds__(256) k_col_scan(const uint32_t* __restrict__ cntp,
                                                  const uint32_t* __restrict__ ptab, int R,
                                                  const sgs_camera* cams, int n_views,
                                                  uint32_t* __restrict__ pre_col, uint32_t* __restrict__ cnt_tile,
                                                  uint32_t n_tiles) {
  __shared__ ViewTable vt;
  load_views(cams, n_views, vt);
  const uint32_t r = blockIdx.x;
  const uint32_t c = threadIdx.x;
  const uint32_t p0 = ptab[r], p1 = ptab[r + 1];
  uint32_t run = 0;
  uint32_t p = p0;
  for (; p + 8 <= p1; p += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = cntp[(uint64_t)(p + k) * 256 + c];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      pre_col[(uint64_t)(p + k) * 256 + c] = run;
      run += v[k];
    }
  }
  for (; p < p1; ++p) {
    pre_col[(uint64_t)p * 256 + c] = run;
    run += cntp[(uint64_t)p * 256 + c];
  }
  __syncthreads();
  uint32_t t0, tx;
  row_view(vt, n_views, r, t0, tx);
  if (c < tx && (uint64_t)t0 + c < n_tiles) cnt_tile[t0 + c] = run;
}

// Mode 2, step 8: placement, one block per piece (grid-stride), its items
// in groups of 256 (one per thread, in order).  Within a group, wave w
// marks in LDS, per column, the lanes whose item starts there and those
// whose item ends there; OR prefixes over the columns turn them into the
// lanes covering each column, so an instance (item, column) ranks among the
// group's items by popcount (lanes below it in its wave, plus the earlier
// waves' counts).  Its position: the tile's start + the row's count before
// this piece + the earlier groups' count + that rank.  The group's
// placements are staged column by column in LDS and written out in that
// order (runs of consecutive positions); a group with more than RB_STG
// placements (or with keys requested) writes them directly.
template <int NCOL>
__global__ void __launch_bounds__(256) k_row_place(const uint32_t* __restrict__ ik, const uint32_t* __restrict__ iv,
                                                   const uint32_t* __restrict__ ptab, int R, int nb_shift,
                                                   const sgs_camera* cams, int n_views,
                                                   const uint32_t* __restrict__ pre_col,
                                                   const uint32_t* __restrict__ ranges, uint32_t n_tiles,
                                                   uint32_t cap, uint32_t* __restrict__ vals,
                                                   uint64_t* __restrict__ keys, const float* __restrict__ depth,
                                                   uint64_t m, const uint32_t* __restrict__ n_total) {
  // NCOL columns (128 or 256: at least the widest view's tiles per row);
  // per-column arrays are indexed by pc(c) = c + c / 32: lane l scans
  // columns CPL l .. CPL l + CPL - 1, which the padding spreads over the banks
  constexpr int CPL = NCOL / 64;
  constexpr int PC = NCOL + NCOL / 32;
  auto pc = [](uint32_t c) { return c + (c >> 5); };
  // (LDS sized for four workgroups per CU, five with 128 columns: the end
  // masks and the column counts share the staging area, and the piece table
  // takes only the launch's rows)
  __shared__ uint64_t S[4][PC];               // per wave: lanes whose item starts at / covers each column
  __shared__ uint2 BS[4][PC];                 // per wave and column: (staging base, global base)
  __shared__ union {
    uint2 st[RB_STG + 64];                    // staged placements (record, global position),
                                              // then one spare slot per lane
    struct {
      uint64_t e[4][PC];                      // per wave: lanes whose item ends at each column
      uint32_t cnt[4][PC];                    // per wave: covering lanes per column
    } c;                                      // (both before staging)
  } SG;
  __shared__ uint32_t ws[4];
  __shared__ uint32_t s_info[4];
  __shared__ uint32_t s_tot;
  extern __shared__ uint32_t pt[];            // the piece table, 2 (R + 1) words
  __shared__ ViewTable vt;
  auto& E = SG.c.e;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t P = ptab[R];
  // every position below the capacity (the usual case): the write-out
  // stores need no test
  const bool fits = *n_total <= cap;
  for (int k = t; k < 2 * (R + 1); k += 256) pt[k] = ptab[k];
  load_views(cams, n_views, vt);
#pragma unroll
  for (int q = 0; q < CPL; ++q) S[wv][pc(CPL * lane + q)] = 0ull;
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  uint32_t gb = 0;   // thread t < NCOL: next global position of column t in this piece
  // pieces in 8 contiguous chunks, one per XCD (workgroup i runs on XCD
  // i mod 8): neighbouring pieces, whose runs of a column abut in the
  // output, share an L2 and complete each other's lines there
  const uint32_t xcd = blockIdx.x & 7u, nx = gridDim.x >> 3;
  const uint32_t chunk = (P + 7) >> 3;
  const uint32_t pend = min((xcd + 1) * chunk, P);
  for (uint32_t p = xcd * chunk + (blockIdx.x >> 3); p < pend; p += nx) {
    if (t == 0) {
      const uint32_t r = piece_row(pt, R, p);
      const uint32_t s = pt[R + 1 + r] + ((p - pt[r]) << nb_shift);
      uint32_t t0, tx;
      row_view(vt, n_views, r, t0, tx);
      s_info[0] = s;
      s_info[1] = min(s + (1u << nb_shift), pt[R + 1 + r + 1]);
      s_info[2] = t0;
      s_info[3] = tx;
    }
    __syncthreads();
    const uint32_t s = s_info[0], e = s_info[1], t0 = s_info[2], tx = s_info[3];
    if (t < NCOL) {
      const bool ok = (uint32_t)t < tx && (uint64_t)t0 + t < n_tiles;
      gb = (ok ? ranges[2 * (uint64_t)(t0 + t)] : 0u) + pre_col[(uint64_t)p * 256 + t];
    }
    uint32_t nkey = s + t < e ? ik[s + t] : 0u;
    uint32_t nval = s + t < e ? iv[s + t] : 0u;
    for (uint32_t g0 = s; g0 < e; g0 += 256) {
      const uint32_t i = g0 + t;
      const bool valid = i < e;
      const uint32_t key = nkey, val = nval;
      {
        // the next group's items, in flight during this group
        const uint32_t i2 = i + 256;
        nkey = i2 < e ? ik[i2] : 0u;
        nval = i2 < e ? iv[i2] : 0u;
      }
      const uint32_t x0 = item_x0(key), w = valid ? item_w(key) : 0u;
      // (this wave's S row is zero here; its E row shares the staging area,
      // which every wave has finished reading, and is cleared first)
#pragma unroll
      for (int q = 0; q < CPL; ++q) E[wv][pc(CPL * lane + q)] = 0ull;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        atomicOr(reinterpret_cast<unsigned long long*>(&S[wv][pc(x0)]), 1ull << lane);
        if (x0 + w < (uint32_t)NCOL) atomicOr(reinterpret_cast<unsigned long long*>(&E[wv][pc(x0 + w)]), 1ull << lane);
      }
      __builtin_amdgcn_wave_barrier();
      {
        // inclusive OR prefixes over the columns (lane l: its CPL columns),
        // then cover = started & ~ended
        uint64_t a[CPL], b[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          a[q] = S[wv][pc(CPL * lane + q)];
          b[q] = E[wv][pc(CPL * lane + q)];
          if (q > 0) {
            a[q] |= a[q - 1];
            b[q] |= b[q - 1];
          }
        }
        // inclusive OR over the lanes' totals (DPP, per 32-bit half), then
        // the exclusive one from the lane below
        const uint64_t xa = ((uint64_t)wave_incl_or((uint32_t)(a[CPL - 1] >> 32)) << 32) |
                            wave_incl_or((uint32_t)a[CPL - 1]);
        const uint64_t xb = ((uint64_t)wave_incl_or((uint32_t)(b[CPL - 1] >> 32)) << 32) |
                            wave_incl_or((uint32_t)b[CPL - 1]);
        uint64_t pa = __shfl_up(xa, 1), pb = __shfl_up(xb, 1);
        if (lane == 0) pa = pb = 0ull;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          const uint64_t cov = (a[q] | pa) & ~(b[q] | pb);
          S[wv][pc(CPL * lane + q)] = cov;
          SG.c.cnt[wv][pc(CPL * lane + q)] = (uint32_t)__popcll(cov);
        }
      }
      __syncthreads();
      uint32_t c0 = 0, c1 = 0, c2 = 0, gc = 0;   // (threads past the columns: none)
      if (t < NCOL) {
        const uint32_t pt_ = pc(t);
        c0 = SG.c.cnt[0][pt_];
        c1 = SG.c.cnt[1][pt_];
        c2 = SG.c.cnt[2][pt_];
        gc = c0 + c1 + c2 + SG.c.cnt[3][pt_];
      }
      // staging start of column t: an exclusive scan over the columns (DPP
      // within each wave, the waves' totals through LDS)
      const uint32_t inc = wave_incl_scan(gc);
      if (lane == 63) ws[wv] = inc;
      __syncthreads();
      uint32_t gs = inc - gc;
      for (int q = 0; q < wv; ++q) gs += ws[q];
      const uint32_t T = ws[0] + ws[1] + ws[2] + ws[3];
      if (t < NCOL) {
        const uint32_t g = gb, pt_ = pc(t);
        BS[0][pt_] = make_uint2(gs, g);
        BS[1][pt_] = make_uint2(gs + c0, g + c0);
        BS[2][pt_] = make_uint2(gs + c0 + c1, g + c0 + c1);
        BS[3][pt_] = make_uint2(gs + c0 + c1 + c2, g + c0 + c1 + c2);
        gb = g + gc;
      }
      __syncthreads();
      // (block-uniform, tested once: two loops rather than a test per
      // column; four columns per step, their LDS reads in flight together)
      const bool stage = __builtin_amdgcn_readfirstlane(T) <= (uint32_t)RB_STG && !keys;
      if (stage) {
        for (uint32_t kk = 0; kk < w; kk += 4) {
          uint2 bs[4];
          uint64_t cv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = pc(min(x0 + kk + u, (uint32_t)NCOL - 1u));
            bs[u] = BS[wv][c];
            cv[u] = S[wv][c];
          }
          // (columns past the item's end go to the lane's spare slot: no
          // branch per column)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t rank = (uint32_t)__popcll(cv[u] & lt);
            const uint32_t slot = kk + u < w ? bs[u].x + rank : (uint32_t)RB_STG + (uint32_t)lane;
            SG.st[slot] = make_uint2(val, bs[u].y + rank);
          }
        }
      } else {
        for (uint32_t kk = 0; kk < w; kk += 4) {
          uint2 bs[4];
          uint64_t cv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = pc(min(x0 + kk + u, (uint32_t)NCOL - 1u));
            bs[u] = BS[wv][c];
            cv[u] = S[wv][c];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (kk + u < w) {
              const uint32_t rank = (uint32_t)__popcll(cv[u] & lt);
              if (bs[u].y + rank < cap) {
                vals[bs[u].y + rank] = val;
                if (keys)
                  keys[bs[u].y + rank] = ((uint64_t)(t0 + x0 + kk + u) << 32) |
                                         (val < m ? (uint64_t)__float_as_uint(depth[val]) : 0ull);
              }
            }
          }
        }
      }
      __syncthreads();
      if (stage && fits) {
        uint32_t q = t;
        for (; q + 768 < T; q += 1024) {
          uint2 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = SG.st[q + 256 * u];
#pragma unroll
          for (int u = 0; u < 4; ++u) vals[v[u].y] = v[u].x;
        }
        for (; q < T; q += 256) {
          const uint2 v = SG.st[q];
          vals[v.y] = v.x;
        }
      } else if (stage) {
        uint32_t q = t;
        for (; q + 768 < T; q += 1024) {
          uint2 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = SG.st[q + 256 * u];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (v[u].y < cap) vals[v[u].y] = v[u].x;
        }
        for (; q < T; q += 256) {
          const uint2 v = SG.st[q];
          if (v.y < cap) vals[v.y] = v.x;
        }
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q) S[wv][pc(CPL * lane + q)] = 0ull;
      __syncthreads();
    }
  }
}

// Mode 2, step 7: tile ranges from the tile counts (one workgroup): an
// exclusive scan, [start, end) clamped to the capacity, [0, 0) for empty
// tiles; with order, the tile order by decreasing count (as k_order_tiles).
__global__ void __launch_bounds__(1024) k_tile_scan(const uint32_t* __restrict__ cnt_tile, uint32_t T, uint32_t cap,
                                                    uint32_t* __restrict__ ranges, uint32_t* __restrict__ order) {
  __shared__ uint64_t wsum[16];
  __shared__ uint64_t carry_s;
  __shared__ uint32_t bcnt[OT_BUCKETS], bpos[OT_BUCKETS];
  __shared__ uint32_t s_w0;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) carry_s = 0;
  if (t < OT_BUCKETS) bcnt[t] = 0;
  __syncthreads();
  for (uint64_t base = 0; base < T; base += 4096) {
    uint32_t c[4];
    uint64_t v[4], loc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t idx = base + (uint64_t)t * 4 + k;
      c[k] = idx < T ? cnt_tile[idx] : 0u;
      v[k] = loc;
      loc += c[k];
    }
    uint64_t inc = loc;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
      const uint64_t s0 = lane < 16 ? wsum[lane] : 0ull;
      uint64_t wi = s0;
      for (int off = 1; off < 16; off <<= 1) {
        const uint64_t y = __shfl_up(wi, off);
        if (lane >= off) wi += y;
      }
      if (lane < 16) wsum[lane] = wi - s0;
    }
    __syncthreads();
    const uint64_t pre = carry_s + wsum[w] + inc - loc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t idx = base + (uint64_t)t * 4 + k;
      if (idx < T) {
        const uint64_t st = pre + v[k];
        const uint32_t a0 = c[k] ? (uint32_t)min(st, (uint64_t)cap) : 0u;
        const uint32_t a1 = c[k] ? (uint32_t)min(st + c[k], (uint64_t)cap) : 0u;
        ranges[2 * idx] = a0;
        ranges[2 * idx + 1] = a1;
        if (order) atomicAdd(&bcnt[len_bucket(c[k])], 1u);
      }
    }
    __syncthreads();
    if (t == 1023) carry_s = pre + loc;
    __syncthreads();
  }
  if (!order) return;
  static_assert(OT_BUCKETS == 128, "two full waves scan the buckets");
  uint32_t cb = 0, incb = 0;
  if (t < OT_BUCKETS) {
    cb = bcnt[OT_BUCKETS - 1 - t];
    incb = wave_incl_scan(cb);
    if (t == 63) s_w0 = incb;
  }
  __syncthreads();
  if (t < OT_BUCKETS) bpos[OT_BUCKETS - 1 - t] = incb - cb + (t >= 64 ? s_w0 : 0u);
  __syncthreads();
  for (uint32_t i = t; i < T; i += 1024) {
    const uint32_t p = atomicAdd(&bpos[len_bucket(cnt_tile[i])], 1u);
    if (p < T) order[p] = i;
  }
}

// ------------------------------------------------------------------ host side
static inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
// Passes of at most 8 bits (dbits = 10: 10 bits, for the wide digits of
// small depth sorts); the digit width spreads the bits evenly over them (13
// bits: 7 + 6, not 8 + 5): fewer digits per block, longer runs.
static int rs_passes(int bits, int dbits = 8) { return (bits + dbits - 1) / dbits; }
static int rs_width(int bits, int dbits = 8) {
  return (bits + rs_passes(bits, dbits) - 1) / rs_passes(bits, dbits);
}
static uint64_t rs_blocks(uint64_t cap) { return std::max<uint64_t>(1, cdiv(cap, (uint64_t)RS_T * RS_IPT)); }

// Scratch of one sort of up to `cap` keys in `passes` passes of db-bin
// digits, contiguous so that it is zeroed as one region: block counters [64]
// (one per pass), digit histograms [passes][db] u32, their partial copies
// [HC][passes][db] u32, look-back status [passes][blocks][db] u64.
static size_t rs_words(uint64_t cap, int passes, int db = 256) {
  return 64 + (size_t)passes * db * (1 + HC) + (size_t)passes * rs_blocks(cap) * db * 2;
}

struct RsScratch {
  uint32_t* counters;
  uint32_t* ghist;
  uint32_t* hpart;
  uint64_t* status;
  uint32_t* err;        // shared error word of the bin_sort call
  uint32_t* n_fold;     // instance count to mark N_INVALID on failure, or null
};

static RsScratch rs_carve(uint32_t* p, int passes, uint32_t* err, uint32_t* n_fold, int db = 256) {
  RsScratch s;
  s.counters = p;
  s.ghist = p + 64;
  s.hpart = s.ghist + (size_t)passes * db;
  s.status = reinterpret_cast<uint64_t*>(p + 64 + (size_t)passes * db * (1 + HC));
  s.err = err;
  s.n_fold = n_fold;
  return s;
}

// Sorts by bits [0, bits), one kernel per pass of rs_width(bits) bits.  Pass 0 reads
// (kin, vin) (vin == nullptr: values are the positions); the result lands in
// (kb[0], vb[0]).  kin may be kb[passes & 1] (sorting in place) or another
// buffer.  pre0: precomputed per-block digit offsets for the first pass (see
// k_os_pass).  The scratch must be zero, except that with hist_done the digit
// histograms already hold the counts of the keys: in the partial copies when
// the hist_blocks_done blocks that counted them exceed HC_MIN_BLOCKS, else in
// the final histograms.  With ranges, the last
// pass also writes the tile ranges of the sorted keys (see k_os_pass).
// DB = 1024 (10-bit digits) only for small sorts (at most RS_WIDE_MAX_BLOCKS
// blocks, 1024-thread pass blocks) without precomputed first-pass offsets;
// xf (32-bit keys) transforms the keys as the first pass and the histogram
// read them.
template <typename K, int DB = 256>
static sgs_status radix_sort(const K* kin, const uint32_t* vin, K* kb[2], uint32_t* vb[2],
                             const uint32_t* n_dev, uint32_t n_host, uint64_t cap, int bits,
                             RsScratch sc, hipStream_t s, bool hist_done = false,
                             uint64_t hist_blocks_done = 0, uint32_t* ranges = nullptr,
                             uint32_t n_tiles = 0, const uint32_t* pre0 = nullptr,
                             const uint32_t* pre0_tot = nullptr, KeyXf xf = KeyXf{0u, 0u, false}) {
  constexpr int DBITS = DB == 1024 ? 10 : 8;
  const uint64_t blocks = rs_blocks(cap);
  const int passes = rs_passes(bits, DBITS);
  const int width = rs_width(bits, DBITS);
  const uint64_t hist_blocks = hist_done ? hist_blocks_done : blocks;
  const bool copies = hist_blocks > HC_MIN_BLOCKS;
  if (DB != 256 && (blocks > RS_WIDE_MAX_BLOCKS || pre0 || hist_done)) return SGS_EINVAL;
  if (!hist_done) {
    // small sorts: twice as many blocks of 2048 keys (a block's LDS counts
    // of the few high digits that most keys share are serialised; 1024-key
    // blocks measured slower at 1M keys)
    if (blocks <= RS_WIDE_MAX_BLOCKS)
      k_os_hist<K, 8, DB><<<(unsigned)cdiv(cap, (uint64_t)RS_T * 8), RS_T, 0, s>>>(
          kin, n_dev, n_host, (uint32_t)cap, passes, width, copies ? sc.hpart : sc.ghist,
          copies ? HC : 1, xf);
    else
      k_os_hist<K, RS_IPT, DB><<<(unsigned)blocks, RS_T, 0, s>>>(kin, n_dev, n_host, (uint32_t)cap,
                                                                  passes, width,
                                                                  copies ? sc.hpart : sc.ghist,
                                                                  copies ? HC : 1, xf);
    SGS_LAUNCH_CHECK();
  }
  if (copies) {
    k_hist_final<<<dim3(passes, DB / 256), 256, 0, s>>>(sc.hpart, passes, DB, sc.ghist);
    SGS_LAUNCH_CHECK();
  }
  const KeyXf none = {0u, 0u, false};
  for (int p = 0; p < passes; ++p) {
    const int nb = std::min(width, bits - width * p);
    const int dst = (passes - 1 - p) & 1;
    const K* ki = p == 0 ? kin : kb[dst ^ 1];
    const uint32_t* vi = p == 0 ? vin : vb[dst ^ 1];
    // (grids of at most the workgroups that fit at once: they loop over
    // the block ids, so a capacity far above the count costs no launches)
#define SGS_PASS_ARGS(D)                                                                          \
  ki, vi, kb[dst], vb[dst], n_dev, n_host, (uint32_t)cap, width * p, nb, sc.ghist + p * (D),        \
      sc.status + (size_t)p * blocks * (D), sc.counters + p, sc.err, sc.n_fold,                     \
      p == passes - 1 ? ranges : nullptr, n_tiles, p == 0 ? pre0 : nullptr, pre0_tot, p == 0 ? xf : none
    if (blocks <= RS_WIDE_MAX_BLOCKS) {
      if (blocks <= RS_GRID_1024)
        k_os_pass<K, 1024, LB_W, DB, false><<<(unsigned)blocks, 1024, 0, s>>>(SGS_PASS_ARGS(DB));
      else
        k_os_pass<K, 1024, LB_W, DB, true><<<(unsigned)RS_GRID_1024, 1024, 0, s>>>(SGS_PASS_ARGS(DB));
    } else if constexpr (DB == 256) {
      k_os_pass<K, 512, LB_W, 256, true><<<(unsigned)std::min<uint64_t>(blocks, RS_GRID_512), 512, 0, s>>>(
          SGS_PASS_ARGS(256));
    }
#undef SGS_PASS_ARGS
    SGS_LAUNCH_CHECK();
  }
  return SGS_OK;
}

static int tile_bits(int64_t total_tiles) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) < total_tiles) ++b;
  return std::max(b, 1);
}

// Layout of the scratch of one bin_sort call.  Computed from a base address
// (0 to size it): every buffer is 256-byte aligned.
struct BinLayout {
  uint32_t* misc;                 // [64]: error word at 0
  uint32_t* rs_main;              // main sort (64-bit keys, or tile keys)
  int main_passes;
  uint32_t* rs_depth;             // mode 1: depth presort
  uint32_t* so_status;            // mode 1: offsets scan: [64] counter, then u64 status
  size_t so_words;
  uint64_t* kalt;                 // mode 0: alternate 64-bit keys
  uint32_t* valt;                 // alternate values
  uint32_t* dk[2];                // mode 1: depth keys
  uint32_t* dv[2];                // mode 1: record order
  uint32_t* offs;                 // mode 1: per-record instance offsets
  uint32_t* bstart;               // mode 1: first record of each expansion block
  uint64_t n_bstart;              //         (= number of expansion blocks)
  uint32_t* cnt0;                 // mode 1: [expansion blocks][256] first-digit counts
  uint32_t* ctot;                 // mode 1: [chunks][256] their chunk totals
  uint32_t* tk[2];                // mode 1: tile keys; mode 2: row items
  uint32_t* cntp;                 // mode 2: per piece, items covering each column [pieces][256]
  uint32_t* pre_col;              // mode 2: the row's count before each piece [pieces][256]
  uint32_t* ptab;                 // mode 2: piece table [2][RB_MAX_ROWS + 1]
  uint32_t* cnt_tile;             // mode 2: instances per tile [T], then items per row [RB_MAX_ROWS]
  size_t bytes;
};

static BinLayout bin_layout(uintptr_t base, int64_t m, int64_t cap, int64_t total_tiles, int mode) {
  BinLayout L = {};
  uintptr_t p = (base + 255) & ~(uintptr_t)255;
  const uintptr_t p0 = p;
  auto take = [&](size_t bytes) { uintptr_t r = p; p += align_up(bytes); return r; };
  const uint64_t T = (uint64_t)total_tiles, C = (uint64_t)cap, M = (uint64_t)m;
  const int tb = tile_bits(total_tiles);
  // (mode 2 sorts row items over at most 16 bits: room for 2 passes, or
  // for the tile-key passes of mode 1 when it falls back)
  L.main_passes = rs_passes(mode == 0 ? 32 + tb : tb);
  if (mode == 2) L.main_passes = std::max(L.main_passes, 2);
  L.misc = reinterpret_cast<uint32_t*>(take(64 * 4));
  L.rs_main = reinterpret_cast<uint32_t*>(take(rs_words(C, L.main_passes) * 4));
  if (mode == 0) {
    L.kalt = reinterpret_cast<uint64_t*>(take(C * 8));
    L.valt = reinterpret_cast<uint32_t*>(take(C * 4));
  } else {
    // depth presort: 4 passes of 8-bit digits, or 3 of 10 bits (room for either)
    L.rs_depth = reinterpret_cast<uint32_t*>(take(std::max(rs_words(M, 4), rs_words(M, 3, 1024)) * 4));
    L.so_words = 64 + 2 * (size_t)cdiv(std::max<uint64_t>(M, 1), SO_TILE);
    L.so_status = reinterpret_cast<uint32_t*>(take(L.so_words * 4));
    for (int k = 0; k < 2; ++k) {
      L.dk[k] = reinterpret_cast<uint32_t*>(take(M * 4));
      L.dv[k] = reinterpret_cast<uint32_t*>(take(M * 4));
      L.tk[k] = reinterpret_cast<uint32_t*>(take(C * 4));
    }
    L.offs = reinterpret_cast<uint32_t*>(take(M * 4));
    L.n_bstart = std::max<uint64_t>(cdiv(C, 1ull << ex_shift_for(C)), 1);
    L.bstart = reinterpret_cast<uint32_t*>(take(L.n_bstart * 4));
    if (cdiv(C, (uint64_t)RS_T * RS_IPT) > RS_WIDE_MAX_BLOCKS) {
      L.cnt0 = reinterpret_cast<uint32_t*>(take(L.n_bstart * 256 * 4));
      L.ctot = reinterpret_cast<uint32_t*>(take(cdiv(L.n_bstart, EC) * 256 * 4));
    }
    L.valt = reinterpret_cast<uint32_t*>(take(C * 4));
    if (mode == 2) {
      const uint64_t pieces = cdiv(C, 1ull << nb_shift_for(C)) + RB_MAX_ROWS;
      L.cntp = reinterpret_cast<uint32_t*>(take(pieces * 256 * 4));
      L.pre_col = reinterpret_cast<uint32_t*>(take(pieces * 256 * 4));
      L.ptab = reinterpret_cast<uint32_t*>(take(2 * (RB_MAX_ROWS + 1) * 4));
      L.cnt_tile = reinterpret_cast<uint32_t*>(take((T + RB_MAX_ROWS) * 4));
    }
  }
  L.bytes = (size_t)(p - p0) + 256;
  return L;
}

size_t bin_sort_scratch_bytes(int64_t m, int64_t cap, int64_t total_tiles, int mode) {
  return bin_layout(0, m, cap, total_tiles, mode).bytes;
}

// Wide (10-bit) depth digits: for depth sorts of at most RS_WIDE_MAX_BLOCKS
// blocks, when every view's near plane is positive.  The keys, transformed
// by KeyXf with base = the bits of the nearest near plane, take 30 bits: 3
// passes instead of 4.
static bool wide_depth(uint64_t m, float near_min) {
  return m > 0 && rs_blocks(m) <= RS_WIDE_MAX_BLOCKS && near_min > 0.0f && std::isfinite(near_min);
}
constexpr int DEPTH_BITS_WIDE = 30;

// Sort mode 2 after the depth presort (see the row binning kernels).
static sgs_status bin_rows(const sgs_geom* g, DupArgs a, const BinLayout& L, const RsScratch& sc_main,
                           const uint32_t* order, int64_t m, int32_t n_views, const sgs_camera* cams_dev,
                           uint64_t T, uint64_t C, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           uint32_t* n_inst, uint32_t* tile_order, int32_t rb_rows, int32_t rb_tx,
                           hipStream_t s) {
  uint32_t* err = L.misc;
  uint32_t* n_items = L.misc + 1;   // row items (zeroed with misc)
  uint32_t* row_cnt = L.cnt_tile + T;
  const uint64_t mm = (uint64_t)m;
  const int ex_shift = ex_shift_for(C);
  const int nb_shift = nb_shift_for(C);
  const int R = rb_rows;
  const uint64_t nb_total = (uint64_t)a.nbx * (uint64_t)n_views;
  k_sorted_offsets<<<(unsigned)cdiv(mm, SO_TILE), 256, 0, s>>>(
      order, g->rows, m, L.offs, n_items, reinterpret_cast<uint64_t*>(L.so_status + 64), L.so_status, err,
      L.bstart, (uint32_t)L.n_bstart, ex_shift, g->block_off + nb_total, n_inst);
  SGS_LAUNCH_CHECK();
  const int rbits = tile_bits(R);
  const int rpasses = rs_passes(rbits);
  uint32_t* ik[2] = {L.tk[0], L.tk[1]};
  uint32_t* iv[2] = {L.valt, vals};   // sorted items land in (tk[0], valt); vals is free until the placement
  const int src = rpasses & 1;
  a.order = order;
  a.offs = L.offs;
  a.bstart = L.bstart;
  a.rows = g->rows;
  a.keys32 = ik[src];
  a.vals = iv[src];
  const uint64_t ex_blocks = cdiv(C, 1ull << ex_shift);
  a.hcopies = ex_blocks > HC_MIN_BLOCKS ? HC : 1;
  a.hpart = a.hcopies > 1 ? sc_main.hpart : sc_main.ghist;
  const bool scan0 = cdiv(C, (uint64_t)RS_T * RS_IPT) > RS_WIDE_MAX_BLOCKS;
  a.cnt0 = scan0 ? L.cnt0 : nullptr;
  a.hpasses = rpasses;
  a.hwidth = rs_width(rbits);
  const unsigned pgrid = (unsigned)std::min<uint64_t>(cdiv(C, 1ull << nb_shift) + (uint64_t)R, RB_MAX_GRID);
  if (C > 0) {
    const unsigned egrid = (unsigned)std::min<uint64_t>(ex_blocks, RB_MAX_GRID);
    if (ex_shift == 10)
      k_emit_rows<EX_TILE_S><<<egrid, 256, 0, s>>>(a, n_items, row_cnt, R, n_views, (uint32_t)ex_blocks);
    else
      k_emit_rows<EX_TILE><<<egrid, 256, 0, s>>>(a, n_items, row_cnt, R, n_views, (uint32_t)ex_blocks);
    SGS_LAUNCH_CHECK();
    if (scan0) {
      const uint32_t nch = (uint32_t)cdiv(ex_blocks, EC);
      k_chunk_scan<<<nch, 256, 0, s>>>(L.cnt0, (uint32_t)ex_blocks, L.ctot, n_items, (uint32_t)C, ex_shift);
      SGS_LAUNCH_CHECK();
      k_chunk_totals<<<256, 256, 0, s>>>(L.ctot, nch);
      SGS_LAUNCH_CHECK();
    }
    const sgs_status st = radix_sort<uint32_t>(ik[src], iv[src], ik, iv, n_items, 0, C, rbits, sc_main, s, true,
                                               ex_blocks, nullptr, 0, a.cnt0, scan0 ? L.ctot : nullptr);
    if (st != SGS_OK) return st;
    k_piece_count<<<pgrid, 256, 0, s>>>(ik[0], row_cnt, R, nb_shift, L.cntp, L.ptab);
    SGS_LAUNCH_CHECK();
    k_col_scan<<<(unsigned)R, 256, 0, s>>>(L.cntp, L.ptab, R, cams_dev, n_views, L.pre_col, L.cnt_tile,
                                           (uint32_t)T);
    SGS_LAUNCH_CHECK();
  }
  k_tile_scan<<<1, 1024, 0, s>>>(L.cnt_tile, (uint32_t)T, (uint32_t)C, ranges, tile_order);
  SGS_LAUNCH_CHECK();
  if (C > 0) {
    const unsigned rgrid = (pgrid + 7u) & ~7u;   // a multiple of 8 (the XCD chunks)
    const size_t pt_bytes = 2 * ((size_t)R + 1) * sizeof(uint32_t);   // (the piece table)
    // (128 columns when every view's rows have at most 128 tiles: half the
    // per-column LDS and scan work, five workgroups per CU instead of four)
    if (rb_tx <= 128)
      k_row_place<128><<<rgrid, 256, pt_bytes, s>>>(ik[0], iv[0], L.ptab, R, nb_shift, cams_dev, n_views,
                                                    L.pre_col, ranges, (uint32_t)T, (uint32_t)C, vals, keys,
                                                    g->depth, mm, n_inst);
    else
      k_row_place<256><<<rgrid, 256, pt_bytes, s>>>(ik[0], iv[0], L.ptab, R, nb_shift, cams_dev, n_views,
                                                    L.pre_col, ranges, (uint32_t)T, (uint32_t)C, vals, keys,
                                                    g->depth, mm, n_inst);
    SGS_LAUNCH_CHECK();
  }
  return SGS_OK;
}

sgs_status launch_bin_sort(const sgs_geom* g, int64_t m, int64_t n, const sgs_camera* cams_dev,
                           int32_t n_views, int64_t total_tiles, const sgs_options* opt,
                           int64_t cap, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           uint32_t* n_inst, uint32_t* tile_order, void* scratch, float near_min,
                           int32_t rb_rows, int32_t rb_tx, hipStream_t s) {
  // sort mode 2 runs when the caller found its conditions met (rb_rows > 0:
  // the global tile rows; rb_tx: the most tiles per row of any view);
  // otherwise mode 1, in the same (larger) scratch layout
  const int mode = opt->sort_mode == 2 && rb_rows == 0 ? 1 : opt->sort_mode;
  const bool wide = mode >= 1 && opt->depth_digit_bits == 10 && wide_depth((uint64_t)m, near_min);
  const BinLayout L = bin_layout(reinterpret_cast<uintptr_t>(scratch), m, cap, total_tiles, opt->sort_mode);
  const uint64_t T = (uint64_t)total_tiles, C = (uint64_t)cap;
  uint32_t* err = L.misc;
  // one fill zeroes the ranges, the instance count and every sort's state
  ZeroList z = {};
  int nz = 0;
  bool z_overflow = false;
  auto zero = [&](uint32_t* ptr, uint64_t words, uint32_t ev = 0u) {
    if (nz == ZL_MAX) {
      z_overflow = true;
      return;
    }
    z.p[nz] = ptr;
    z.n[nz] = words;
    z.ev[nz] = ev;
    ++nz;
  };
  // mode 1 writes ranges from the last sort pass by atomic min / max; mode
  // 2 writes every range from the tile counts
  if (mode != 2) zero(ranges, 2 * T, mode == 1 ? 0xffffffffu : 0u);
  if (mode == 2) zero(L.cnt_tile, T + RB_MAX_ROWS);   // tile counts and row item counts
  zero(n_inst, 1);
  zero(L.misc, 64);
  if (C > 0) {
    // block statuses of the passes that look back: large sorts take scanned
    // offsets in their first pass (its statuses stay untouched), and the row
    // sort of mode 2 runs its own (fewer) passes in the tile sort's layout
    const bool scan0 = mode >= 1 && cdiv(C, (uint64_t)RS_T * RS_IPT) > RS_WIDE_MAX_BLOCKS;
    const uint64_t head = 64 + (uint64_t)L.main_passes * 256 * (1 + HC);   // counters, histograms
    const uint64_t st0 = rs_blocks(C) * 256 * 2;                             // one pass's statuses
    const int used = mode == 2 ? rs_passes(tile_bits(rb_rows)) : L.main_passes;
    const int first = scan0 ? 1 : 0;
    zero(L.rs_main, head);
    if (used > first) zero(L.rs_main + head + (uint64_t)first * st0, (uint64_t)(used - first) * st0);
  }
  if (mode >= 1 && m > 0) {
    zero(L.rs_depth, wide ? rs_words((uint64_t)m, 3, 1024) : rs_words((uint64_t)m, 4));
    zero(L.so_status, L.so_words);
    zero(L.bstart, L.n_bstart);
  }
  if (z_overflow) return SGS_EINVAL;   // (at most ZL_MAX regions are ever listed)
  uint64_t zmax = 0;
  for (int k = 0; k < nz; ++k) zmax = std::max(zmax, z.n[k]);
  k_zero<<<dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>(cdiv(zmax, 256), 1), 2048), nz), 256, 0, s>>>(z);
  SGS_LAUNCH_CHECK();

  // tiles by decreasing list length (after the ranges are known)
  auto order_tiles = [&]() -> sgs_status {
    if (!tile_order && mode == 0) return SGS_OK;
    k_order_tiles<<<1, 1024, 0, s>>>(ranges, (uint32_t)T, tile_order);
    SGS_LAUNCH_CHECK();
    return SGS_OK;
  };
  DupArgs a = {};
  const uint64_t mm = (uint64_t)m;
  a.rec = reinterpret_cast<const float4*>(g->rec);
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
  a.enhanced = g->enhanced;
  a.m = m;
  const RsScratch sc_main = rs_carve(L.rs_main, L.main_passes, err, n_inst);
  if (mode == 0) {
    const int passes = L.main_passes;
    const int tb = tile_bits(total_tiles);
    uint64_t* kb[2] = {keys, L.kalt};
    uint32_t* vb[2] = {vals, L.valt};
    const int src = passes & 1;             // so that the result lands in buffer 0
    a.block_off = g->block_off;
    a.nb_total = a.nbx * n_views;
    a.keys64 = kb[src];
    a.vals = vb[src];
    if (n > 0) {
      k_duplicate64<<<dim3(a.nbx, n_views), 256, 0, s>>>(a);
      SGS_LAUNCH_CHECK();
    }
    if (cap > 0) {
      sgs_status st = radix_sort<uint64_t>(kb[src], vb[src], kb, vb, n_inst, 0, C, 32 + tb, sc_main, s);
      if (st != SGS_OK) return st;
      k_tile_ranges<uint64_t><<<(unsigned)cdiv(C, 256), 256, 0, s>>>(keys, 32, n_inst, (uint32_t)C,
                                                                      (uint32_t)T, ranges);
      SGS_LAUNCH_CHECK();
    }
    return order_tiles();
  }
  // mode 1
  if (m == 0) {
    if (mode != 2) return order_tiles();
    k_tile_scan<<<1, 1024, 0, s>>>(L.cnt_tile, (uint32_t)T, (uint32_t)C, ranges, tile_order);   // all empty
    SGS_LAUNCH_CHECK();
    return SGS_OK;
  }
  const int tb = tile_bits(total_tiles);
  uint32_t* dk[2] = {L.dk[0], L.dk[1]};
  uint32_t* dv[2] = {L.dv[0], L.dv[1]};
  // depth presort straight from the depth buffer (all-ones for tile-less records)
  sgs_status st;
  if (wide) {
    KeyXf xf;
    uint32_t nb;
    memcpy(&nb, &near_min, 4);
    xf.base = nb;
    xf.lim = (1u << DEPTH_BITS_WIDE) - 1u;
    xf.on = true;
    st = radix_sort<uint32_t, 1024>(reinterpret_cast<const uint32_t*>(g->depth), nullptr, dk, dv, nullptr,
                                    (uint32_t)m, mm, DEPTH_BITS_WIDE,
                                    rs_carve(L.rs_depth, 3, err, nullptr, 1024), s, false, 0, nullptr, 0,
                                    nullptr, nullptr, xf);
  } else {
    st = radix_sort<uint32_t>(reinterpret_cast<const uint32_t*>(g->depth), nullptr, dk, dv, nullptr,
                              (uint32_t)m, mm, 32, rs_carve(L.rs_depth, 4, err, nullptr), s);
  }
  if (st != SGS_OK) return st;
  const uint32_t* order = dv[0];
  if (mode == 2) return bin_rows(g, a, L, sc_main, order, m, n_views, cams_dev, T, C, keys, vals, ranges, n_inst,
                                 tile_order, rb_rows, rb_tx, s);
  k_sorted_offsets<<<(unsigned)cdiv(mm, SO_TILE), 256, 0, s>>>(
      order, g->tiles, m, L.offs, n_inst, reinterpret_cast<uint64_t*>(L.so_status + 64), L.so_status, err,
      L.bstart, (uint32_t)L.n_bstart, ex_shift_for(C), nullptr, nullptr);
  SGS_LAUNCH_CHECK();
  const int passes = L.main_passes;
  const int src = passes & 1;
  uint32_t* tk[2] = {L.tk[0], L.tk[1]};
  uint32_t* vb[2] = {vals, L.valt};
  a.order = order;
  a.offs = L.offs;
  a.bstart = L.bstart;
  a.keys32 = tk[src];
  a.vals = vb[src];
  const int ex_shift = ex_shift_for(C);
  const uint64_t ex_blocks = cdiv(C, 1ull << ex_shift);
  a.hcopies = ex_blocks > HC_MIN_BLOCKS ? HC : 1;
  a.hpart = a.hcopies > 1 ? sc_main.hpart : sc_main.ghist;
  // large sorts scan the expansion blocks' first-digit counts instead of
  // looking back over the blocks of the first pass
  // (their expansion blocks are EX_TILE long)
  static_assert(RS_WIDE_MAX_BLOCKS * RS_T * RS_IPT >= EX_SMALL_CAP, "scanned first pass needs EX_TILE");
  const bool scan0 = cdiv(C, (uint64_t)RS_T * RS_IPT) > RS_WIDE_MAX_BLOCKS;
  a.cnt0 = scan0 ? L.cnt0 : nullptr;
  a.hpasses = passes;
  a.hwidth = rs_width(tb);
  if (cap > 0) {
    if (ex_shift == 10)
      k_expand32<EX_TILE_S><<<(unsigned)ex_blocks, 256, 0, s>>>(a);
    else
      k_expand32<EX_TILE><<<(unsigned)ex_blocks, 256, 0, s>>>(a);
    SGS_LAUNCH_CHECK();
    if (scan0) {
      const uint32_t nch = (uint32_t)cdiv(ex_blocks, EC);
      k_chunk_scan<<<nch, 256, 0, s>>>(L.cnt0, (uint32_t)ex_blocks, L.ctot, n_inst, (uint32_t)C, ex_shift);
      SGS_LAUNCH_CHECK();
      k_chunk_totals<<<256, 256, 0, s>>>(L.ctot, nch);
      SGS_LAUNCH_CHECK();
    }
    st = radix_sort<uint32_t>(tk[src], vb[src], tk, vb, n_inst, 0, C, tb, sc_main, s, true, ex_blocks,
                              ranges, (uint32_t)T, a.cnt0, scan0 ? L.ctot : nullptr);
    if (st != SGS_OK) return st;
    if (keys) {
      k_make_keys64<<<(unsigned)cdiv(C, 256), 256, 0, s>>>(tk[0], vals, g->depth, mm, n_inst,
                                                            (uint32_t)C, keys);
      SGS_LAUNCH_CHECK();
    }
  }
  return order_tiles();
}

}  // namespace sgs
