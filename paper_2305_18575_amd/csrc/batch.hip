// Batched solver: one workgroup runs the complete search of one instance
// (Algorithm 1's cost loop, Algorithm 2's constructors, uniqueness, ordered
// append, precision) with barriers as the only synchronisation, so many small
// instances progress side by side in one launch and no host round trip is
// needed per level or chunk.  Results are bit-identical to the per-chunk grid
// path: the same enumeration order, the same deterministic winner rule
// (smallest enumeration index), the same ordered append.
#include <algorithm>
#include <mutex>

#include "device_common.h"

namespace rei {

// Arenas of the allocation-free batched entry point.  In host code this name
// stands for the array only through hipGetSymbolAddress (static_scratch);
// kernels receive the address that call returns.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr uint32_t kWords = kBatchChunk / 32;  // winner bitmap words per chunk
constexpr int kMaxBlocks = 2 + 2 * (int)kBatchMaxCost;
constexpr uint32_t kTreeMax = kBatchTreeNodes;  // nodes of the answer tree written back

struct BlockD {
  uint32_t op, L, R, same;
  uint64_t count;
};

// Work items of block b's candidates [e0, e1) in the current chunk: 64
// consecutive candidates each, or one 64-candidate concatenation tile (64
// right operands of one left operand, or 64 left operands of one right
// operand when the right level is small and shorter than the left).
__device__ inline uint64_t block_items(const BlockD& b, uint64_t e0, uint64_t e1, uint64_t nL, uint64_t nR) {
  if (b.op != OP_CONCAT) return (e1 - e0 + 63) / 64;
  if (nR >= 64 || nR >= nL) {
    const uint64_t nT = (nR + 63) / 64;
    const uint64_t f0 = (e0 / nR) * nT + (e0 % nR) / 64;
    const uint64_t f1 = ((e1 - 1) / nR) * nT + ((e1 - 1) % nR) / 64;
    return f1 - f0 + 1;
  }
  return ((e1 - 1) / nR / 64 - (e0 / nR) / 64 + 1) * nR;
}

// Barrier between phases whose global-memory effects later phases read.  An
// instance's buffers are touched by its own workgroup only, and all waves of
// a workgroup run on one CU, so workgroup scope suffices: the barrier makes
// every store and atomic issued before it visible to every wave after it.
// (Agent scope would write back and invalidate the whole L2 at each phase.)
__device__ __forceinline__ void phase_barrier() { __syncthreads(); }


// Concatenation of 64 candidates that share one operand ("uniform") while the
// other operand varies over the 64 bit positions of the transposed tile T.
// kLeft = false: tile = right rows, out_t(w) = OR over cuts (u, v) of w with
//                uniform(u) of T[v];
// kLeft = true:  tile = left rows,  out_t(w) = OR over cuts (u, v) with
//                uniform(v) of T[u].
// Lane t receives the W words of candidate t.
// The guide table (gto, gtp) is the workgroup's LDS copy.
// qn: most cuts of any word (the longest word's length + 1).  From 8 words
// on, cut position q is the outer loop and the lane's W words the inner one
// (each word's read clamped to its last cut and masked after), so 24
// independent LDS reads are in flight per round of eight words instead of a
// chain of three per cut; below that the per-word loop keeps the register
// count of the 1024-thread instantiations down.
template <int W, bool kLeft>
__device__ __forceinline__ void concat_tile(const uint64_t* T, const uint64_t* uni, const uint32_t* gto,
                                            const uint32_t* gtp, uint32_t n, uint32_t qn, uint64_t (&key)[W]) {
  const uint32_t lane = lane_id();
  if constexpr (W >= 8) {
    // eight words at a time keeps the registers of the 16- and 32-word
    // instantiations within their launch bounds
#pragma unroll
    for (int k0 = 0; k0 < W; k0 += 8) {
      uint32_t first[8], last[8], cnt[8];
      uint64_t acc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t w = 64u * (k0 + k) + lane;
        first[k] = w < n ? gto[w] : 0u;
        cnt[k] = w < n ? gto[w + 1] - first[k] : 0u;
        last[k] = first[k] + (cnt[k] ? cnt[k] - 1 : 0u);
        acc[k] = 0;
      }
      for (uint32_t q = 0; q < qn; ++q) {
        uint32_t p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = gtp[min(first[k] + q, last[k])];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t ui = kLeft ? (p[k] & 0xFFFFu) : (p[k] >> 16);
          const uint32_t si = kLeft ? (p[k] >> 16) : (p[k] & 0xFFFFu);
          const uint64_t t = T[si];
          const bool on = q < cnt[k] && ((uni[ui >> 6] >> (ui & 63)) & 1ull);
          acc[k] |= on ? t : 0ull;
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) key[k0 + k] = transpose64(acc[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const uint32_t w = 64u * k + lane;
      uint64_t acc = 0;
      if (w < n) {
        const uint32_t q1 = gto[w + 1];
        for (uint32_t q = gto[w]; q < q1; ++q) {
          const uint32_t p = gtp[q];
          const uint32_t ui = kLeft ? (p & 0xFFFFu) : (p >> 16);
          const uint32_t si = kLeft ? (p >> 16) : (p & 0xFFFFu);
          if ((uni[ui >> 6] >> (ui & 63)) & 1ull) acc |= T[si];
        }
      }
      key[k] = transpose64(acc);
    }
  }
}

// Decodes level index e of level c into its constructor and operands (rows),
// walking the level's blocks in enumeration order (Q, S, C by left cost, U by
// left cost); the counts of levels below c are final.  lstart and lcount are
// the workgroup's level tables in LDS.
__device__ __forceinline__ bool decode_index(const BatchDesc& d, const uint64_t* lstart, const uint64_t* lcount,
                                             uint32_t c, uint64_t e, uint32_t* op, uint64_t* a, uint64_t* b) {
  const int64_t c1 = d.c1, cc = c;
  auto lc = [&](int64_t k) -> uint64_t { return (k >= c1 && k < cc) ? lcount[k] : 0ull; };
  *b = 0;
  if (cc == c1) {
    *op = OP_CHAR;
    *a = e;
    return e < d.nsigma;
  }
  uint64_t n = lc(cc - d.c2);
  if (e < n) {
    *op = OP_QUESTION;
    *a = lstart[cc - d.c2] + e;
    return true;
  }
  e -= n;
  n = lc(cc - d.c3);
  if (e < n) {
    *op = OP_STAR;
    *a = lstart[cc - d.c3] + e;
    return true;
  }
  e -= n;
  for (int64_t L = c1; cc - (int64_t)d.c4 - L >= c1; ++L) {
    const int64_t R = cc - d.c4 - L;
    n = lc(L) * lc(R);
    if (e < n) {
      *op = OP_CONCAT;
      *a = lstart[L] + e / lc(R);
      *b = lstart[R] + e % lc(R);
      return true;
    }
    e -= n;
  }
  for (int64_t L = c1; L <= cc - (int64_t)d.c5 - L; ++L) {
    const int64_t R = cc - d.c5 - L;
    const uint64_t x = lc(L), y = lc(R);
    n = (L < R) ? x * y : (x ? x * (x - 1) / 2 : 0);
    if (e < n) {
      *op = OP_UNION;
      if (L == R) {
        uint64_t i = 0, j = 0;
        tri_decode(e, x, &i, &j);
        *a = lstart[L] + i;
        *b = lstart[L] + j;
      } else {
        *a = lstart[L] + e / y;
        *b = lstart[R] + e % y;
      }
      return true;
    }
    e -= n;
  }
  return false;
}

// kT threads per instance (256, 512 or 1024; at most batch_max_threads(W),
// so that the per-wave operand tiles and the guide table fit the LDS):
// many waves shorten one instance's search, few let more instances share a
// CU.  The host picks kT per launch (tuned or from the batch size).
// Two launch forms.  next == nullptr: workgroup b solves instance b.
// Persistent (next != nullptr): a grid of at most the resident workgroups;
// each takes the next item from the device counter *next (zero at launch)
// and solves instance order[item] (or item itself when order is null),
// until the items run out, so the longest instances can start first
// whatever the grid size.
// Queue (qc != nullptr, with next): descs is a ring the host fills while the
// launch runs (n_inst slots, published up to qc->tail); a workgroup claims
// the next published slot by compare-and-swap on *next (zero at launch), so
// a slot is taken only once it exists and exactly once.  Every workgroup
// leaves once it has waited qc->idle_ticks without finding a slot, or when
// the host sets qc->closing; slots published after the last one left are
// found unsolved by the host and published again in its next launch.
template <int W, bool kInl, uint32_t kT>
__global__ __launch_bounds__(kT) void solve_batch(const BatchDesc* descs, uint32_t n_inst, const uint32_t* order,
                                                  uint32_t* next, const QueueCtl* qc) {
  static_assert(kT >= kBatchChunk / 32 && kT <= batch_max_threads(W) && kT % 64 == 0, "one scan value per thread");
  constexpr uint32_t kIc = batch_max_ic(W), kPairs = batch_max_pairs(W);
  constexpr uint32_t kWaves = kT / 64;
  __shared__ uint64_t s_lstart[kBatchMaxCost + 2], s_lcount[kBatchMaxCost + 2];
  __shared__ uint64_t s_uniq[kBatchMaxCost + 2], s_cand[kBatchMaxCost + 2];
  __shared__ BlockD s_blk[kMaxBlocks];
  __shared__ uint64_t s_bstart[kMaxBlocks + 1];  // level index of each block's first candidate
  __shared__ uint32_t s_item0[kMaxBlocks + 1];   // each block's first work item in the current chunk
  __shared__ uint32_t s_nblk;
  __shared__ uint32_t s_nsurv, s_ans, s_rank, s_over, s_stop, s_resume;
  __shared__ uint64_t s_total;
  __shared__ uint32_t s_bm[kWords], s_pre[kWords];
  __shared__ uint32_t s_winners;
  __shared__ uint64_t s_tile[kWaves][64 * W];
  static_assert(W < 8 || sizeof(s_tile) >= kBatchChunk * sizeof(uint16_t), "ranks of a chunk fit the tiles");
  static_assert(kBatchChunk <= 0xFFFFu, "ranks of a chunk fit 16 bits");
  __shared__ uint64_t s_uni[kWaves][W];
  __shared__ uint32_t s_gto[kIc + 1], s_gtp[kPairs], s_lo[kIc + 2];
  __shared__ uint32_t s_item;

  for (uint32_t pass = 0;; ++pass) {
  uint32_t item;
  if (!next) {
    if (pass || blockIdx.x >= n_inst) return;
    item = blockIdx.x;
  } else if (qc) {
    if (threadIdx.x == 0) {
      uint32_t got = ~0u;
      const long long t_wait = wall_clock64();
      for (;;) {
        const uint32_t tail = __hip_atomic_load(&qc->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t h = __hip_atomic_load(next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < tail && h < n_inst) {
          if (atomicCAS(next, h, h + 1) == h) {
            got = h;
            break;
          }
          continue;  // another workgroup took it: look again
        }
        const uint32_t closing = __hip_atomic_load(&qc->closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (closing || (uint64_t)(wall_clock64() - t_wait) > qc->idle_ticks) break;
        __builtin_amdgcn_s_sleep(16);
      }
      s_item = got;
    }
    __syncthreads();
    item = s_item;
    __syncthreads();
    if (item >= n_inst) return;
  } else {
    if (threadIdx.x == 0) s_item = atomicAdd(next, 1u);
    __syncthreads();
    item = s_item;
    __syncthreads();  // read by every wave before thread 0 writes the next one
    if (item >= n_inst) return;
    if (order) item = order[item];
  }
  const BatchDesc d = descs[item];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The dedup table starts small and grows (cleared and rebuilt from the
  // stored rows) while rows accumulate, up to the arena's slot_mask: a
  // small instance clears a few KB instead of its whole arena.
  uint64_t tmask = min(d.slot_mask, (uint64_t)1023);
  Probe probe{d.rows, d.slots, tmask, d.pmask, d.nmask, d.max_err};
  const Sink sink{d.skey, d.se, d.spos, &s_nsurv, &s_ans};

  // start: empty table, zero counters
  for (uint64_t i = tid; i <= tmask; i += kT) {
    d.slots[i] = kEmpty;
    if (kInl) d.sref[i] = kEmpty;
  }
  // guide table and words-by-length offsets into LDS (batchable instances
  // have at most batch_max_ic(W) words and batch_max_pairs(W) cuts)
  for (uint32_t i = tid; i <= d.n; i += kT) s_gto[i] = d.gt_off[i];
  for (uint32_t i = tid; i < d.n_pairs; i += kT) s_gtp[i] = d.gt_pair[i];
  for (uint32_t i = tid; i < d.max_len + 2; i += kT) s_lo[i] = d.len_off[i];
  for (uint32_t c = tid; c < kBatchMaxCost + 2; c += kT) {
    s_lstart[c] = 0;
    s_lcount[c] = 0;
    s_uniq[c] = 0;
    s_cand[c] = 0;
  }
  if (tid == 0) {
    s_total = 0;
    s_stop = STOP_NONE;
    s_resume = 0;
  }
  phase_barrier();

  uint32_t ans_cost = 0;
  uint64_t ans_e = 0;
  const long long t_start = wall_clock64();
  for (uint32_t c = d.c1; c <= d.max_cost && s_stop == STOP_NONE; ++c) {
    if (tid == 0) {
      s_lstart[c] = s_total;
      // constructor blocks of level c, in enumeration order
      uint32_t nb = 0;
      auto lc = [&](int64_t k) -> uint64_t { return (k >= (int64_t)d.c1 && k < (int64_t)c) ? s_lcount[k] : 0ull; };
      if (c == d.c1) {
        s_blk[nb++] = {OP_CHAR, 0, 0, 0, (uint64_t)d.nsigma};
      } else {
        const int64_t cc = c;
        if (lc(cc - d.c2)) s_blk[nb++] = {OP_QUESTION, (uint32_t)(cc - d.c2), 0, 0, lc(cc - d.c2)};
        if (lc(cc - d.c3)) s_blk[nb++] = {OP_STAR, (uint32_t)(cc - d.c3), 0, 0, lc(cc - d.c3)};
        for (int64_t L = d.c1; cc - (int64_t)d.c4 - L >= (int64_t)d.c1; ++L) {
          const int64_t R = cc - d.c4 - L;
          const uint64_t n = lc(L) * lc(R);
          if (n) s_blk[nb++] = {OP_CONCAT, (uint32_t)L, (uint32_t)R, 0, n};
        }
        for (int64_t L = d.c1; L <= cc - (int64_t)d.c5 - L; ++L) {
          const int64_t R = cc - d.c5 - L;
          const uint64_t a = lc(L), b = lc(R);
          const uint64_t n = (L < R) ? a * b : (a ? a * (a - 1) / 2 : 0);
          if (n) s_blk[nb++] = {OP_UNION, (uint32_t)L, (uint32_t)R, L == R ? 1u : 0u, n};
        }
      }
      s_nblk = nb;
      s_bstart[0] = 0;
      for (uint32_t b = 0; b < nb; ++b) s_bstart[b + 1] = s_bstart[b] + s_blk[b].count;
      // a level this large is work for the whole device: hand the instance,
      // with its lower levels stored, to the per-chunk path; so is a
      // mid-sized level of an instance that has kept its workgroup long
      // (the deep searches of a batch), while the device has room beside it
      const bool late = d.time_ticks && s_bstart[nb] > kBatchTimeMinLevel &&
                        (uint64_t)(wall_clock64() - t_start) > d.time_ticks;
      if (s_bstart[nb] > d.level_max || late) {
        s_stop = STOP_HANDOFF;
        s_resume = c;
      }
    }
    __syncthreads();
    const uint32_t nblk = s_nblk;
    const uint64_t level_total = s_bstart[nblk];
    // Chunks cover consecutive level indices [E0, E1) and may span several
    // constructor blocks, so small blocks share one round of phases.
    for (uint64_t E0 = 0; E0 < level_total && s_stop == STOP_NONE; E0 += kBatchChunk) {
      const uint64_t E1 = min(level_total, E0 + (uint64_t)kBatchChunk);
      const uint32_t len = (uint32_t)(E1 - E0);
      {
        // keep the load at most 1/2 with this chunk's survivors inserted
        const uint64_t total = s_total;
        if (2 * (total + len) > tmask + 1) {
          uint64_t cap = tmask + 1;
          while (cap < 4 * (total + len) && cap <= d.slot_mask) cap *= 2;
          tmask = min(d.slot_mask, cap - 1);
          for (uint64_t i = tid; i <= tmask; i += kT) {
            d.slots[i] = kEmpty;
            if (kInl) d.sref[i] = kEmpty;
          }
          __syncthreads();
          for (uint64_t row = tid; row < total; row += kT) {
            uint64_t key[W];
#pragma unroll
            for (int k = 0; k < W; ++k) key[k] = d.rows[row * W + k];
            table_rebuild_one<W, kInl>(d.slots, tmask, key, row);
          }
          probe.slot_mask = tmask;
          __syncthreads();
        }
      }
      if (tid == 0) {
        s_nsurv = 0;
        s_ans = ~0u;
        s_rank = ~0u;
        s_over = ~0u;
      }
      __syncthreads();
      // Star blocks first, one at a time: they pair the waves and need the
      // workgroup barriers around them.
      for (uint32_t bi = 0; bi < nblk; ++bi) {
        const uint64_t bs = s_bstart[bi], be = s_bstart[bi + 1];
        if (be <= E0) continue;
        if (bs >= E1) break;
        const BlockD blk = s_blk[bi];
        if (blk.op != OP_STAR) continue;
        const uint64_t lst = s_lstart[blk.L];
        // block-local candidate range of this chunk; candidate e of the block
        // has chunk-relative index bs + e - E0
        const uint64_t e0 = max(E0, bs) - bs, e1 = min(E1, be) - bs;
        const uint64_t rel0 = bs - E0;  // modulo 2^64: rel0 + e >= 0 for e >= e0
        // r* for 64 rows per wave pair: the even wave of each pair owns
        // the pair's two tiles (Xt = its own, Yt = its partner's), so
        // kWaves/2 groups of rows run at once with wave-level syncs only.
        // The workgroup barriers around the block keep the partner's tile
        // out of the neighbouring blocks' per-wave use.
        __syncthreads();
        if ((wave & 1u) == 0) {
          uint64_t* Xt = s_tile[wave];
          uint64_t* Yt = s_tile[wave + 1];
          constexpr uint32_t kPairs = kWaves / 2;
          for (uint64_t g0 = e0 + 64 * (uint64_t)(wave >> 1); g0 < e1; g0 += 64 * (uint64_t)kPairs) {
            const uint64_t e = g0 + lane;
#pragma unroll
            for (int k = 0; k < W; ++k) {
              const uint64_t v = (e < e1) ? d.rows[(lst + e) * W + k] : 0ull;
              Xt[64 * k + lane] = transpose64(v);
            }
            for (uint32_t w = lane; w < 64u * W; w += 64) Yt[w] = (w == 0) ? ~0ull : 0ull;
            wave_sync_lds();
            // Y(eps) = 1; by increasing length, Y(w) = OR over cuts w = u v
            // with u non-empty of X(u) & Y(v) (v is shorter)
            for (uint32_t l = 1; l <= d.max_len; ++l) {
              const uint32_t lo = s_lo[l], hi = s_lo[l + 1];
              for (uint32_t w = lo + lane; w < hi; w += 64) {
                // a word of length l has cuts 0..l; cut 0 has u = eps
                Yt[w] = star_fold(Xt, Yt, s_gtp, s_gto[w], l);
              }
              wave_sync_lds();
            }
            uint64_t key[W];
#pragma unroll
            for (int k = 0; k < W; ++k) key[k] = transpose64(Yt[64 * k + lane]);
            filter_emit<W, kInl>(probe, sink, e < e1, false, key, (uint32_t)(rel0 + e));
            wave_sync_lds();  // the tiles are rewritten by the next group
          }
        }
        __syncthreads();
      }
      // Every other block's work items (64 consecutive candidates, or one
      // concatenation tile) are dealt to the waves together, so a chunk that
      // spans many small blocks keeps every wave busy.
      if (tid == 0) {
        uint32_t n = 0;
        for (uint32_t bi = 0; bi < nblk; ++bi) {
          s_item0[bi] = n;
          const uint64_t bs = s_bstart[bi], be = s_bstart[bi + 1];
          const BlockD blk = s_blk[bi];
          if (be > E0 && bs < E1 && blk.op != OP_STAR)
            n += (uint32_t)block_items(blk, max(E0, bs) - bs, min(E1, be) - bs, s_lcount[blk.L], s_lcount[blk.R]);
        }
        s_item0[nblk] = n;
      }
      __syncthreads();
      {
        const uint32_t n_items = s_item0[nblk];
        uint32_t bi = 0;
        for (uint32_t it = wave; it < n_items; it += kWaves) {
          while (s_item0[bi + 1] <= it) ++bi;  // blocks with no items here are skipped
          const uint32_t li = it - s_item0[bi];
          const uint64_t bs = s_bstart[bi], be = s_bstart[bi + 1];
          const BlockD blk = s_blk[bi];
          const uint64_t lst = s_lstart[blk.L], lct = s_lcount[blk.L];
          const uint64_t rst = s_lstart[blk.R], rct = s_lcount[blk.R];
          const uint64_t e0 = max(E0, bs) - bs, e1 = min(E1, be) - bs;
          const uint64_t rel0 = bs - E0;
          if (blk.op != OP_CONCAT) {
            const uint64_t e = e0 + 64 * (uint64_t)li + lane;
            const bool valid = e < e1;
            uint64_t key[W];
            bool dup = false;
            if (blk.op == OP_CHAR) {
              const int idx = valid ? d.char_index[e] : -1;
#pragma unroll
              for (int k = 0; k < W; ++k) key[k] = (idx >= 0 && (idx >> 6) == k) ? (1ull << (idx & 63)) : 0ull;
            } else if (blk.op == OP_QUESTION) {
              const uint64_t* src = d.rows + (lst + (valid ? e : 0)) * W;
#pragma unroll
              for (int k = 0; k < W; ++k) key[k] = valid ? src[k] : 0ull;
              dup = (key[0] & 1ull) != 0;
              key[0] |= 1ull;
            } else {
              uint64_t i = 0, j = 0;
              if (valid) {
                if (blk.same) {
                  tri_decode(e, lct, &i, &j);
                } else {
                  i = e / rct;
                  j = e - i * rct;
                }
              }
              const uint64_t* x = d.rows + (lst + i) * W;
              const uint64_t* y = d.rows + (rst + j) * W;
              bool eqx = true, eqy = true;
#pragma unroll
              for (int k = 0; k < W; ++k) {
                const uint64_t xv = valid ? x[k] : 0ull, yv = valid ? y[k] : 0ull;
                key[k] = xv | yv;
                eqx = eqx && key[k] == xv;
                eqy = eqy && key[k] == yv;
              }
              dup = eqx || eqy;
            }
            filter_emit<W, kInl>(probe, sink, valid, dup, key, (uint32_t)(rel0 + e));
            continue;
          }
          uint64_t* T = s_tile[wave];
          uint64_t* U = s_uni[wave];
          const uint64_t nL = lct, nR = rct;
          if (nR >= 64 || nR >= nL) {
            // right operands across the lanes: tile f = i * nT + jt holds
            // candidates i * nR + 64 * jt + lane; the block's items are the
            // tiles from the one holding e0 to the one holding e1 - 1
            const uint64_t nT = (nR + 63) / 64;
            const uint64_t f = (e0 / nR) * nT + (e0 % nR) / 64 + li;
            const uint64_t i = f / nT, jt = f - i * nT;
            const uint64_t jr = 64 * jt + lane;
#pragma unroll
            for (int k = 0; k < W; ++k)
              T[64 * k + lane] = transpose64(jr < nR ? d.rows[(rst + jr) * W + k] : 0ull);
            if (lane < (uint32_t)W) U[lane] = d.rows[(lst + i) * W + lane];
            wave_sync_lds();
            uint64_t key[W];
            concat_tile<W, false>(T, U, s_gto, s_gtp, d.n, d.max_len + 1, key);
            const uint64_t e = i * nR + jr;
            filter_emit<W, kInl>(probe, sink, jr < nR && e >= e0 && e < e1, false, key, (uint32_t)(rel0 + e));
            wave_sync_lds();
          } else {
            // left operands across the lanes (the right level is small):
            // item li is (left tile xt, right operand j)
            const uint64_t xt = (e0 / nR) / 64 + li / nR, j = li % nR;
            const uint64_t ef = (64 * xt) * nR + j, el = (64 * xt + 63) * nR + j;
            if (el < e0 || ef >= e1) continue;
            const uint64_t ir = 64 * xt + lane;
#pragma unroll
            for (int k = 0; k < W; ++k)
              T[64 * k + lane] = transpose64(ir < nL ? d.rows[(lst + ir) * W + k] : 0ull);
            if (lane < (uint32_t)W) U[lane] = d.rows[(rst + j) * W + lane];
            wave_sync_lds();
            uint64_t key[W];
            concat_tile<W, true>(T, U, s_gto, s_gtp, d.n, d.max_len + 1, key);
            const uint64_t e = ir * nR + j;
            filter_emit<W, kInl>(probe, sink, ir < nL && e >= e0 && e < e1, false, key, (uint32_t)(rel0 + e));
            wave_sync_lds();
          }
        }
      }
      phase_barrier();

        // ---- insert survivors
        const uint32_t ns = s_nsurv;
        for (uint32_t sid = tid; sid < ns; sid += kT) {
          uint64_t key[W];
#pragma unroll
          for (int k = 0; k < W; ++k) key[k] = d.skey[(uint64_t)sid * W + k];
          const uint64_t h = d.spos[sid];
          const uint64_t pos = table_insert<W, kInl>(d.slots, d.sref, tmask, d.rows, d.skey, key, h,
                                                     new_ref(d.se[sid], sid));
          d.spos[sid] = spos_pack(pos, h);
        }
        phase_barrier();

        // ---- winners, ranks, ordered append, accounting
        const uint32_t words = (len + 31) / 32;
        for (uint32_t i = tid; i < words; i += kT) s_bm[i] = 0;
        __syncthreads();
        for (uint32_t sid = tid; sid < ns; sid += kT) {
          const uint32_t e = d.se[sid];
          if (table_is_winner<kInl>(d.slots, d.sref, d.spos[sid], new_ref(e, sid)))
            atomicOr(&s_bm[e >> 5], 1u << (e & 31));
        }
        __syncthreads();
        if (wave == 0) {
          const uint32_t t = wave_popc_scan<kWords / 64>(s_bm, s_pre, words);
          if (lane == 0) s_winners = t;
        }
        __syncthreads();
        const uint32_t winners = s_winners;
        const uint64_t total = s_total;
        const uint64_t room = d.row_cap > total ? d.row_cap - total : 0;
        const uint64_t alloc_room = d.rows_alloc > total ? d.rows_alloc - total : 0;
        const uint32_t ans = s_ans;
        // each survivor's rank among the stored rows (kNotStored: not stored)
        constexpr uint32_t kNotStored = 0xFFFFu;  // ranks are below kBatchChunk
        auto place = [&](uint32_t sid, uint32_t e) -> uint32_t {
          const uint32_t word = s_bm[e >> 5];
          const uint32_t bit = 1u << (e & 31);
          if (!(word & bit)) return kNotStored;
          const uint32_t rank = s_pre[e >> 5] + (uint32_t)__popc(word & (bit - 1));
          if (e == ans) s_rank = rank;
          if (ans != ~0u && e >= ans) return kNotStored;
          if (rank < room && rank < alloc_room) return rank;
          if (rank == room) s_over = e;
          return kNotStored;
        };
        if constexpr (W < 8) {
          for (uint32_t sid = tid; sid < ns; sid += kT) {
            const uint32_t e = d.se[sid];
            const uint32_t rank = place(sid, e);
            if (rank == kNotStored) continue;
            const uint64_t row = total + rank;
#pragma unroll
            for (int k = 0; k < W; ++k) d.rows[row * W + k] = d.skey[(uint64_t)sid * W + k];
            d.aux[row] = E0 + e;
            table_publish<kInl>(d.slots, d.sref, d.spos[sid], row);
          }
        } else {
          // wide rows: ranks into LDS (over the tiles, idle in this phase),
          // then W consecutive lanes copy one row, whole rows per wave
          uint16_t* s_dst = reinterpret_cast<uint16_t*>(&s_tile[0][0]);
          for (uint32_t sid = tid; sid < ns; sid += kT) s_dst[sid] = (uint16_t)place(sid, d.se[sid]);
          __syncthreads();
          constexpr uint32_t kPer = kT / W;  // rows per round
          const uint32_t k = tid % W;
          for (uint32_t q = tid / W; q < ns; q += kPer) {
            const uint32_t rank = s_dst[q];
            if (rank == kNotStored) continue;
            const uint64_t row = total + rank;
            d.rows[row * W + k] = d.skey[(uint64_t)q * W + k];
            if (k == 0) {
              d.aux[row] = E0 + d.se[q];
              table_publish<kInl>(d.slots, d.sref, d.spos[q], row);
            }
          }
        }
        __syncthreads();
        if (tid == 0) {
          uint64_t stored, du, dc;
          uint32_t stop = STOP_NONE;
          if (ans != ~0u) {
            if ((uint64_t)s_rank > room) {
              stored = room;
              dc = (uint64_t)s_over + 1;
              du = room;
              stop = STOP_OOM;
            } else {
              stored = s_rank;
              dc = (uint64_t)ans + 1;
              du = (uint64_t)s_rank + 1;
              stop = STOP_ANSWER;
              ans_cost = c;
              ans_e = E0 + ans;
            }
          } else if ((uint64_t)winners > room) {
            stored = room;
            dc = (uint64_t)s_over + 1;
            du = room;
            stop = STOP_OOM;
          } else {
            stored = winners;
            dc = len;
            du = winners;
          }
          if (stored > alloc_room) {
            stop = STOP_CAPACITY;
          } else {
            s_total = total + stored;
            s_lcount[c] += stored;
            s_uniq[c] += du;
            s_cand[c] += dc;
          }
          s_stop = stop;
        }
        phase_barrier();
    }
  }

  // ---- results, written straight to the instance's host-visible buffers
  if (tid == 0) {
    // The answer's expression tree (A12): the answer candidate, then every
    // stored row below it, each decoded from its back-pointer (level index)
    // with the block structure of its level.  Trees have at most one node
    // per unit of cost; a count of 0 tells the host to decode from the
    // back-pointers itself.
    uint32_t k = 0;
    if (s_stop == STOP_ANSWER) {
      uint64_t* stk = s_tile[0];  // free after the search
      uint32_t sp = 0;
      bool ok = true;
      auto node = [&](uint64_t row, uint32_t c, uint64_t e) {
        uint32_t op = 0;
        uint64_t a = 0, b = 0;
        if (k >= kTreeMax || sp + 2 > 64 || !decode_index(d, s_lstart, s_lcount, c, e, &op, &a, &b)) {
          ok = false;
          return;
        }
        uint64_t* o = d.htree + 1 + 4 * k++;
        o[0] = row;
        o[1] = op;
        o[2] = a;
        o[3] = b;
        if (op != OP_CHAR) stk[sp++] = a;
        if (op == OP_CONCAT || op == OP_UNION) stk[sp++] = b;
      };
      node(~0ull, ans_cost, ans_e);
      while (ok && sp) {
        const uint64_t row = stk[--sp];
        uint32_t rc = 0;
        for (uint32_t c = d.c1; c <= d.max_cost; ++c)
          if (row >= s_lstart[c] && row < s_lstart[c] + s_lcount[c]) rc = c;
        if (!rc) {
          ok = false;
          break;
        }
        node(row, rc, d.aux[row]);
      }
      if (!ok) k = 0;
    }
    d.htree[0] = k;
    d.hst->total_rows = s_total;
    d.hst->row_cap = d.row_cap;
    d.hst->stop = s_stop;
    d.hst->answer_cost = ans_cost;
    d.hst->answer_e = ans_e;
    d.hst->resume_level = s_resume;
  }
  const uint32_t L = d.max_cost + 2;
  for (uint32_t i = tid; i < L; i += kT) {
    d.hlev[i] = s_lcount[i];
    d.hlev[L + i] = s_uniq[i];
    d.hlev[2 * L + i] = s_cand[i];
  }
  // Publish: every result above, and the rows and table in device memory,
  // become visible to the host and to other kernels before the flag does,
  // so the host may hand the instance to the per-chunk path while the rest
  // of the launch still runs.
  __threadfence_system();
  __syncthreads();
  if (tid == 0) __hip_atomic_store(&d.hst->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }  // next instance
}

// Writes up to kDescPack descriptors, passed by value, to device memory (the
// allocation-free entry point sets its descriptors up with no copy API).
struct DescPack {
  BatchDesc d[kDescPack];
  uint32_t n;
};
__global__ void put_descs(BatchDesc* dst, DescPack p) {
  static_assert(sizeof(BatchDesc) % 8 == 0, "descriptors copy as 64-bit words");
  const uint32_t words = p.n * (uint32_t)(sizeof(BatchDesc) / 8);
  const uint64_t* src = reinterpret_cast<const uint64_t*>(p.d);
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) reinterpret_cast<uint64_t*>(dst)[i] = src[i];
}

// Puts the work counters of the persistent launches back to zero (a kernel,
// so that it can sit in a captured graph).
__global__ void reset_counters(uint32_t* c, uint32_t n) {
  if (threadIdx.x < n) c[threadIdx.x] = 0;
}

}  // namespace

hipError_t set_hash_mask_batch(uint64_t mask) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_hash_mask), &mask, sizeof(mask));
}

hipError_t launch_solve_batch(int W, bool inl, uint32_t threads, const BatchDesc* d_descs, uint32_t n,
                              hipStream_t s, const uint32_t* order, uint32_t* next, uint32_t grid,
                              const QueueCtl* qc) {
  if (n == 0) return hipSuccess;
  if (!next) grid = n;
  if (qc && !next) return hipErrorInvalidValue;
  if (grid == 0 || (grid > n && !qc)) return hipErrorInvalidValue;
#define REI_BATCH_L(WW, II, TT)                                                                          \
  launch_timed(solve_batch<WW, II, std::min(TT, batch_max_threads(WW))>, dim3(grid), dim3(TT), 0, s, d_descs, n, \
               order, next, qc)
#define REI_BATCH_T(WW, II)                                              \
  if (threads > batch_max_threads(WW)) return hipErrorInvalidValue;      \
  switch (threads) {                                                     \
    case 256: REI_BATCH_L(WW, II, 256u); break;                          \
    case 512: REI_BATCH_L(WW, II, 512u); break;                          \
    case 1024: REI_BATCH_L(WW, II, 1024u); break;                        \
    default: return hipErrorInvalidValue;                                \
  }
  switch (W) {
    case 1:
      if (inl) {
        REI_BATCH_T(1, true)
      } else {
        REI_BATCH_T(1, false)
      }
      break;
    case 2: REI_BATCH_T(2, false) break;
    case 4: REI_BATCH_T(4, false) break;
    case 8: REI_BATCH_T(8, false) break;
    case 16: REI_BATCH_T(16, false) break;
    case 32: REI_BATCH_T(32, false) break;
    default: return hipErrorInvalidValue;
  }
#undef REI_BATCH_L
#undef REI_BATCH_T
  return hipGetLastError();
}

hipError_t batch_resident(int W, bool inl, uint32_t threads, uint32_t* per_cu) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define REI_OCC_L(WW, II, TT)                                                                          \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_batch<WW, II, std::min(TT, batch_max_threads(WW))>, \
                                                   (int)TT, 0)
#define REI_OCC(WW, II)                                              \
  if (threads > batch_max_threads(WW)) return hipErrorInvalidValue;  \
  switch (threads) {                                                 \
    case 256: REI_OCC_L(WW, II, 256u); break;                        \
    case 512: REI_OCC_L(WW, II, 512u); break;                        \
    case 1024: REI_OCC_L(WW, II, 1024u); break;                      \
    default: return hipErrorInvalidValue;                            \
  }
  switch (W) {
    case 1:
      if (inl) {
        REI_OCC(1, true)
      } else {
        REI_OCC(1, false)
      }
      break;
    case 2: REI_OCC(2, false) break;
    case 4: REI_OCC(4, false) break;
    case 8: REI_OCC(8, false) break;
    case 16: REI_OCC(16, false) break;
    case 32: REI_OCC(32, false) break;
    default: return hipErrorInvalidValue;
  }
#undef REI_OCC_L
#undef REI_OCC
  if (e == hipSuccess) *per_cu = (uint32_t)std::max(nb, 1);
  return e;
}

hipError_t launch_put_descs(BatchDesc* dst, const BatchDesc* src, uint32_t n, hipStream_t s) {
  for (uint32_t k = 0; k < n; k += kDescPack) {
    DescPack p;
    p.n = std::min<uint32_t>(kDescPack, n - k);
    for (uint32_t i = 0; i < p.n; ++i) p.d[i] = src[k + i];
    hipLaunchKernelGGL(put_descs, dim3(1), dim3(256), 0, s, dst + k, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t static_scratch(void** out) {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static void* addr[kDevices] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_reset_counters(uint32_t* c, uint32_t n, hipStream_t s) {
  if (n == 0 || n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, c, n);
  return hipGetLastError();
}

}  // namespace rei
