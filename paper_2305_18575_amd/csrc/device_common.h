// Device helpers shared by the per-chunk grid kernels and the batched
// workgroup solver: hashing, the wave bit-matrix transpose, the dedup probe
// with survivor append, and index decoding.
#pragma once

#include "internal.h"

namespace rei {
namespace {

constexpr int kWave = 64;

// 64-bit finalizer of MurmurHash3 (fmix64, Austin Appleby's published
// constants): every input bit affects every output bit.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Bits of the language hash that are kept: all, unless a test narrows them
// to force collisions, equal fingerprints and long probe sequences (results
// must not change).  Each translation unit has its own copy (set_hash_mask).
__constant__ uint64_t g_hash_mask = ~0ull;

template <int W>
__device__ __forceinline__ uint64_t hash_key(const uint64_t (&k)[W]) {
  uint64_t h = mix64(k[0] ^ 0x9e3779b97f4a7c15ull);
#pragma unroll
  for (int i = 1; i < W; ++i) h = mix64(h ^ k[i]);
  return h & g_hash_mask;
}

__device__ __forceinline__ uint64_t fingerprint(uint64_t h) { return (h >> 40) & 0xFFFFFFull; }

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The value of lane (lane ^ J) for one 32-bit register, J a power of two
// below 64, by the cheapest cross-lane route: DPP quad permutes for 1 and 2,
// a DPP rotate by 8 within each 16-lane row for 8 (i + 8 mod 16 = i ^ 8),
// a ds_swizzle in bit-mask mode (and 0x1f, xor J, within 32 lanes) for 4
// and 16, and a ds_bpermute for 32.
template <int J>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v) {
  if constexpr (J == 1)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
  else if constexpr (J == 2)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  else if constexpr (J == 8)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);  // row_ror:8
  else if constexpr (J == 4 || J == 16)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
  else
    return (uint32_t)__shfl_xor((int)v, J, kWave);
}

// One stage of the transpose on one 32-bit half, J < 32: swaps bit J of the
// row index with bit J of the column index.  M has the bits whose index has
// bit J clear.  A lane with bit J clear keeps its M bits and takes the
// partner's M bits moved up by J (a left rotate by J puts them there); a
// lane with bit J set keeps ~M and takes the partner's ~M bits moved down
// (a right rotate by J).  One cross-lane move, one rotate (alignbit with a
// per-lane amount), one bit select.
template <int J, uint32_t M>
__device__ __forceinline__ uint32_t transpose_stage32(uint32_t x, uint32_t lane) {
  const bool up = (lane & J) != 0;
  const uint32_t keep = up ? ~M : M;
  const uint32_t rot = up ? (uint32_t)J : 32u - J;  // right-rotate amount
  const uint32_t b = lane_xor32<J>(x);
  const uint32_t moved = __builtin_amdgcn_alignbit(b, b, rot);
  return (x & keep) | (moved & ~keep);
}

// 64x64 bit-matrix transpose across a wave: on entry lane r holds row r, on
// exit lane c holds column c (bit r of the result = bit c of row r).  The
// first stage (bit 5) exchanges 32-bit halves between lanes 32 apart; the
// other five work on each half alone.
__device__ __forceinline__ uint64_t transpose64(uint64_t a) {
  const uint32_t lane = lane_id();
  uint32_t lo = (uint32_t)a, hi = (uint32_t)(a >> 32);
  {
    const uint32_t blo = lane_xor32<32>(lo), bhi = lane_xor32<32>(hi);
    const bool up = (lane & 32) != 0;
    const uint32_t nlo = up ? bhi : lo, nhi = up ? hi : blo;
    lo = nlo;
    hi = nhi;
  }
  lo = transpose_stage32<16, 0x0000FFFFu>(lo, lane);
  hi = transpose_stage32<16, 0x0000FFFFu>(hi, lane);
  lo = transpose_stage32<8, 0x00FF00FFu>(lo, lane);
  hi = transpose_stage32<8, 0x00FF00FFu>(hi, lane);
  lo = transpose_stage32<4, 0x0F0F0F0Fu>(lo, lane);
  hi = transpose_stage32<4, 0x0F0F0F0Fu>(hi, lane);
  lo = transpose_stage32<2, 0x33333333u>(lo, lane);
  hi = transpose_stage32<2, 0x33333333u>(hi, lane);
  lo = transpose_stage32<1, 0x55555555u>(lo, lane);
  hi = transpose_stage32<1, 0x55555555u>(hi, lane);
  return ((uint64_t)hi << 32) | lo;
}

// The W words of row `row` (zeros when !valid), read as 16-byte loads that
// are all issued before any is used (rows are 16-byte aligned for W >= 2).
template <int W>
__device__ __forceinline__ void load_row(const uint64_t* rows, uint64_t row, bool valid, uint64_t (&v)[W]) {
  if constexpr (W == 1) {
    v[0] = valid ? rows[row] : 0ull;
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = 0;
    if (valid) {
      const ulonglong2* p = reinterpret_cast<const ulonglong2*>(rows + row * W);
      ulonglong2 t[W / 2];
#pragma unroll
      for (int k = 0; k < W / 2; ++k) t[k] = p[k];
#pragma unroll
      for (int k = 0; k < W / 2; ++k) {
        v[2 * k] = t[k].x;
        v[2 * k + 1] = t[k].y;
      }
    }
  }
}

// Copies n 32-bit values from global memory to LDS with threads tid, tid +
// nt, ...: 16-byte loads, four in flight per thread, when both ends are
// 16-byte aligned; single values otherwise and for the tail.
__device__ __forceinline__ void stage_u32(uint32_t* dst, const uint32_t* src, uint32_t n, uint32_t tid, uint32_t nt) {
  uint32_t done = 0;
  if ((((size_t)dst | (size_t)src) & 15) == 0) {
    const uint32_t n4 = n / 4;
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    uint32_t q = tid;
    for (; q + 3 * nt < n4; q += 4 * nt) {
      const uint4 v0 = s4[q], v1 = s4[q + nt], v2 = s4[q + 2 * nt], v3 = s4[q + 3 * nt];
      d4[q] = v0;
      d4[q + nt] = v1;
      d4[q + 2 * nt] = v2;
      d4[q + 3 * nt] = v3;
    }
    for (; q < n4; q += nt) d4[q] = s4[q];
    done = 4 * n4;
  }
  uint32_t q = done + tid;
  for (; q + 3 * nt < n; q += 4 * nt) {
    const uint32_t v0 = src[q], v1 = src[q + nt], v2 = src[q + 2 * nt], v3 = src[q + 3 * nt];
    dst[q] = v0;
    dst[q + nt] = v1;
    dst[q + 2 * nt] = v2;
    dst[q + 3 * nt] = v3;
  }
  for (; q < n; q += nt) dst[q] = src[q];
}

// One word of the star's fixed point: OR over the cuts q = 1..l of a word of
// length l (guide entries gt[off + q], cut 0 being u = eps) of X(u) & Y(v),
// four cuts' reads in flight at a time (l is the same for every lane).
template <typename GT>
__device__ __forceinline__ uint64_t star_fold(const uint64_t* X, const uint64_t* Y, GT gt, uint32_t off, uint32_t l) {
  uint64_t acc = 0;
  uint32_t q = 1;
  for (; q + 3 <= l; q += 4) {
    const uint32_t p0 = gt[off + q], p1 = gt[off + q + 1], p2 = gt[off + q + 2], p3 = gt[off + q + 3];
    acc |= (X[p0 >> 16] & Y[p0 & 0xFFFFu]) | (X[p1 >> 16] & Y[p1 & 0xFFFFu]) | (X[p2 >> 16] & Y[p2 & 0xFFFFu]) |
           (X[p3 >> 16] & Y[p3 & 0xFFFFu]);
  }
  for (; q <= l; ++q) {
    const uint32_t p = gt[off + q];
    acc |= X[p >> 16] & Y[p & 0xFFFFu];
  }
  return acc;
}

// ---- dedup table -----------------------------------------------------------
// Fingerprint form (any W): a slot holds EMPTY, a stored row
// (0 | fingerprint | row) or a survivor of the running chunk (1 | e | sid);
// equal keys are confirmed against the row or the survivor's key.
// Inline form (kInl: one word per language and |ic| <= 63, so no language is
// all ones): a slot holds the key itself; sref[pos] holds the smallest
// survivor reference of the running chunk for that key (EMPTY otherwise).
// A probe is then a single read.

template <int W>
__device__ __forceinline__ bool key_eq(const uint64_t* p, const uint64_t (&key)[W]) {
  bool eq = true;
#pragma unroll
  for (int k = 0; k < W; ++k) eq = eq && p[k] == key[k];
  return eq;
}

__device__ __forceinline__ uint64_t new_ref(uint32_t e, uint32_t sid) {
  return kNewFlag | ((uint64_t)e << 32) | sid;
}

// Is the key stored?  The table holds stored rows only while generators run.
template <int W, bool kInl>
__device__ __forceinline__ bool table_find(const uint64_t* slots, uint64_t mask, const uint64_t* rows,
                                           const uint64_t (&key)[W], uint64_t h) {
  uint64_t pos = h & mask;
  if constexpr (kInl) {
    for (;;) {
      const uint64_t v = slots[pos];
      if (v == kEmpty) return false;
      if (v == key[0]) return true;
      pos = (pos + 1) & mask;
    }
  } else {
    const uint64_t fp = fingerprint(h);
    for (;;) {
      const uint64_t v = slots[pos];
      if (v == kEmpty) return false;
      if (((v >> kRowBits) & 0xFFFFFFull) == fp && key_eq<W>(rows + (v & kRowMask) * W, key)) return true;
      pos = (pos + 1) & mask;
    }
  }
}

// Inserts a survivor (reference `mine` = 1 | e | sid); equal keys meet in one
// slot and keep the smallest reference.  Returns the slot.
template <int W, bool kInl>
__device__ __forceinline__ uint64_t table_insert(uint64_t* slots, uint64_t* sref, uint64_t mask,
                                                 const uint64_t* rows, const uint64_t* skey,
                                                 const uint64_t (&key)[W], uint64_t h, uint64_t mine) {
  uint64_t pos = h & mask;
  if constexpr (kInl) {
    for (;;) {
      uint64_t v = slots[pos];
      if (v == kEmpty) {
        v = atomicCAS((unsigned long long*)&slots[pos], (unsigned long long)kEmpty,
                      (unsigned long long)key[0]);
        if (v == kEmpty) v = key[0];  // claimed
      }
      if (v == key[0]) {
        atomicMin((unsigned long long*)&sref[pos], (unsigned long long)mine);
        return pos;
      }
      pos = (pos + 1) & mask;
    }
  } else {
    const uint64_t fp = fingerprint(h);
    for (;;) {
      uint64_t v = slots[pos];
      if (v == kEmpty) {
        v = atomicCAS((unsigned long long*)&slots[pos], (unsigned long long)kEmpty,
                      (unsigned long long)mine);
        if (v == kEmpty) return pos;  // claimed
      }
      if (v & kNewFlag) {
        // another survivor owns the slot; its key never changes
        if (key_eq<W>(skey + (uint64_t)(uint32_t)v * W, key)) {
          atomicMin((unsigned long long*)&slots[pos], (unsigned long long)mine);
          return pos;
        }
      } else if (((v >> kRowBits) & 0xFFFFFFull) == fp && key_eq<W>(rows + (v & kRowMask) * W, key)) {
        return pos;  // stored already (the generators filter these; kept for safety)
      }
      pos = (pos + 1) & mask;
    }
  }
}

// A survivor's slot record (spos): written by the generator as the key's
// hash, replaced at insertion by the slot position with the hash's 24-bit
// fingerprint above bit 40 (table positions stay below 2^40), so that
// inserting and publishing a survivor never hash its key again.
constexpr uint64_t kPosMask = (1ull << 40) - 1;
__device__ __forceinline__ uint64_t spos_pack(uint64_t pos, uint64_t h) { return pos | (fingerprint(h) << 40); }

// After all inserts of the chunk: does `mine` own its key's slot?  rec is
// the survivor's slot record.
template <bool kInl>
__device__ __forceinline__ bool table_is_winner(const uint64_t* slots, const uint64_t* sref, uint64_t rec,
                                                uint64_t mine) {
  const uint64_t pos = rec & kPosMask;
  return kInl ? sref[pos] == mine : slots[pos] == mine;
}

// The winner (slot record rec) is now stored as `row`.
template <bool kInl>
__device__ __forceinline__ void table_publish(uint64_t* slots, uint64_t* sref, uint64_t rec, uint64_t row) {
  const uint64_t pos = rec & kPosMask;
  if constexpr (kInl)
    sref[pos] = kEmpty;  // the key is in the slot already
  else
    slots[pos] = ((rec >> 40) << kRowBits) | row;
}

// Stores a row's key during a rebuild (all keys distinct).
template <int W, bool kInl>
__device__ __forceinline__ void table_rebuild_one(uint64_t* slots, uint64_t mask, const uint64_t (&key)[W],
                                                  uint64_t row) {
  const uint64_t h = hash_key<W>(key);
  const uint64_t v = kInl ? key[0] : ((fingerprint(h) << kRowBits) | row);
  uint64_t pos = h & mask;
  while (atomicCAS((unsigned long long*)&slots[pos], (unsigned long long)kEmpty, (unsigned long long)v) !=
         kEmpty)
    pos = (pos + 1) & mask;
}

// Examples a language misclassifies: positives it lacks, negatives it has.
template <int W>
__device__ __forceinline__ int misclassified(const uint64_t* pmask, const uint64_t* nmask,
                                             const uint64_t (&key)[W]) {
  int bad = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) bad += __popcll(pmask[k] & ~key[k]) + __popcll(nmask[k] & key[k]);
  return bad;
}

// Where a generator probes: the cache rows and the dedup table, and the
// precision masks.
struct Probe {
  const uint64_t* rows;
  const uint64_t* slots;
  uint64_t slot_mask;
  const uint64_t* pmask;
  const uint64_t* nmask;
  uint32_t max_err;
};

// Where survivors go: keys, chunk-relative indices, the survivor counter and
// the smallest precise index (counters may live in global memory or LDS).
struct Sink {
  uint64_t* skey;
  uint32_t* se;
  uint64_t* spos;  // the survivor's hash, for its insertion
  uint32_t* n_surv;
  uint32_t* answer_e;
};

// Probe the table for the candidate's language and append it as a survivor
// if it is not stored yet; survivors that satisfy the specification (at most
// max_err misclassified examples) lower answer_e.  Must be called by every
// lane of the wave.
template <int W, bool kInl>
__device__ __forceinline__ void filter_emit(const Probe& a, const Sink& o, bool valid, bool known_dup,
                                            const uint64_t (&key)[W], uint32_t e_rel) {
  bool surv = false;
  uint64_t h = 0;
  if (valid && !known_dup) {
    h = hash_key<W>(key);
    surv = !table_find<W, kInl>(a.slots, a.slot_mask, a.rows, key, h);
  }
  const uint64_t m = __ballot(surv);
  if (m == 0) return;
  const uint32_t lane = lane_id();
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if ((int)lane == leader) base = atomicAdd(o.n_surv, (uint32_t)__popcll(m));
  base = __shfl((int)base, leader, kWave);
  if (surv) {
    const uint32_t sid = base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
    uint64_t* dst = o.skey + (uint64_t)sid * W;
#pragma unroll
    for (int k = 0; k < W; ++k) dst[k] = key[k];
    o.se[sid] = e_rel;
    o.spos[sid] = h;
    if (misclassified<W>(a.pmask, a.nmask, key) <= (int)a.max_err) atomicMin(o.answer_e, e_rel);
  }
}

// Exclusive prefix sums of the popcounts of bm[0, words) into pre[], by one
// wave (all 64 lanes call it; words <= 64 * kPer); returns the total.  Lane
// l takes words l*kPer .. l*kPer + kPer - 1, so one shuffle scan over the
// lanes replaces a workgroup-wide scan with a barrier per step.
template <int kPer>
__device__ __forceinline__ uint32_t wave_popc_scan(const uint32_t* bm, uint32_t* pre, uint32_t words) {
  const uint32_t lane = lane_id();
  uint32_t c[kPer];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t idx = lane * kPer + k;
    c[k] = idx < words ? (uint32_t)__popc(bm[idx]) : 0u;
    sum += c[k];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)incl, off, kWave);
    if ((int)lane >= off) incl += v;
  }
  uint32_t run = incl - sum;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t idx = lane * kPer + k;
    if (idx < words) pre[idx] = run;
    run += c[k];
  }
  return (uint32_t)__shfl((int)incl, kWave - 1, kWave);
}

// Orders a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Pairs (i, j) with i < j of an n-row level, row-major: index of the first
// pair of row i is i*n - i*(i+1)/2.
__device__ __forceinline__ void tri_decode(uint64_t e, uint64_t n, uint64_t* pi, uint64_t* pj) {
  const double b = 2.0 * (double)n - 1.0;
  double d = b * b - 8.0 * (double)e;
  if (d < 0) d = 0;
  int64_t i = (int64_t)((b - sqrt(d)) * 0.5);
  if (i < 0) i = 0;
  auto first = [n](int64_t r) -> uint64_t { return (uint64_t)r * n - (uint64_t)r * (uint64_t)(r + 1) / 2; };
  while (i > 0 && first(i) > e) --i;
  while ((uint64_t)(i + 1) < n && first(i + 1) <= e) ++i;
  *pi = (uint64_t)i;
  *pj = (uint64_t)i + 1 + (e - first(i));
}

}  // namespace
}  // namespace rei
