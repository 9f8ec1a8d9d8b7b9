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

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor((int)lo, m, kWave);
  hi = __shfl_xor((int)hi, m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// 64x64 bit-matrix transpose across a wave: on entry lane r holds row r, on
// exit lane c holds column c (bit r of the result = bit c of row r).  Each
// stage swaps one bit of the row index with the same bit of the column index.
__device__ __forceinline__ uint64_t transpose64(uint64_t a) {
  const uint32_t lane = lane_id();
  const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                             0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int j = 32 >> s;
    const uint64_t m = masks[s];
    uint64_t b = shfl_xor64(a, j);
    a = (lane & j) ? ((a & ~m) | ((b >> j) & m)) : ((a & m) | ((b & m) << j));
  }
  return a;
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

// After all inserts of the chunk: does `mine` own its key's slot?
template <bool kInl>
__device__ __forceinline__ bool table_is_winner(const uint64_t* slots, const uint64_t* sref, uint64_t pos,
                                                uint64_t mine) {
  return kInl ? sref[pos] == mine : slots[pos] == mine;
}

// The winner's key is now stored as `row`.
template <int W, bool kInl>
__device__ __forceinline__ void table_publish(uint64_t* slots, uint64_t* sref, uint64_t pos,
                                              const uint64_t (&key)[W], uint64_t row) {
  if constexpr (kInl)
    sref[pos] = kEmpty;  // the key is in the slot already
  else
    slots[pos] = (fingerprint(hash_key<W>(key)) << kRowBits) | row;
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
  if (valid && !known_dup) surv = !table_find<W, kInl>(a.slots, a.slot_mask, a.rows, key, hash_key<W>(key));
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
