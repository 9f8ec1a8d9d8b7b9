// Device kernels of the REI search for CDNA4 (gfx950), wave64.
//
// One chunk of candidates (a contiguous range of level indices, spanning one
// or more constructor blocks of a cost level) goes through:
//   gen_*     build each candidate's language (characteristic sequence over
//             ic, W 64-bit words) and probe the dedup table read-only; a
//             candidate whose language is not yet stored is a survivor and
//             is appended with its chunk-relative index; precise survivors
//             lower ctrl->answer_e (Algorithm 2: uniqueness, then precision);
//   insert    survivors claim table slots; equal languages meet in one slot
//             and keep the smallest enumeration index (deterministic
//             atomicMin), so the first occurrence wins;
//   mark      winners set their bit in a per-chunk bitmap indexed by
//             enumeration index;
//   scan      exclusive prefix of the bitmap popcounts = rank of each winner
//             in enumeration order;
//   compact   winners before the answer are appended to the level in rank
//             order (new languages wait in temporary storage and only the
//             unique ones enter the cache: Sec. 3, GPU language cache).
#include <algorithm>

#include <cstdlib>

#include "device_common.h"

namespace rei {

namespace {

// Probe the table and append survivors (see filter_emit in device_common.h).
// In OnTheFly mode (Sec. 3) the cache is full: no probe and no survivors,
// only the precision test (a known duplicate equals a stored language, which
// is not precise, or the search would have stopped there).
template <int W, bool kInl>
__device__ __forceinline__ void filter_emit(const GenArgs& a, bool valid, bool known_dup,
                                            const uint64_t (&key)[W], uint32_t e_rel) {
  if (a.st->otf) {
    if (valid && !known_dup && misclassified<W>(a.pmask, a.nmask, key) <= (int)a.max_err)
      atomicMin(&a.ctrl->answer_e, e_rel);
    return;
  }
  const Probe p{a.rows, a.slots, a.slot_mask, a.pmask, a.nmask, a.max_err};
  const Sink k{a.skey, a.se, a.spos, &a.ctrl->n_surv, &a.ctrl->answer_e};
  filter_emit<W, kInl>(p, k, valid, known_dup, key, e_rel);
}

// ---- generators -----------------------------------------------------------

template <int W, bool kInl>
__global__ __launch_bounds__(256) void gen_char(GenArgs a) {
  if (a.st->stop) return;
  const uint64_t e = a.e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = e < a.e1;
  uint64_t key[W];
  const int idx = valid ? a.char_index[e] : -1;
#pragma unroll
  for (int k = 0; k < W; ++k) key[k] = (idx >= 0 && (idx >> 6) == k) ? (1ull << (idx & 63)) : 0ull;
  filter_emit<W, kInl>(a, valid, false, key, (uint32_t)(e - a.e0) + a.rel0);
}

// r? = eps + r; eps is word 0 of ic (shortlex puts the empty word first).
template <int W, bool kInl>
__global__ __launch_bounds__(256) void gen_question(GenArgs a) {
  if (a.st->stop) return;
  const uint64_t e = a.e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = e < a.e1;
  uint64_t key[W];
  const uint64_t* src = a.rows + (a.lstart + (valid ? e : 0)) * W;
#pragma unroll
  for (int k = 0; k < W; ++k) key[k] = valid ? src[k] : 0ull;
  const bool dup = (key[0] & 1ull) != 0;  // already contains eps: r? = r
  key[0] |= 1ull;
  filter_emit<W, kInl>(a, valid, dup, key, (uint32_t)(e - a.e0) + a.rel0);
}

// r* for 64 rows per workgroup, bit-sliced: Xt[w] / Yt[w] hold bit t = row t's
// membership of word w.  Y(eps) = 1 and, by increasing length,
// Y(w) = OR over cuts w = u v with u non-empty of X(u) & Y(v) (v is shorter).
template <int W, bool kInl>
__global__ __launch_bounds__(256) void gen_star(GenArgs a) {
  __shared__ uint64_t Xt[64 * W];
  __shared__ uint64_t Yt[64 * W];
  if (a.st->stop) return;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t base = a.e0 + (uint64_t)blockIdx.x * 64;
  for (int k = wave; k < W; k += 4) {
    const uint64_t e = base + lane;
    const uint64_t v = (e < a.e1) ? a.rows[(a.lstart + e) * W + k] : 0ull;
    Xt[64 * k + lane] = transpose64(v);
  }
  for (uint32_t w = threadIdx.x; w < 64u * W; w += 256) Yt[w] = (w == 0) ? ~0ull : 0ull;
  __syncthreads();
  for (uint32_t l = 1; l <= a.max_len; ++l) {
    const uint32_t lo = a.len_off[l], hi = a.len_off[l + 1];
    for (uint32_t w = lo + threadIdx.x; w < hi; w += 256)
      Yt[w] = star_fold(Xt, Yt, a.gt_pair, a.gt_off[w], l);  // cuts 1..l (cut 0 has u = eps)
    __syncthreads();
  }
  if (wave == 0) {
    uint64_t key[W];
#pragma unroll
    for (int k = 0; k < W; ++k) key[k] = transpose64(Yt[64 * k + lane]);
    const uint64_t e = base + lane;
    filter_emit<W, kInl>(a, e < a.e1, false, key, (uint32_t)(e - a.e0) + a.rel0);
  }
}

// x.y, bit-sliced over 64 right operands.  A workgroup owns YT tiles of 64
// rows of the right level (transposed into LDS: Yt[tile][w], bit t = row t
// contains word w) and a group of left rows.  For a left row x, lane l of a
// wave owns word w = 64k + l of output word k; the cuts (u, v) of w with u in
// x select which Yt[v] are or-ed:  out_t(w) = OR_{(u,v) cut of w, x(u)=1} y_t(v)
// (Algorithm 2, the fold over the guide table, done for 64 candidates at once).
// A wave transpose then gives lane t the W words of candidate (x, y_t).
constexpr int kConcatYT = 8;

// kShort: every word has at most 32 cuts (length <= 31), so the cuts whose
// prefix is in x fit one 32-bit mask per output word; otherwise the prefix
// bit is tested inside the fold.
// kGtLds: the guide table is staged in LDS.  The choice is made at compile
// time so that every access has a fixed address space: reading LDS through a
// generic pointer (chosen at run time between LDS and global memory) gave
// wrong prefix bits now and then on gfx950.
template <int W, bool kShort, bool kInl, bool kGtLds>
__global__ __launch_bounds__(256) void gen_concat(GenArgs a, ConcatSet cs) {
  extern __shared__ uint64_t lds[];
  if (a.st->stop) return;
  // this workgroup's part (block) and its place in the part's grid
  uint32_t part = 0;
  while (part + 1 < cs.n && cs.p[part + 1].wg0 <= blockIdx.x) ++part;
  const ConcatPart& cp = cs.p[part];
  a.lstart = cp.lstart;
  a.rstart = cp.rstart;
  a.rcount = cp.rcount;
  a.e0 = cp.e0;
  a.e1 = cp.e1;
  a.rel0 = cp.rel0;
  const uint32_t yt_per_wg = cp.yt, xi_per_wg = cp.xi, n_tile_groups = cp.gx;
  const uint64_t i_lo = cp.i_lo, i_hi = cp.i_hi;
  const uint32_t bid = blockIdx.x - cp.wg0;
  uint64_t* Yt = lds;                                        // [yt_per_wg][64W]
  uint64_t* Xs = Yt + (size_t)yt_per_wg * 64 * W;            // [xi_per_wg][W]
  uint32_t* G = (uint32_t*)(Xs + (size_t)xi_per_wg * W);     // guide pairs (if gt_lds)
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t nR = a.rcount;
  const uint64_t nT = (nR + 63) / 64;
  // flat grid: workgroup -> (group of right tiles, group of left rows)
  const uint64_t t0 = (uint64_t)(bid % n_tile_groups) * yt_per_wg;
  const uint32_t nt = (uint32_t)min<uint64_t>(yt_per_wg, nT - t0);
  const uint64_t x0 = i_lo + (uint64_t)(bid / n_tile_groups) * xi_per_wg;
  const uint32_t nx = (uint32_t)min<uint64_t>(xi_per_wg, i_hi + 1 - x0);

  // stage right tiles (transposed), left rows and guide table; every load
  // of a thread is issued before the first is used
  for (uint32_t tq = wave; tq < nt; tq += 4) {
    const uint64_t j = (t0 + tq) * 64 + lane;
    uint64_t v[W];
    load_row<W>(a.rows, a.rstart + j, j < nR, v);
#pragma unroll
    for (int k = 0; k < W; ++k) Yt[(size_t)tq * 64 * W + 64 * k + lane] = transpose64(v[k]);
  }
  {
    const uint64_t* src = a.rows + (a.lstart + x0) * W;
    const uint32_t total = nx * W;
    uint32_t q = threadIdx.x;
    for (; q + 3 * 256 < total; q += 4 * 256) {
      const uint64_t v0 = src[q], v1 = src[q + 256], v2 = src[q + 512], v3 = src[q + 768];
      Xs[q] = v0;
      Xs[q + 256] = v1;
      Xs[q + 512] = v2;
      Xs[q + 768] = v3;
    }
    for (; q < total; q += 256) Xs[q] = src[q];
  }
  if constexpr (kGtLds) stage_u32(G, a.gt_pair, a.n_pairs, threadIdx.x, 256);
  __syncthreads();
  const uint32_t* gp;
  if constexpr (kGtLds)
    gp = G;
  else
    gp = a.gt_pair;

  // cut ranges of this lane's words
  uint32_t off[W], cnt[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const uint32_t w = 64u * k + lane;
    off[k] = (w < a.n) ? a.gt_off[w] : 0u;
    cnt[k] = (w < a.n) ? a.gt_off[w + 1] - off[k] : 0u;
  }

  for (uint32_t xi = wave; xi < nx; xi += 4) {
    const uint64_t i = x0 + xi;
    const uint64_t* xr = Xs + (size_t)xi * W;
    // bit q of m[k]: x contains the prefix of cut q of word 64k+lane
    uint32_t m[W];
    if constexpr (kShort) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        uint32_t mm = 0;
        for (uint32_t q0 = 0; q0 < cnt[k]; q0 += 4) {
          // four cuts at a time: their reads overlap
          uint32_t u[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) u[t] = (q0 + t < cnt[k]) ? gp[off[k] + q0 + t] >> 16 : 0u;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (q0 + t < cnt[k]) mm |= (uint32_t)((xr[u[t] >> 6] >> (u[t] & 63)) & 1ull) << (q0 + t);
        }
        m[k] = mm;
      }
    }
    for (uint32_t tq = 0; tq < nt; ++tq) {
      const uint64_t* Y = Yt + (size_t)tq * 64 * W;
      uint64_t key[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        uint64_t acc = 0;
        if constexpr (kShort) {
          for (uint32_t mm = m[k]; mm; mm &= mm - 1) {
            const uint32_t q = __ffs(mm) - 1;
            acc |= Y[gp[off[k] + q] & 0xFFFFu];
          }
        } else {
          for (uint32_t q = 0; q < cnt[k]; ++q) {
            const uint32_t p = gp[off[k] + q];
            const uint32_t u = p >> 16;
            if ((xr[u >> 6] >> (u & 63)) & 1ull) acc |= Y[p & 0xFFFFu];
          }
        }
        key[k] = transpose64(acc);
      }
      const uint64_t j = (t0 + tq) * 64 + lane;
      const uint64_t e = i * nR + j;
      const bool valid = (j < nR) && (e >= a.e0) && (e < a.e1);
      filter_emit<W, kInl>(a, valid, false, key, (uint32_t)(e - a.e0) + a.rel0);
    }
  }
}

// One thread per candidate x + y; several union blocks of a chunk share a
// launch (UnionSet), each workgroup in one block.
template <int W, bool kInl>
__global__ __launch_bounds__(256) void gen_union(GenArgs a, UnionSet us) {
  if (a.st->stop) return;
  uint32_t part = 0;
  while (part + 1 < us.n && us.p[part + 1].wg0 <= blockIdx.x) ++part;
  const UnionPart& up = us.p[part];
  a.e0 = up.e0;
  a.rel0 = up.rel0;
  const uint64_t e = up.e0 + (uint64_t)(blockIdx.x - up.wg0) * blockDim.x + threadIdx.x;
  const bool valid = e < up.e1;
  uint64_t i = 0, j = 0;
  if (valid) {
    if (up.same) {
      tri_decode(e, up.lcount, &i, &j);
    } else {
      i = e / up.rcount;
      j = e - i * up.rcount;
    }
  }
  const uint64_t* x = a.rows + (up.lstart + i) * W;
  const uint64_t* y = a.rows + (up.rstart + j) * W;
  uint64_t key[W];
  bool eqx = true, eqy = true;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const uint64_t xv = valid ? x[k] : 0ull, yv = valid ? y[k] : 0ull;
    key[k] = xv | yv;
    eqx = eqx && key[k] == xv;
    eqy = eqy && key[k] == yv;
  }
  // x+y equals x or y (one contains the other): that language is stored
  filter_emit<W, kInl>(a, valid, eqx || eqy, key, (uint32_t)(e - a.e0) + a.rel0);
}

// Many small pieces of one chunk (see PieceArgs): one wave per item of 64
// candidates, so a level's small constructor blocks cost one launch.  The
// constructors are those of the kernels above, at wave scale; the guide
// table is read through the caches.

// An item of 64 candidates of a CHAR, QUESTION, UNION or STAR piece (the
// star with the wave's tiles X and Y): lane t's candidate key.
template <int W>
__device__ __forceinline__ void piece_simple(const GenArgs& a, const PieceD& p, uint64_t li, uint32_t lane,
                                             uint64_t* X, uint64_t* Y, uint64_t (&key)[W], bool* valid,
                                             bool* dup, uint64_t* e_out) {
  const uint64_t e = p.e0 + 64 * li + lane;
  *valid = e < p.e1;
  *dup = false;
  *e_out = e;
  if (p.op == OP_CHAR) {
    const int idx = *valid ? a.char_index[p.char_off + e] : -1;
#pragma unroll
    for (int q = 0; q < W; ++q) key[q] = (idx >= 0 && (idx >> 6) == q) ? (1ull << (idx & 63)) : 0ull;
  } else if (p.op == OP_QUESTION) {
    const uint64_t* src = a.rows + (p.lstart + (*valid ? e : 0)) * W;
#pragma unroll
    for (int q = 0; q < W; ++q) key[q] = *valid ? src[q] : 0ull;
    *dup = (key[0] & 1ull) != 0;
    key[0] |= 1ull;
  } else if (p.op == OP_UNION) {
    uint64_t i = 0, j = 0;
    if (*valid) {
      if (p.same) {
        tri_decode(e, p.lcount, &i, &j);
      } else {
        i = e / p.rcount;
        j = e - i * p.rcount;
      }
    }
    const uint64_t* x = a.rows + (p.lstart + i) * W;
    const uint64_t* y = a.rows + (p.rstart + j) * W;
    bool eqx = true, eqy = true;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const uint64_t xv = *valid ? x[q] : 0ull, yv = *valid ? y[q] : 0ull;
      key[q] = xv | yv;
      eqx = eqx && key[q] == xv;
      eqy = eqy && key[q] == yv;
    }
    *dup = eqx || eqy;
  } else {  // OP_STAR: Y(eps) = 1; by increasing length, Y(w) = OR over
            // cuts with a non-empty first factor of X(u) & Y(v)
#pragma unroll
    for (int q = 0; q < W; ++q) {
      X[64 * q + lane] = transpose64(*valid ? a.rows[(p.lstart + e) * W + q] : 0ull);
      Y[64 * q + lane] = (q == 0 && lane == 0) ? ~0ull : 0ull;
    }
    wave_sync_lds();
    for (uint32_t l = 1; l <= a.max_len; ++l) {
      const uint32_t lo = a.len_off[l], hi = a.len_off[l + 1];
      for (uint32_t w = lo + lane; w < hi; w += 64) Y[w] = star_fold(X, Y, a.gt_pair, a.gt_off[w], l);
      wave_sync_lds();
    }
#pragma unroll
    for (int q = 0; q < W; ++q) key[q] = transpose64(Y[64 * q + lane]);
  }
}

// A CONCAT item: its varying operand's rows across the lanes (right rows
// with one left row, or left rows with one right row when the right level
// is small), staged transposed in X for words [q_lo, q_hi), the uniform
// operand's row in U (when stage_u).  Returns lane t's candidate index and
// whether it is one.
template <int W>
__device__ __forceinline__ void concat_stage(const GenArgs& a, const PieceD& p, uint64_t li, uint32_t lane,
                                             uint64_t* X, uint64_t* U, int q_lo, int q_hi, bool stage_u,
                                             uint64_t* e_out, bool* valid) {
  const uint64_t nR = p.rcount, nL = p.lcount;
  uint64_t i, j, row, urow;
  bool have;
  if (!p.left_lanes) {
    i = p.t0 + li / p.nt;
    j = 64 * (li % p.nt) + lane;
    have = j < nR;
    row = p.rstart + j;
    urow = p.lstart + i;
  } else {
    i = 64 * (p.t0 + li / p.nt) + lane;
    j = li % p.nt;
    have = i < nL;
    row = p.lstart + i;
    urow = p.rstart + j;
  }
#pragma unroll
  for (int q = 0; q < W; ++q)
    if (q >= q_lo && q < q_hi) X[64 * q + lane] = transpose64(have ? a.rows[row * W + q] : 0ull);
  if (stage_u && lane < (uint32_t)W) U[lane] = a.rows[urow * W + lane];
  const uint64_t e = i * nR + j;
  *e_out = e;
  *valid = have && e >= p.e0 && e < p.e1;
}

// The fold of a CONCAT item for output words [q_lo, q_hi) (X and U staged;
// q_lo and q_hi multiples of kG): key[q] for those q.  From 8 words, cut
// position outer over kG of the lane's words at a time, 3 kG independent
// reads per round (each word's read clamped to its last cut, masked
// after); below, per word.
template <int W, int kG = 8>
__device__ __forceinline__ void concat_fold(const GenArgs& a, const PieceD& p, uint32_t lane, const uint64_t* X,
                                            const uint64_t* U, int q_lo, int q_hi, uint64_t (&key)[W]) {
  if constexpr (W >= 8) {
#pragma unroll
    for (int q0 = 0; q0 < W; q0 += kG) {
      if (q0 < q_lo || q0 >= q_hi) continue;
      uint32_t first[kG], last[kG], cnt[kG];
      uint64_t acc[kG];
#pragma unroll
      for (int q = 0; q < kG; ++q) {
        const uint32_t w = 64u * (q0 + q) + lane;
        first[q] = w < a.n ? a.gt_off[w] : 0u;
        cnt[q] = w < a.n ? a.gt_off[w + 1] - first[q] : 0u;
        last[q] = first[q] + (cnt[q] ? cnt[q] - 1 : 0u);
        acc[q] = 0;
      }
      for (uint32_t c = 0; c <= a.max_len; ++c) {
        uint32_t pr[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) pr[q] = a.gt_pair[min(first[q] + c, last[q])];
#pragma unroll
        for (int q = 0; q < kG; ++q) {
          const uint32_t uu = p.left_lanes ? (pr[q] & 0xFFFFu) : (pr[q] >> 16);  // index into the uniform row
          const uint32_t tt = p.left_lanes ? (pr[q] >> 16) : (pr[q] & 0xFFFFu);  // index into the tile
          const uint64_t xv = X[tt];
          const bool on = c < cnt[q] && ((U[uu >> 6] >> (uu & 63)) & 1ull);
          acc[q] |= on ? xv : 0ull;
        }
      }
#pragma unroll
      for (int q = 0; q < kG; ++q) key[q0 + q] = transpose64(acc[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < W; ++q) {
      if (q < q_lo || q >= q_hi) continue;
      const uint32_t w = 64u * q + lane;
      uint64_t acc = 0;
      if (w < a.n) {
        const uint32_t q1 = a.gt_off[w + 1];
        for (uint32_t c = a.gt_off[w]; c < q1; ++c) {
          const uint32_t pr = a.gt_pair[c];
          const uint32_t uu = p.left_lanes ? (pr & 0xFFFFu) : (pr >> 16);   // index into the uniform row
          const uint32_t tt = p.left_lanes ? (pr >> 16) : (pr & 0xFFFFu);   // index into the tile
          if ((U[uu >> 6] >> (uu & 63)) & 1ull) acc |= X[tt];
        }
      }
      key[q] = transpose64(acc);
    }
  }
}

__device__ __forceinline__ uint32_t piece_of(const PieceArgs& pa, uint64_t it) {
  uint32_t k = 0;
  while (k + 1 < pa.n && pa.p[k + 1].item0 <= it) ++k;
  return k;
}

// kSplit (from 16 words, launches of few items, where one item's latency
// is the launch's): kSplit waves (2 or 4) share each CONCAT item, each
// staging and folding W / kSplit of the words, and each STAR item (each
// stages its words; the words of each length are dealt to all of them);
// the others hand their key words to the first through LDS, which probes.
// Other items are the first wave's.
template <int W, bool kInl, int kSplit>
__global__ __launch_bounds__(256) void gen_pieces(GenArgs a, PieceArgs pa) {
  __shared__ uint64_t lds[4][2 * 64 * W + W];
  if (a.st->stop) return;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (kSplit == 1) {
    uint64_t* X = lds[wave];       // star: X tile; concat: operand tile
    uint64_t* Y = X + 64 * W;      // star: Y tile
    uint64_t* U = Y + 64 * W;      // concat: the uniform operand
    for (uint64_t it = (uint64_t)blockIdx.x * 4 + wave; it < pa.items; it += (uint64_t)gridDim.x * 4) {
      const PieceD& p = pa.p[piece_of(pa, it)];
      const uint64_t li = it - p.item0;
      uint64_t key[W];
      bool valid = false, dup = false;
      uint64_t e = 0;
      if (p.op != OP_CONCAT) {
        piece_simple<W>(a, p, li, lane, X, Y, key, &valid, &dup, &e);
      } else {
        concat_stage<W>(a, p, li, lane, X, U, 0, W, true, &e, &valid);
        wave_sync_lds();
        concat_fold<W>(a, p, lane, X, U, 0, W, key);
      }
      filter_emit<W, kInl>(a, valid, dup, key, valid ? (uint32_t)(e - p.e0) + p.rel0 : 0u);
      wave_sync_lds();  // the tiles are rewritten by the next item
    }
  } else {
    constexpr int kPart = W / kSplit;          // words per wave
    constexpr int kG = kPart < 8 ? kPart : 8;  // fold group
    constexpr uint32_t kItems = 4 / kSplit;    // items per workgroup round
    static_assert((kSplit == 2 || kSplit == 4) && kPart >= 4 && kPart % kG == 0, "whole fold groups per wave");
    const uint32_t slot = wave / kSplit, part = wave % kSplit;
    uint64_t* X = lds[kSplit * slot];
    uint64_t* Y = X + 64 * W;
    uint64_t* U = Y + 64 * W;
    uint64_t* K = lds[kSplit * slot + 1];  // the other waves' key words, [q - kPart][lane]
    const int q_lo = (int)part * kPart, q_hi = q_lo + kPart;  // this wave's words
    // every wave takes the same number of rounds (workgroup barriers inside)
    for (uint64_t base = (uint64_t)blockIdx.x * kItems; base < pa.items; base += (uint64_t)gridDim.x * kItems) {
      const uint64_t it = base + slot;
      const bool have = it < pa.items;
      const PieceD& p = pa.p[have ? piece_of(pa, it) : 0];
      const uint64_t li = have ? it - p.item0 : 0;
      const bool cat = have && p.op == OP_CONCAT;
      const bool star = have && p.op == OP_STAR;
      uint64_t key[W];
      bool valid = false, dup = false;
      uint64_t e = 0;
      if (cat) concat_stage<W>(a, p, li, lane, X, U, q_lo, q_hi, part == 0, &e, &valid);
      if (star) {
        // r* of 64 rows: each wave stages its words of X and Y
        e = p.e0 + 64 * li + lane;
        valid = e < p.e1;
#pragma unroll
        for (int q = 0; q < W; ++q)
          if (q >= q_lo && q < q_hi) {
            X[64 * q + lane] = transpose64(valid ? a.rows[(p.lstart + e) * W + q] : 0ull);
            Y[64 * q + lane] = (q == 0 && lane == 0) ? ~0ull : 0ull;
          }
      }
      // (uniform over the workgroup: the star's barriers below are taken by
      // all of its waves or by none)
      const bool any_star = __syncthreads_or(star);
      if (any_star) {
        // Y(w) by increasing length from shorter words' Y: the words of one
        // length dealt to the item's waves, a barrier per length
        for (uint32_t l = 1; l <= a.max_len; ++l) {
          if (star) {
            const uint32_t lo = a.len_off[l], hi = a.len_off[l + 1];
            for (uint32_t w = lo + lane + 64 * part; w < hi; w += 64 * kSplit)
              Y[w] = star_fold(X, Y, a.gt_pair, a.gt_off[w], l);
          }
          __syncthreads();
        }
      }
      if (cat) concat_fold<W, kG>(a, p, lane, X, U, q_lo, q_hi, key);
      if (star) {
#pragma unroll
        for (int q = 0; q < W; ++q)
          if (q >= q_lo && q < q_hi) key[q] = transpose64(Y[64 * q + lane]);
      }
      if ((cat || star) && part != 0) {
#pragma unroll
        for (int q = 0; q < W; ++q)
          if (q >= q_lo && q < q_hi) K[64 * (q - kPart) + lane] = key[q];
      }
      __syncthreads();
      if (part == 0 && have) {
        if (cat || star) {
#pragma unroll
          for (int q = kPart; q < W; ++q) key[q] = K[64 * (q - kPart) + lane];
        } else {
          piece_simple<W>(a, p, li, lane, X, Y, key, &valid, &dup, &e);
        }
        filter_emit<W, kInl>(a, valid, dup, key, valid ? (uint32_t)(e - p.e0) + p.rel0 : 0u);
      }
      __syncthreads();  // the tiles are rewritten in the next round
    }
  }
}

// ---- chunk pipeline ------------------------------------------------------

__global__ void fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ void ctrl_clear(Ctrl* c) {
  c->n_surv = 0;
  c->answer_e = ~0u;
  c->answer_rank = ~0u;
  c->winners = 0;
  c->overflow_e = ~0u;
}

__global__ void state_reset(Ctrl* c, DevState* st, uint64_t row_cap, uint32_t otf_on) {
  ctrl_clear(c);
  st->total_rows = 0;
  st->row_cap = row_cap;
  st->stop = STOP_NONE;
  st->answer_cost = 0;
  st->answer_e = 0;
  st->resume_level = 0;
  st->otf_on = otf_on;
  st->otf = 0;
  st->chunks = 0;
}

template <int W, bool kInl>
__global__ __launch_bounds__(256) void rehash_rows(const uint64_t* rows, uint64_t nrows, uint64_t* slots,
                                                   uint64_t mask) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
       r += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t key[W];
#pragma unroll
    for (int k = 0; k < W; ++k) key[k] = rows[r * W + k];
    table_rebuild_one<W, kInl>(slots, mask, key, r);
  }
}

template <int W, bool kInl>
__global__ __launch_bounds__(256) void insert_survivors(ChunkArgs a) {
  if (a.st->stop) return;
  // the winner bitmap of the grid finalize path starts empty
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < a.clear_words; w += gridDim.x * blockDim.x)
    a.bitmap[w] = 0;
  const uint32_t ns = a.ctrl->n_surv;
  for (uint32_t sid = blockIdx.x * blockDim.x + threadIdx.x; sid < ns; sid += gridDim.x * blockDim.x) {
    uint64_t key[W];
#pragma unroll
    for (int k = 0; k < W; ++k) key[k] = a.skey[(uint64_t)sid * W + k];
    const uint64_t h = a.spos[sid];
    const uint64_t pos = table_insert<W, kInl>(a.slots, a.sref, a.slot_mask, a.rows, a.skey, key, h,
                                               new_ref(a.se[sid], sid));
    a.spos[sid] = spos_pack(pos, h);
  }
}

// Outcome of a chunk, in enumeration order: the answer (first precise
// candidate) if its winners before it fit the row cap, else out of memory at
// the first winner that does not fit; otherwise all winners are stored.
// With OnTheFly allowed, the first winner that does not fit switches the
// search to OnTheFly mode instead: the winners that fit are stored, and the
// rest of the chunk (and of the search) is tested for precision only.
__device__ void account_chunk(const ChunkArgs& a, uint32_t ans, uint32_t answer_rank, uint32_t winners,
                              uint32_t overflow_e) {
  DevState* st = a.st;
  const uint64_t room = st->row_cap > st->total_rows ? st->row_cap - st->total_rows : 0;
  const uint32_t c = a.cost;
  uint64_t stored;
  if (st->otf) {
    stored = 0;
    if (ans != ~0u) {
      a.cand[c] += (uint64_t)ans + 1;
      st->stop = STOP_ANSWER;
      st->answer_cost = c;
      st->answer_e = a.chunk_e0 + ans;
    } else {
      a.cand[c] += a.len;
    }
  } else if (ans != ~0u) {
    if ((uint64_t)answer_rank > room && st->otf_on) {
      // the cache filled before the answer, which is found on the fly
      stored = room;
      a.cand[c] += (uint64_t)ans + 1;
      a.uniq[c] += room;
      st->stop = STOP_ANSWER;
      st->answer_cost = c;
      st->answer_e = a.chunk_e0 + ans;
    } else if ((uint64_t)answer_rank > room) {
      stored = room;
      a.cand[c] += (uint64_t)overflow_e + 1;
      a.uniq[c] += room;
      st->stop = STOP_OOM;
    } else {
      stored = answer_rank;
      a.cand[c] += (uint64_t)ans + 1;
      a.uniq[c] += (uint64_t)answer_rank + 1;
      st->stop = STOP_ANSWER;
      st->answer_cost = c;
      st->answer_e = a.chunk_e0 + ans;
    }
  } else if ((uint64_t)winners > room && st->otf_on) {
    stored = room;
    a.cand[c] += a.len;
    a.uniq[c] += room;
    st->otf = 1;
  } else if ((uint64_t)winners > room) {
    stored = room;
    a.cand[c] += (uint64_t)overflow_e + 1;
    a.uniq[c] += room;
    st->stop = STOP_OOM;
  } else {
    stored = winners;
    a.cand[c] += a.len;
    a.uniq[c] += winners;
  }
  st->total_rows += stored;
  a.lcount[c] += stored;
  ctrl_clear(a.ctrl);
  // the host reads these at level boundaries without a copy
  DevState* h = a.hst;
  h->total_rows = st->total_rows;
  h->row_cap = st->row_cap;
  h->stop = st->stop;
  h->answer_cost = st->answer_cost;
  h->answer_e = st->answer_e;
  h->resume_level = st->resume_level;
  h->otf_on = st->otf_on;
  h->otf = st->otf;
  a.hlev[c] = a.lcount[c];
  a.hlev[a.nlev + c] = a.uniq[c];
  a.hlev[2 * a.nlev + c] = a.cand[c];
  // the count last: a host that sees it sees everything above
  st->chunks += 1;
  __hip_atomic_store(&h->chunks, st->chunks, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int W, bool kInl>
__device__ __forceinline__ void store_winner(const ChunkArgs& a, uint32_t sid, uint32_t e, uint64_t row) {
  uint64_t key[W];
#pragma unroll
  for (int k = 0; k < W; ++k) key[k] = a.skey[(uint64_t)sid * W + k];
  const uint64_t rec = a.spos[sid];
#pragma unroll
  for (int k = 0; k < W; ++k) a.rows_w[row * W + k] = key[k];
  a.aux[row] = a.chunk_e0 + e;
  table_publish<kInl>(a.slots, a.sref, rec, row);
}

constexpr uint32_t kSmallWords = (uint32_t)(kSmallChunk / 32);
constexpr uint64_t kSmallCopyWords = 1ull << 16;
static_assert(kSmallChunk <= 0xFFFFu, "survivor ranks of a small chunk fit 16 bits");

// Whole finalization of a small chunk in one workgroup: winner bitmap in LDS,
// its prefix scan, ordered append, accounting.
template <int W, bool kInl>
__global__ __launch_bounds__(1024) void finalize_small(ChunkArgs a) {
  __shared__ uint32_t bm[kSmallWords];
  __shared__ uint32_t pre[kSmallWords];
  __shared__ uint32_t s_rank, s_over, s_total;
  __shared__ uint16_t dst[W <= 2 ? 1 : kSmallChunk];  // wide rows: each survivor's rank
  constexpr uint32_t kNotStored = 0xFFFFu;             // ranks are below kSmallChunk
  if (a.st->stop) return;
  const uint32_t t = threadIdx.x;
  const uint32_t ns = a.ctrl->n_surv, ans = a.ctrl->answer_e;
  const uint32_t words = (uint32_t)((a.len + 31) / 32);
  for (uint32_t i = t; i < words; i += 1024) bm[i] = 0;
  if (t == 0) {
    s_rank = ~0u;
    s_over = ~0u;
  }
  __syncthreads();
  // four survivors per thread and round, their reads issued together
  auto mark = [&](uint32_t sid, uint32_t e, uint64_t pos) {
    if (table_is_winner<kInl>(a.slots, a.sref, pos, new_ref(e, sid))) atomicOr(&bm[e >> 5], 1u << (e & 31));
  };
  uint32_t sid = t;
  for (; sid + 3 * 1024 < ns; sid += 4 * 1024) {
    const uint32_t e0 = a.se[sid], e1 = a.se[sid + 1024], e2 = a.se[sid + 2048], e3 = a.se[sid + 3072];
    const uint64_t p0 = a.spos[sid], p1 = a.spos[sid + 1024], p2 = a.spos[sid + 2048], p3 = a.spos[sid + 3072];
    mark(sid, e0, p0);
    mark(sid + 1024, e1, p1);
    mark(sid + 2048, e2, p2);
    mark(sid + 3072, e3, p3);
  }
  for (; sid < ns; sid += 1024) mark(sid, a.se[sid], a.spos[sid]);
  __syncthreads();
  if (t < 64) {
    const uint32_t tot = wave_popc_scan<kSmallWords / 64>(bm, pre, words);
    if (t == 0) s_total = tot;
  }
  __syncthreads();
  const uint32_t total = s_total;
  const uint64_t row_base = a.st->total_rows;
  const uint64_t room = a.st->row_cap > row_base ? a.st->row_cap - row_base : 0;
  // each survivor's rank among the stored rows (kNotStored: not stored)
  auto place = [&](uint32_t sid, uint32_t e) -> uint32_t {
    const uint32_t word = bm[e >> 5];
    const uint32_t bit = 1u << (e & 31);
    if (!(word & bit)) return kNotStored;  // e is unique per survivor: the bit marks this one
    const uint32_t rank = pre[e >> 5] + (uint32_t)__popc(word & (bit - 1));
    if (e == ans) s_rank = rank;
    if (ans != ~0u && e >= ans) return kNotStored;  // the answer and later ones are not stored
    if (rank < room) return rank;
    if (rank == room) s_over = e;
    return kNotStored;
  };
  if constexpr (W <= 2) {
    sid = t;
    for (; sid + 3 * 1024 < ns; sid += 4 * 1024) {
      const uint32_t e0 = a.se[sid], e1 = a.se[sid + 1024], e2 = a.se[sid + 2048], e3 = a.se[sid + 3072];
      const uint32_t r0 = place(sid, e0), r1 = place(sid + 1024, e1), r2 = place(sid + 2048, e2),
                     r3 = place(sid + 3072, e3);
      if (r0 != kNotStored) store_winner<W, kInl>(a, sid, e0, row_base + r0);
      if (r1 != kNotStored) store_winner<W, kInl>(a, sid + 1024, e1, row_base + r1);
      if (r2 != kNotStored) store_winner<W, kInl>(a, sid + 2048, e2, row_base + r2);
      if (r3 != kNotStored) store_winner<W, kInl>(a, sid + 3072, e3, row_base + r3);
    }
    for (; sid < ns; sid += 1024) {
      const uint32_t e = a.se[sid];
      const uint32_t r = place(sid, e);
      if (r != kNotStored) store_winner<W, kInl>(a, sid, e, row_base + r);
    }
  } else {
    // wide rows: ranks first, then W consecutive lanes copy one row, so
    // that each wave reads and writes whole rows (coalesced)
    sid = t;
    for (; sid + 3 * 1024 < ns; sid += 4 * 1024) {
      const uint32_t e0 = a.se[sid], e1 = a.se[sid + 1024], e2 = a.se[sid + 2048], e3 = a.se[sid + 3072];
      dst[sid] = (uint16_t)place(sid, e0);
      dst[sid + 1024] = (uint16_t)place(sid + 1024, e1);
      dst[sid + 2048] = (uint16_t)place(sid + 2048, e2);
      dst[sid + 3072] = (uint16_t)place(sid + 3072, e3);
    }
    for (; sid < ns; sid += 1024) dst[sid] = (uint16_t)place(sid, a.se[sid]);
    __syncthreads();
    constexpr uint32_t kPer = 1024 / W;  // rows per round
    const uint32_t k = t % W;
    for (uint32_t q = t / W; q < ns; q += kPer) {
      const uint32_t r = dst[q];
      if (r == kNotStored) continue;
      const uint64_t row = row_base + r;
      a.rows_w[row * W + k] = a.skey[(uint64_t)q * W + k];
      if (k == 0) {
        a.aux[row] = a.chunk_e0 + a.se[q];
        table_publish<kInl>(a.slots, a.sref, a.spos[q], row);
      }
    }
  }
  __syncthreads();
  if (t == 0) account_chunk(a, ans, s_rank, total, s_over);
}

// ---- grid path for large chunks ----

template <bool kInl>
__global__ __launch_bounds__(256) void mark_winners(ChunkArgs a) {
  if (a.st->stop) return;
  const uint32_t ns = a.ctrl->n_surv;
  for (uint32_t sid = blockIdx.x * blockDim.x + threadIdx.x; sid < ns; sid += gridDim.x * blockDim.x) {
    const uint32_t e = a.se[sid];
    if (table_is_winner<kInl>(a.slots, a.sref, a.spos[sid], new_ref(e, sid)))
      atomicOr(&a.bitmap[e >> 5], 1u << (e & 31));
  }
}

constexpr uint32_t kScanBlock = 1024;  // bitmap words per scan block (256 threads x 4)

__global__ __launch_bounds__(256) void scan_reduce(ChunkArgs a) {
  __shared__ uint32_t red[256];
  if (a.st->stop) return;
  const uint32_t b = blockIdx.x, t = threadIdx.x;
  uint32_t s = 0;
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t w = b * kScanBlock + t * 4 + q;
    if (w < a.n_bitmap_words) s += __popc(a.bitmap[w]);
  }
  red[t] = s;
  __syncthreads();
  for (uint32_t st = 128; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0) a.block_sums[b] = red[0];
}

// Chunks whose bitmap has at most kScanSingleWords words (2^18 candidates,
// eight words per thread): the whole exclusive scan of the winner bitmap in
// one workgroup (each thread a contiguous run of words), total ->
// ctrl->winners.  Replaces the three launches below for the mid-sized
// chunks a level starts with; larger bitmaps scan faster spread out.
constexpr uint32_t kScanSingleWords = 8192;
__global__ __launch_bounds__(1024) void scan_single(ChunkArgs a) {
  __shared__ uint32_t part[1024];
  if (a.st->stop) return;
  const uint32_t t = threadIdx.x;
  const uint32_t words = a.n_bitmap_words;
  const uint32_t per = (words + 1023) / 1024;
  const uint32_t lo = min(words, t * per), hi = min(words, lo + per);
  uint32_t s = 0;
  for (uint32_t w = lo; w < hi; ++w) s += __popc(a.bitmap[w]);
  part[t] = s;
  __syncthreads();
  for (uint32_t st = 1; st < 1024; st <<= 1) {
    const uint32_t v = (t >= st) ? part[t - st] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive
  for (uint32_t w = lo; w < hi; ++w) {
    a.word_prefix[w] = run;
    run += __popc(a.bitmap[w]);
  }
  if (t == 1023) a.ctrl->winners = part[1023];
}

// single workgroup: exclusive scan of the block sums, total -> ctrl->winners
__global__ __launch_bounds__(1024) void scan_top(ChunkArgs a, uint32_t nb) {
  __shared__ uint32_t part[1024];
  if (a.st->stop) return;
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t lo = min(nb, t * per), hi = min(nb, lo + per);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a.block_sums[i];
  part[t] = s;
  __syncthreads();
  for (uint32_t st = 1; st < 1024; st <<= 1) {
    const uint32_t v = (t >= st) ? part[t - st] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a.block_sums[i];
    a.block_sums[i] = run;
    run += v;
  }
  if (t == 1023) a.ctrl->winners = part[1023];
}

__global__ __launch_bounds__(256) void scan_down(ChunkArgs a) {
  __shared__ uint32_t part[256];
  if (a.st->stop) return;
  const uint32_t b = blockIdx.x, t = threadIdx.x;
  uint32_t c[4], s = 0;
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t w = b * kScanBlock + t * 4 + q;
    c[q] = (w < a.n_bitmap_words) ? __popc(a.bitmap[w]) : 0u;
    s += c[q];
  }
  part[t] = s;
  __syncthreads();
  for (uint32_t st = 1; st < 256; st <<= 1) {
    const uint32_t v = (t >= st) ? part[t - st] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = a.block_sums[b] + part[t] - s;
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t w = b * kScanBlock + t * 4 + q;
    if (w < a.n_bitmap_words) a.word_prefix[w] = run;
    run += c[q];
  }
}

template <int W, bool kInl>
__global__ __launch_bounds__(256) void compact_winners(ChunkArgs a) {
  if (a.st->stop) return;
  const uint32_t ns = a.ctrl->n_surv;
  const uint32_t ans = a.ctrl->answer_e;
  const uint64_t row_base = a.st->total_rows;
  const uint64_t room = a.st->row_cap > row_base ? a.st->row_cap - row_base : 0;
  for (uint32_t sid = blockIdx.x * blockDim.x + threadIdx.x; sid < ns; sid += gridDim.x * blockDim.x) {
    const uint32_t e = a.se[sid];
    const uint32_t word = a.bitmap[e >> 5];
    const uint32_t bit = 1u << (e & 31);
    if (!(word & bit)) continue;
    const uint32_t rank = a.word_prefix[e >> 5] + (uint32_t)__popc(word & (bit - 1));
    if (e == ans) a.ctrl->answer_rank = rank;
    if (ans != ~0u && e >= ans) continue;
    if (rank < room)
      store_winner<W, kInl>(a, sid, e, row_base + rank);
    else if (rank == room)
      a.ctrl->overflow_e = e;
  }
}

__global__ void account_large(ChunkArgs a) {
  if (a.st->stop) return;
  account_chunk(a, a.ctrl->answer_e, a.ctrl->answer_rank, a.ctrl->winners, a.ctrl->overflow_e);
}

inline uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap = 0x7fffffffu) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

template <int W, bool kInl>
hipError_t launch_concat_w(const GenArgs& a, ConcatSet cs, hipStream_t s) {
  if (cs.n == 0 || cs.n > (uint32_t)kMaxConcatParts) return hipErrorInvalidValue;
  // right tiles in LDS: at most 32 KB
  const uint32_t yt_cap = (uint32_t)std::max(1, std::min(kConcatYT, 32768 / (512 * W)));
  // per part: left rows per workgroup at most concat_xi (16 by default),
  // fewer (down to 4), then fewer right tiles, while its grid has under
  // concat_wg workgroups (2048 by default)
  const uint64_t target = a.concat_wg ? a.concat_wg : 2048;
  const uint32_t xi_max = a.concat_xi ? std::min<uint32_t>(a.concat_xi, 64) : 16;
  size_t lds = 0;
  uint64_t wgs_total = 0;
  for (uint32_t k = 0; k < cs.n; ++k) {
    ConcatPart& p = cs.p[k];
    const uint64_t nR = p.rcount;
    if (nR == 0 || p.e1 <= p.e0) return hipErrorInvalidValue;
    p.i_lo = p.e0 / nR;
    p.i_hi = (p.e1 - 1) / nR;
    const uint64_t rowsx = p.i_hi - p.i_lo + 1;
    const uint64_t nT = (nR + 63) / 64;
    uint32_t yt = (uint32_t)std::min<uint64_t>(yt_cap, nT);
    uint32_t xi = xi_max;
    auto wgs = [&](uint32_t y, uint32_t x) { return ((nT + y - 1) / y) * ((rowsx + x - 1) / x); };
    while (xi > 4 && wgs(yt, xi) < target) xi /= 2;
    while (yt > 1 && wgs(yt, xi) < target) yt /= 2;
    lds = std::max(lds, (size_t)yt * 64 * W * 8 + (size_t)xi * W * 8);
    const uint64_t gx = (nT + yt - 1) / yt, gy = (rowsx + xi - 1) / xi;
    p.yt = yt;
    p.xi = xi;
    p.gx = (uint32_t)gx;
    p.wg0 = (uint32_t)wgs_total;
    wgs_total += gx * gy;
    if (wgs_total > 0x7fffffffull) return hipErrorInvalidConfiguration;
  }
  const uint32_t gt_lds = (lds + (size_t)a.n_pairs * 4 <= 60 * 1024) ? 1u : 0u;
  if (gt_lds) lds += (size_t)a.n_pairs * 4;
  const dim3 grid((uint32_t)wgs_total);
  const bool shrt = a.max_len < 32;
  if (shrt && gt_lds)
    launch_timed(gen_concat<W, true, kInl, true>, grid, dim3(256), lds, s, a, cs);
  else if (shrt)
    launch_timed(gen_concat<W, true, kInl, false>, grid, dim3(256), lds, s, a, cs);
  else if (gt_lds)
    launch_timed(gen_concat<W, false, kInl, true>, grid, dim3(256), lds, s, a, cs);
  else
    launch_timed(gen_concat<W, false, kInl, false>, grid, dim3(256), lds, s, a, cs);
  return hipGetLastError();
}

// One block of candidates [a.e0, a.e1) as a one-part set.
template <int W, bool kInl>
hipError_t launch_concat_one(const GenArgs& a, hipStream_t s) {
  ConcatSet cs{};
  cs.n = 1;
  cs.p[0].lstart = a.lstart;
  cs.p[0].rstart = a.rstart;
  cs.p[0].rcount = a.rcount;
  cs.p[0].e0 = a.e0;
  cs.p[0].e1 = a.e1;
  cs.p[0].rel0 = a.rel0;
  return launch_concat_w<W, kInl>(a, cs, s);
}

template <int W, bool kInl>
hipError_t launch_union_w(const GenArgs& a, UnionSet us, hipStream_t s) {
  if (us.n == 0 || us.n > (uint32_t)kMaxUnionParts) return hipErrorInvalidValue;
  uint64_t wgs = 0;
  for (uint32_t k = 0; k < us.n; ++k) {
    UnionPart& p = us.p[k];
    if (p.e1 <= p.e0 || p.lcount == 0 || (!p.same && p.rcount == 0)) return hipErrorInvalidValue;
    p.wg0 = (uint32_t)wgs;
    wgs += (p.e1 - p.e0 + 255) / 256;
    if (wgs > 0x7fffffffull) return hipErrorInvalidConfiguration;
  }
  launch_timed(gen_union<W, kInl>, dim3((uint32_t)wgs), dim3(256), 0, s, a, us);
  return hipGetLastError();
}

template <int W, bool kInl>
hipError_t launch_gen_w(int op, const GenArgs& a, bool same_level, hipStream_t s) {
  const uint64_t cnt = a.e1 - a.e0;
  switch (op) {
    case OP_CHAR:
      launch_timed(gen_char<W, kInl>, dim3(grid_for(cnt, 256)), dim3(256), 0, s, a);
      break;
    case OP_QUESTION:
      launch_timed(gen_question<W, kInl>, dim3(grid_for(cnt, 256)), dim3(256), 0, s, a);
      break;
    case OP_STAR:
      launch_timed(gen_star<W, kInl>, dim3(grid_for(cnt, 64)), dim3(256), 0, s, a);
      break;
    case OP_CONCAT:
      return launch_concat_one<W, kInl>(a, s);
    case OP_UNION: {
      UnionSet us{};
      us.n = 1;
      us.p[0] = UnionPart{a.lstart, a.lcount, a.rstart, a.rcount, a.e0, a.e1, a.rel0, same_level ? 1u : 0u, 0, 0};
      return launch_union_w<W, kInl>(a, us, s);
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// W words per language; inl selects the inline-key table (only with W = 1).
#define REI_DISPATCH_WI(W, INL, CALL)                                        \
  switch (W) {                                                               \
    case 1:                                                                  \
      if (INL) {                                                             \
        constexpr int kW = 1;                                                \
        constexpr bool kI = true;                                            \
        CALL;                                                                \
      } else {                                                               \
        constexpr int kW = 1;                                                \
        constexpr bool kI = false;                                           \
        CALL;                                                                \
      }                                                                      \
      break;                                                                 \
    case 2: { constexpr int kW = 2; constexpr bool kI = false; CALL; } break;   \
    case 4: { constexpr int kW = 4; constexpr bool kI = false; CALL; } break;   \
    case 8: { constexpr int kW = 8; constexpr bool kI = false; CALL; } break;   \
    case 16: { constexpr int kW = 16; constexpr bool kI = false; CALL; } break; \
    case 32: { constexpr int kW = 32; constexpr bool kI = false; CALL; } break; \
    default: return hipErrorInvalidValue;                                    \
  }

hipError_t launch_fill(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_state_reset(Ctrl* c, DevState* st, uint64_t row_cap, bool otf_on, hipStream_t s) {
  hipLaunchKernelGGL(state_reset, dim3(1), dim3(1), 0, s, c, st, row_cap, otf_on ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_rehash(int W, bool inl, const uint64_t* rows, uint64_t nrows, uint64_t* slots,
                         uint64_t slot_mask, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  REI_DISPATCH_WI(W, inl, hipLaunchKernelGGL((rehash_rows<kW, kI>), dim3(grid_for(nrows, 256, 65536)),
                                             dim3(256), 0, s, rows, nrows, slots, slot_mask));
  return hipGetLastError();
}

hipError_t launch_gen(int W, int op, const GenArgs& a, bool same_level, hipStream_t s) {
  if (a.e1 <= a.e0) return hipSuccess;
  REI_DISPATCH_WI(W, a.inl, return (launch_gen_w<kW, kI>(op, a, same_level, s)));
  return hipGetLastError();
}

hipError_t launch_union_set(int W, const GenArgs& a, const UnionSet& us, hipStream_t s) {
  if (us.n == 0) return hipSuccess;
  if (!a.rows || !a.st || !a.ctrl) return hipErrorInvalidValue;
  REI_DISPATCH_WI(W, a.inl, return (launch_union_w<kW, kI>(a, us, s)));
  return hipGetLastError();
}

hipError_t launch_concat_set(int W, const GenArgs& a, const ConcatSet& cs, hipStream_t s) {
  if (cs.n == 0) return hipSuccess;
  if (!a.rows || !a.gt_off || !a.gt_pair || !a.st || !a.ctrl) return hipErrorInvalidValue;
  REI_DISPATCH_WI(W, a.inl, return (launch_concat_w<kW, kI>(a, cs, s)));
  return hipGetLastError();
}

constexpr uint64_t kPairItemsMax = 1024;  // gen_pieces items up to which a wide item takes two waves
constexpr uint64_t kQuadItemsMax = 256;   // ... and up to which four

hipError_t launch_gen_pieces(int W, const GenArgs& a, const PieceArgs& p, hipStream_t s) {
  if (p.items == 0) return hipSuccess;
  if (W > kPiecesMaxW || p.n > (uint32_t)kMaxPieces) return hipErrorInvalidValue;
  // every table a piece reads must be there, and every range non-empty
  if (!a.char_index || !a.gt_off || !a.gt_pair || !a.len_off || !a.st || !a.ctrl) return hipErrorInvalidValue;
  for (uint32_t k = 0; k < p.n; ++k) {
    const PieceD& d = p.p[k];
    if (d.op != OP_CHAR && !a.rows) return hipErrorInvalidValue;  // (no rows yet: only characters)
    if (d.e1 <= d.e0 || (k && d.item0 < p.p[k - 1].item0) || d.item0 >= p.items) return hipErrorInvalidValue;
    if (d.op == OP_CONCAT && (d.rcount == 0 || d.lcount == 0 || d.nt == 0)) return hipErrorInvalidValue;
    if ((d.op == OP_UNION && !d.same && d.rcount == 0) || (d.op != OP_CHAR && d.lcount == 0))
      return hipErrorInvalidValue;
  }
  // few items (one item's latency is the launch's): from 16 words, two or
  // four waves per concatenation or star item
  const int split = W < 16 ? 1 : p.items <= kQuadItemsMax ? 4 : p.items <= kPairItemsMax ? 2 : 1;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((p.items * split + 3) / 4, 4096);
#define REI_PIECES_SPLIT(WW)                                                                   \
  do {                                                                                         \
    if (split == 4)                                                                            \
      launch_timed(gen_pieces<WW, false, 4>, dim3(grid), dim3(256), 0, s, a, p);                \
    else if (split == 2)                                                                       \
      launch_timed(gen_pieces<WW, false, 2>, dim3(grid), dim3(256), 0, s, a, p);                \
    else                                                                                       \
      launch_timed(gen_pieces<WW, false, 1>, dim3(grid), dim3(256), 0, s, a, p);                \
  } while (0)
  switch (W) {
    case 1:
      if (a.inl)
        launch_timed(gen_pieces<1, true, 1>, dim3(grid), dim3(256), 0, s, a, p);
      else
        launch_timed(gen_pieces<1, false, 1>, dim3(grid), dim3(256), 0, s, a, p);
      break;
    case 2: launch_timed(gen_pieces<2, false, 1>, dim3(grid), dim3(256), 0, s, a, p); break;
    case 4: launch_timed(gen_pieces<4, false, 1>, dim3(grid), dim3(256), 0, s, a, p); break;
    case 8: launch_timed(gen_pieces<8, false, 1>, dim3(grid), dim3(256), 0, s, a, p); break;
    case 16: REI_PIECES_SPLIT(16); break;
    case 32: REI_PIECES_SPLIT(32); break;
    default: return hipErrorInvalidValue;
  }
#undef REI_PIECES_SPLIT
  return hipGetLastError();
}

hipError_t launch_insert(int W, const ChunkArgs& a, hipStream_t s) {
  REI_DISPATCH_WI(W, a.inl, hipLaunchKernelGGL((insert_survivors<kW, kI>), dim3(grid_for(a.len, 256, 8192)),
                                               dim3(256), 0, s, a));
  return hipGetLastError();
}

bool finalize_in_one_workgroup(int W, uint64_t len) {
  // one workgroup moves at most kSmallCopyWords words of rows: a chunk
  // with more is finalized by the grid kernels, spread over the device
  return len <= kSmallChunk && len * (uint64_t)W <= kSmallCopyWords;
}

hipError_t launch_finalize(int W, const ChunkArgs& a, hipStream_t s) {
  if (finalize_in_one_workgroup(W, a.len)) {
    REI_DISPATCH_WI(W, a.inl, hipLaunchKernelGGL((finalize_small<kW, kI>), dim3(1), dim3(1024), 0, s, a));
    return hipGetLastError();
  }
  // the bitmap was cleared by insert_survivors
  if (a.clear_words != a.n_bitmap_words) return hipErrorInvalidValue;
  const uint32_t g = grid_for(a.len, 256, 8192);
  if (a.inl)
    hipLaunchKernelGGL(mark_winners<true>, dim3(g), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(mark_winners<false>, dim3(g), dim3(256), 0, s, a);
  if (a.n_bitmap_words <= kScanSingleWords) {
    hipLaunchKernelGGL(scan_single, dim3(1), dim3(1024), 0, s, a);
  } else {
    const uint32_t nb = (a.n_bitmap_words + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, a, nb);
    hipLaunchKernelGGL(scan_down, dim3(nb), dim3(256), 0, s, a);
  }
  REI_DISPATCH_WI(W, a.inl, hipLaunchKernelGGL((compact_winners<kW, kI>), dim3(g), dim3(256), 0, s, a));
  hipLaunchKernelGGL(account_large, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}

namespace {
__global__ void noop_kernel() {}
}

namespace {
// Decodes level index e of level c: the characters of cost c, then r? over
// c - c2, r* over c - c3, concatenations by left cost and unions by left cost
// (Sec. 3 enumeration order; the counts of the levels below c are final).
__device__ bool tree_decode_index(const TreeArgs& t, const uint64_t* lstart, const uint64_t* lcount, uint32_t c,
                                  uint64_t e, uint32_t* op, uint64_t* a, uint64_t* b) {
  const int64_t c1 = t.c1, cc = c;
  auto lc = [&](int64_t k) -> uint64_t { return (k >= c1 && k < cc) ? lcount[k] : 0ull; };
  *b = 0;
  uint32_t first = 0, cnt = 0;
  for (uint32_t k = 0; k < t.nsigma; ++k) {
    first += t.ccost[k] < c;
    cnt += t.ccost[k] == c;
  }
  if (e < cnt) {
    *op = OP_CHAR;
    *a = first + e;
    return true;
  }
  e -= cnt;
  uint64_t n = lc(cc - t.c2);
  if (e < n) {
    *op = OP_QUESTION;
    *a = lstart[cc - t.c2] + e;
    return true;
  }
  e -= n;
  n = lc(cc - t.c3);
  if (e < n) {
    *op = OP_STAR;
    *a = lstart[cc - t.c3] + e;
    return true;
  }
  e -= n;
  for (int64_t L = c1; cc - (int64_t)t.c4 - L >= c1; ++L) {
    const int64_t R = cc - t.c4 - L;
    n = lc(L) * lc(R);
    if (e < n) {
      *op = OP_CONCAT;
      *a = lstart[L] + e / lc(R);
      *b = lstart[R] + e % lc(R);
      return true;
    }
    e -= n;
  }
  for (int64_t L = c1; L <= cc - (int64_t)t.c5 - L; ++L) {
    const int64_t R = cc - t.c5 - L;
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

__global__ __launch_bounds__(64) void decode_tree(TreeArgs t) {
  __shared__ uint64_t lstart[kTreeMaxLevels], lcount[kTreeMaxLevels];
  __shared__ uint64_t stk[64];
  const uint32_t ans_c = t.st->answer_cost;
  const uint64_t ans_e = t.st->answer_e;
  const bool have = t.st->stop == STOP_ANSWER && ans_c < kTreeMaxLevels && ans_c >= t.c1;
  // level sizes loaded by the whole wave, prefix sums by lane 0
  if (have)
    for (uint32_t c = threadIdx.x; c <= ans_c; c += blockDim.x) lcount[c] = c >= t.c1 ? t.levels[c] : 0ull;
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (!have) {
    t.out[0] = 0;
    return;
  }
  uint64_t start = 0;
  for (uint32_t c = 0; c <= ans_c; ++c) {
    lstart[c] = start;
    start += lcount[c];
  }
  uint32_t k = 0, sp = 0;
  bool ok = true;
  auto node = [&](uint64_t row, uint32_t c, uint64_t e) {
    uint32_t op = 0;
    uint64_t a = 0, b = 0;
    if (k >= t.max_nodes || sp + 2 > 64 || !tree_decode_index(t, lstart, lcount, c, e, &op, &a, &b)) {
      ok = false;
      return;
    }
    uint64_t* o = t.out + 1 + 4 * k++;
    o[0] = row;
    o[1] = op;
    o[2] = a;
    o[3] = b;
    if (op != OP_CHAR) stk[sp++] = a;
    if (op == OP_CONCAT || op == OP_UNION) stk[sp++] = b;
  };
  node(~0ull, ans_c, ans_e);
  while (ok && sp) {
    const uint64_t row = stk[--sp];
    uint32_t rc = 0;
    for (uint32_t c = t.c1; c < ans_c; ++c)
      if (row >= lstart[c] && row < lstart[c] + lcount[c]) rc = c;
    if (!rc) {
      ok = false;
      break;
    }
    node(row, rc, t.aux[row]);
  }
  t.out[0] = ok ? k : 0;
}
}  // namespace

hipError_t launch_decode_tree(const TreeArgs& t, hipStream_t s) {
  if (!t.levels || !t.aux || !t.st || !t.out || t.nsigma > kTreeMaxChars || t.max_nodes == 0)
    return hipErrorInvalidValue;
  launch_timed(decode_tree, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

hipError_t set_hash_mask_kernels(uint64_t mask) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_hash_mask), &mask, sizeof(mask));
}

hipError_t launch_noop_timed(hipStream_t s) {
  launch_timed(noop_kernel, dim3(1), dim3(64), 0, s);
  return hipGetLastError();
}

hipError_t launch_account(const ChunkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(account_large, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}


}  // namespace rei
