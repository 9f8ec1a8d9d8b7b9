// Host driver of the REI search (Algorithm 1): the cost-level loop, the
// constructor blocks of each level, chunking, device memory, reconstruction
// of the answer from the per-row back-pointers, and the C ABI.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace rei;

namespace rei {
thread_local KernelTimer g_kernel_timer{nullptr, nullptr};
}

namespace {

thread_local std::string g_create_error;

constexpr uint64_t kDefaultChunk = 1ull << 24;
constexpr uint64_t kDefaultArena = 16ull << 20;  // bytes per batched instance
// Work (weighted candidates) below which an instance always stays in a
// captured graph, however uneven the batch.
constexpr double kGraphHeavyMin = 1e5;

struct Block {
  int op;
  uint32_t L, R;     // operand levels (costs)
  uint64_t count;    // candidates
  bool same;         // union of a level with itself (pairs x before y)
};

// Device memory of an instance: hipMalloc / hipFree, or the caller's pair
// (rei_set_allocator) captured when the instance is created.
struct DevAlloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
DevAlloc g_alloc;

struct ProfRec {
  int k;
  hipEvent_t a, b;
  uint64_t units;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct rei_instance {
  Staged st;
  rei_costs costs{};
  uint32_t max_cost = 0;
  uint64_t cache_bytes = 0;
  uint64_t row_cap = 0;
  uint32_t max_err = 0;
  uint64_t chunk_max = kDefaultChunk;
  // grid-path launch parameters set for this instance (0: the process table
  // for its word width, else the defaults)
  GridTune grid_set{0, 0, 0, 0};
  uint64_t batch_level_max = 0;  // 0: the tuned value, else kBatchLevelMax
  int64_t batch_time_us = -1;    // -1: kBatchTimeUs; 0: no hand-off on time
  int device = 0;
  DevAlloc alloc;  // how this instance's device memory is obtained and released
  double t_seen = -1;  // seconds into a batched call when its completion flag showed
  double seconds_stage = 0;

  // staged tables on the device
  uint32_t* d_gt_off = nullptr;
  uint32_t* d_gt_pair = nullptr;
  uint32_t* d_len_off = nullptr;
  uint64_t* d_pmask = nullptr;
  uint64_t* d_nmask = nullptr;
  int32_t* d_char_index = nullptr;  // ic index of each character, in char_order
  // per-character costs (empty: every character costs c_char, which is then
  // the smallest character cost) and the characters ordered by (cost,
  // alphabet position): level c's base block is a contiguous run of it
  std::vector<uint32_t> char_cost;
  std::vector<uint32_t> char_order;

  // language cache
  uint64_t* d_rows = nullptr;
  uint64_t* d_aux = nullptr;
  uint64_t rows_alloc = 0;
  // dedup table
  uint64_t* d_slots = nullptr;
  uint64_t* d_sref = nullptr;  // inline-key table only
  uint64_t slots_cap = 0;
  bool inl = false;            // one word per language and |ic| <= 63: keys live in the slots
  // chunk buffers
  uint64_t* d_skey = nullptr;
  uint32_t* d_se = nullptr;
  uint64_t* d_spos = nullptr;
  uint64_t surv_cap = 0;
  uint32_t* d_bitmap = nullptr;
  uint32_t* d_prefix = nullptr;
  uint32_t* d_bsums = nullptr;
  uint64_t bitmap_cap = 0;  // words
  Ctrl* d_ctrl = nullptr;
  DevState* d_state = nullptr;
  // per-cost counters on the device: stored rows [0, L), unique [L, 2L),
  // candidates [2L, 3L) with L = max_cost + 2
  uint64_t* d_levels = nullptr;
  DevState* h_state = nullptr;    // pinned mirrors
  uint64_t* h_levels = nullptr;
  uint64_t* h_tree = nullptr;     // answer tree written by the batched solver
  // the same pinned buffers as the device addresses them
  DevState* v_state = nullptr;
  uint64_t* v_levels = nullptr;
  uint64_t* v_tree = nullptr;
  // nodes of the answer tree (row, op, a, b) decoded on the device by the
  // batched solver; printing looks rows up here before reading back-pointers
  std::vector<uint64_t> tree;

  // rows known stored at the last synchronisation, candidates enqueued since
  uint64_t known_rows = 0;
  // set when the batched solver handed the instance over at this level
  uint32_t resume_level = 0;
  // OnTheFly mode (Sec. 3): allowed, level where the cache filled (0: not
  // yet), and whether a level needed an incomplete one
  bool otf_on = false;
  uint32_t otf_level = 0;
  bool otf_blocked = false;
  uint64_t pending = 0;
  uint32_t chunks_enq = 0;  // chunks enqueued on the per-chunk path since the state was reset

  // levels, indexed by cost
  std::vector<uint64_t> lstart, lcount;
  // host copy of the back-pointers for printing (filled on first use)
  std::vector<uint64_t> h_aux;
  bool h_aux_valid = false;
  // set by rei_solve_batch_noalloc: the last search's rows lived in the
  // shared static array, not in this instance's buffers; aux_view points at
  // its back-pointers while that call prints the answer
  bool rows_elsewhere = false;
  const uint64_t* aux_view = nullptr;

  // result
  std::vector<uint64_t> uniq, cand;
  std::string regex;
  rei_result res{};
  std::string err;

  // profiling
  int prof = 0;  // 0 off, 1 generators and batched solver, 2 every class, 3 prof_class only
  int prof_class = 0;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  uint64_t st_launch[REI_K_COUNT] = {0};
  double st_ms[REI_K_COUNT] = {0};
  uint64_t st_units[REI_K_COUNT] = {0};
};

namespace {

#define HIP_OK(inst, call)                                                             \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (inst)->err = std::string(#call) + ": " + hipGetErrorString(e_);                \
      return REI_ERR_DEVICE;                                                           \
    }                                                                                  \
  } while (0)

// A caller's allocator may order its reuse of memory by some stream of its
// own, which the library's streams do not follow: the device is drained after
// taking memory from it and before handing memory back, as hipMalloc and
// hipFree would do by themselves.
template <class T>
hipError_t dev_alloc(const rei_instance* in, T** p, size_t bytes) {
  if (in->alloc.alloc) {
    *p = (T*)in->alloc.alloc(bytes, in->alloc.ctx);
    if (!*p) return hipErrorOutOfMemory;
    return hipDeviceSynchronize();
  }
  return hipMalloc(p, bytes);
}

template <class T>
void dfree(const rei_instance* in, T*& p) {
  if (p) {
    if (in->alloc.free_) {
      (void)hipDeviceSynchronize();
      in->alloc.free_((void*)p, in->alloc.ctx);
    } else {
      (void)hipFree(p);
    }
  }
  p = nullptr;
}

// Grid-path launch parameters by word width, from rei_tune_grid or a tuning
// file; widths without an entry use GridTune's defaults.
std::mutex g_grid_mu;
std::map<int, GridTune> g_grid_tuned;

GridTune grid_params(const rei_instance* in);

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Timing-only events: no system-scope fence (cache write-back and
// invalidation) when they complete, so they neither perturb nor pad the
// launches they bracket.  They are read only after the stream has drained.
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

// Generators and the batched solver are launched through launch_timed, which
// records the pair at the kernel's own start and end; the other launchers
// (several small kernels each) are bracketed by events on the stream.
bool self_timed(int k) { return k <= REI_K_GEN_UNION || k == REI_K_BATCH || k == REI_K_GEN_MIXED; }

rei_status prof_event(rei_instance* in, hipEvent_t* ev) {
  if (in->pool.empty()) {
    hipEvent_t e;
    HIP_OK(in, hipEventCreateWithFlags(&e, kTimingEvent));
    in->pool.push_back(e);
  }
  *ev = in->pool.back();
  in->pool.pop_back();
  return REI_OK;
}

bool profiled(const rei_instance* in, int k) {
  return in->prof == 2 || (in->prof == 1 && self_timed(k)) || (in->prof == 3 && k == in->prof_class);
}

rei_status prof_begin(rei_instance* in, hipStream_t s, int k, hipEvent_t* a, hipEvent_t* b) {
  if (!profiled(in, k)) return REI_OK;
  rei_status r;
  if ((r = prof_event(in, a)) != REI_OK || (r = prof_event(in, b)) != REI_OK) return r;
  if (self_timed(k))
    g_kernel_timer = KernelTimer{*a, *b};
  else
    HIP_OK(in, hipEventRecord(*a, s));
  return REI_OK;
}

rei_status prof_end(rei_instance* in, hipStream_t s, int k, hipEvent_t a, hipEvent_t b, uint64_t units) {
  if (!profiled(in, k)) return REI_OK;
  if (self_timed(k)) {
    if (g_kernel_timer.start) {  // the launcher launched nothing
      g_kernel_timer = KernelTimer{nullptr, nullptr};
      HIP_OK(in, hipEventRecord(a, s));
      HIP_OK(in, hipEventRecord(b, s));
    }
  } else {
    HIP_OK(in, hipEventRecord(b, s));
  }
  in->recs.push_back({k, a, b, units});
  return REI_OK;
}

// Folds finished event pairs into the statistics (the stream must be idle).
rei_status prof_collect(rei_instance* in) {
  for (auto& r : in->recs) {
    float ms = 0;
    HIP_OK(in, hipEventElapsedTime(&ms, r.a, r.b));
    in->st_launch[r.k] += 1;
    in->st_ms[r.k] += ms;
    in->st_units[r.k] += r.units;
    in->pool.push_back(r.a);
    in->pool.push_back(r.b);
  }
  in->recs.clear();
  return REI_OK;
}

#define LAUNCH(in, s, k, units, call)                     \
  do {                                                    \
    hipEvent_t ev_ = nullptr, ev2_ = nullptr;             \
    rei_status ps_ = prof_begin(in, s, k, &ev_, &ev2_);   \
    if (ps_ != REI_OK) return ps_;                        \
    HIP_OK(in, call);                                     \
    ps_ = prof_end(in, s, k, ev_, ev2_, units);           \
    if (ps_ != REI_OK) return ps_;                        \
  } while (0)

rei_status ensure_rows(rei_instance* in, uint64_t need, hipStream_t s) {
  if (need <= in->rows_alloc) return REI_OK;
  uint64_t cap = std::max<uint64_t>({need, 2 * in->rows_alloc, 1024});
  const int W = in->st.W;
  uint64_t* nr = nullptr;
  uint64_t* na = nullptr;
  HIP_OK(in, dev_alloc(in, &nr, cap * W * 8));
  if (dev_alloc(in, &na, cap * 8) != hipSuccess) {
    dfree(in, nr);
    in->err = "hipMalloc of the back-pointer array failed";
    return REI_ERR_DEVICE;
  }
  if (in->known_rows) {
    HIP_OK(in, hipMemcpyAsync(nr, in->d_rows, in->known_rows * W * 8, hipMemcpyDeviceToDevice, s));
    HIP_OK(in, hipMemcpyAsync(na, in->d_aux, in->known_rows * 8, hipMemcpyDeviceToDevice, s));
  }
  HIP_OK(in, hipStreamSynchronize(s));
  dfree(in, in->d_rows);
  dfree(in, in->d_aux);
  in->d_rows = nr;
  in->d_aux = na;
  in->rows_alloc = cap;
  return REI_OK;
}

// The table keeps its load at most 1/2: entries = stored rows + possible new ones.
rei_status ensure_table(rei_instance* in, uint64_t entries, hipStream_t s, bool force) {
  if (!force && in->slots_cap >= 2 * entries) return REI_OK;
  uint64_t cap = std::max<uint64_t>(4096, pow2_at_least(4 * entries));
  if (force && in->slots_cap >= cap) cap = in->slots_cap;
  if (cap != in->slots_cap) {
    dfree(in, in->d_slots);
    dfree(in, in->d_sref);
    in->slots_cap = 0;
    HIP_OK(in, dev_alloc(in, &in->d_slots, cap * 8));
    if (in->inl) HIP_OK(in, dev_alloc(in, &in->d_sref, cap * 8));
    in->slots_cap = cap;
  }
  LAUNCH(in, s, REI_K_OTHER, cap, launch_fill(in->d_slots, cap, kEmpty, s));
  if (in->inl) LAUNCH(in, s, REI_K_OTHER, cap, launch_fill(in->d_sref, cap, kEmpty, s));
  LAUNCH(in, s, REI_K_OTHER, in->known_rows,
         launch_rehash(in->st.W, in->inl, in->d_rows, in->known_rows, in->d_slots, cap - 1, s));
  return REI_OK;
}

rei_status ensure_chunk_buffers(rei_instance* in, uint64_t len) {
  const int W = in->st.W;
  if (len > in->surv_cap) {
    dfree(in, in->d_skey);
    dfree(in, in->d_se);
    dfree(in, in->d_spos);
    HIP_OK(in, dev_alloc(in, &in->d_skey, len * W * 8));
    HIP_OK(in, dev_alloc(in, &in->d_se, len * 4));
    HIP_OK(in, dev_alloc(in, &in->d_spos, len * 8));
    in->surv_cap = len;
  }
  const uint64_t words = (len + 31) / 32;
  if (words > in->bitmap_cap) {
    dfree(in, in->d_bitmap);
    dfree(in, in->d_prefix);
    dfree(in, in->d_bsums);
    HIP_OK(in, dev_alloc(in, &in->d_bitmap, words * 4));
    HIP_OK(in, dev_alloc(in, &in->d_prefix, words * 4));
    HIP_OK(in, dev_alloc(in, &in->d_bsums, ((words + 1023) / 1024 + 1) * 4));
    in->bitmap_cap = words;
  }
  return REI_OK;
}

// The characters of cost c: positions [*first, *first + *count) of char_order.
void chars_at(const rei_instance* in, int64_t c, uint32_t* first, uint32_t* count) {
  *first = *count = 0;
  for (uint32_t a : in->char_order) {
    const uint32_t ca = in->char_cost.empty() ? in->costs.c_char : in->char_cost[a];
    if ((int64_t)ca < c) ++*first;
    if ((int64_t)ca == c) ++*count;
  }
}

GridTune grid_params(const rei_instance* in) {
  GridTune t;
  {
    std::lock_guard<std::mutex> lk(g_grid_mu);
    auto it = g_grid_tuned.find(in->st.W);
    if (it != g_grid_tuned.end()) t = it->second;
  }
  if (in->grid_set.first_chunk) t.first_chunk = in->grid_set.first_chunk;
  if (in->grid_set.chunk_max) t.chunk_max = in->grid_set.chunk_max;
  if (in->grid_set.concat_wg) t.concat_wg = in->grid_set.concat_wg;
  if (in->grid_set.concat_xi) t.concat_xi = in->grid_set.concat_xi;
  return t;
}

uint64_t level_n(const rei_instance* in, int64_t c) {
  if (c < (int64_t)in->costs.c_char || c >= (int64_t)in->lcount.size()) return 0;
  return in->lcount[c];
}

bool mul_ok(uint64_t a, uint64_t b, uint64_t* out) { return !__builtin_mul_overflow(a, b, out); }

// Constructor blocks of level c in enumeration order.  In OnTheFly mode the
// list ends before the first block that needs an incomplete level (the one
// where the cache filled, or a later one) and *blocked is set, unless a
// complete operand level of that block is empty (it has no candidates).
bool make_blocks(const rei_instance* in, uint32_t c, std::vector<Block>* out, bool* blocked = nullptr) {
  out->clear();
  if (blocked) *blocked = false;
  const rei_costs& k = in->costs;
  // the characters of this cost come first (all of them at c_char when the
  // characters cost the same)
  uint32_t ch_first = 0, ch_count = 0;
  chars_at(in, c, &ch_first, &ch_count);
  if (ch_count) out->push_back({OP_CHAR, c, 0, ch_count, false});
  const int64_t cc = c;
  const int64_t full = in->otf_level;
  auto usable = [&](int64_t a, int64_t b) -> bool {
    if (!full || a < (int64_t)k.c_char || (b >= 0 && b < (int64_t)k.c_char)) return true;
    const bool ca = a < full, cb = b < 0 || b < full;
    if (ca && cb) return true;
    if ((ca && level_n(in, a) == 0) || (b >= 0 && cb && level_n(in, b) == 0)) return true;
    if (blocked) *blocked = true;
    return false;
  };
  if (!usable(cc - k.c_question, -1)) return true;
  if (level_n(in, cc - k.c_question))
    out->push_back({OP_QUESTION, (uint32_t)(cc - k.c_question), 0, level_n(in, cc - k.c_question), false});
  if (!usable(cc - k.c_star, -1)) return true;
  if (level_n(in, cc - k.c_star))
    out->push_back({OP_STAR, (uint32_t)(cc - k.c_star), 0, level_n(in, cc - k.c_star), false});
  for (int64_t L = k.c_char; cc - (int64_t)k.c_concat - L >= (int64_t)k.c_char; ++L) {
    const int64_t R = cc - k.c_concat - L;
    if (!usable(L, R)) return true;
    uint64_t n;
    if (!mul_ok(level_n(in, L), level_n(in, R), &n)) return false;
    if (n) out->push_back({OP_CONCAT, (uint32_t)L, (uint32_t)R, n, false});
  }
  for (int64_t L = k.c_char; L <= cc - (int64_t)k.c_union - L; ++L) {
    const int64_t R = cc - k.c_union - L;
    if (!usable(L, R)) return true;
    const uint64_t a = level_n(in, L), b = level_n(in, R);
    uint64_t n;
    if (L < R) {
      if (!mul_ok(a, b, &n)) return false;
    } else {
      if (!mul_ok(a, a ? a - 1 : 0, &n)) return false;
      n /= 2;
    }
    if (n) out->push_back({OP_UNION, (uint32_t)L, (uint32_t)R, n, L == R});
  }
  return true;
}

// Waits until every chunk enqueued so far is accounted; the search state is
// then in the host mirrors (h_state, h_levels), which the accounting writes
// with the device state, its chunk count last.  At a level boundary
// (drain = false) the host watches that count (a few microseconds sooner
// than the stream's completion) for at most kSpinUs; a search that stopped
// (whose later chunks account nothing), or one still running then, waits
// for the stream.  drain = true waits for the stream in any case: buffers
// may be freed next, and other work on the stream (fills, rehashes, copies)
// may still use them.
constexpr double kSpinUs = 2000;
rei_status sync_state(rei_instance* in, hipStream_t s, bool drain) {
  const double t0 = now_s();
  bool seen = false;
  for (; !drain;) {
    const uint32_t got = __atomic_load_n(&in->h_state->chunks, __ATOMIC_ACQUIRE);
    if (got == in->chunks_enq && !__atomic_load_n(&in->h_state->stop, __ATOMIC_ACQUIRE)) {
      seen = true;
      break;
    }
    if (__atomic_load_n(&in->h_state->stop, __ATOMIC_ACQUIRE) || (now_s() - t0) * 1e6 > kSpinUs) break;
  }
  if (!seen) HIP_OK(in, hipStreamSynchronize(s));
  in->known_rows = in->h_state->total_rows;
  in->pending = 0;
  return REI_OK;
}

// Enqueues one chunk (no host synchronisation unless a buffer may have to
// grow: then the stream is drained first and the buffer grown for the worst
// case of this chunk).
// A piece of a chunk: candidates [e0, e1) of one block, whose first
// candidate has level index e_base.  The pieces of a chunk are consecutive
// in level index, so small blocks share one insert and one finalize.
struct Piece {
  Block b;
  uint64_t e_base, e0, e1;
};

rei_status enqueue_chunk(rei_instance* in, hipStream_t s, uint32_t c, const std::vector<Piece>& pieces,
                         bool* stopped) {
  const int W = in->st.W;
  uint64_t len = 0;
  for (const Piece& p : pieces) len += p.e1 - p.e0;
  const uint64_t chunk_e0 = pieces[0].e_base + pieces[0].e0;
  const uint64_t words = (len + 31) / 32;
  rei_status r;
  auto worst_rows = [&] { return std::min(in->row_cap, in->known_rows + in->pending + len); };
  auto worst_entries = [&] { return in->known_rows + in->pending + len; };
  // a level enumerated in OnTheFly mode stores nothing: no buffer grows
  const bool otf_level = in->otf_level != 0;
  if (!otf_level && (worst_rows() > in->rows_alloc || 2 * worst_entries() > in->slots_cap ||
                     len > in->surv_cap || words > in->bitmap_cap)) {
    if ((r = sync_state(in, s, true)) != REI_OK) return r;
    if (in->h_state->stop) {
      *stopped = true;
      return REI_OK;
    }
    if ((r = ensure_chunk_buffers(in, len)) != REI_OK) return r;
    if ((r = ensure_rows(in, std::min(in->row_cap, in->known_rows + len), s)) != REI_OK) return r;
    if ((r = ensure_table(in, in->known_rows + len, s, false)) != REI_OK) return r;
  }

  GenArgs g{};
  g.rows = in->d_rows;
  g.slots = in->d_slots;
  g.slot_mask = in->slots_cap - 1;
  g.skey = in->d_skey;
  g.se = in->d_se;
  g.spos = in->d_spos;
  g.ctrl = in->d_ctrl;
  g.pmask = in->d_pmask;
  g.nmask = in->d_nmask;
  g.max_err = in->max_err;
  g.gt_off = in->d_gt_off;
  g.gt_pair = in->d_gt_pair;
  g.len_off = in->d_len_off;
  g.max_len = in->st.max_len;
  g.n = in->st.n;
  g.n_pairs = (uint32_t)in->st.gt_pair.size();
  g.st = in->d_state;
  g.inl = in->inl ? 1u : 0u;
  {
    const GridTune gt = grid_params(in);
    g.concat_wg = gt.concat_wg;
    g.concat_xi = gt.concat_xi;
  }
  // small pieces (W <= kPiecesMaxW) share gen_pieces launches of up to
  // kMaxPieces pieces; larger ones get their constructor's kernel
  PieceArgs pa{};
  // large concatenation blocks share gen_concat launches of up to
  // kMaxConcatParts blocks
  ConcatSet cset{};
  uint64_t cset_cand = 0;
  auto flush_concat = [&]() -> rei_status {
    if (!cset.n) return REI_OK;
    LAUNCH(in, s, REI_K_GEN_CONCAT, cset_cand, launch_concat_set(W, g, cset, s));
    cset = ConcatSet{};
    cset_cand = 0;
    return REI_OK;
  };
  // large union blocks share gen_union launches likewise
  UnionSet uset{};
  uint64_t uset_cand = 0;
  auto flush_union = [&]() -> rei_status {
    if (!uset.n) return REI_OK;
    LAUNCH(in, s, REI_K_GEN_UNION, uset_cand, launch_union_set(W, g, uset, s));
    uset = UnionSet{};
    uset_cand = 0;
    return REI_OK;
  };
  auto flush_pieces = [&]() -> rei_status {
    if (!pa.n) return REI_OK;
    GenArgs gp = g;  // pieces carry their own ranges; characters index from the table's start
    gp.char_index = in->d_char_index;
    LAUNCH(in, s, REI_K_GEN_MIXED, pa.items_cand, launch_gen_pieces(W, gp, pa, s));
    pa = PieceArgs{};
    return REI_OK;
  };
  for (const Piece& p : pieces) {
    const Block& b = p.b;
    if (W <= kPiecesMaxW && p.e1 - p.e0 <= kSmallPiece) {
      PieceD& d = pa.p[pa.n];
      d = PieceD{};
      d.op = (uint32_t)b.op;
      d.same = b.same ? 1u : 0u;
      d.e0 = p.e0;
      d.e1 = p.e1;
      d.rel0 = (uint32_t)(p.e_base + p.e0 - chunk_e0);
      if (b.op == OP_CHAR) {
        uint32_t first = 0, count = 0;
        chars_at(in, c, &first, &count);
        d.char_off = first;
      } else {
        d.lstart = in->lstart[b.L];
        d.lcount = in->lcount[b.L];
        if (b.op == OP_CONCAT || b.op == OP_UNION) {
          d.rstart = in->lstart[b.R];
          d.rcount = in->lcount[b.R];
        }
      }
      d.item0 = pa.items;
      uint64_t items;
      if (b.op == OP_CONCAT) {
        const uint64_t nR = d.rcount, nL = d.lcount;
        const uint64_t i_lo = p.e0 / nR, i_hi = (p.e1 - 1) / nR;
        d.left_lanes = (nR < 64 && nR < nL) ? 1u : 0u;
        if (!d.left_lanes) {
          d.t0 = i_lo;
          d.nt = (nR + 63) / 64;
          items = (i_hi - i_lo + 1) * d.nt;
        } else {
          d.t0 = i_lo / 64;
          d.nt = nR;
          items = (i_hi / 64 - i_lo / 64 + 1) * nR;
        }
      } else {
        items = (p.e1 - p.e0 + 63) / 64;
      }
      pa.items += items;
      pa.items_cand += p.e1 - p.e0;
      if (++pa.n == kMaxPieces && (r = flush_pieces()) != REI_OK) return r;
      continue;
    }
    if (b.op == OP_CONCAT) {
      ConcatPart& cp = cset.p[cset.n];
      cp = ConcatPart{};
      cp.lstart = in->lstart[b.L];
      cp.rstart = in->lstart[b.R];
      cp.rcount = in->lcount[b.R];
      cp.e0 = p.e0;
      cp.e1 = p.e1;
      cp.rel0 = (uint32_t)(p.e_base + p.e0 - chunk_e0);
      cset_cand += p.e1 - p.e0;
      if (++cset.n == (uint32_t)kMaxConcatParts && (r = flush_concat()) != REI_OK) return r;
      continue;
    }
    if (b.op == OP_UNION) {
      uset.p[uset.n] = UnionPart{in->lstart[b.L], in->lcount[b.L], in->lstart[b.R], in->lcount[b.R], p.e0, p.e1,
                                 (uint32_t)(p.e_base + p.e0 - chunk_e0), b.same ? 1u : 0u, 0, 0};
      uset_cand += p.e1 - p.e0;
      if (++uset.n == (uint32_t)kMaxUnionParts && (r = flush_union()) != REI_OK) return r;
      continue;
    }
    g.e0 = p.e0;
    g.e1 = p.e1;
    g.rel0 = (uint32_t)(p.e_base + p.e0 - chunk_e0);
    g.char_index = in->d_char_index;
    if (b.op == OP_CHAR) {
      uint32_t first = 0, count = 0;
      chars_at(in, c, &first, &count);
      g.char_index = in->d_char_index + first;
    }
    g.lstart = g.lcount = g.rstart = g.rcount = 0;
    if (b.op != OP_CHAR) {
      g.lstart = in->lstart[b.L];
      g.lcount = in->lcount[b.L];
      if (b.op == OP_CONCAT || b.op == OP_UNION) {
        g.rstart = in->lstart[b.R];
        g.rcount = in->lcount[b.R];
      }
    }
    LAUNCH(in, s, REI_K_GEN_CHAR + b.op, p.e1 - p.e0, launch_gen(W, b.op, g, b.same, s));
  }
  if ((r = flush_pieces()) != REI_OK) return r;
  if ((r = flush_concat()) != REI_OK) return r;
  if ((r = flush_union()) != REI_OK) return r;

  ChunkArgs ca{};
  ca.rows = in->d_rows;
  ca.rows_w = in->d_rows;
  ca.aux = in->d_aux;
  ca.slots = in->d_slots;
  ca.sref = in->d_sref;
  ca.inl = in->inl ? 1u : 0u;
  ca.slot_mask = in->slots_cap - 1;
  ca.skey = in->d_skey;
  ca.se = in->d_se;
  ca.spos = in->d_spos;
  ca.bitmap = in->d_bitmap;
  ca.word_prefix = in->d_prefix;
  ca.block_sums = in->d_bsums;
  ca.n_bitmap_words = (uint32_t)words;
  ca.ctrl = in->d_ctrl;
  ca.st = in->d_state;
  const uint64_t L = in->max_cost + 2;
  ca.lcount = in->d_levels;
  ca.uniq = in->d_levels + L;
  ca.cand = in->d_levels + 2 * L;
  ca.cost = c;
  ca.chunk_e0 = chunk_e0;
  ca.len = len;
  ca.hst = in->v_state;
  ca.hlev = in->v_levels;
  ca.nlev = L;
  ca.clear_words = finalize_in_one_workgroup(W, len) ? 0u : (uint32_t)words;
  if (otf_level) {
    LAUNCH(in, s, REI_K_COMPACT, len, launch_account(ca, s));
    ++in->chunks_enq;
    return REI_OK;
  }
  LAUNCH(in, s, REI_K_INSERT, len, launch_insert(W, ca, s));
  LAUNCH(in, s, REI_K_COMPACT, len, launch_finalize(W, ca, s));
  ++in->chunks_enq;
  in->pending += len;
  return REI_OK;
}

// ---- reconstruction --------------------------------------------------------

struct Node {
  int op;
  uint64_t a, b;  // child rows (or char index)
};

uint64_t tri_first(uint64_t i, uint64_t n) { return i * n - i * (i + 1) / 2; }

bool decode(const rei_instance* in, uint32_t c, uint64_t e, Node* out) {
  std::vector<Block> blocks;
  if (!make_blocks(in, c, &blocks)) return false;
  for (const Block& b : blocks) {
    if (e >= b.count) {
      e -= b.count;
      continue;
    }
    out->op = b.op;
    if (b.op == OP_CHAR) {
      uint32_t first = 0, count = 0;
      chars_at(in, c, &first, &count);
      out->a = in->char_order[first + e];  // alphabet position
      out->b = 0;
    } else if (b.op == OP_QUESTION || b.op == OP_STAR) {
      out->a = in->lstart[b.L] + e;
      out->b = 0;
    } else if (b.op == OP_UNION && b.same) {
      const uint64_t n = in->lcount[b.L];
      uint64_t lo = 0, hi = n - 1;  // largest i with tri_first(i) <= e
      while (lo < hi) {
        uint64_t mid = (lo + hi + 1) / 2;
        if (tri_first(mid, n) <= e) lo = mid; else hi = mid - 1;
      }
      out->a = in->lstart[b.L] + lo;
      out->b = in->lstart[b.L] + lo + 1 + (e - tri_first(lo, n));
    } else {
      const uint64_t nR = in->lcount[b.R];
      out->a = in->lstart[b.L] + e / nR;
      out->b = in->lstart[b.R] + e % nR;
    }
    return true;
  }
  return false;
}

uint32_t row_cost(const rei_instance* in, uint64_t row) {
  for (uint32_t c = in->costs.c_char; c < in->lstart.size(); ++c)
    if (in->lcount[c] && row >= in->lstart[c] && row < in->lstart[c] + in->lcount[c]) return c;
  return 0;
}

// Back-pointer of a stored row.  Caches with up to 4M rows are copied to the
// host in one transfer on first use; larger ones are read row by row.
rei_status row_aux(rei_instance* in, uint64_t row, uint64_t* e) {
  const uint64_t* aux = in->aux_view ? in->aux_view : in->d_aux;
  if (!in->h_aux_valid) {
    uint64_t rows = 0;
    for (uint32_t c = in->costs.c_char; c < in->lcount.size(); ++c) rows += in->lcount[c];
    if (rows <= (4ull << 20)) {
      in->h_aux.resize(rows);
      if (rows) HIP_OK(in, hipMemcpy(in->h_aux.data(), aux, rows * 8, hipMemcpyDeviceToHost));
      in->h_aux_valid = true;
    }
  }
  if (in->h_aux_valid && row < in->h_aux.size()) {
    *e = in->h_aux[row];
    return REI_OK;
  }
  HIP_OK(in, hipMemcpy(e, aux + row, 8, hipMemcpyDeviceToHost));
  return REI_OK;
}

rei_status row_node(rei_instance* in, uint64_t row, Node* nd) {
  for (size_t k = 0; k + 3 < in->tree.size(); k += 4)
    if (in->tree[k] == row) {
      nd->op = (int)in->tree[k + 1];
      nd->a = in->tree[k + 2];
      nd->b = in->tree[k + 3];
      return REI_OK;
    }
  uint64_t e = 0;
  rei_status r = row_aux(in, row, &e);
  if (r != REI_OK) return r;
  const uint32_t c = row_cost(in, row);
  if (!c || !decode(in, c, e, nd)) {
    in->err = "corrupt back-pointer";
    return REI_ERR_DEVICE;
  }
  return REI_OK;
}

// Printing: x? and x* parenthesise x iff x is a concatenation or a union; a
// concatenation parenthesises a union child; a union never parenthesises.
rei_status print_node(rei_instance* in, const Node& nd, std::string* out);

rei_status print_row(rei_instance* in, uint64_t row, std::string* out, int* op) {
  Node nd;
  rei_status r = row_node(in, row, &nd);
  if (r != REI_OK) return r;
  *op = nd.op;
  return print_node(in, nd, out);
}

rei_status print_node(rei_instance* in, const Node& nd, std::string* out) {
  rei_status r;
  if (nd.op == OP_CHAR) {
    *out = std::string(1, in->st.sigma[nd.a]);
    return REI_OK;
  }
  std::string x, y;
  int xo = 0, yo = 0;
  if ((r = print_row(in, nd.a, &x, &xo)) != REI_OK) return r;
  if (nd.op == OP_QUESTION || nd.op == OP_STAR) {
    if (xo == OP_CONCAT || xo == OP_UNION) x = "(" + x + ")";
    *out = x + (nd.op == OP_QUESTION ? "?" : "*");
    return REI_OK;
  }
  if ((r = print_row(in, nd.b, &y, &yo)) != REI_OK) return r;
  if (nd.op == OP_CONCAT) {
    if (xo == OP_UNION) x = "(" + x + ")";
    if (yo == OP_UNION) y = "(" + y + ")";
    *out = x + y;
  } else {
    *out = x + "+" + y;
  }
  return REI_OK;
}

void fill_result(rei_instance* in, rei_status st, uint32_t cost, uint32_t last_level, double t0) {
  const uint32_t c1 = in->costs.c_char;
  rei_result& r = in->res;
  r = rei_result{};
  r.status = st;
  r.cost = cost;
  r.regex = in->regex.c_str();
  r.first_level = c1;
  r.n_levels = last_level >= c1 ? last_level - c1 + 1 : 0;
  r.unique_per_level = r.n_levels ? in->uniq.data() + c1 : nullptr;
  r.candidates_per_level = r.n_levels ? in->cand.data() + c1 : nullptr;
  r.total_unique = 0;
  for (uint32_t i = 0; i < r.n_levels; ++i) r.total_unique += in->uniq[c1 + i];
  r.ic_size = in->st.n;
  r.cs_words = (uint32_t)in->st.W;
  r.seconds_stage = in->seconds_stage;
  r.seconds_solve = now_s() - t0;
}

// Resets the host-side result state; answers the trivial specifications
// (Algorithm 1: P = {} gives the empty language, P = {eps} gives eps, both at
// the character cost) and max_cost below the character cost.  Returns true
// when the result is complete without a search.
bool begin_solve(rei_instance* in, double t0) {
  const uint32_t c1 = in->costs.c_char;
  in->lstart.assign(in->max_cost + 2, 0);
  in->lcount.assign(in->max_cost + 2, 0);
  in->uniq.assign(in->max_cost + 2, 0);
  in->cand.assign(in->max_cost + 2, 0);
  in->regex.clear();
  in->known_rows = 0;
  in->pending = 0;
  in->h_aux_valid = false;
  in->rows_elsewhere = false;
  in->aux_view = nullptr;
  in->tree.clear();
  in->resume_level = 0;
  in->otf_level = 0;
  in->otf_blocked = false;
  if (in->max_cost < c1) {
    fill_result(in, REI_NOT_FOUND, 0, 0, t0);
    return true;
  }
  if (in->st.P.size() <= in->max_err) {
    in->regex = "\xE2\x88\x85";
    fill_result(in, REI_OK, c1, 0, t0);
    return true;
  }
  uint64_t bad = 0;
  for (auto& w : in->st.P) bad += w.empty() ? 0 : 1;
  for (auto& w : in->st.N) bad += w.empty() ? 1 : 0;
  if (bad <= in->max_err) {
    in->regex = "\xCE\xB5";
    fill_result(in, REI_OK, c1, 0, t0);
    return true;
  }
  return false;
}

// Builds the result from the device state mirrored by sync_state: level
// sizes and counters, the stop code, and the answer's expression.
rei_status finish_solve(rei_instance* in, double t0) {
  const uint64_t L = in->max_cost + 2;
  const uint32_t c1 = in->costs.c_char;
  uint64_t start = 0;
  uint32_t last_used = c1;
  for (uint64_t c = 0; c < L; ++c) {
    in->lcount[c] = in->h_levels[c];
    in->uniq[c] = in->h_levels[L + c];
    in->cand[c] = in->h_levels[2 * L + c];
    if (c >= c1) {
      in->lstart[c] = start;
      start += in->lcount[c];
      if (in->cand[c]) last_used = (uint32_t)c;
    }
  }
  rei_status final_status = REI_NOT_FOUND;
  uint32_t cost = 0, last = in->max_cost;
  rei_status r;
  if (in->h_state->stop == STOP_OOM || (in->h_state->stop == STOP_NONE && in->otf_blocked)) {
    final_status = REI_OUT_OF_MEMORY;
    last = last_used;
  }
  if (in->h_state->stop == STOP_ANSWER) {
    final_status = REI_OK;
    cost = in->h_state->answer_cost;
    last = cost;
    Node nd;
    if (!decode(in, cost, in->h_state->answer_e, &nd)) {
      in->err = "answer index does not decode";
      return REI_ERR_DEVICE;
    }
    if (!in->tree.empty() && (in->tree[0] != ~0ull || in->tree[1] != (uint64_t)nd.op || in->tree[2] != nd.a ||
                              in->tree[3] != nd.b)) {
      in->err = "device answer tree disagrees with the host decode";
      return REI_ERR_DEVICE;
    }
    if ((r = print_node(in, nd, &in->regex)) != REI_OK) return r;
  }
  if (in->prof && (r = prof_collect(in)) != REI_OK) return r;
  fill_result(in, final_status, cost, last, t0);
  return REI_OK;
}

// The answer's expression tree from the device (decode_tree): in->tree then
// answers the printer's back-pointer reads.  Left empty (the printer reads
// back-pointers itself) in OnTheFly mode, whose levels are not all stored,
// or past the kernel's limits.
rei_status device_tree(rei_instance* in, hipStream_t s) {
  in->tree.clear();
  if (in->otf_on || in->max_cost + 2 > kTreeMaxLevels || in->char_order.size() > kTreeMaxChars) return REI_OK;
  TreeArgs t{};
  t.levels = in->d_levels;
  t.aux = in->d_aux;
  t.st = in->d_state;
  t.out = in->v_tree;
  t.c1 = in->costs.c_char;
  t.c2 = in->costs.c_question;
  t.c3 = in->costs.c_star;
  t.c4 = in->costs.c_concat;
  t.c5 = in->costs.c_union;
  t.nsigma = (uint32_t)in->char_order.size();
  t.max_nodes = kBatchTreeNodes;
  for (size_t k = 0; k < in->char_order.size(); ++k) {
    const uint32_t a = in->char_order[k];
    t.ccost[k] = in->char_cost.empty() ? in->costs.c_char : in->char_cost[a];
  }
  in->h_tree[0] = 0;
  LAUNCH(in, s, REI_K_OTHER, 1, launch_decode_tree(t, s));
  HIP_OK(in, hipStreamSynchronize(s));
  const uint64_t k = std::min<uint64_t>(in->h_tree[0], kBatchTreeNodes);
  in->tree.assign(in->h_tree + 1, in->h_tree + 1 + 4 * k);
  for (size_t q = 0; q + 3 < in->tree.size(); q += 4)
    if (in->tree[q + 1] == OP_CHAR) {
      if (in->tree[q + 2] >= in->char_order.size()) {
        in->tree.clear();  // not a character position: leave it to the printer
        break;
      }
      in->tree[q + 2] = in->char_order[in->tree[q + 2]];  // enumeration -> alphabet position
    }
  return REI_OK;
}

// The per-chunk search on the grid: chunks are enqueued without waiting,
// with one wait per cost level.
rei_status search_levels(rei_instance* in, hipStream_t s) {
  const uint32_t c1 = in->costs.c_char;
  const uint64_t L = in->max_cost + 2;
  rei_status r;
  in->pending = 0;
  in->tree.clear();
  std::fill(in->lstart.begin(), in->lstart.end(), 0);
  std::fill(in->lcount.begin(), in->lcount.end(), 0);
  const uint32_t c_from = in->resume_level;
  in->resume_level = 0;
  in->otf_level = 0;
  in->otf_blocked = false;
  LAUNCH(in, s, REI_K_OTHER, 1, launch_state_reset(in->d_ctrl, in->d_state, in->row_cap, in->otf_on, s));
  in->chunks_enq = 0;
  if (c_from > c1) {
    // The batched solver stored every level below c_from (rows and
    // back-pointers) and wrote its state and counters to the pinned mirrors:
    // put them back on the device, rebuild the table from the rows and
    // continue from level c_from.
    in->known_rows = in->h_state->total_rows;
    uint64_t start = 0;
    for (uint32_t c = c1; c < c_from; ++c) {
      in->lstart[c] = start;
      in->lcount[c] = in->h_levels[c];
      start += in->lcount[c];
    }
    if (start != in->known_rows) {
      in->err = "batched solver state is inconsistent";
      return REI_ERR_DEVICE;
    }
    DevState* hs = in->h_state;
    hs->row_cap = in->row_cap;
    hs->stop = STOP_NONE;
    hs->answer_cost = 0;
    hs->answer_e = 0;
    hs->resume_level = 0;
    hs->chunks = 0;
    HIP_OK(in, hipMemcpyAsync(in->d_state, hs, sizeof(DevState), hipMemcpyHostToDevice, s));
    HIP_OK(in, hipMemcpyAsync(in->d_levels, in->h_levels, 3 * L * 8, hipMemcpyHostToDevice, s));
    // the batched solver used a prefix of the table: rebuild it at full size
    if ((r = ensure_table(in, in->known_rows + 1024, s, true)) != REI_OK) return r;
  } else {
    // a fresh search: nothing stored yet (also when a batched attempt ran out
    // of its preallocated rows and left some behind)
    in->known_rows = 0;
    LAUNCH(in, s, REI_K_OTHER, 3 * L, launch_fill(in->d_levels, 3 * L, 0, s));
    // the host mirrors of the state just reset (the stream has no earlier
    // work of this instance that writes them)
    std::memset(in->h_levels, 0, 3 * L * 8);
    DevState* hs = in->h_state;
    hs->total_rows = 0;
    hs->row_cap = in->row_cap;
    hs->stop = STOP_NONE;
    hs->answer_cost = 0;
    hs->answer_e = 0;
    hs->resume_level = 0;
    hs->otf_on = in->otf_on ? 1u : 0u;
    hs->otf = 0;
    hs->chunks = 0;
    if ((r = ensure_table(in, 1024, s, true)) != REI_OK) return r;
  }
  std::vector<Block> blocks;
  bool stopped = false;
  for (uint32_t c = c_from > c1 ? c_from : c1; c <= in->max_cost && !stopped; ++c) {
    in->lstart[c] = in->known_rows;
    bool blocked = false;
    if (!make_blocks(in, c, &blocks, &blocked)) {
      in->err = "candidate count overflows 64 bits";
      return REI_ERR_TOO_LARGE;
    }
    // chunks of consecutive level indices: large blocks are split, small
    // ones share a chunk.  Chunks grow from the first chunk size to the
    // largest (grid_params, capped by rei_set_chunk) within a
    // level: an answer early in a large level ends it after a few small
    // chunks (later chunks see the stop flag and exit at once), while a level
    // without one costs a handful of extra launches.
    uint64_t e_base = 0, acc = 0;
    const GridTune gt = grid_params(in);
    const uint64_t cmax = std::max<uint64_t>(1, std::min(in->chunk_max, gt.chunk_max));
    uint64_t cur = std::min(cmax, gt.first_chunk);
    std::vector<Piece> pieces;
    for (const Block& b : blocks) {
      for (uint64_t e0 = 0; e0 < b.count && !stopped;) {
        const uint64_t e1 = std::min(b.count, e0 + (cur - acc));
        pieces.push_back({b, e_base, e0, e1});
        acc += e1 - e0;
        e0 = e1;
        if (acc == cur) {
          if ((r = enqueue_chunk(in, s, c, pieces, &stopped)) != REI_OK) return r;
          pieces.clear();
          acc = 0;
          cur = std::min(cmax, 2 * cur);
        }
      }
      if (stopped) break;
      e_base += b.count;
    }
    if (!stopped && !pieces.empty() && (r = enqueue_chunk(in, s, c, pieces, &stopped)) != REI_OK) return r;
    // level boundary: the next level's blocks depend on this level's size
    if ((r = sync_state(in, s, false)) != REI_OK) return r;
    in->lcount[c] = in->h_levels[c];
    if (in->h_state->stop) stopped = true;
    if (!stopped && blocked) {
      in->otf_blocked = true;  // a block needs a level that is not stored
      stopped = true;
    }
    if (in->h_state->otf && !in->otf_level) in->otf_level = c;
  }
  // a stopped search's last wait was on the stream; one that ran out of
  // levels last waited on the mirrors: its launches end before the caller
  // gets the result
  if (in->h_state->stop == STOP_ANSWER) return device_tree(in, s);
  if (!in->h_state->stop) HIP_OK(in, hipStreamSynchronize(s));
  return REI_OK;
}

rei_status solve_impl(rei_instance* in, hipStream_t s, rei_result* out) {
  const double t0 = now_s();
  HIP_OK(in, hipSetDevice(in->device));
  rei_status r;
  if (!begin_solve(in, t0)) {
    if ((r = search_levels(in, s)) != REI_OK) return r;
    if ((r = finish_solve(in, t0)) != REI_OK) return r;
  }
  *out = in->res;
  return REI_OK;
}

// Rows the batched solver preallocates for one instance (its cache budget,
// capped by a per-instance arena size).
uint64_t batch_rows(const rei_instance* in, uint64_t arena_bytes) {
  const uint64_t per_row = 8ull * in->st.W + 8 + 32;  // row, back-pointer, table share
  return std::max<uint64_t>(1024, std::min<uint64_t>(in->row_cap, arena_bytes / per_row));
}

bool batchable(const rei_instance* in) {
  bool same_char_cost = true;
  for (uint32_t ca : in->char_cost) same_char_cost = same_char_cost && ca == in->costs.c_char;
  return in->st.W <= kBatchMaxW && in->max_cost <= kBatchMaxCost && in->st.gt_pair.size() <= batch_max_pairs(in->st.W) &&
         !in->otf_on && same_char_cost;
}

// ---- batched solving -------------------------------------------------------

// Descriptor arrays (pinned host memory the kernel reads directly), side
// streams and events for the batched launches, kept for reuse: allocating
// or freeing them per solve would wait for the whole device.
struct DescBuf {
  BatchDesc* h = nullptr;
  BatchDesc* d = nullptr;  // the device's address of the same memory
  size_t cap = 0;
};
struct SideStream {
  int device = 0;
  hipStream_t s = nullptr;
  hipEvent_t join = nullptr;
};
std::mutex g_pool_mu;
std::vector<DescBuf> g_desc_free;
std::vector<SideStream> g_side_free;
std::vector<std::pair<int, hipEvent_t>> g_event_free;

rei_status desc_acquire(rei_instance* in, size_t n, DescBuf* out) {
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (size_t k = 0; k < g_desc_free.size(); ++k)
      if (g_desc_free[k].cap >= n) {
        *out = g_desc_free[k];
        g_desc_free.erase(g_desc_free.begin() + k);
        return REI_OK;
      }
  }
  DescBuf b;
  b.cap = std::max<size_t>(n, 256);
  HIP_OK(in, hipHostMalloc((void**)&b.h, b.cap * sizeof(BatchDesc), hipHostMallocMapped | hipHostMallocPortable));
  HIP_OK(in, hipHostGetDevicePointer((void**)&b.d, b.h, 0));
  *out = b;
  return REI_OK;
}

rei_status side_acquire(rei_instance* in, SideStream* out) {
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (size_t k = 0; k < g_side_free.size(); ++k)
      if (g_side_free[k].device == in->device) {
        *out = g_side_free[k];
        g_side_free.erase(g_side_free.begin() + k);
        return REI_OK;
      }
  }
  SideStream ss;
  ss.device = in->device;
  HIP_OK(in, hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
  HIP_OK(in, hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
  *out = ss;
  return REI_OK;
}

rei_status event_acquire(rei_instance* in, hipEvent_t* out) {
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (size_t k = 0; k < g_event_free.size(); ++k)
      if (g_event_free[k].first == in->device) {
        *out = g_event_free[k].second;
        g_event_free.erase(g_event_free.begin() + k);
        return REI_OK;
      }
  }
  HIP_OK(in, hipEventCreateWithFlags(out, hipEventDisableTiming));
  return REI_OK;
}

struct BatchRun;
void batch_release(BatchRun* run);

struct BatchRun {
  hipStream_t s = nullptr;
  double t0 = 0;
  std::vector<rei_instance*> grid;                    // per-chunk path afterwards
  // batched, by group: index 0 = one word with keys inline, else W
  std::vector<rei_instance*> members[kBatchMaxW + 1];
  std::vector<rei_instance*> finished;                // results complete
  std::vector<DescBuf> descs;                         // pooled, returned by batch_release
  std::vector<SideStream> sides;
  hipEvent_t fork = nullptr;
  rei_instance* pin = nullptr;  // holds the batched launches' timings
  std::vector<ProfRec> brecs;   // the batched launches' event pairs
  std::vector<int> rec_w;
  // launch shape: threads per instance of each group (forced by the tuner,
  // else tuned or from the batch size)
  uint32_t threads[kBatchMaxW + 1] = {0};
};

// ---- launch shape of the batched solver ---------------------------------
// Threads per instance for a group of n instances of word width W: the
// tuner's choice for this size class when there is one, else enough waves
// per instance to fill the device's wave slots (32 per CU) with n instances.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, uint32_t> g_tuned;  // (group, size class) -> threads
int g_cus = 0;

// Hand-off level size of instances that leave it at the default, per word
// width group (slot 0: one word with keys in the table slots, then 1 + log2
// W): the tuner's choice + 1, or 0 for none (then kBatchLevelMax).  A size
// of 0 sends the group's instances to rei_solve's path at once.
constexpr int kSlots = 7;
std::atomic<uint64_t> g_level_max[kSlots];
// Threads per instance forced on every group while the tuner times a shape.
std::atomic<uint32_t> g_force_threads{0};

int width_slot(int g) { return g == 0 ? 0 : 1 + __builtin_ctz((unsigned)g); }
int group_of(const rei_instance* in) { return in->inl ? 0 : in->st.W; }

uint64_t tuned_level_max(int slot) {
  const uint64_t v = g_level_max[slot].load();
  return v ? v - 1 : kBatchLevelMax;
}

// The instance's hand-off level size (its own setting, else its group's).
uint64_t level_max_of(const rei_instance* in) {
  return in->batch_level_max ? in->batch_level_max : tuned_level_max(width_slot(group_of(in)));
}

// Whether rei_solve_batch (and the server) start the instance in the
// one-workgroup solver: it fits there, and its hand-off size is not 0.
bool batch_path(const rei_instance* in) { return batchable(in) && level_max_of(in) > 0; }

int size_class(size_t n) {
  int k = 0;
  while ((size_t(1) << k) < n) ++k;
  return k;
}

uint32_t max_threads(int g) { return batch_max_threads(g ? g : 1); }

uint32_t choose_threads(int g, size_t n) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find({g, size_class(n)});
    if (it != g_tuned.end()) return it->second;
    if (!g_cus) {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        g_cus = cus;
      else
        g_cus = 256;
    }
  }
  const uint64_t waves = (uint64_t)g_cus * 32 / std::max<size_t>(1, n);
  uint32_t t = waves >= 16 ? 1024u : waves >= 8 ? 512u : 256u;
  return std::min(t, max_threads(g));
}

// Wall-clock counter ticks per microsecond of a device (its counter runs at a
// fixed rate, independent of the shader clock).
uint64_t wall_ticks_per_us(int device) {
  static std::mutex mu;
  static std::map<int, uint64_t> rate;
  std::lock_guard<std::mutex> lk(mu);
  auto it = rate.find(device);
  if (it != rate.end()) return it->second;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0)
    khz = 100000;  // the usual 100 MHz
  const uint64_t t = std::max<uint64_t>(1, (uint64_t)khz / 1000);
  rate[device] = t;
  return t;
}

// Compute units of a device.
uint32_t device_cus(int device) {
  static std::mutex mu;
  static std::map<int, uint32_t> cus;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cus.find(device);
  if (it != cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
  cus[device] = (uint32_t)n;
  return (uint32_t)n;
}

BatchDesc make_desc(const rei_instance* in) {
  BatchDesc d{};
  d.gt_off = in->d_gt_off;
  d.gt_pair = in->d_gt_pair;
  d.len_off = in->d_len_off;
  d.pmask = in->d_pmask;
  d.nmask = in->d_nmask;
  d.char_index = in->d_char_index;
  d.n = in->st.n;
  d.n_pairs = (uint32_t)in->st.gt_pair.size();
  d.max_len = in->st.max_len;
  d.nsigma = (uint32_t)in->st.sigma.size();
  d.c1 = in->costs.c_char;
  d.c2 = in->costs.c_question;
  d.c3 = in->costs.c_star;
  d.c4 = in->costs.c_concat;
  d.c5 = in->costs.c_union;
  d.max_cost = in->max_cost;
  d.max_err = in->max_err;
  d.rows = in->d_rows;
  d.aux = in->d_aux;
  d.rows_alloc = in->rows_alloc;
  d.row_cap = in->row_cap;
  d.slots = in->d_slots;
  d.sref = in->d_sref;
  d.inl = in->inl ? 1u : 0u;
  d.level_max = level_max_of(in);
  const int64_t us = in->batch_time_us < 0 ? kBatchTimeUs : in->batch_time_us;
  d.time_ticks = us ? (uint64_t)us * wall_ticks_per_us(in->device) : 0;
  d.slot_mask = in->slots_cap - 1;
  d.skey = in->d_skey;
  d.se = in->d_se;
  d.spos = in->d_spos;
  d.hst = in->v_state;
  d.hlev = in->v_levels;
  d.htree = in->v_tree;
  return d;
}

// Device bytes a batched instance uses (rows, back-pointers, table, survivors).
uint64_t batch_reserve(const rei_instance* in, uint64_t arena_bytes) {
  const uint64_t R = batch_rows(in, arena_bytes);
  const uint64_t W = in->st.W;
  return R * (8 * W + 8) + pow2_at_least(4 * (R + kBatchChunk)) * 8 + kBatchChunk * (8 * W + 12);
}

// Trivial instances are finished at once, others that cannot be batched go to
// run->grid; the rest are staged and launched (one launch per word width) on
// run->s.  Nothing waits for the device.
rei_status batch_launch(rei_instance* const* insts, size_t n, hipStream_t s, uint64_t arena_bytes,
                        BatchRun* run) {
  run->s = s;
  run->t0 = now_s();
  std::vector<BatchDesc> groups[kBatchMaxW + 1];
  rei_status r;
  for (size_t i = 0; i < n; ++i) {
    rei_instance* in = insts[i];
    in->err.clear();
    HIP_OK(in, hipSetDevice(in->device));
    if (begin_solve(in, run->t0)) {
      run->finished.push_back(in);
      continue;
    }
    if (!batch_path(in)) {
      run->grid.push_back(in);
      continue;
    }
    const uint64_t R = batch_rows(in, arena_bytes);
    if ((r = ensure_chunk_buffers(in, kBatchChunk)) != REI_OK) return r;
    if ((r = ensure_rows(in, R, s)) != REI_OK) return r;
    if ((r = ensure_table(in, in->rows_alloc + kBatchChunk, s, false)) != REI_OK) return r;
    const int g = in->inl ? 0 : in->st.W;
    groups[g].push_back(make_desc(in));
    run->members[g].push_back(in);
    __atomic_store_n(&in->h_state->done, 0u, __ATOMIC_RELEASE);
  }
  run->pin = n ? insts[0] : nullptr;
  // Hand-off on time moves deep searches onto compute units the batch leaves
  // idle; a batch with a workgroup for every compute unit leaves none.
  size_t batched = 0;
  for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1) batched += groups[g].size();
  if (n && batched >= device_cus(insts[0]->device))
    for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
      for (BatchDesc& d : groups[g]) d.time_ticks = 0;
  // One launch per word width; the first on s, the others on side streams
  // that start after s's earlier work and that s waits for, so the groups
  // run side by side.  The fork is recorded before the first launch: after
  // it, the side streams would wait for the first group to finish.
  {
    rei_instance* lead = nullptr;
    int n_groups = 0;
    for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
      if (!groups[g].empty()) {
        if (!lead) lead = run->members[g][0];
        ++n_groups;
      }
    if (n_groups > 1) {
      if ((r = event_acquire(lead, &run->fork)) != REI_OK) return r;
      HIP_OK(lead, hipEventRecord(run->fork, s));
    }
  }
  bool first = true;
  for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1) {
    if (groups[g].empty()) continue;
    rei_instance* in0 = run->members[g][0];
    DescBuf db;
    if ((r = desc_acquire(in0, groups[g].size(), &db)) != REI_OK) return r;
    run->descs.push_back(db);
    std::memcpy(db.h, groups[g].data(), groups[g].size() * sizeof(BatchDesc));
    hipStream_t gs = s;
    if (!first) {
      SideStream ss;
      if ((r = side_acquire(in0, &ss)) != REI_OK) return r;
      run->sides.push_back(ss);
      HIP_OK(in0, hipStreamWaitEvent(ss.s, run->fork, 0));
      gs = ss.s;
    }
    const uint32_t forced = g_force_threads.load();
    const uint32_t th = forced ? std::min(forced, max_threads(g)) : choose_threads(g, groups[g].size());
    run->threads[g] = th;
    hipEvent_t ev = nullptr, ev2 = nullptr;
    if ((r = prof_begin(run->pin, gs, REI_K_BATCH, &ev, &ev2)) != REI_OK) return r;
    HIP_OK(in0, launch_solve_batch(g ? g : 1, g == 0, th, db.d, (uint32_t)groups[g].size(), gs));
    if ((r = prof_end(run->pin, gs, REI_K_BATCH, ev, ev2, 0)) != REI_OK) return r;
    if (profiled(run->pin, REI_K_BATCH)) {
      // kept apart from the instance's own records until the launch is
      // known to have finished (the instance may continue on the grid)
      run->brecs.push_back(run->pin->recs.back());
      run->pin->recs.pop_back();
      run->rec_w.push_back(g);
    }
    if (!first) {
      HIP_OK(in0, hipEventRecord(run->sides.back().join, gs));
      HIP_OK(in0, hipStreamWaitEvent(s, run->sides.back().join, 0));
    }
    first = false;
  }
  return REI_OK;
}

// Returns the run's pooled resources; the launches must have finished (or
// never been enqueued).
void batch_release(BatchRun* run) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  for (auto& d : run->descs) g_desc_free.push_back(d);
  run->descs.clear();
  for (auto& ss : run->sides) g_side_free.push_back(ss);
  run->sides.clear();
  if (run->fork) g_event_free.push_back({run->pin ? run->pin->device : 0, run->fork});
  run->fork = nullptr;
}

// After run->s has finished the launches: results of the batched instances;
// those that outgrew their preallocated rows are appended to run->grid.
// Reads a batched instance's final state from its pinned buffers (the
// kernel wrote them); true when it continues on the per-chunk path.
bool batch_take_state(rei_instance* in) {
  in->known_rows = in->h_state->total_rows;
  in->pending = 0;
  const uint64_t k = std::min<uint64_t>(in->h_tree[0], kBatchTreeNodes);
  in->tree.assign(in->h_tree + 1, in->h_tree + 1 + 4 * k);
  if (in->h_state->stop == STOP_CAPACITY || in->h_state->stop == STOP_HANDOFF) {
    in->resume_level = in->h_state->stop == STOP_HANDOFF ? (uint32_t)in->h_state->resume_level : 0;
    return true;
  }
  return false;
}

// The batched launches' event pairs go into the statistics of insts[0];
// call once nothing else uses that instance.
rei_status batch_fold_prof(BatchRun* run) {
  if (!run->pin || run->brecs.empty()) return REI_OK;
  uint64_t group_cand[kBatchMaxW + 1] = {0};
  for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
    for (rei_instance* in : run->members[g]) {
      const uint64_t L = in->max_cost + 2;
      for (uint64_t c = 0; c < L; ++c) group_cand[g] += in->h_levels[2 * L + c];
    }
  for (size_t q = 0; q < run->brecs.size(); ++q) run->brecs[q].units = group_cand[run->rec_w[q]];
  run->pin->recs.insert(run->pin->recs.end(), run->brecs.begin(), run->brecs.end());
  run->brecs.clear();
  return prof_collect(run->pin);
}

// After run->s has finished the launches: results of the batched instances
// (those already taken, listed in `taken`, are skipped); those that
// continue on the per-chunk path are appended to run->grid.
rei_status batch_collect(BatchRun* run, const std::vector<rei_instance*>* taken = nullptr,
                         bool fold_prof = true) {
  rei_status r;
  if (run->pin) HIP_OK(run->pin, hipStreamSynchronize(run->s));
  batch_release(run);
  std::vector<rei_instance*> done;
  for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
    for (rei_instance* in : run->members[g]) {
      if (taken && std::find(taken->begin(), taken->end(), in) != taken->end()) continue;
      if (batch_take_state(in))
        run->grid.push_back(in);
      else
        done.push_back(in);
    }
  for (rei_instance* in : done) {
    if ((r = finish_solve(in, run->t0)) != REI_OK) return r;
    // latency of an instance the launch finished: when its flag showed
    if (in->t_seen >= 0) in->res.seconds_solve = in->t_seen;
    in->t_seen = -1;
    run->finished.push_back(in);
  }
  if (fold_prof && (r = batch_fold_prof(run)) != REI_OK) return r;
  return REI_OK;
}

constexpr int kGridWorkers = 8;

// Worker threads that run the per-chunk path for instances handed to them
// while a batched launch still runs: 8 threads for the whole process, each
// driving its own pooled stream per device, started on first use and kept
// (starting threads per call cost the polling thread tens of microseconds
// per hand-off).  A GridPool is one call's group of instances on them.
class Workers {
 public:
  struct Group {
    double t0 = 0;
    size_t pending = 0;
    rei_status status = REI_OK;
  };
  static Workers& get() {
    // never destroyed: threads parked on its condition variable at process
    // exit must not see it torn down
    static Workers* w = new Workers();
    return *w;
  }
  void submit(Group* g, rei_instance* in) {
    std::lock_guard<std::mutex> lk(mu_);
    ++g->pending;
    q_.push_back({g, in});
    if (idle_ == 0 && threads_ < kThreads) {
      ++threads_;
      std::thread([this] { work(); }).detach();
    }
    cv_.notify_one();
  }
  // Waits until every instance of the group is done; the first error.
  rei_status wait(Group* g) {
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return g->pending == 0; });
    return g->status;
  }

 private:
  static constexpr int kThreads = kGridWorkers;
  struct Job {
    Group* g;
    rei_instance* in;
  };
  void work() {
    std::vector<SideStream> streams;  // one per device this thread has served
    for (;;) {
      Job job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        ++idle_;
        cv_.wait(lk, [&] { return !q_.empty(); });
        --idle_;
        job = q_.front();
        q_.pop_front();
      }
      rei_instance* in = job.in;
      rei_status r = REI_OK;
      try {
        if (hipSetDevice(in->device) != hipSuccess) r = REI_ERR_DEVICE;
        SideStream* ss = nullptr;
        for (auto& x : streams)
          if (x.device == in->device) ss = &x;
        if (r == REI_OK && !ss) {
          SideStream n;
          r = side_acquire(in, &n);
          if (r == REI_OK) {
            streams.push_back(n);
            ss = &streams.back();
          }
        }
        if (r == REI_OK) r = search_levels(in, ss->s);
        if (r == REI_OK) r = finish_solve(in, job.g->t0);
        // the instance's work is on ss: finished before the caller sees it
        if (r == REI_OK && hipStreamSynchronize(ss->s) != hipSuccess) r = REI_ERR_DEVICE;
      } catch (const std::bad_alloc&) {
        r = REI_ERR_HOST_ALLOC;
      }
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (r != REI_OK && job.g->status == REI_OK) job.g->status = r;
        --job.g->pending;
      }
      done_cv_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Job> q_;
  int threads_ = 0;
  int idle_ = 0;
};

class GridPool {
 public:
  explicit GridPool(double t0) { g_.t0 = t0; }
  ~GridPool() { (void)join(); }
  void submit(rei_instance* in) { Workers::get().submit(&g_, in); }
  rei_status join() { return Workers::get().wait(&g_); }

 private:
  Workers::Group g_;
};

// Frees the language cache, the table and the chunk buffers (the staged
// tables and the result stay).
void free_search_buffers(rei_instance* in) {
  (void)hipSetDevice(in->device);
  dfree(in, in->d_rows);
  dfree(in, in->d_aux);
  dfree(in, in->d_slots);
  dfree(in, in->d_sref);
  dfree(in, in->d_skey);
  dfree(in, in->d_se);
  dfree(in, in->d_spos);
  dfree(in, in->d_bitmap);
  dfree(in, in->d_prefix);
  dfree(in, in->d_bsums);
  in->rows_alloc = 0;
  in->slots_cap = 0;
  in->surv_cap = 0;
  in->bitmap_cap = 0;
  in->known_rows = 0;
  in->h_aux_valid = false;
}

void free_device(rei_instance* in) {
  (void)hipSetDevice(in->device);
  dfree(in, in->d_gt_off);
  dfree(in, in->d_gt_pair);
  dfree(in, in->d_len_off);
  dfree(in, in->d_pmask);
  dfree(in, in->d_nmask);
  dfree(in, in->d_char_index);
  dfree(in, in->d_rows);
  dfree(in, in->d_aux);
  dfree(in, in->d_slots);
  dfree(in, in->d_sref);
  dfree(in, in->d_skey);
  dfree(in, in->d_se);
  dfree(in, in->d_spos);
  dfree(in, in->d_bitmap);
  dfree(in, in->d_prefix);
  dfree(in, in->d_bsums);
  dfree(in, in->d_ctrl);
  dfree(in, in->d_state);
  dfree(in, in->d_levels);
  if (in->h_state) (void)hipHostFree(in->h_state);
  if (in->h_levels) (void)hipHostFree(in->h_levels);
  if (in->h_tree) (void)hipHostFree(in->h_tree);
  in->h_state = nullptr;
  in->h_levels = nullptr;
  in->h_tree = nullptr;
  for (auto& r : in->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  in->recs.clear();
  for (auto e : in->pool) (void)hipEventDestroy(e);
  in->pool.clear();
}

template <class T>
rei_status upload(rei_instance* in, T** dst, const std::vector<T>& src) {
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  HIP_OK(in, dev_alloc(in, dst, bytes));
  if (!src.empty()) HIP_OK(in, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return REI_OK;
}

rei_status create_device(rei_instance* in) {
  HIP_OK(in, hipGetDevice(&in->device));
  rei_status r;
  if ((r = upload(in, &in->d_gt_off, in->st.gt_off)) != REI_OK) return r;
  if ((r = upload(in, &in->d_gt_pair, in->st.gt_pair)) != REI_OK) return r;
  if ((r = upload(in, &in->d_len_off, in->st.len_off)) != REI_OK) return r;
  if ((r = upload(in, &in->d_pmask, in->st.pmask)) != REI_OK) return r;
  if ((r = upload(in, &in->d_nmask, in->st.nmask)) != REI_OK) return r;
  in->char_order.resize(in->st.sigma.size());
  for (uint32_t a = 0; a < in->char_order.size(); ++a) in->char_order[a] = a;
  if ((r = upload(in, &in->d_char_index, in->st.char_index)) != REI_OK) return r;
  HIP_OK(in, dev_alloc(in, &in->d_ctrl, sizeof(Ctrl)));
  HIP_OK(in, dev_alloc(in, &in->d_state, sizeof(DevState)));
  const uint64_t L = in->max_cost + 2;
  HIP_OK(in, dev_alloc(in, &in->d_levels, 3 * L * 8));
  // coherent (fine-grained): the batched solver's completion flag is read
  // by the host while the launch still runs
  const unsigned fl = hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent;
  HIP_OK(in, hipHostMalloc((void**)&in->h_state, sizeof(DevState), fl));
  HIP_OK(in, hipHostMalloc((void**)&in->h_levels, 3 * L * 8, fl));
  HIP_OK(in, hipHostMalloc((void**)&in->h_tree, (1 + 4 * kBatchTreeNodes) * 8, fl));
  in->h_tree[0] = 0;
  HIP_OK(in, hipHostGetDevicePointer((void**)&in->v_state, in->h_state, 0));
  HIP_OK(in, hipHostGetDevicePointer((void**)&in->v_levels, in->h_levels, 0));
  HIP_OK(in, hipHostGetDevicePointer((void**)&in->v_tree, in->h_tree, 0));
  return REI_OK;
}

// Reads a tuning file as rei_tune_save writes it: objects of integer
// fields under "batch_threads", "batch_level_max" and "grid".  Entries
// with values out of range are rejected as a whole (nothing is applied).
bool tune_parse(const std::string& text) {
  auto section = [&](const char* key, std::string* out) -> bool {
    const size_t k = text.find(std::string("\"") + key + "\"");
    if (k == std::string::npos) return false;
    const size_t a = text.find('[', k), b = text.find(']', k);
    if (a == std::string::npos || b == std::string::npos || b < a) return false;
    *out = text.substr(a + 1, b - a - 1);
    return true;
  };
  auto field = [](const std::string& obj, const char* key, uint64_t* v) -> bool {
    const size_t k = obj.find(std::string("\"") + key + "\"");
    if (k == std::string::npos) return false;
    size_t c = obj.find(':', k);
    if (c == std::string::npos) return false;
    ++c;
    while (c < obj.size() && (obj[c] == ' ' || obj[c] == '\t' || obj[c] == '\n')) ++c;
    if (c >= obj.size() || obj[c] < '0' || obj[c] > '9') return false;
    *v = std::strtoull(obj.c_str() + c, nullptr, 10);
    return true;
  };
  auto objects = [](const std::string& arr) {
    std::vector<std::string> out;
    size_t p = 0;
    while ((p = arr.find('{', p)) != std::string::npos) {
      const size_t q = arr.find('}', p);
      if (q == std::string::npos) break;
      out.push_back(arr.substr(p, q - p + 1));
      p = q + 1;
    }
    return out;
  };
  std::map<std::pair<int, int>, uint32_t> bt;
  std::map<int, GridTune> gr;
  uint64_t lm[kSlots] = {0};
  std::string arr;
  if (section("batch_threads", &arr))
    for (const std::string& o : objects(arr)) {
      uint64_t g = 0, c = 0, t = 0;
      if (!field(o, "group", &g) || !field(o, "size_class", &c) || !field(o, "threads", &t)) return false;
      if (g > (uint64_t)kBatchMaxW || (g & (g - 1)) || c > 40 || (t != 256 && t != 512 && t != 1024) ||
          t > batch_max_threads(g ? (int)g : 1))
        return false;
      bt[{(int)g, (int)c}] = (uint32_t)t;
    }
  if (section("grid", &arr))
    for (const std::string& o : objects(arr)) {
      uint64_t w = 0, fc = 0, cm = 0, wg = 0, xi = 0;
      if (!field(o, "words", &w) || !field(o, "first_chunk", &fc) || !field(o, "chunk_max", &cm) ||
          !field(o, "concat_wg", &wg) || !field(o, "concat_xi", &xi))
        return false;
      if (w < 1 || w > (uint64_t)kMaxWords || (w & (w - 1)) || fc < 1 || cm < 1 || cm > kMaxChunk || wg < 1 ||
          wg > (1u << 24) || xi < 1 || xi > 64)
        return false;
      gr[(int)w] = GridTune{fc, cm, (uint32_t)wg, (uint32_t)xi};
    }
  if (section("batch_level_max", &arr))
    for (const std::string& o : objects(arr)) {
      uint64_t g = 0, v = 0;
      if (!field(o, "group", &g) || !field(o, "level_max", &v)) return false;
      if (g > (uint64_t)kBatchMaxW || (g & (g - 1)) || v > (1ull << 40)) return false;
      lm[width_slot((int)g)] = v + 1;
    }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : bt) g_tuned[kv.first] = kv.second;
  }
  {
    std::lock_guard<std::mutex> lk(g_grid_mu);
    for (auto& kv : gr) g_grid_tuned[kv.first] = kv.second;
  }
  for (int k = 0; k < kSlots; ++k)
    if (lm[k]) g_level_max[k].store(lm[k]);
  return true;
}

// REI_TUNE_FILE names a tuning file (as rei_tune_save writes it) that the
// process loads once, when its first instance is created.
void load_tune_file_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* p = std::getenv("REI_TUNE_FILE");
    if (!p || !*p) return;
    FILE* f = std::fopen(p, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    std::fclose(f);
    (void)tune_parse(text);
  });
}

}  // namespace

extern "C" {

rei_status rei_create(const char* alphabet, const char* const* pos, size_t n_pos, const char* const* neg,
                      size_t n_neg, rei_costs costs, uint32_t max_cost, uint64_t cache_bytes,
                      rei_instance** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "null output pointer";
    return REI_ERR_INVALID_ARG;
  }
  *out = nullptr;
  const double t0 = now_s();
  load_tune_file_once();
  if (costs.c_char < 1 || costs.c_question < 1 || costs.c_star < 1 || costs.c_concat < 1 ||
      costs.c_union < 1) {
    g_create_error = "every constructor cost must be at least 1";
    return REI_ERR_INVALID_ARG;
  }
  if (max_cost > (1u << 20)) {
    g_create_error = "max_cost above 2^20";
    return REI_ERR_INVALID_ARG;
  }
  rei_instance* in = new (std::nothrow) rei_instance();
  if (!in) return REI_ERR_HOST_ALLOC;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    in->alloc = g_alloc;
  }
  rei_status st;
  try {
    st = stage(alphabet, pos, n_pos, neg, n_neg, &in->st, &g_create_error);
  } catch (const std::bad_alloc&) {
    st = REI_ERR_HOST_ALLOC;
  } catch (...) {
    st = REI_ERR_INVALID_ARG;
  }
  if (st != REI_OK) {
    delete in;
    return st;
  }
  in->costs = costs;
  in->max_cost = max_cost;
  in->cache_bytes = cache_bytes;
  in->row_cap = cache_bytes / (8ull * in->st.W + 8);
  in->inl = in->st.W == 1 && in->st.n <= 63;
  if ((st = create_device(in)) != REI_OK) {
    g_create_error = in->err;
    free_device(in);
    delete in;
    return st;
  }
  in->seconds_stage = now_s() - t0;
  *out = in;
  return REI_OK;
}

rei_status rei_solve(rei_instance* inst, void* hip_stream, rei_result* out) {
  if (!inst || !out) return REI_ERR_INVALID_ARG;
  inst->err.clear();
  try {
    return solve_impl(inst, (hipStream_t)hip_stream, out);
  } catch (const std::bad_alloc&) {
    inst->err = "host allocation failed";
    return REI_ERR_HOST_ALLOC;
  }
}

rei_status rei_solve_batch(rei_instance* const* insts, size_t n, void* hip_stream, uint64_t arena_bytes,
                           rei_result* out) {
  if (n && (!insts || !out)) return REI_ERR_INVALID_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!insts[i]) return REI_ERR_INVALID_ARG;
  if (arena_bytes == 0) arena_bytes = kDefaultArena;
  hipStream_t s = (hipStream_t)hip_stream;
  BatchRun run;
  rei_status r;
  try {
    if ((r = batch_launch(insts, n, s, arena_bytes, &run)) != REI_OK) {
      (void)hipStreamSynchronize(s);
      batch_release(&run);
      return r;
    }
    // Instances that are not batched start on the per-chunk path at once;
    // batched ones that hand off (or outgrow their rows) follow as soon as
    // their completion flag shows, while the launches still run.
    GridPool pool(run.t0);
    for (rei_instance* in : run.grid) pool.submit(in);
    run.grid.clear();
    std::vector<rei_instance*> members, taken;
    for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
      members.insert(members.end(), run.members[g].begin(), run.members[g].end());
    std::vector<char> seen(members.size(), 0);
    size_t left = members.size();
    bool launches_done = false;
    double last_query = 0;
    while (left) {
      bool progress = false;
      for (size_t i = 0; i < members.size(); ++i) {
        if (seen[i] || !__atomic_load_n(&members[i]->h_state->done, __ATOMIC_ACQUIRE)) continue;
        seen[i] = 1;
        members[i]->t_seen = now_s() - run.t0;
        --left;
        progress = true;
        if (batch_take_state(members[i])) {
          taken.push_back(members[i]);
          pool.submit(members[i]);
        }
      }
      if (!left || progress) continue;
      if (launches_done) break;  // every flag is final: collected below
      // the flags are plain host memory, read at every pass; the stream is
      // asked (a runtime call the workers' launches contend with) every
      // 50 us at most
      if (now_s() - last_query < 50e-6) {
        // a sleep would round up to the timer slack (tens of microseconds),
        // which the deep instances' hand-offs would wait for
        std::this_thread::yield();
        continue;
      }
      last_query = now_s();
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        launches_done = true;  // one more pass sees every flag
      } else if (q != hipErrorNotReady) {
        for (size_t i = 0; i < n; ++i) insts[i]->err = std::string("batched launch: ") + hipGetErrorString(q);
        (void)pool.join();
        (void)hipStreamSynchronize(s);
        batch_release(&run);
        return REI_ERR_DEVICE;
      } else {
        std::this_thread::yield();
      }
    }
    hipError_t se = hipStreamSynchronize(s);
    if (se != hipSuccess) {
      for (size_t i = 0; i < n; ++i) insts[i]->err = std::string("batched launch: ") + hipGetErrorString(se);
      (void)pool.join();
      batch_release(&run);
      return REI_ERR_DEVICE;
    }
    r = batch_collect(&run, &taken, false);
    for (rei_instance* in : run.grid) pool.submit(in);
    const rei_status rp = pool.join();
    if (r != REI_OK) return r;
    if (rp != REI_OK) return rp;
    if ((r = batch_fold_prof(&run)) != REI_OK) return r;
    // seconds_solve: when each result was known (its flag, or the end of
    // its per-chunk levels), counted from the start of the call
    for (size_t i = 0; i < n; ++i) out[i] = insts[i]->res;
  } catch (const std::bad_alloc&) {
    return REI_ERR_HOST_ALLOC;
  }
  return REI_OK;
}

rei_status rei_solve_batch_noalloc(rei_instance* const* insts, size_t n, void* hip_stream, rei_result* out) {
  if (n && (!insts || !out)) return REI_ERR_INVALID_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!insts[i]) return REI_ERR_INVALID_ARG;
  if (n == 0) return REI_OK;
  auto fail = [&](rei_status st, size_t i, const std::string& msg) {
    insts[i]->err = msg;
    return st;
  };
  if (n > kStaticMaxInstances)
    return fail(REI_ERR_TOO_LARGE, 0,
                "at most " + std::to_string(kStaticMaxInstances) + " instances per allocation-free call");
  int dev = 0;
  HIP_OK(insts[0], hipGetDevice(&dev));
  for (size_t i = 0; i < n; ++i)
    if (insts[i]->device != dev) return fail(REI_ERR_INVALID_ARG, i, "instance lives on another device");
  void* base = nullptr;
  HIP_OK(insts[0], static_scratch(&base));
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    const double t0 = now_s();
    // searches to run (trivial specifications are answered here), then
    // ordered by word width (group 0: one word with keys inline)
    uint32_t todo[kStaticMaxInstances], idx[kStaticMaxInstances];
    uint32_t nt = 0, m = 0;
    for (size_t i = 0; i < n; ++i) {
      rei_instance* in = insts[i];
      in->err.clear();
      if (begin_solve(in, t0)) continue;
      if (!batchable(in))
        return fail(REI_ERR_TOO_LARGE, i,
                    "instance cannot run in the one-workgroup solver (more than 32 words, max_cost above 63, "
                    "too many cuts, OnTheFly mode or per-character costs)");
      todo[nt++] = (uint32_t)i;
    }
    auto group = [&](uint32_t i) { return insts[i]->inl ? 0 : insts[i]->st.W; };
    for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
      for (uint32_t k = 0; k < nt; ++k)
        if (group(todo[k]) == g) idx[m++] = todo[k];
    // equal shares of the array after the descriptor header, 256-byte aligned
    const uint64_t share = m ? ((kStaticScratchBytes - kStaticHeaderBytes) / m) & ~255ull : 0;
    BatchDesc stage[kStaticMaxInstances];
    uint64_t rows_of[kStaticMaxInstances];
    const uint64_t* aux_of[kStaticMaxInstances];
    unsigned char* const arena0 = (unsigned char*)base + kStaticHeaderBytes;
    for (uint32_t k = 0; k < m; ++k) {
      rei_instance* in = insts[idx[k]];
      const uint64_t W = in->st.W;
      const uint64_t tab = in->inl ? 16 : 8;  // table bytes per slot
      auto up = [](uint64_t b) { return (b + 255) & ~255ull; };
      const uint64_t fixed = up(kBatchChunk * W * 8) + up(kBatchChunk * 4) + up(kBatchChunk * 8);
      // largest row count R (and table of T slots, T >= 2 (R + chunk), a
      // power of two) whose buffers fit the share
      uint64_t R = 0, T = 0;
      for (uint64_t t = 1ull << 40; t >= 4096; t >>= 1) {
        if (fixed + t * tab + 2 * 256 > share) continue;
        const uint64_t by_mem = (share - fixed - t * tab - 2 * 256) / (8 * W + 8);
        const uint64_t by_tab = t / 2 > kBatchChunk ? t / 2 - kBatchChunk : 0;
        const uint64_t r = std::min(std::min(by_mem, by_tab), in->row_cap);
        if (r > R) {
          R = r;
          T = t;
        }
      }
      if (R < 1024 && R < in->row_cap)
        return fail(REI_ERR_TOO_LARGE, idx[k], "the static array's share per instance is too small; call with fewer instances");
      unsigned char* p = arena0 + (uint64_t)k * share;
      BatchDesc d = make_desc(in);
      d.skey = (uint64_t*)p;
      p += up(kBatchChunk * W * 8);
      d.se = (uint32_t*)p;
      p += up(kBatchChunk * 4);
      d.spos = (uint64_t*)p;
      p += up(kBatchChunk * 8);
      d.rows = (uint64_t*)p;
      p += up(R * W * 8);
      d.aux = (uint64_t*)p;
      p += up(R * 8);
      d.slots = (uint64_t*)p;
      p += T * 8;
      d.sref = in->inl ? (uint64_t*)p : nullptr;
      d.rows_alloc = R;
      d.slot_mask = T - 1;
      d.level_max = ~0ull;  // the whole search stays in the workgroup
      d.time_ticks = 0;
      stage[k] = d;
      rows_of[k] = R;
      aux_of[k] = d.aux;
      __atomic_store_n(&in->h_state->done, 0u, __ATOMIC_RELEASE);
    }
    BatchDesc* d_desc = (BatchDesc*)base;
    if (m) HIP_OK(insts[0], launch_put_descs(d_desc, stage, m, s));
    // one launch per word width, one after another on the caller's stream
    for (uint32_t k = 0; k < m;) {
      rei_instance* in0 = insts[idx[k]];
      const int g = group(idx[k]);
      uint32_t e = k;
      while (e < m && group(idx[e]) == g) ++e;
      HIP_OK(in0, launch_solve_batch(g ? g : 1, g == 0, choose_threads(g, e - k), d_desc + k, e - k, s));
      k = e;
    }
    HIP_OK(insts[0], hipStreamSynchronize(s));
    rei_status r = REI_OK;
    for (uint32_t k = 0; k < m; ++k) {
      rei_instance* in = insts[idx[k]];
      const bool more = batch_take_state(in);
      in->rows_elsewhere = true;
      if (more) {
        r = fail(REI_ERR_TOO_LARGE, idx[k],
                 "the search outgrew its share of the static array (" + std::to_string(rows_of[k]) +
                     " rows); call with fewer instances");
        continue;
      }
      in->aux_view = aux_of[k];  // valid until this call returns
      const rei_status f = finish_solve(in, t0);
      in->aux_view = nullptr;
      in->h_aux_valid = false;
      if (f != REI_OK && r == REI_OK) r = f;
    }
    if (r != REI_OK) return r;
    for (size_t i = 0; i < n; ++i) out[i] = insts[i]->res;
  } catch (const std::bad_alloc&) {
    return REI_ERR_HOST_ALLOC;
  }
  return REI_OK;
}

rei_status rei_tune_batch(rei_instance* const* insts, size_t n, void* hip_stream, uint64_t arena_bytes,
                          uint32_t* threads_out, uint64_t* level_max_out) {
  if (n == 0 || !insts) return REI_ERR_INVALID_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!insts[i]) return REI_ERR_INVALID_ARG;
  if (arena_bytes == 0) arena_bytes = kDefaultArena;
  try {
    const uint32_t cand[3] = {256, 512, 1024};
    std::vector<rei_result> res(n);
    rei_status r;
    // the shortest of five whole calls (batched launches and the hand-offs
    // they start), with the current shape and hand-off settings
    auto time_calls = [&](double* best) -> rei_status {
      for (int q = 0; q < 5; ++q) {
        const double t = now_s();
        rei_status st = rei_solve_batch(insts, n, hip_stream, arena_bytes, res.data());
        if (st != REI_OK) return st;
        *best = std::min(*best, now_s() - t);
      }
      return REI_OK;
    };
    // Launch shape: every group at one shape, whole calls timed (what the
    // caller waits for, hand-offs included, not the launches alone); the
    // shapes take turns, one call each per round over five rounds, so that
    // drift during tuning favours none of them.
    double shape_s[3] = {1e300, 1e300, 1e300};
    for (int round = 0; round < 5; ++round)
      for (int q = 0; q < 3; ++q) {
        g_force_threads.store(cand[q]);
        const double t = now_s();
        r = rei_solve_batch(insts, n, hip_stream, arena_bytes, res.data());
        shape_s[q] = std::min(shape_s[q], now_s() - t);
        g_force_threads.store(0);
        if (r != REI_OK) return r;
      }
    const int bq = (int)(std::min_element(shape_s, shape_s + 3) - shape_s);
    size_t group_n[kBatchMaxW + 1] = {0};
    for (size_t i = 0; i < n; ++i)
      if (batchable(insts[i])) ++group_n[insts[i]->inl ? 0 : insts[i]->st.W];
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1) {
        const int slot = width_slot(g);  // W1-inline, W1, W2, W4, ..., W32
        const uint32_t t = group_n[g] ? std::min(cand[bq], max_threads(g)) : 0u;
        if (t) g_tuned[{g, size_class(group_n[g])}] = t;
        if (threads_out) threads_out[slot] = t;
      }
    }
    // Hand-off level size (instances left at the default), whole calls with
    // the shape just chosen.  First one size for every group present: 2^8,
    // 2^10, 2^12, then 2^13 .. 2^19, the shortest wins.  Then, widest group
    // first, each group no larger than the worker pool (which runs that many
    // at once) tries 0: its instances take rei_solve's path from the start;
    // kept only if at least 3 % faster (timing noise must not move a group).
    static const uint64_t sizes[] = {1u << 8, 1u << 10, 1u << 12, 1u << 13, 1u << 14, 1u << 15,
                                     1u << 16, 1u << 17, 1u << 18, 1u << 19};
    uint64_t keep[kSlots];
    for (int k = 0; k < kSlots; ++k) keep[k] = g_level_max[k].load();
    auto set_all = [&](uint64_t l) {
      for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
        if (group_n[g]) g_level_max[width_slot(g)].store(l + 1);
    };
    auto restore = [&] {
      for (int k = 0; k < kSlots; ++k) g_level_max[k].store(keep[k]);
    };
    double best_s = 1e300;
    uint64_t best_l = kBatchLevelMax;
    for (uint64_t l : sizes) {
      set_all(l);
      double t = 1e300;
      if ((r = time_calls(&t)) != REI_OK) {
        restore();
        return r;
      }
      if (t < best_s) {
        best_s = t;
        best_l = l;
      }
    }
    set_all(best_l);
    for (int g = kBatchMaxW; g >= 0; g = g > 1 ? g / 2 : g - 1) {
      if (!group_n[g] || group_n[g] > (size_t)kGridWorkers) continue;
      const int slot = width_slot(g);
      g_level_max[slot].store(0 + 1);
      double t = 1e300;
      if ((r = time_calls(&t)) != REI_OK) {
        restore();
        return r;
      }
      if (t < 0.97 * best_s)
        best_s = t;
      else
        g_level_max[slot].store(best_l + 1);
    }
    if (level_max_out) {
      std::fill(level_max_out, level_max_out + kSlots, ~0ull);
      for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1)
        if (group_n[g]) level_max_out[width_slot(g)] = tuned_level_max(width_slot(g));
    }
    return REI_OK;
  } catch (const std::bad_alloc&) {
    g_force_threads.store(0);
    return REI_ERR_HOST_ALLOC;
  }
}

rei_status rei_set_grid_tuning(rei_instance* inst, uint64_t first_chunk, uint64_t chunk_max, uint32_t concat_wg,
                               uint32_t concat_xi) {
  if (!inst || concat_xi > 64) return REI_ERR_INVALID_ARG;
  inst->grid_set = GridTune{first_chunk, chunk_max, concat_wg, concat_xi};
  return REI_OK;
}

rei_status rei_tune_grid(rei_instance* const* insts, size_t n, void* hip_stream, uint64_t* params_out) {
  if (n == 0 || !insts) return REI_ERR_INVALID_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!insts[i]) return REI_ERR_INVALID_ARG;
  try {
    std::map<int, std::vector<rei_instance*>> by_w;
    for (size_t i = 0; i < n; ++i) by_w[insts[i]->st.W].push_back(insts[i]);
    if (params_out) std::fill(params_out, params_out + 24, 0ull);
    for (auto& kv : by_w) {
      std::vector<rei_instance*>& grp = kv.second;
      std::vector<GridTune> saved;
      for (rei_instance* in : grp) saved.push_back(in->grid_set);
      GridTune base;
      {
        std::lock_guard<std::mutex> lk(g_grid_mu);
        auto it = g_grid_tuned.find(kv.first);
        if (it != g_grid_tuned.end()) base = it->second;
      }
      rei_result res;
      rei_status r = REI_OK;
      // the group's rei_solve calls one after another, best of three
      auto time_group = [&](const GridTune& t, double* out) -> rei_status {
        for (rei_instance* in : grp) in->grid_set = t;
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
          const double t0 = now_s();
          for (rei_instance* in : grp) {
            in->err.clear();
            rei_status st = solve_impl(in, (hipStream_t)hip_stream, &res);
            if (st != REI_OK) return st;
          }
          best = std::min(best, now_s() - t0);
        }
        *out = best;
        return REI_OK;
      };
      double cur = 1e300;
      if ((r = time_group(base, &cur)) != REI_OK) {
        for (size_t k = 0; k < grp.size(); ++k) grp[k]->grid_set = saved[k];
        return r;
      }
      // one parameter at a time, each over a few values around the defaults
      const uint64_t firsts[] = {1ull << 14, 1ull << 15, 1ull << 16, 1ull << 17, 1ull << 18, 1ull << 19};
      const uint64_t maxes[] = {1ull << 20, 1ull << 22, 1ull << 24};
      const uint32_t wgs[] = {512, 1024, 2048, 4096, 8192};
      const uint32_t xis[] = {4, 8, 16, 32, 64};
      auto sweep = [&](const auto& values, auto set) -> rei_status {
        GridTune keep = base;
        for (auto v : values) {
          GridTune t = base;
          set(t, v);
          double tt = 1e300;
          rei_status st = time_group(t, &tt);
          if (st != REI_OK) return st;
          if (tt < cur) {
            cur = tt;
            keep = t;
          }
        }
        base = keep;
        return REI_OK;
      };
      if ((r = sweep(firsts, [](GridTune& t, uint64_t v) { t.first_chunk = v; })) == REI_OK &&
          (r = sweep(maxes, [](GridTune& t, uint64_t v) { t.chunk_max = v; })) == REI_OK &&
          (r = sweep(wgs, [](GridTune& t, uint32_t v) { t.concat_wg = v; })) == REI_OK)
        r = sweep(xis, [](GridTune& t, uint32_t v) { t.concat_xi = v; });
      for (size_t k = 0; k < grp.size(); ++k) grp[k]->grid_set = saved[k];
      if (r != REI_OK) return r;
      {
        std::lock_guard<std::mutex> lk(g_grid_mu);
        g_grid_tuned[kv.first] = base;
      }
      const int slot = __builtin_ctz((unsigned)kv.first);  // W = 1, 2, 4, ..., 32
      if (params_out && slot < 6) {
        params_out[4 * slot + 0] = base.first_chunk;
        params_out[4 * slot + 1] = base.chunk_max;
        params_out[4 * slot + 2] = base.concat_wg;
        params_out[4 * slot + 3] = base.concat_xi;
      }
    }
    return REI_OK;
  } catch (const std::bad_alloc&) {
    return REI_ERR_HOST_ALLOC;
  }
}

rei_status rei_tune_save(const char* path) {
  if (!path) return REI_ERR_INVALID_ARG;
  std::string js = "{\n  \"batch_threads\": [";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool first = true;
    for (auto& kv : g_tuned) {
      js += std::string(first ? "" : ",") + "\n    {\"group\": " + std::to_string(kv.first.first) +
            ", \"size_class\": " + std::to_string(kv.first.second) + ", \"threads\": " + std::to_string(kv.second) + "}";
      first = false;
    }
  }
  js += "\n  ],\n  \"batch_level_max\": [";
  {
    bool first = true;
    for (int g = 0; g <= kBatchMaxW; g = g ? 2 * g : 1) {
      const uint64_t v = g_level_max[width_slot(g)].load();
      if (!v) continue;
      js += std::string(first ? "" : ",") + "\n    {\"group\": " + std::to_string(g) +
            ", \"level_max\": " + std::to_string(v - 1) + "}";
      first = false;
    }
  }
  js += "\n  ],\n  \"grid\": [";
  {
    std::lock_guard<std::mutex> lk(g_grid_mu);
    bool first = true;
    for (auto& kv : g_grid_tuned) {
      const GridTune& t = kv.second;
      js += std::string(first ? "" : ",") + "\n    {\"words\": " + std::to_string(kv.first) +
            ", \"first_chunk\": " + std::to_string(t.first_chunk) + ", \"chunk_max\": " + std::to_string(t.chunk_max) +
            ", \"concat_wg\": " + std::to_string(t.concat_wg) + ", \"concat_xi\": " + std::to_string(t.concat_xi) + "}";
      first = false;
    }
  }
  js += "\n  ]\n}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return REI_ERR_INVALID_ARG;
  const bool ok = std::fwrite(js.data(), 1, js.size(), f) == js.size();
  return (std::fclose(f) == 0 && ok) ? REI_OK : REI_ERR_INVALID_ARG;
}

rei_status rei_tune_load(const char* path) {
  if (!path) return REI_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return REI_ERR_INVALID_ARG;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  try {
    return tune_parse(text) ? REI_OK : REI_ERR_INVALID_ARG;
  } catch (const std::bad_alloc&) {
    return REI_ERR_HOST_ALLOC;
  }
}

void rei_destroy(rei_instance* inst) {
  if (!inst) return;
  free_device(inst);
  delete inst;
}

const char* rei_status_str(rei_status s) {
  switch (s) {
    case REI_OK: return "REI_OK";
    case REI_NOT_FOUND: return "REI_NOT_FOUND";
    case REI_OUT_OF_MEMORY: return "REI_OUT_OF_MEMORY";
    case REI_ERR_INVALID_ARG: return "REI_ERR_INVALID_ARG";
    case REI_ERR_INCONSISTENT: return "REI_ERR_INCONSISTENT";
    case REI_ERR_BAD_CHAR: return "REI_ERR_BAD_CHAR";
    case REI_ERR_TOO_LARGE: return "REI_ERR_TOO_LARGE";
    case REI_ERR_DEVICE: return "REI_ERR_DEVICE";
    case REI_ERR_HOST_ALLOC: return "REI_ERR_HOST_ALLOC";
  }
  return "REI_UNKNOWN";
}

const char* rei_last_error(const rei_instance* inst) { return inst ? inst->err.c_str() : ""; }
const char* rei_create_error(void) { return g_create_error.c_str(); }

rei_status rei_ic_word(const rei_instance* inst, uint32_t i, char* buf, size_t cap) {
  if (!inst || !buf || i >= inst->st.n) return REI_ERR_INVALID_ARG;
  const std::string& w = inst->st.ic[i];
  if (w.size() + 1 > cap) return REI_ERR_INVALID_ARG;
  std::memcpy(buf, w.c_str(), w.size() + 1);
  return REI_OK;
}

rei_status rei_level_size(const rei_instance* inst, uint32_t cost, uint64_t* out) {
  if (!inst || !out) return REI_ERR_INVALID_ARG;
  *out = cost < inst->lcount.size() ? inst->lcount[cost] : 0;
  return REI_OK;
}

rei_status rei_row_bits(rei_instance* inst, uint32_t cost, uint64_t i, uint64_t* words_out) {
  if (!inst || !words_out || cost >= inst->lcount.size() || i >= inst->lcount[cost])
    return REI_ERR_INVALID_ARG;
  if (inst->rows_elsewhere) {
    inst->err = "the last search ran in the shared static array; its rows were not kept";
    return REI_ERR_INVALID_ARG;
  }
  const int W = inst->st.W;
  HIP_OK(inst, hipMemcpy(words_out, inst->d_rows + (inst->lstart[cost] + i) * W, W * 8,
                         hipMemcpyDeviceToHost));
  return REI_OK;
}

rei_status rei_row_regex(rei_instance* inst, uint32_t cost, uint64_t i, char* buf, size_t cap) {
  if (!inst || !buf || cost >= inst->lcount.size() || i >= inst->lcount[cost]) return REI_ERR_INVALID_ARG;
  if (inst->rows_elsewhere) {
    inst->err = "the last search ran in the shared static array; its rows were not kept";
    return REI_ERR_INVALID_ARG;
  }
  std::string s;
  int op;
  rei_status r = print_row(inst, inst->lstart[cost] + i, &s, &op);
  if (r != REI_OK) return r;
  if (s.size() + 1 > cap) return REI_ERR_INVALID_ARG;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return REI_OK;
}

rei_status rei_set_chunk(rei_instance* inst, uint64_t max_candidates) {
  if (!inst) return REI_ERR_INVALID_ARG;
  if (max_candidates == 0) max_candidates = kDefaultChunk;
  if (max_candidates > kMaxChunk) return REI_ERR_INVALID_ARG;
  inst->chunk_max = max_candidates;
  return REI_OK;
}

rei_status rei_set_batch_level(rei_instance* inst, uint64_t max_candidates) {
  if (!inst) return REI_ERR_INVALID_ARG;
  inst->batch_level_max = max_candidates;
  return REI_OK;
}

rei_status rei_set_batch_time(rei_instance* inst, int64_t microseconds) {
  if (!inst || microseconds < -1) return REI_ERR_INVALID_ARG;
  inst->batch_time_us = microseconds;
  return REI_OK;
}

rei_status rei_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return REI_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.free_ = free_;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return REI_OK;
}

rei_status rei_trim(rei_instance* inst) {
  if (!inst) return REI_ERR_INVALID_ARG;
  HIP_OK(inst, hipSetDevice(inst->device));
  HIP_OK(inst, hipDeviceSynchronize());
  free_search_buffers(inst);
  // no rows left to inspect (the result's counts live in uniq / cand)
  std::fill(inst->lstart.begin(), inst->lstart.end(), 0);
  std::fill(inst->lcount.begin(), inst->lcount.end(), 0);
  inst->tree.clear();
  return REI_OK;
}

rei_status rei_set_char_costs(rei_instance* inst, const uint32_t* costs, size_t n) {
  if (!inst || (n && !costs) || n != inst->st.sigma.size() || n == 0) return REI_ERR_INVALID_ARG;
  uint32_t lo = costs[0];
  for (size_t a = 0; a < n; ++a) {
    if (costs[a] < 1) return REI_ERR_INVALID_ARG;
    lo = std::min(lo, costs[a]);
  }
  inst->char_cost.assign(costs, costs + n);
  inst->costs.c_char = lo;
  for (uint32_t a = 0; a < inst->char_order.size(); ++a) inst->char_order[a] = a;
  std::stable_sort(inst->char_order.begin(), inst->char_order.end(),
                   [&](uint32_t x, uint32_t y) { return inst->char_cost[x] < inst->char_cost[y]; });
  std::vector<int32_t> idx(n);
  for (size_t i = 0; i < n; ++i) idx[i] = inst->st.char_index[inst->char_order[i]];
  HIP_OK(inst, hipSetDevice(inst->device));
  HIP_OK(inst, hipMemcpy(inst->d_char_index, idx.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  return REI_OK;
}

rei_status rei_set_on_the_fly(rei_instance* inst, int enable) {
  if (!inst) return REI_ERR_INVALID_ARG;
  inst->otf_on = enable != 0;
  return REI_OK;
}

rei_status rei_set_max_errors(rei_instance* inst, uint32_t max_errors) {
  if (!inst) return REI_ERR_INVALID_ARG;
  inst->max_err = max_errors;
  return REI_OK;
}

rei_status rei_set_profiling_class(rei_instance* inst, rei_kernel_class k) {
  if (!inst || (int)k < 0 || (int)k >= REI_K_COUNT) return REI_ERR_INVALID_ARG;
  for (int q = 0; q < REI_K_COUNT; ++q) {
    inst->st_launch[q] = 0;
    inst->st_ms[q] = 0;
    inst->st_units[q] = 0;
  }
  inst->prof = 3;
  inst->prof_class = (int)k;
  return REI_OK;
}

rei_status rei_set_profiling(rei_instance* inst, int enable) {
  if (!inst) return REI_ERR_INVALID_ARG;
  if (enable < 0 || enable > 2) return REI_ERR_INVALID_ARG;
  if (enable && !inst->prof)
    for (int k = 0; k < REI_K_COUNT; ++k) {
      inst->st_launch[k] = 0;
      inst->st_ms[k] = 0;
      inst->st_units[k] = 0;
    }
  inst->prof = enable;
  return REI_OK;
}

rei_status rei_set_hash_bits(uint32_t bits) {
  const uint64_t mask = (bits == 0 || bits >= 64) ? ~0ull : ((1ull << bits) - 1);
  if (set_hash_mask_kernels(mask) != hipSuccess || set_hash_mask_batch(mask) != hipSuccess) return REI_ERR_DEVICE;
  return REI_OK;
}

rei_status rei_timing_overhead(double* us) {
  if (!us) return REI_ERR_INVALID_ARG;
  *us = 0;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return REI_ERR_DEVICE;
  constexpr int kRuns = 64;
  std::vector<hipEvent_t> ev(2 * kRuns, nullptr);
  rei_status st = REI_OK;
  for (auto& e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) st = REI_ERR_DEVICE;
  for (int k = 0; st == REI_OK && k < kRuns; ++k) {
    g_kernel_timer = KernelTimer{ev[2 * k], ev[2 * k + 1]};
    if (launch_noop_timed(s) != hipSuccess) st = REI_ERR_DEVICE;
  }
  g_kernel_timer = KernelTimer{nullptr, nullptr};
  if (st == REI_OK && hipStreamSynchronize(s) != hipSuccess) st = REI_ERR_DEVICE;
  std::vector<float> ms;
  for (int k = 8; st == REI_OK && k < kRuns; ++k) {  // the first launches warm up
    float m = 0;
    if (hipEventElapsedTime(&m, ev[2 * k], ev[2 * k + 1]) != hipSuccess) st = REI_ERR_DEVICE;
    ms.push_back(m);
  }
  if (st == REI_OK) *us = 1e3 * *std::min_element(ms.begin(), ms.end());
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(s);
  return st;
}

rei_status rei_measure_peak(rei_peak_kind kind, uint64_t size, double* rate, double* seconds) {
  if (!rate || !seconds || (int)kind < 0 || (int)kind > (int)REI_PEAK_BITWISE) return REI_ERR_INVALID_ARG;
  if ((kind == REI_PEAK_COPY || kind == REI_PEAK_PROBE || kind == REI_PEAK_PROBE_ATOMIC) && size < 4096)
    return REI_ERR_INVALID_ARG;
  return measure_peak((int)kind, size, rate, seconds) == hipSuccess ? REI_OK : REI_ERR_DEVICE;
}

rei_status rei_kernel_stats(const rei_instance* inst, rei_kernel_class k, uint64_t* launches, double* ms,
                            uint64_t* units) {
  if (!inst || k < 0 || k >= REI_K_COUNT) return REI_ERR_INVALID_ARG;
  if (launches) *launches = inst->st_launch[k];
  if (ms) *ms = inst->st_ms[k];
  if (units) *units = inst->st_units[k];
  return REI_OK;
}

const char* rei_kernel_name(rei_kernel_class k) {
  switch (k) {
    case REI_K_GEN_CHAR: return "gen_char";
    case REI_K_GEN_QUESTION: return "gen_question";
    case REI_K_GEN_STAR: return "gen_star";
    case REI_K_GEN_CONCAT: return "gen_concat";
    case REI_K_GEN_UNION: return "gen_union";
    case REI_K_INSERT: return "insert_survivors";
    case REI_K_COMPACT: return "compact_winners";
    case REI_K_OTHER: return "other";
    case REI_K_BATCH: return "solve_batch";
    case REI_K_GEN_MIXED: return "gen_pieces";
    default: return "?";
  }
}

}  // extern "C"

// ---- serving: continuous batching -----------------------------------------
//
// Requests (staged instances) queue on submit.  A scheduler thread admits
// them in arrival order while their device bytes fit the budget (their
// arenas are allocated at admission), and hands instances that cannot be
// batched, or that outgrew their preallocated rows or reached a level too
// large for one workgroup, to worker threads that run the per-chunk path on
// their own streams.  Batchable requests reach the device one of two ways:
//  * queue mode (the default): per word-width group, a persistent launch of
//    the batched solver takes requests from a ring in pinned memory while it
//    runs; the scheduler writes each admitted request's descriptor into the
//    ring and publishes it, so a request arriving while others are on the
//    device starts as soon as a workgroup is free, with no launch.  A launch
//    ends when its workgroups have found no work for a while; the next
//    admission starts a new one.
//  * launch mode: each admitted group is one batched solve on a free stream
//    (groups that arrive while others run overlap on the device).
// Every result equals rei_solve's for that instance.

struct rei_server {
  uint64_t budget = 0;
  uint64_t in_use = 0;
  uint32_t max_batch = 64;
  uint64_t arena = kDefaultArena;
  int device = 0;
  struct Req {
    rei_instance* in = nullptr;
    uint64_t reserve = 0;
    double t_submit = 0, t_done = 0;
    bool begun = false;  // begin_solve ran (a batched launch took it): the grid path resumes it
    bool done = false;
    rei_status status = REI_OK;
    rei_result res{};
  };
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_grid;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;       // waiting for admission
  std::deque<uint64_t> grid_queue;  // admitted, per-chunk path
  uint64_t next_ticket = 1;
  bool stopping = false;
  struct Flight {
    BatchRun run;
    std::vector<uint64_t> tickets;
    int stream = -1;
    hipEvent_t ev = nullptr;
  };
  std::list<Flight> flights;
  std::vector<hipStream_t> streams;
  std::vector<bool> stream_busy;
  std::thread sched;
  std::vector<std::thread> workers;
  int busy_workers = 0;
  // queue mode: one ring and persistent launch per word-width group (slot
  // 0: one word with keys inline; slot 1 + log2 W otherwise)
  bool queue_mode = true;
  struct QGroup {
    BatchDesc* h_ring = nullptr;  // pinned, read by the launch
    BatchDesc* d_ring = nullptr;
    QueueCtl* h_ctl = nullptr;    // pinned control block
    QueueCtl* d_ctl = nullptr;
    uint32_t* d_next = nullptr;   // next slot to claim (device)
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;      // recorded after the launch
    bool running = false;
    uint32_t tail = 0;            // slots published to the current launch
    std::vector<uint64_t> slot;   // ticket of each published slot
    std::deque<uint64_t> pending; // admitted, not yet published
    uint32_t threads = 0, grid = 0;
  };
  QGroup qg[8];
  std::vector<uint64_t> published;  // tickets published, results not yet taken
  hipStream_t setup = nullptr;      // arena set-up at admission
  uint64_t idle_ticks = 0;
};

namespace {

void server_finish(rei_server* sv, uint64_t t, rei_status st) {
  // caller holds sv->mu
  auto& q = sv->reqs[t];
  q.status = st;
  q.res = q.in->res;
  q.t_done = now_s();
  q.res.seconds_solve = q.t_done - q.t_submit;
  q.done = true;
  sv->in_use -= q.reserve;
  sv->cv_done.notify_all();
  sv->cv_sched.notify_all();
}

void server_worker(rei_server* sv, hipStream_t s) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv_grid.wait(lk, [&] { return sv->stopping || !sv->grid_queue.empty(); });
    if (sv->grid_queue.empty()) {
      if (sv->stopping) return;
      continue;
    }
    const uint64_t t = sv->grid_queue.front();
    sv->grid_queue.pop_front();
    rei_instance* in = sv->reqs[t].in;
    const double t0 = sv->reqs[t].t_submit;
    const bool begun = sv->reqs[t].begun;
    sv->busy_workers++;
    lk.unlock();
    rei_status r = REI_OK;
    try {
      in->err.clear();
      // A request that never went through a batched launch starts here:
      // reset its result state (counts, expression, hand-off level, OnTheFly
      // state of an earlier solve) and answer the trivial specifications at
      // once, exactly as rei_solve does.  A hand-off or a restart from a
      // batched launch was begun there and continues.
      const bool trivial = !begun && begin_solve(in, t0);
      if (!trivial) {
        if (hipSetDevice(in->device) != hipSuccess) r = REI_ERR_DEVICE;
        if (r == REI_OK) r = search_levels(in, s);
        if (r == REI_OK) r = finish_solve(in, t0);
        if (r == REI_OK && hipStreamSynchronize(s) != hipSuccess) r = REI_ERR_DEVICE;
      }
    } catch (const std::bad_alloc&) {
      r = REI_ERR_HOST_ALLOC;
    }
    lk.lock();
    sv->busy_workers--;
    server_finish(sv, t, r);
  }
}

constexpr uint32_t kRing = 4096;  // ring slots per queue launch
// A queue launch's workgroups leave after this long without work, and a
// group's launch has one workgroup per kQueueCuShare compute units: idle
// workgroups hold their compute units, which the per-chunk kernels of
// handed-off requests need (a 2 ms idle time on a quarter of the device
// tripled the served p99 of the serving mix; 100-300 us on an eighth made
// it lower than one launch per admitted group).
constexpr uint32_t kQueueIdleUs = 150;
constexpr uint32_t kQueueCuShare = 8;

int queue_slot(const rei_instance* in) {
  if (in->inl) return 0;
  int k = 1;
  for (int w = in->st.W; w > 1; w >>= 1) ++k;
  return k;
}

// The ring, control block, counter, stream and event of a group, on first use.
rei_status queue_group_init(rei_server* sv, int slot, rei_instance* in) {
  rei_server::QGroup& q = sv->qg[slot];
  if (q.h_ring) return REI_OK;
  const unsigned fl = hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent;
  HIP_OK(in, hipHostMalloc((void**)&q.h_ring, kRing * sizeof(BatchDesc), fl));
  HIP_OK(in, hipHostGetDevicePointer((void**)&q.d_ring, q.h_ring, 0));
  HIP_OK(in, hipHostMalloc((void**)&q.h_ctl, sizeof(QueueCtl), fl));
  HIP_OK(in, hipHostGetDevicePointer((void**)&q.d_ctl, q.h_ctl, 0));
  q.h_ctl->tail = 0;
  q.h_ctl->closing = 0;
  q.h_ctl->idle_ticks = sv->idle_ticks;
  HIP_OK(in, hipMalloc((void**)&q.d_next, 64 * sizeof(uint32_t)));
  HIP_OK(in, hipStreamCreateWithFlags(&q.s, hipStreamNonBlocking));
  HIP_OK(in, hipEventCreateWithFlags(&q.ev, hipEventDisableTiming));
  // 512 threads per workgroup (256 for 32 words) on an eighth of the
  // compute units per group: a workgroup of the batched solver fills most of
  // a compute unit's registers, so the launches of several groups are
  // resident side by side, the per-chunk path of hand-offs finds room, and
  // one group busy with a stream of requests does not keep another group's
  // launch from starting for longer than its idle time
  const int g = slot == 0 ? 0 : 1 << (slot - 1);
  q.threads = std::min<uint32_t>(512, max_threads(g));
  q.grid = std::max<uint32_t>(1, device_cus(sv->device) / kQueueCuShare);
  return REI_OK;
}

// Starts a queue launch of group slot over the slots published so far.
rei_status queue_launch(rei_server* sv, int slot, rei_instance* in) {
  rei_server::QGroup& q = sv->qg[slot];
  const int g = slot == 0 ? 0 : 1 << (slot - 1);
  q.h_ctl->closing = 0;
  q.h_ctl->idle_ticks = sv->idle_ticks;
  HIP_OK(in, launch_reset_counters(q.d_next, 1, q.s));
  HIP_OK(in, launch_solve_batch(g ? g : 1, g == 0, q.threads, q.d_ring, kRing, q.s, nullptr, q.d_next, q.grid,
                                q.d_ctl));
  HIP_OK(in, hipEventRecord(q.ev, q.s));
  q.running = true;
  return REI_OK;
}

uint64_t request_reserve(const rei_server* sv, const rei_instance* in) {
  uint64_t b = batch_path(in) ? batch_reserve(in, sv->arena)
                             : in->cache_bytes + pow2_at_least(4 * (in->row_cap + 1)) * 8;
  return std::min(b, sv->budget);
}

// The descriptor of a served request: hand-off of large levels, and of
// mid-sized ones after the workgroup's time, as for rei_solve_batch (the
// per-chunk path runs beside the persistent launches, which hold a quarter
// of the compute units per group).
BatchDesc queue_desc(const rei_instance* in) { return make_desc(in); }

void server_sched_queue(rei_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool worked = false, any_running = false;
    // launches that ended: published slots still unsolved were never
    // claimed; they go back to the front of their group, in order
    for (int k = 0; k < 8; ++k) {
      rei_server::QGroup& q = sv->qg[k];
      if (!q.running) continue;
      if (hipEventQuery(q.ev) != hipSuccess) {
        any_running = true;
        continue;
      }
      q.running = false;
      std::vector<uint64_t> again;
      for (uint32_t i = 0; i < q.tail; ++i) {
        const uint64_t t = q.slot[i];
        auto it = std::find(sv->published.begin(), sv->published.end(), t);
        if (it == sv->published.end()) continue;  // result taken already
        if (__atomic_load_n(&sv->reqs[t].in->h_state->done, __ATOMIC_ACQUIRE)) continue;  // taken below
        sv->published.erase(it);
        again.push_back(t);
      }
      for (auto it = again.rbegin(); it != again.rend(); ++it) q.pending.push_front(*it);
      q.tail = 0;
      q.slot.clear();
      __atomic_store_n(&q.h_ctl->tail, 0u, __ATOMIC_RELEASE);
      worked = true;
    }
    // finished requests: results from their pinned buffers
    struct Fin {
      uint64_t t;
      rei_instance* in;
      double t0;
      bool more;
      rei_status r;
    };
    std::vector<Fin> fin;
    for (size_t i = 0; i < sv->published.size();) {
      const uint64_t t = sv->published[i];
      const auto& rq = sv->reqs[t];
      if (__atomic_load_n(&rq.in->h_state->done, __ATOMIC_ACQUIRE)) {
        fin.push_back({t, rq.in, rq.t_submit, false, REI_OK});
        sv->published.erase(sv->published.begin() + (long)i);
      } else {
        ++i;
      }
    }
    if (!fin.empty()) {
      lk.unlock();
      for (Fin& f : fin) {
        try {
          f.more = batch_take_state(f.in);
          if (!f.more) f.r = finish_solve(f.in, f.t0);
        } catch (const std::bad_alloc&) {
          f.r = REI_ERR_HOST_ALLOC;
        }
      }
      lk.lock();
      for (const Fin& f : fin) {
        if (f.more) {
          sv->reqs[f.t].begun = true;  // begun at admission: the per-chunk path continues it
          sv->grid_queue.push_back(f.t);
          sv->cv_grid.notify_one();
        } else {
          server_finish(sv, f.t, f.r);
        }
      }
      worked = true;
    }
    // admission in arrival order while the bytes fit; arenas allocated now
    struct Adm {
      uint64_t t;
      rei_instance* in;
      double t0;
      bool trivial;
      rei_status r;
    };
    std::vector<Adm> adm;
    while (!sv->queue.empty()) {
      const uint64_t t = sv->queue.front();
      auto& rq = sv->reqs[t];
      if (sv->in_use + rq.reserve > sv->budget) break;
      sv->in_use += rq.reserve;
      sv->queue.pop_front();
      if (batch_path(rq.in)) {
        adm.push_back({t, rq.in, rq.t_submit, false, REI_OK});
      } else {
        sv->grid_queue.push_back(t);
        sv->cv_grid.notify_one();
      }
    }
    if (!adm.empty()) {
      lk.unlock();
      bool setup_used = false;
      for (Adm& a : adm) {
        rei_instance* in = a.in;
        try {
          in->err.clear();
          if (begin_solve(in, a.t0)) {
            a.trivial = true;
            continue;
          }
          const uint64_t R = batch_rows(in, sv->arena);
          if ((a.r = ensure_chunk_buffers(in, kBatchChunk)) != REI_OK) continue;
          if ((a.r = ensure_rows(in, R, sv->setup)) != REI_OK) continue;
          if ((a.r = ensure_table(in, in->rows_alloc + kBatchChunk, sv->setup, false)) != REI_OK) continue;
          setup_used = true;
          __atomic_store_n(&in->h_state->done, 0u, __ATOMIC_RELEASE);
        } catch (const std::bad_alloc&) {
          a.r = REI_ERR_HOST_ALLOC;
        }
      }
      if (setup_used && hipStreamSynchronize(sv->setup) != hipSuccess)
        for (Adm& a : adm)
          if (a.r == REI_OK && !a.trivial) a.r = REI_ERR_DEVICE;
      lk.lock();
      for (const Adm& a : adm) {
        if (a.r != REI_OK || a.trivial) {
          server_finish(sv, a.t, a.r);
          continue;
        }
        const int k = queue_slot(a.in);
        rei_status r = queue_group_init(sv, k, a.in);
        if (r != REI_OK) {
          server_finish(sv, a.t, r);
          continue;
        }
        sv->qg[k].pending.push_back(a.t);
      }
      worked = true;
    }
    // publish pending requests into their group's ring; start a launch
    // where none runs; a full ring is closed and published again once its
    // launch has ended
    for (int k = 0; k < 8; ++k) {
      rei_server::QGroup& q = sv->qg[k];
      if (q.pending.empty()) continue;
      if (q.tail >= kRing) {
        if (q.running) __atomic_store_n(&q.h_ctl->closing, 1u, __ATOMIC_RELEASE);
        continue;
      }
      rei_instance* first = sv->reqs[q.pending.front()].in;
      const uint32_t before = q.tail;
      while (!q.pending.empty() && q.tail < kRing) {
        const uint64_t t = q.pending.front();
        q.pending.pop_front();
        q.h_ring[q.tail] = queue_desc(sv->reqs[t].in);
        q.slot.push_back(t);
        sv->published.push_back(t);
        ++q.tail;
      }
      std::atomic_thread_fence(std::memory_order_release);
      __atomic_store_n(&q.h_ctl->tail, q.tail, __ATOMIC_RELEASE);
      if (!q.running) {
        const rei_status r = queue_launch(sv, k, first);
        if (r != REI_OK) {
          // nothing of this launch runs: its slots fail
          for (uint32_t i = before; i < q.tail; ++i) {
            const uint64_t t = q.slot[i];
            sv->published.erase(std::find(sv->published.begin(), sv->published.end(), t));
            server_finish(sv, t, r);
          }
          q.tail = before;
          q.slot.resize(before);
          __atomic_store_n(&q.h_ctl->tail, q.tail, __ATOMIC_RELEASE);
          continue;
        }
      }
      any_running = true;
      worked = true;
    }
    bool idle = sv->queue.empty() && sv->published.empty();
    for (int k = 0; k < 8; ++k) idle = idle && sv->qg[k].pending.empty();
    if (sv->stopping && idle) {
      // no more work: end the launches still waiting for some
      for (int k = 0; k < 8; ++k)
        if (sv->qg[k].running) __atomic_store_n(&sv->qg[k].h_ctl->closing, 1u, __ATOMIC_RELEASE);
      bool any = false;
      for (int k = 0; k < 8; ++k) any = any || sv->qg[k].running;
      if (!any) return;
    }
    if (!worked) sv->cv_sched.wait_for(lk, std::chrono::microseconds(any_running || !sv->published.empty() ? 10 : 2000));
  }
}

void server_sched(rei_server* sv) {
  {
    // the mode is fixed once the first request is in
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_sched.wait(lk, [&] { return sv->stopping || !sv->queue.empty(); });
  }
  if (sv->queue_mode) {
    server_sched_queue(sv);
    return;
  }
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // finished groups
    for (auto it = sv->flights.begin(); it != sv->flights.end();) {
      if (hipEventQuery(it->ev) != hipSuccess) {
        ++it;
        continue;
      }
      rei_server::Flight f = std::move(*it);
      it = sv->flights.erase(it);
      lk.unlock();
      rei_status r = batch_collect(&f.run);
      lk.lock();
      (void)hipEventDestroy(f.ev);
      sv->stream_busy[f.stream] = false;
      std::unordered_map<rei_instance*, uint64_t> by_inst;
      for (uint64_t t : f.tickets) by_inst[sv->reqs[t].in] = t;
      if (r != REI_OK) {
        for (uint64_t t : f.tickets) server_finish(sv, t, r);
        continue;
      }
      for (rei_instance* in : f.run.finished) server_finish(sv, by_inst[in], REI_OK);
      for (rei_instance* in : f.run.grid) {
        sv->reqs[by_inst[in]].begun = true;  // batch_launch began it
        sv->grid_queue.push_back(by_inst[in]);
        sv->cv_grid.notify_one();
      }
    }
    // admission in arrival order, while the bytes fit and a stream is free
    int free_stream = -1;
    for (size_t k = 0; k < sv->streams.size(); ++k)
      if (!sv->stream_busy[k]) free_stream = (int)k;
    std::vector<uint64_t> take;
    while (!sv->queue.empty()) {
      const uint64_t t = sv->queue.front();
      auto& q = sv->reqs[t];
      if (sv->in_use + q.reserve > sv->budget) break;
      if (batch_path(q.in)) {
        if (free_stream < 0 || take.size() >= sv->max_batch) break;
        take.push_back(t);
      } else {
        sv->grid_queue.push_back(t);
        sv->cv_grid.notify_one();
      }
      sv->in_use += q.reserve;
      sv->queue.pop_front();
    }
    if (!take.empty()) {
      sv->flights.emplace_back();
      rei_server::Flight& f = sv->flights.back();
      f.tickets = take;
      f.stream = free_stream;
      sv->stream_busy[free_stream] = true;
      std::vector<rei_instance*> ins;
      for (uint64_t t : take) ins.push_back(sv->reqs[t].in);
      hipStream_t s = sv->streams[free_stream];
      lk.unlock();
      rei_status r = batch_launch(ins.data(), ins.size(), s, sv->arena, &f.run);
      hipError_t e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(f.ev, s);
      lk.lock();
      if (r != REI_OK || e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        batch_release(&f.run);
        if (f.ev) (void)hipEventDestroy(f.ev);
        sv->stream_busy[free_stream] = false;
        for (uint64_t t : take) server_finish(sv, t, r != REI_OK ? r : REI_ERR_DEVICE);
        sv->flights.pop_back();
      }
      continue;  // look again at once: more may be admissible
    }
    if (sv->stopping && sv->queue.empty() && sv->flights.empty()) return;
    // wait for an arrival, a freed budget, or poll running groups
    sv->cv_sched.wait_for(lk, std::chrono::microseconds(sv->flights.empty() ? 2000 : 20));
  }
}

}  // namespace

extern "C" {

rei_status rei_server_create(uint64_t hbm_budget, uint32_t max_batch, uint32_t n_streams,
                             uint32_t n_workers, rei_server** out) {
  if (!out) return REI_ERR_INVALID_ARG;
  *out = nullptr;
  rei_server* sv = new (std::nothrow) rei_server();
  if (!sv) return REI_ERR_HOST_ALLOC;
  sv->max_batch = max_batch ? max_batch : 64;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return REI_ERR_DEVICE;
  }
  if (hbm_budget == 0) {
    // the device's free memory now, less a reserve for everything else
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete sv;
      return REI_ERR_DEVICE;
    }
    const uint64_t reserve = 8ull << 30;
    hbm_budget = free_b > 2 * reserve ? free_b - reserve : free_b / 2;
  }
  sv->budget = hbm_budget;
  sv->idle_ticks = (uint64_t)kQueueIdleUs * wall_ticks_per_us(sv->device);
  if (hipStreamCreateWithFlags(&sv->setup, hipStreamNonBlocking) != hipSuccess) {
    delete sv;
    return REI_ERR_DEVICE;
  }
  const uint32_t ns = n_streams ? n_streams : 4;
  for (uint32_t k = 0; k < ns; ++k) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto q : sv->streams) (void)hipStreamDestroy(q);
      delete sv;
      return REI_ERR_DEVICE;
    }
    sv->streams.push_back(s);
    sv->stream_busy.push_back(false);
  }
  const uint32_t nw = n_workers ? n_workers : 4;
  for (uint32_t k = 0; k < nw; ++k) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
    sv->streams.push_back(s);  // owned here, destroyed with the others
    sv->stream_busy.push_back(true);  // never used for batches
    sv->workers.emplace_back(server_worker, sv, s);
  }
  sv->sched = std::thread(server_sched, sv);
  *out = sv;
  return REI_OK;
}

rei_status rei_server_submit(rei_server* sv, rei_instance* inst, uint64_t* ticket) {
  if (!sv || !inst || !ticket) return REI_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->stopping) return REI_ERR_INVALID_ARG;
  const uint64_t t = sv->next_ticket++;
  rei_server::Req q;
  q.in = inst;
  q.t_submit = now_s();
  q.reserve = request_reserve(sv, inst);
  sv->reqs[t] = q;
  sv->queue.push_back(t);
  sv->cv_sched.notify_all();
  *ticket = t;
  return REI_OK;
}

rei_status rei_server_poll(rei_server* sv, uint64_t ticket, int wait, int* done, rei_result* out,
                           double* latency_s) {
  if (!sv || !done) return REI_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->reqs.find(ticket) == sv->reqs.end()) return REI_ERR_INVALID_ARG;
  // submits during the wait may rehash the map: look the ticket up afresh
  if (wait)
    sv->cv_done.wait(lk, [&] {
      auto i = sv->reqs.find(ticket);
      return i == sv->reqs.end() || i->second.done;
    });
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return REI_ERR_INVALID_ARG;  // retired by a concurrent poll
  *done = it->second.done ? 1 : 0;
  if (!*done) return REI_OK;
  if (out) *out = it->second.res;
  if (latency_s) *latency_s = it->second.t_done - it->second.t_submit;
  const rei_status st = it->second.status;
  sv->reqs.erase(it);
  return st;
}

void rei_server_destroy(rei_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stopping = true;
    sv->cv_sched.notify_all();
    sv->cv_grid.notify_all();
  }
  if (sv->sched.joinable()) sv->sched.join();
  {
    // the scheduler has drained the queue; let the workers finish theirs
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->grid_queue.empty() && sv->busy_workers == 0; });
    sv->cv_grid.notify_all();
  }
  for (auto& w : sv->workers)
    if (w.joinable()) w.join();
  for (auto& q : sv->qg) {
    if (q.s) (void)hipStreamSynchronize(q.s);
    if (q.ev) (void)hipEventDestroy(q.ev);
    if (q.s) (void)hipStreamDestroy(q.s);
    if (q.d_next) (void)hipFree(q.d_next);
    if (q.h_ctl) (void)hipHostFree(q.h_ctl);
    if (q.h_ring) (void)hipHostFree(q.h_ring);
  }
  if (sv->setup) (void)hipStreamDestroy(sv->setup);
  for (auto s : sv->streams) (void)hipStreamDestroy(s);
  delete sv;
}

rei_status rei_server_set_queue_mode(rei_server* sv, int enable) {
  if (!sv) return REI_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->next_ticket != 1) return REI_ERR_INVALID_ARG;  // fixed once a request was submitted
  sv->queue_mode = enable != 0;
  return REI_OK;
}

}  // extern "C"

// ---- the batched solver as one captured graph --------------------------------
//
// rei_batch_graph_create prepares every batchable instance once (arena,
// descriptor), runs the persistent launches eagerly to measure each
// instance's work, orders each word-width group longest first and splits
// the device's resident workgroups between the groups by their work, then
// captures the step (counter reset, one persistent launch per group on
// forked streams, join) as one hipGraph.  A replay is one graph launch; the
// host then only reads each instance's results from its pinned buffers.

struct rei_batch_graph {
  int device = 0;
  std::vector<rei_instance*> insts;   // caller's order
  std::vector<rei_instance*> batched; // in descriptor order (groups concatenated)
  std::vector<rei_instance*> other;   // not batchable, or too heavy for one workgroup: rei_solve's
                                      // path on the worker threads, beside each replay
  struct Group {
    int g = 0;            // 0 = one word with keys inline, else W
    uint32_t off = 0, n = 0, threads = 0, grid = 0;
  };
  std::vector<Group> groups;
  BatchDesc* h_desc = nullptr;  // pinned, read by the kernels
  BatchDesc* d_desc = nullptr;
  uint32_t* d_order = nullptr;  // per group: item -> descriptor index within the group
  uint32_t* d_next = nullptr;   // per group: work counter
  hipStream_t cap = nullptr;    // capture stream (owned)
  std::vector<hipStream_t> sides;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t launched_on = nullptr;
  uint64_t arena = 0;
  bool in_flight = false;
  double t0 = 0;
  std::unique_ptr<GridPool> pool;     // the replay's instances on the worker threads
  std::string err;
};

namespace {

void graph_free(rei_batch_graph* g) {
  if (g->pool) (void)g->pool->join();
  g->pool.reset();
  if (g->in_flight && g->launched_on) (void)hipStreamSynchronize(g->launched_on);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (auto e : g->joins) (void)hipEventDestroy(e);
  if (g->fork) (void)hipEventDestroy(g->fork);
  for (auto s : g->sides) (void)hipStreamDestroy(s);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->d_order) (void)hipFree(g->d_order);
  if (g->d_next) (void)hipFree(g->d_next);
  if (g->h_desc) (void)hipHostFree(g->h_desc);
  delete g;
}

#define G_OK(g, call)                                                    \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      (g)->err = std::string(#call) + ": " + hipGetErrorString(e_);      \
      return REI_ERR_DEVICE;                                             \
    }                                                                    \
  } while (0)

// Enqueues the persistent launches of every group on g->cap and the side
// streams (eagerly, or into a capture).
rei_status graph_enqueue(rei_batch_graph* g) {
  G_OK(g, launch_reset_counters(g->d_next, (uint32_t)g->groups.size(), g->cap));
  G_OK(g, hipEventRecord(g->fork, g->cap));
  for (size_t k = 0; k < g->groups.size(); ++k) {
    const auto& q = g->groups[k];
    hipStream_t s = k ? g->sides[k - 1] : g->cap;
    if (k) G_OK(g, hipStreamWaitEvent(s, g->fork, 0));
    G_OK(g, launch_solve_batch(q.g ? q.g : 1, q.g == 0, q.threads, g->d_desc + q.off, q.n, s, g->d_order + q.off,
                               g->d_next + k, q.grid));
    if (k) {
      G_OK(g, hipEventRecord(g->joins[k - 1], s));
      G_OK(g, hipStreamWaitEvent(g->cap, g->joins[k - 1], 0));
    }
  }
  return REI_OK;
}

// The descriptor of a graph's instance, as every replay reads it: the whole
// search stays in the launch (no hand-off on size or time).
BatchDesc graph_desc(const rei_instance* in) {
  BatchDesc d = make_desc(in);
  d.level_max = ~0ull;
  d.time_ticks = 0;
  return d;
}

// Arena of a graph's instance: rows, chunk buffers, and a table that holds
// every row plus a chunk at load at most 1/2.
rei_status graph_arena(rei_instance* in, uint64_t arena_bytes, hipStream_t s) {
  rei_status r;
  const uint64_t R = batch_rows(in, arena_bytes);
  if ((r = ensure_chunk_buffers(in, kBatchChunk)) != REI_OK) return r;
  if ((r = ensure_rows(in, R, s)) != REI_OK) return r;
  return ensure_table(in, in->rows_alloc + kBatchChunk, s, false);
}

// Results of one run of the launches (they have finished): every batched
// instance's state from its pinned buffers.  Instances that ran out of
// their preallocated rows, and those that are not batchable, run
// rei_solve's path on the worker threads; the former then get an arena that
// holds their rows, and their descriptors follow the buffers they now have,
// so the next replay reads no freed memory.
rei_status graph_collect(rei_batch_graph* g, hipStream_t s) {
  rei_status r;
  GridPool& pool = *g->pool;  // holds the other instances since the launch
  std::vector<size_t> refresh;
  for (size_t i = 0; i < g->batched.size(); ++i) {
    rei_instance* in = g->batched[i];
    in->err.clear();
    const double seen = in->t_seen;
    (void)begin_solve(in, g->t0);  // batchable instances are never trivial
    if (batch_take_state(in)) {
      in->resume_level = 0;  // a fresh search: the arena was not enough
      refresh.push_back(i);
      pool.submit(in);
      continue;
    }
    if ((r = finish_solve(in, g->t0)) != REI_OK) {
      (void)pool.join();
      return r;
    }
    if (seen >= 0) in->res.seconds_solve = seen;
    in->t_seen = -1;
  }
  r = pool.join();
  g->pool.reset();
  if (r != REI_OK) return r;
  for (size_t i : refresh) {
    rei_instance* in = g->batched[i];
    if ((r = graph_arena(in, g->arena, s)) != REI_OK) return r;
    HIP_OK(in, hipStreamSynchronize(s));
    g->h_desc[i] = graph_desc(in);
  }
  return REI_OK;
}

}  // namespace

extern "C" {

rei_status rei_batch_graph_create(rei_instance* const* insts, size_t n, uint64_t arena_bytes,
                                  rei_batch_graph** out) {
  if (!out || (n && !insts)) return REI_ERR_INVALID_ARG;
  *out = nullptr;
  for (size_t i = 0; i < n; ++i)
    if (!insts[i]) return REI_ERR_INVALID_ARG;
  if (arena_bytes == 0) arena_bytes = kDefaultArena;
  rei_batch_graph* g = new (std::nothrow) rei_batch_graph();
  if (!g) return REI_ERR_HOST_ALLOC;
  rei_status r = REI_OK;
  try {
    G_OK(g, hipGetDevice(&g->device));
    G_OK(g, hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    g->insts.assign(insts, insts + n);
    std::vector<BatchDesc> descs;
    const double t0 = now_s();
    std::vector<rei_instance*> members[kBatchMaxW + 1];
    for (rei_instance* in : g->insts) {
      if (in->device != g->device) {
        g->err = "instances of one graph must live on the current device";
        graph_free(g);
        return REI_ERR_INVALID_ARG;
      }
      if (begin_solve(in, t0)) continue;  // trivial: answered at results time
      if (!batch_path(in)) {
        g->other.push_back(in);
        continue;
      }
      members[in->inl ? 0 : in->st.W].push_back(in);
    }
    // arenas (device memory is taken here, not at replay)
    g->arena = arena_bytes;
    for (int w = 0; w <= kBatchMaxW; w = w ? 2 * w : 1)
      for (rei_instance* in : members[w])
        if ((r = graph_arena(in, arena_bytes, g->cap)) != REI_OK) {
          g->err = in->err;
          graph_free(g);
          return r;
        }
    G_OK(g, hipStreamSynchronize(g->cap));
    auto regroup = [&] {
      descs.clear();
      g->groups.clear();
      g->batched.clear();
      for (int w = 0; w <= kBatchMaxW; w = w ? 2 * w : 1) {
        if (members[w].empty()) continue;
        rei_batch_graph::Group q;
        q.g = w;
        q.off = (uint32_t)descs.size();
        q.n = (uint32_t)members[w].size();
        q.threads = choose_threads(w, members[w].size());
        for (rei_instance* in : members[w]) {
          descs.push_back(graph_desc(in));  // no hand-off: the whole search stays in the graph
          g->batched.push_back(in);
        }
        g->groups.push_back(q);
      }
    };
    regroup();
    const size_t nd = std::max<size_t>(1, descs.size());
    G_OK(g, hipHostMalloc((void**)&g->h_desc, nd * sizeof(BatchDesc), hipHostMallocMapped | hipHostMallocPortable));
    G_OK(g, hipHostGetDevicePointer((void**)&g->d_desc, g->h_desc, 0));
    if (!descs.empty()) std::memcpy(g->h_desc, descs.data(), descs.size() * sizeof(BatchDesc));
    G_OK(g, hipMalloc((void**)&g->d_order, nd * sizeof(uint32_t)));
    G_OK(g, hipMalloc((void**)&g->d_next, 64 * sizeof(uint32_t)));
    G_OK(g, hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
    for (size_t k = 1; k < g->groups.size(); ++k) {
      hipStream_t s;
      hipEvent_t e;
      G_OK(g, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      g->sides.push_back(s);
      G_OK(g, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      g->joins.push_back(e);
    }
    if (g->groups.empty()) {
      *out = g;
      return REI_OK;
    }
    // a measuring run: every group in index order on a grid of its size
    std::vector<uint32_t> order(descs.size());
    for (const auto& q : g->groups)
      for (uint32_t i = 0; i < q.n; ++i) order[q.off + i] = i;
    G_OK(g, hipMemcpy(g->d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice));
    const uint32_t cus = device_cus(g->device);
    std::vector<uint32_t> per_cu(g->groups.size(), 1);
    for (size_t k = 0; k < g->groups.size(); ++k) {
      auto& q = g->groups[k];
      G_OK(g, batch_resident(q.g ? q.g : 1, q.g == 0, q.threads, &per_cu[k]));
      q.grid = std::min<uint32_t>(q.n, per_cu[k] * cus);
    }
    for (rei_instance* in : g->batched) __atomic_store_n(&in->h_state->done, 0u, __ATOMIC_RELEASE);
    if ((r = graph_enqueue(g)) != REI_OK) {
      graph_free(g);
      return r;
    }
    G_OK(g, hipStreamSynchronize(g->cap));
    // work of each instance: its candidates (all levels), and its largest level
    std::map<const rei_instance*, double> work_of;
    std::map<const rei_instance*, uint64_t> widest_of;
    double all_work = 0, resident = 0;
    for (size_t k = 0; k < g->groups.size(); ++k) {
      const auto& q = g->groups[k];
      resident += (double)per_cu[k] * cus;
      for (uint32_t i = 0; i < q.n; ++i) {
        rei_instance* in = g->batched[q.off + i];
        const uint64_t L = in->max_cost + 2;
        double c = 0;
        uint64_t widest = 0;
        for (uint64_t l = 0; l < L; ++l) {
          c += (double)in->h_levels[2 * L + l];
          widest = std::max(widest, in->h_levels[2 * L + l]);
        }
        // a candidate of a wider language costs more (W words per operation)
        const double w = c * (1.0 + 0.25 * std::max(1, in->st.W)) + 1000.0;
        work_of[in] = w;
        widest_of[in] = widest;
        all_work += w;
      }
    }
    // An instance with more than twice a resident workgroup's fair share of
    // the work would decide the replay's length alone, and one with a level
    // larger than rei_solve_batch's hand-off size is, there, solved from that
    // level by the whole device: either leaves the graph and runs
    // rei_solve's path on the worker threads while each replay runs.
    const double heavy = 2.0 * all_work / std::max(1.0, resident);
    bool moved = false;
    for (int w = 0; w <= kBatchMaxW; w = w ? 2 * w : 1) {
      auto& m = members[w];
      for (auto it = m.begin(); it != m.end();) {
        if ((work_of[*it] > heavy && work_of[*it] > kGraphHeavyMin) || widest_of[*it] > level_max_of(*it)) {
          g->other.push_back(*it);
          it = m.erase(it);
          moved = true;
        } else {
          ++it;
        }
      }
    }
    if (moved) {
      regroup();
      if (!descs.empty()) std::memcpy(g->h_desc, descs.data(), descs.size() * sizeof(BatchDesc));
      order.assign(descs.size(), 0);
      for (const auto& q : g->groups)
        for (uint32_t i = 0; i < q.n; ++i) order[q.off + i] = i;
      for (size_t k = 0; k < g->groups.size(); ++k) {
        auto& q = g->groups[k];
        G_OK(g, batch_resident(q.g ? q.g : 1, q.g == 0, q.threads, &per_cu[k]));
      }
    }
    // longest first within each group
    std::vector<double> work(descs.size(), 0);
    double total = 0;
    std::vector<double> gwork(g->groups.size(), 0);
    for (size_t k = 0; k < g->groups.size(); ++k) {
      const auto& q = g->groups[k];
      for (uint32_t i = 0; i < q.n; ++i) {
        work[q.off + i] = work_of[g->batched[q.off + i]];
        gwork[k] += work[q.off + i];
      }
      total += gwork[k];
      std::stable_sort(order.begin() + q.off, order.begin() + q.off + q.n,
                       [&](uint32_t a, uint32_t b) { return work[q.off + a] > work[q.off + b]; });
    }
    G_OK(g, hipMemcpy(g->d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice));
    // resident workgroups shared between the groups in proportion to their work
    for (size_t k = 0; k < g->groups.size(); ++k) {
      auto& q = g->groups[k];
      const double share = total > 0 ? gwork[k] / total : 1.0 / g->groups.size();
      const uint32_t want = (uint32_t)std::llround(share * per_cu[k] * cus);
      q.grid = std::max<uint32_t>(1, std::min<uint32_t>(q.n, want));
    }
    if (g->groups.empty()) {  // every batchable instance was too heavy: nothing to capture
      *out = g;
      return REI_OK;
    }
    G_OK(g, hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    r = graph_enqueue(g);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
    g->graph = graph;
    if (r != REI_OK) {
      graph_free(g);
      return r;
    }
    G_OK(g, ec);
    G_OK(g, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  } catch (const std::bad_alloc&) {
    graph_free(g);
    return REI_ERR_HOST_ALLOC;
  }
  *out = g;
  return REI_OK;
}

rei_status rei_batch_graph_launch(rei_batch_graph* g, void* hip_stream) {
  if (!g) return REI_ERR_INVALID_ARG;
  if (g->in_flight) {
    g->err = "the previous launch's results were not collected";
    return REI_ERR_INVALID_ARG;
  }
  G_OK(g, hipSetDevice(g->device));
  for (rei_instance* in : g->batched) {
    __atomic_store_n(&in->h_state->done, 0u, __ATOMIC_RELEASE);
    in->t_seen = -1;
  }
  g->t0 = now_s();
  g->launched_on = (hipStream_t)hip_stream;
  if (g->exec) G_OK(g, hipGraphLaunch(g->exec, g->launched_on));
  g->in_flight = true;
  // the instances outside the graph start now, beside the replay
  g->pool.reset(new GridPool(g->t0));
  for (rei_instance* in : g->other) {
    in->err.clear();
    if (!begin_solve(in, g->t0)) g->pool->submit(in);
  }
  return REI_OK;
}

rei_status rei_batch_graph_results(rei_batch_graph* g, rei_result* out) {
  if (!g || (!out && !g->insts.empty())) return REI_ERR_INVALID_ARG;
  if (!g->in_flight) {
    g->err = "no launch to collect";
    return REI_ERR_INVALID_ARG;
  }
  rei_status r = REI_OK;
  try {
    G_OK(g, hipSetDevice(g->device));
    // read completion flags while the launches run: the time each result
    // was known
    size_t left = g->batched.size();
    std::vector<char> seen(g->batched.size(), 0);
    while (left) {
      bool progress = false;
      for (size_t i = 0; i < g->batched.size(); ++i) {
        if (seen[i] || !__atomic_load_n(&g->batched[i]->h_state->done, __ATOMIC_ACQUIRE)) continue;
        seen[i] = 1;
        g->batched[i]->t_seen = now_s() - g->t0;
        --left;
        progress = true;
      }
      if (!left) break;
      if (!progress) {
        const hipError_t q = hipStreamQuery(g->launched_on);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) G_OK(g, q);
        std::this_thread::yield();
      }
    }
    G_OK(g, hipStreamSynchronize(g->launched_on));
    g->in_flight = false;
    r = graph_collect(g, g->launched_on);
    if (r != REI_OK) {
      for (rei_instance* in : g->insts)
        if (!in->err.empty()) {
          g->err = in->err;
          break;
        }
      return r;
    }
    for (size_t i = 0; i < g->insts.size(); ++i) {
      rei_instance* in = g->insts[i];
      out[i] = in->res;
    }
  } catch (const std::bad_alloc&) {
    return REI_ERR_HOST_ALLOC;
  }
  return REI_OK;
}

const char* rei_batch_graph_error(const rei_batch_graph* g) { return g ? g->err.c_str() : ""; }

size_t rei_batch_graph_outside(const rei_batch_graph* g) { return g ? g->other.size() : 0; }

void rei_batch_graph_destroy(rei_batch_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  graph_free(g);
}

}  // extern "C"
