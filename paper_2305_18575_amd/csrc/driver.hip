// Host driver of the REI search (Algorithm 1): the cost-level loop, the
// constructor blocks of each level, chunking, device memory, reconstruction
// of the answer from the per-row back-pointers, and the C ABI.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace rei;

namespace {

thread_local std::string g_create_error;

constexpr uint64_t kDefaultChunk = 1ull << 24;

struct Block {
  int op;
  uint32_t L, R;     // operand levels (costs)
  uint64_t count;    // candidates
  bool same;         // union of a level with itself (pairs x before y)
};

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
  int device = 0;
  double seconds_stage = 0;

  // staged tables on the device
  uint32_t* d_gt_off = nullptr;
  uint32_t* d_gt_pair = nullptr;
  uint32_t* d_len_off = nullptr;
  uint64_t* d_pmask = nullptr;
  uint64_t* d_nmask = nullptr;
  int32_t* d_char_index = nullptr;

  // language cache
  uint64_t* d_rows = nullptr;
  uint64_t* d_aux = nullptr;
  uint64_t rows_alloc = 0;
  // dedup table
  uint64_t* d_slots = nullptr;
  uint64_t slots_cap = 0;
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

  // rows known stored at the last synchronisation, candidates enqueued since
  uint64_t known_rows = 0;
  uint64_t pending = 0;

  // levels, indexed by cost
  std::vector<uint64_t> lstart, lcount;

  // result
  std::vector<uint64_t> uniq, cand;
  std::string regex;
  rei_result res{};
  std::string err;

  // profiling
  bool prof = false;
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

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

rei_status prof_begin(rei_instance* in, hipStream_t s, hipEvent_t* ev) {
  if (!in->prof) return REI_OK;
  if (in->pool.empty()) {
    hipEvent_t e;
    HIP_OK(in, hipEventCreate(&e));
    in->pool.push_back(e);
  }
  *ev = in->pool.back();
  in->pool.pop_back();
  HIP_OK(in, hipEventRecord(*ev, s));
  return REI_OK;
}

rei_status prof_end(rei_instance* in, hipStream_t s, int k, hipEvent_t a, uint64_t units) {
  if (!in->prof) return REI_OK;
  hipEvent_t b;
  if (in->pool.empty()) {
    HIP_OK(in, hipEventCreate(&b));
  } else {
    b = in->pool.back();
    in->pool.pop_back();
  }
  HIP_OK(in, hipEventRecord(b, s));
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
    hipEvent_t ev_ = nullptr;                             \
    rei_status ps_ = prof_begin(in, s, &ev_);             \
    if (ps_ != REI_OK) return ps_;                        \
    HIP_OK(in, call);                                     \
    ps_ = prof_end(in, s, k, ev_, units);                 \
    if (ps_ != REI_OK) return ps_;                        \
  } while (0)

rei_status ensure_rows(rei_instance* in, uint64_t need, hipStream_t s) {
  if (need <= in->rows_alloc) return REI_OK;
  uint64_t cap = std::max<uint64_t>({need, 2 * in->rows_alloc, 1024});
  const int W = in->st.W;
  uint64_t* nr = nullptr;
  uint64_t* na = nullptr;
  HIP_OK(in, hipMalloc(&nr, cap * W * 8));
  if (hipMalloc(&na, cap * 8) != hipSuccess) {
    (void)hipFree(nr);
    in->err = "hipMalloc of the back-pointer array failed";
    return REI_ERR_DEVICE;
  }
  if (in->known_rows) {
    HIP_OK(in, hipMemcpyAsync(nr, in->d_rows, in->known_rows * W * 8, hipMemcpyDeviceToDevice, s));
    HIP_OK(in, hipMemcpyAsync(na, in->d_aux, in->known_rows * 8, hipMemcpyDeviceToDevice, s));
  }
  HIP_OK(in, hipStreamSynchronize(s));
  dfree(in->d_rows);
  dfree(in->d_aux);
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
    dfree(in->d_slots);
    HIP_OK(in, hipMalloc(&in->d_slots, cap * 8));
    in->slots_cap = cap;
  }
  LAUNCH(in, s, REI_K_OTHER, cap, launch_fill(in->d_slots, cap, kEmpty, s));
  LAUNCH(in, s, REI_K_OTHER, in->known_rows,
         launch_rehash(in->st.W, in->d_rows, in->known_rows, in->d_slots, cap - 1, s));
  return REI_OK;
}

rei_status ensure_chunk_buffers(rei_instance* in, uint64_t len) {
  const int W = in->st.W;
  if (len > in->surv_cap) {
    dfree(in->d_skey);
    dfree(in->d_se);
    dfree(in->d_spos);
    HIP_OK(in, hipMalloc(&in->d_skey, len * W * 8));
    HIP_OK(in, hipMalloc(&in->d_se, len * 4));
    HIP_OK(in, hipMalloc(&in->d_spos, len * 8));
    in->surv_cap = len;
  }
  const uint64_t words = (len + 31) / 32;
  if (words > in->bitmap_cap) {
    dfree(in->d_bitmap);
    dfree(in->d_prefix);
    dfree(in->d_bsums);
    HIP_OK(in, hipMalloc(&in->d_bitmap, words * 4));
    HIP_OK(in, hipMalloc(&in->d_prefix, words * 4));
    HIP_OK(in, hipMalloc(&in->d_bsums, ((words + 1023) / 1024 + 1) * 4));
    in->bitmap_cap = words;
  }
  return REI_OK;
}

uint64_t level_n(const rei_instance* in, int64_t c) {
  if (c < (int64_t)in->costs.c_char || c >= (int64_t)in->lcount.size()) return 0;
  return in->lcount[c];
}

bool mul_ok(uint64_t a, uint64_t b, uint64_t* out) { return !__builtin_mul_overflow(a, b, out); }

// Constructor blocks of level c in enumeration order.
bool make_blocks(const rei_instance* in, uint32_t c, std::vector<Block>* out) {
  out->clear();
  const rei_costs& k = in->costs;
  if (c == k.c_char) {
    out->push_back({OP_CHAR, 0, 0, (uint64_t)in->st.sigma.size(), false});
    return true;
  }
  const int64_t cc = c;
  if (level_n(in, cc - k.c_question))
    out->push_back({OP_QUESTION, (uint32_t)(cc - k.c_question), 0, level_n(in, cc - k.c_question), false});
  if (level_n(in, cc - k.c_star))
    out->push_back({OP_STAR, (uint32_t)(cc - k.c_star), 0, level_n(in, cc - k.c_star), false});
  for (int64_t L = k.c_char; cc - (int64_t)k.c_concat - L >= (int64_t)k.c_char; ++L) {
    const int64_t R = cc - k.c_concat - L;
    uint64_t n;
    if (!mul_ok(level_n(in, L), level_n(in, R), &n)) return false;
    if (n) out->push_back({OP_CONCAT, (uint32_t)L, (uint32_t)R, n, false});
  }
  for (int64_t L = k.c_char; L <= cc - (int64_t)k.c_union - L; ++L) {
    const int64_t R = cc - k.c_union - L;
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

// Waits for the stream and reads the device search state.
rei_status sync_state(rei_instance* in, hipStream_t s) {
  const uint64_t L = in->max_cost + 2;
  HIP_OK(in, hipMemcpyAsync(in->h_state, in->d_state, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_OK(in, hipMemcpyAsync(in->h_levels, in->d_levels, 3 * L * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(in, hipStreamSynchronize(s));
  in->known_rows = in->h_state->total_rows;
  in->pending = 0;
  return REI_OK;
}

// Enqueues one chunk (no host synchronisation unless a buffer may have to
// grow: then the stream is drained first and the buffer grown for the worst
// case of this chunk).
rei_status enqueue_chunk(rei_instance* in, hipStream_t s, uint32_t c, const Block& b, uint64_t e_base,
                         uint64_t e0, uint64_t e1, bool* stopped) {
  const int W = in->st.W;
  const uint64_t len = e1 - e0;
  const uint64_t words = (len + 31) / 32;
  rei_status r;
  auto worst_rows = [&] { return std::min(in->row_cap, in->known_rows + in->pending + len); };
  auto worst_entries = [&] { return in->known_rows + in->pending + len; };
  if (worst_rows() > in->rows_alloc || 2 * worst_entries() > in->slots_cap || len > in->surv_cap ||
      words > in->bitmap_cap) {
    if ((r = sync_state(in, s)) != REI_OK) return r;
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
  g.e0 = e0;
  g.e1 = e1;
  g.char_index = in->d_char_index;
  g.st = in->d_state;
  if (b.op != OP_CHAR) {
    g.lstart = in->lstart[b.L];
    g.lcount = in->lcount[b.L];
    if (b.op == OP_CONCAT || b.op == OP_UNION) {
      g.rstart = in->lstart[b.R];
      g.rcount = in->lcount[b.R];
    }
  }
  LAUNCH(in, s, REI_K_GEN_CHAR + b.op, len, launch_gen(W, b.op, g, b.same, s));

  ChunkArgs ca{};
  ca.rows = in->d_rows;
  ca.rows_w = in->d_rows;
  ca.aux = in->d_aux;
  ca.slots = in->d_slots;
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
  ca.chunk_e0 = e_base + e0;
  ca.len = len;
  LAUNCH(in, s, REI_K_INSERT, len, launch_insert(W, ca, s));
  LAUNCH(in, s, REI_K_COMPACT, len, launch_finalize(W, ca, s));
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
      out->a = e;
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

rei_status row_node(rei_instance* in, uint64_t row, Node* nd) {
  uint64_t e = 0;
  HIP_OK(in, hipMemcpy(&e, in->d_aux + row, 8, hipMemcpyDeviceToHost));
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

rei_status solve_impl(rei_instance* in, hipStream_t s, rei_result* out) {
  const double t0 = now_s();
  HIP_OK(in, hipSetDevice(in->device));
  const rei_costs& k = in->costs;
  const uint32_t c1 = k.c_char;
  in->lstart.assign(in->max_cost + 2, 0);
  in->lcount.assign(in->max_cost + 2, 0);
  in->uniq.assign(in->max_cost + 2, 0);
  in->cand.assign(in->max_cost + 2, 0);
  in->regex.clear();

  if (in->max_cost < c1) {
    fill_result(in, REI_NOT_FOUND, 0, 0, t0);
    *out = in->res;
    return REI_OK;
  }
  // trivial specifications (Algorithm 1): the empty language, then eps
  if (in->st.P.size() <= in->max_err) {
    in->regex = "\xE2\x88\x85";
    fill_result(in, REI_OK, c1, 0, t0);
    *out = in->res;
    return REI_OK;
  }
  {
    uint64_t bad = 0;
    for (auto& w : in->st.P) bad += w.empty() ? 0 : 1;
    for (auto& w : in->st.N) bad += w.empty() ? 1 : 0;
    if (bad <= in->max_err) {
      in->regex = "\xCE\xB5";
      fill_result(in, REI_OK, c1, 0, t0);
      *out = in->res;
      return REI_OK;
    }
  }

  rei_status r;
  const uint64_t L = in->max_cost + 2;
  in->known_rows = 0;
  in->pending = 0;
  LAUNCH(in, s, REI_K_OTHER, 1, launch_state_reset(in->d_ctrl, in->d_state, in->row_cap, s));
  LAUNCH(in, s, REI_K_OTHER, 3 * L, launch_fill(in->d_levels, 3 * L, 0, s));
  if ((r = ensure_table(in, 1024, s, true)) != REI_OK) return r;
  std::vector<Block> blocks;
  uint32_t last = in->max_cost;
  bool stopped = false;
  for (uint32_t c = c1; c <= in->max_cost && !stopped; ++c) {
    in->lstart[c] = in->known_rows;
    if (!make_blocks(in, c, &blocks)) {
      in->err = "candidate count overflows 64 bits";
      return REI_ERR_TOO_LARGE;
    }
    uint64_t e_base = 0;
    for (const Block& b : blocks) {
      for (uint64_t e0 = 0; e0 < b.count && !stopped;) {
        const uint64_t e1 = std::min(b.count, e0 + in->chunk_max);
        if ((r = enqueue_chunk(in, s, c, b, e_base, e0, e1, &stopped)) != REI_OK) return r;
        e0 = e1;
      }
      if (stopped) break;
      e_base += b.count;
    }
    // level boundary: the next level's blocks depend on this level's size
    if ((r = sync_state(in, s)) != REI_OK) return r;
    in->lcount[c] = in->h_levels[c];
    if (in->h_state->stop) {
      stopped = true;
      last = c;
    }
  }
  for (uint64_t c = 0; c < L; ++c) {
    in->lcount[c] = in->h_levels[c];
    in->uniq[c] = in->h_levels[L + c];
    in->cand[c] = in->h_levels[2 * L + c];
  }
  rei_status final_status = REI_NOT_FOUND;
  uint32_t cost = 0;
  if (in->h_state->stop == STOP_OOM) final_status = REI_OUT_OF_MEMORY;
  if (in->h_state->stop == STOP_ANSWER) {
    final_status = REI_OK;
    cost = in->h_state->answer_cost;
    Node nd;
    if (!decode(in, cost, in->h_state->answer_e, &nd)) {
      in->err = "answer index does not decode";
      return REI_ERR_DEVICE;
    }
    if ((r = print_node(in, nd, &in->regex)) != REI_OK) return r;
  }
  if (in->prof && (r = prof_collect(in)) != REI_OK) return r;
  fill_result(in, final_status, cost, last, t0);
  *out = in->res;
  return REI_OK;
}

void free_device(rei_instance* in) {
  (void)hipSetDevice(in->device);
  dfree(in->d_gt_off);
  dfree(in->d_gt_pair);
  dfree(in->d_len_off);
  dfree(in->d_pmask);
  dfree(in->d_nmask);
  dfree(in->d_char_index);
  dfree(in->d_rows);
  dfree(in->d_aux);
  dfree(in->d_slots);
  dfree(in->d_skey);
  dfree(in->d_se);
  dfree(in->d_spos);
  dfree(in->d_bitmap);
  dfree(in->d_prefix);
  dfree(in->d_bsums);
  dfree(in->d_ctrl);
  dfree(in->d_state);
  dfree(in->d_levels);
  if (in->h_state) (void)hipHostFree(in->h_state);
  if (in->h_levels) (void)hipHostFree(in->h_levels);
  in->h_state = nullptr;
  in->h_levels = nullptr;
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
  HIP_OK(in, hipMalloc(dst, bytes));
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
  if ((r = upload(in, &in->d_char_index, in->st.char_index)) != REI_OK) return r;
  HIP_OK(in, hipMalloc(&in->d_ctrl, sizeof(Ctrl)));
  HIP_OK(in, hipMalloc(&in->d_state, sizeof(DevState)));
  const uint64_t L = in->max_cost + 2;
  HIP_OK(in, hipMalloc(&in->d_levels, 3 * L * 8));
  HIP_OK(in, hipHostMalloc((void**)&in->h_state, sizeof(DevState), hipHostMallocDefault));
  HIP_OK(in, hipHostMalloc((void**)&in->h_levels, 3 * L * 8, hipHostMallocDefault));
  return REI_OK;
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
  const int W = inst->st.W;
  HIP_OK(inst, hipMemcpy(words_out, inst->d_rows + (inst->lstart[cost] + i) * W, W * 8,
                         hipMemcpyDeviceToHost));
  return REI_OK;
}

rei_status rei_row_regex(rei_instance* inst, uint32_t cost, uint64_t i, char* buf, size_t cap) {
  if (!inst || !buf || cost >= inst->lcount.size() || i >= inst->lcount[cost]) return REI_ERR_INVALID_ARG;
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

rei_status rei_set_max_errors(rei_instance* inst, uint32_t max_errors) {
  if (!inst) return REI_ERR_INVALID_ARG;
  inst->max_err = max_errors;
  return REI_OK;
}

rei_status rei_set_profiling(rei_instance* inst, int enable) {
  if (!inst) return REI_ERR_INVALID_ARG;
  inst->prof = enable != 0;
  for (int k = 0; k < REI_K_COUNT; ++k) {
    inst->st_launch[k] = 0;
    inst->st_ms[k] = 0;
    inst->st_units[k] = 0;
  }
  return REI_OK;
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
    default: return "?";
  }
}

}  // extern "C"
