// TEST INFRASTRUCTURE ONLY -- the CPU oracle for search-based regular
// expression inference (Valizadeh & Berger, "Search-Based Regular Expression
// Inference on a GPU", PLDI 2023).  Only the test suite, the smoke check and
// the benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or helper with the GPU library; both sides only agree on the
// written specification of the enumeration order below.
//
// What it computes (Sec. 3 "The algorithm", Algorithm 1 and Algorithm 2):
//   * ic = the infix closure of P u N (Definition of infix-closed sets and
//     of infix power series), ordered shortlex: by length, then
//     lexicographically in alphabet-argument order (Definition of the
//     shortlex ordering);
//   * a language is kept as one byte per word of ic (0 or 1): the
//     characteristic sequence restricted to ic;
//   * operations follow the definition of infix power series directly on the
//     strings: union is element-wise or; r? adds the empty word (Definition of
//     regular expressions, r? = eps + r); r.s contains w iff some cut
//     w = u v has u in r and v in s; r* contains w iff w is empty or some cut
//     w = u v with u non-empty has u in r and v in r* (least fixed point of
//     Y = 1 + r.Y, evaluated in increasing length so the shorter suffix is
//     already final);
//   * levels are built bottom-up by cost (Lemma "build up"): level c holds
//     the languages whose cheapest expression costs exactly c, each kept once
//     (global uniqueness, "Uniqueness checking");
//   * the search stops at the first candidate whose language satisfies
//     (P, N) (Definition of specification; Algorithm 2 stops at the first
//     unique precise candidate).
//
// Enumeration order (the paper leaves the order inside a cost level open;
// this is the reading both implementations follow):
//   level c1 (char cost): one candidate per alphabet character, in argument
//   order.  Level c > c1, in this order:
//     Q: r? for r in level c-c2;
//     S: r* for r in level c-c3;
//     C: for L = c1, c1+1, ... with R = c-c4-L >= c1: for x in level L
//        (outer), for y in level R (inner): x.y;
//     U: for L ascending with L <= R = c-c5-L: if L < R all (x, y) row-major;
//        if L == R only pairs x before y, row-major: x+y.
//   A candidate's enumeration index e is its position in this sequence.
//   New languages are appended to the level in order of first occurrence.
//   The answer is the first (lowest cost, then lowest e) candidate whose
//   language satisfies (P, N); it is necessarily new.
//   unique[c*] counts the new languages with e <= e(answer);
//   candidates[c*] = e(answer) + 1.
//
// Trivial specifications (Algorithm 1): P = {} gives the empty language,
// P = {eps} gives eps, both at cost c1.  With an allowed error of k
// misclassified examples (REI with error, Sec. 5.2, Future Work) these read: the empty
// language if |P| <= k, else eps if it misclassifies at most k examples.
//
// Per-character costs (the cost-homomorphism definition allows a different
// cost for each alphabet character): character a enters at level cost(a),
// before every other block of that level, in alphabet order.  The smallest
// character cost takes the place of c1 (first level, cost of the trivial
// answers).  With equal character costs this is the order above.
//
// Row cap: at most row_cap languages are kept (all levels, base level
// included); a new non-answer language beyond it stops the search with
// status OUT_OF_MEMORY (the language cache is full).
//
// OnTheFly mode (Sec. 3, "OnTheFly mode"; optional here): instead of
// stopping at that language, the search goes on without storing and without
// uniqueness checks, testing every further candidate for precision only.
// The level where the cache filled (otf_level) is incomplete, and so is
// every later level (nothing of them is stored).  A later level is still
// enumerated block by block in the usual order while a block's operand
// levels are complete (cost below otf_level); a block that needs an
// incomplete level stops the search with OUT_OF_MEMORY, unless one of its
// operand levels is complete and empty (then the block has no candidates).
// Candidates found this way count in candidates[c]; nothing counts as new in
// unique[c] once the cache is full.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

enum Status {
  ST_OK = 0,
  ST_NOT_FOUND = 1,
  ST_OUT_OF_MEMORY = 2,
  ST_INVALID_ARG = -1,
  ST_INCONSISTENT = -2,
  ST_BAD_CHAR = -3,
};

enum Op { OP_CHAR = 0, OP_QUESTION = 1, OP_STAR = 2, OP_CONCAT = 3, OP_UNION = 4 };

struct Cand {
  int op;
  int64_t x;  // row id (char index for OP_CHAR)
  int64_t y;  // row id or -1
};

struct Oracle {
  // inputs
  std::string sigma;
  std::vector<std::string> P, N;
  int c1 = 1, c2 = 1, c3 = 1, c4 = 1, c5 = 1;
  int max_cost = 0;
  int64_t row_cap = 0;
  int max_err = 0;
  int threads = 1;
  std::vector<int> char_cost;  // per alphabet character (empty: all c1)
  bool otf = false;   // OnTheFly mode allowed
  int otf_level = 0;  // level where the cache filled (0: not reached)

  // staged
  std::vector<std::string> ic;
  std::unordered_map<std::string, int> index;
  // for every word w: all cuts w = u v as (index of u, index of v), cut
  // position 0 .. |w| in increasing order
  std::vector<std::vector<std::pair<int, int>>> cuts;
  int eps = -1;
  std::vector<int> pidx, nidx;

  // language cache
  std::vector<std::string> cs;  // one byte per word of ic
  std::vector<int> op;
  std::vector<int64_t> arg_a, arg_b;
  std::vector<int> row_level;
  std::vector<std::vector<int64_t>> level;  // level[c] = row ids in order
  std::unordered_map<std::string, int64_t> seen;

  // results
  int status = ST_NOT_FOUND;
  int answer_cost = 0;
  Cand answer{-1, -1, -1};
  std::string answer_text;
  std::vector<uint64_t> uniq, cand;
  std::string scratch;  // returned strings live here until the next call
  std::string error;
};

// shortlex: length first, then lexicographic in alphabet-argument order
struct Shortlex {
  const int* rank;
  bool operator()(const std::string& a, const std::string& b) const {
    if (a.size() != b.size()) return a.size() < b.size();
    for (size_t i = 0; i < a.size(); ++i) {
      int ra = rank[(unsigned char)a[i]], rb = rank[(unsigned char)b[i]];
      if (ra != rb) return ra < rb;
    }
    return false;
  }
};

int validate_and_stage(Oracle& o) {
  if (o.sigma.empty()) { o.error = "empty alphabet"; return ST_INVALID_ARG; }
  int rank[256];
  for (int i = 0; i < 256; ++i) rank[i] = -1;
  for (size_t i = 0; i < o.sigma.size(); ++i) {
    unsigned char ch = (unsigned char)o.sigma[i];
    if (ch == 0 || ch >= 0x80 || std::strchr("()+*?", ch) != nullptr) {
      o.error = "alphabet character not allowed";
      return ST_INVALID_ARG;
    }
    if (rank[ch] >= 0) { o.error = "repeated alphabet character"; return ST_INVALID_ARG; }
    rank[ch] = (int)i;
  }
  if (o.c1 < 1 || o.c2 < 1 || o.c3 < 1 || o.c4 < 1 || o.c5 < 1) {
    o.error = "every constructor cost must be at least 1";
    return ST_INVALID_ARG;
  }
  if (o.max_cost < 0 || o.row_cap < 0 || o.max_err < 0) { o.error = "negative limit"; return ST_INVALID_ARG; }
  for (auto* side : {&o.P, &o.N})
    for (auto& w : *side)
      for (unsigned char ch : w)
        if (rank[ch] < 0) { o.error = "example uses a character outside the alphabet"; return ST_BAD_CHAR; }
  // specifications are pairs of sets: duplicates collapse
  auto dedup = [](std::vector<std::string>& v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  };
  dedup(o.P);
  dedup(o.N);
  for (auto& w : o.P)
    if (std::binary_search(o.N.begin(), o.N.end(), w)) {
      o.error = "a string is both positive and negative";
      return ST_INCONSISTENT;
    }
  // infix closure: every substring of every example
  std::vector<std::string> all;
  for (auto* side : {&o.P, &o.N})
    for (auto& w : *side)
      for (size_t i = 0; i <= w.size(); ++i)
        for (size_t j = i; j <= w.size(); ++j) all.push_back(w.substr(i, j - i));
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  std::sort(all.begin(), all.end(), Shortlex{rank});
  o.ic = all;
  for (size_t i = 0; i < o.ic.size(); ++i) o.index[o.ic[i]] = (int)i;
  o.eps = o.index.count("") ? o.index[""] : -1;
  o.cuts.assign(o.ic.size(), {});
  for (size_t i = 0; i < o.ic.size(); ++i) {
    const std::string& w = o.ic[i];
    for (size_t k = 0; k <= w.size(); ++k)
      o.cuts[i].push_back({o.index.at(w.substr(0, k)), o.index.at(w.substr(k))});
  }
  for (auto& w : o.P) o.pidx.push_back(o.index.at(w));
  for (auto& w : o.N) o.nidx.push_back(o.index.at(w));
  return ST_OK;
}

// ---- the four constructors on characteristic sequences over ic ----------

std::string op_question(const Oracle& o, const std::string& x) {
  std::string r = x;
  r[o.eps] = 1;
  return r;
}

std::string op_union(const Oracle& o, const std::string& x, const std::string& y) {
  std::string r(o.ic.size(), 0);
  for (size_t w = 0; w < o.ic.size(); ++w) r[w] = (x[w] || y[w]) ? 1 : 0;
  return r;
}

std::string op_concat(const Oracle& o, const std::string& x, const std::string& y) {
  std::string r(o.ic.size(), 0);
  for (size_t w = 0; w < o.ic.size(); ++w)
    for (auto& uv : o.cuts[w])
      if (x[uv.first] && y[uv.second]) { r[w] = 1; break; }
  return r;
}

std::string op_star(const Oracle& o, const std::string& x) {
  std::string r(o.ic.size(), 0);
  for (size_t w = 0; w < o.ic.size(); ++w) {  // increasing length
    if ((int)w == o.eps) { r[w] = 1; continue; }
    for (auto& uv : o.cuts[w]) {
      if (uv.first == o.eps) continue;  // the first factor is non-empty
      if (x[uv.first] && r[uv.second]) { r[w] = 1; break; }
    }
  }
  return r;
}

int misclassified(const Oracle& o, const std::string& x) {
  int bad = 0;
  for (int p : o.pidx) bad += x[p] ? 0 : 1;
  for (int n : o.nidx) bad += x[n] ? 1 : 0;
  return bad;
}

std::string op_char(const Oracle& o, int64_t a) {
  std::string r(o.ic.size(), 0);
  auto it = o.index.find(std::string(1, o.sigma[a]));
  if (it != o.index.end()) r[it->second] = 1;
  return r;
}

std::string compute(const Oracle& o, const Cand& c) {
  switch (c.op) {
    case OP_CHAR: return op_char(o, c.x);
    case OP_QUESTION: return op_question(o, o.cs[c.x]);
    case OP_STAR: return op_star(o, o.cs[c.x]);
    case OP_CONCAT: return op_concat(o, o.cs[c.x], o.cs[c.y]);
    default: return op_union(o, o.cs[c.x], o.cs[c.y]);
  }
}

// ---- printing -------------------------------------------------------------
// x? and x* parenthesise x iff x is a concatenation or a union; x.y
// parenthesises a child iff it is a union; x+y never parenthesises.

std::string print_node(const Oracle& o, int opk, int64_t a, int64_t b);

std::string print_row(const Oracle& o, int64_t r) { return print_node(o, o.op[r], o.arg_a[r], o.arg_b[r]); }

std::string print_node(const Oracle& o, int opk, int64_t a, int64_t b) {
  if (opk == OP_CHAR) return std::string(1, o.sigma[a]);
  if (opk == OP_QUESTION || opk == OP_STAR) {
    std::string s = print_row(o, a);
    int k = o.op[a];
    if (k == OP_CONCAT || k == OP_UNION) s = "(" + s + ")";
    return s + (opk == OP_QUESTION ? "?" : "*");
  }
  if (opk == OP_CONCAT) {
    std::string l = print_row(o, a), r = print_row(o, b);
    if (o.op[a] == OP_UNION) l = "(" + l + ")";
    if (o.op[b] == OP_UNION) r = "(" + r + ")";
    return l + r;
  }
  return print_row(o, a) + "+" + print_row(o, b);
}

// ---- the search -----------------------------------------------------------

// Processes a buffer of candidates of level c in enumeration order.
// Returns true when the search has to stop (answer or row cap).
bool flush(Oracle& o, int c, std::vector<Cand>& buf) {
  if (buf.empty()) return false;
  std::vector<std::string> out(buf.size());
  int T = std::max(1, o.threads);
  if (T == 1 || buf.size() < 256) {
    for (size_t k = 0; k < buf.size(); ++k) out[k] = compute(o, buf[k]);
  } else {
    std::vector<std::thread> pool;
    size_t per = (buf.size() + T - 1) / T;
    for (int t = 0; t < T; ++t) {
      size_t lo = t * per, hi = std::min(buf.size(), lo + per);
      if (lo >= hi) break;
      pool.emplace_back([&, lo, hi] {
        for (size_t k = lo; k < hi; ++k) out[k] = compute(o, buf[k]);
      });
    }
    for (auto& th : pool) th.join();
  }
  for (size_t k = 0; k < buf.size(); ++k) {
    o.cand[c] += 1;
    if (o.otf_level) {
      // OnTheFly: no storage, no uniqueness check; precision only
      if (misclassified(o, out[k]) <= o.max_err) {
        o.status = ST_OK;
        o.answer_cost = c;
        o.answer = buf[k];
        o.answer_text = print_node(o, buf[k].op, buf[k].x, buf[k].y);
        buf.clear();
        return true;
      }
      continue;
    }
    if (o.seen.count(out[k])) continue;
    if (misclassified(o, out[k]) <= o.max_err) {
      o.uniq[c] += 1;
      o.status = ST_OK;
      o.answer_cost = c;
      o.answer = buf[k];
      o.answer_text = print_node(o, buf[k].op, buf[k].x, buf[k].y);
      buf.clear();
      return true;
    }
    if ((int64_t)o.cs.size() + 1 > o.row_cap) {
      if (o.otf) {
        o.otf_level = c;  // this language is not kept; the rest goes on the fly
        continue;
      }
      o.status = ST_OUT_OF_MEMORY;
      buf.clear();
      return true;
    }
    int64_t id = (int64_t)o.cs.size();
    o.seen.emplace(out[k], id);
    o.cs.push_back(std::move(out[k]));
    o.op.push_back(buf[k].op);
    o.arg_a.push_back(buf[k].x);
    o.arg_b.push_back(buf[k].y);
    o.row_level.push_back(c);
    o.level[c].push_back(id);
    o.uniq[c] += 1;
  }
  buf.clear();
  return false;
}

const size_t kChunk = 1 << 16;

bool build_level(Oracle& o, int c) {
  std::vector<Cand> buf;
  buf.reserve(kChunk);
  auto push = [&](int opk, int64_t x, int64_t y) -> bool {
    buf.push_back({opk, x, y});
    return buf.size() >= kChunk ? flush(o, c, buf) : false;
  };
  auto lvl = [&](int k) -> const std::vector<int64_t>& {
    static const std::vector<int64_t> none;
    return (k >= o.c1 && k < (int)o.level.size()) ? o.level[k] : none;
  };
  // OnTheFly: may a block over operand levels a (and b) be enumerated?  A
  // level is complete when it lies below the level where the cache filled.
  // Returns false after stopping the search (the candidates that come
  // before the block in enumeration order have been processed).
  auto usable = [&](int a, int b) -> bool {
    if (!o.otf_level) return true;
    auto exists = [&](int k) { return k >= o.c1; };
    auto complete = [&](int k) { return k < o.otf_level; };
    if (!exists(a) || (b >= 0 && !exists(b))) return true;  // no such block
    const bool ca = complete(a), cb = b < 0 || complete(b);
    if (ca && cb) return true;
    if ((ca && lvl(a).empty()) || (b >= 0 && cb && lvl(b).empty())) return true;  // no candidates
    if (flush(o, c, buf)) return false;
    o.status = ST_OUT_OF_MEMORY;
    return false;
  };
  // characters of this cost, then Q, then S
  for (size_t a = 0; a < o.sigma.size(); ++a) {
    const int ca = o.char_cost.empty() ? o.c1 : o.char_cost[a];
    if (ca == c && push(OP_CHAR, (int64_t)a, -1)) return true;
  }
  if (!usable(c - o.c2, -1)) return true;
  for (int64_t x : lvl(c - o.c2))
    if (push(OP_QUESTION, x, -1)) return true;
  if (!usable(c - o.c3, -1)) return true;
  for (int64_t x : lvl(c - o.c3))
    if (push(OP_STAR, x, -1)) return true;
  // C: left cost ascending
  for (int L = o.c1; c - o.c4 - L >= o.c1; ++L) {
    if (!usable(L, c - o.c4 - L)) return true;
    const auto& A = lvl(L);
    const auto& B = lvl(c - o.c4 - L);
    for (int64_t x : A)
      for (int64_t y : B)
        if (push(OP_CONCAT, x, y)) return true;
  }
  // U: left cost ascending, left cost <= right cost
  for (int L = o.c1; L <= c - o.c5 - L; ++L) {
    int R = c - o.c5 - L;
    if (!usable(L, R)) return true;
    const auto& A = lvl(L);
    const auto& B = lvl(R);
    if (L < R) {
      for (int64_t x : A)
        for (int64_t y : B)
          if (push(OP_UNION, x, y)) return true;
    } else {
      for (size_t i = 0; i < A.size(); ++i)
        for (size_t j = i + 1; j < A.size(); ++j)
          if (push(OP_UNION, A[i], A[j])) return true;
    }
  }
  return flush(o, c, buf);
}

void solve(Oracle& o) {
  o.status = ST_NOT_FOUND;
  o.otf_level = 0;
  o.uniq.assign(o.max_cost + 1, 0);
  o.cand.assign(o.max_cost + 1, 0);
  o.level.assign(o.max_cost + 1, {});
  if (o.max_cost < o.c1) return;
  // trivial specifications
  if ((int)o.P.size() <= o.max_err) {
    o.status = ST_OK;
    o.answer_cost = o.c1;
    o.answer_text = "\xE2\x88\x85";  // empty set
    return;
  }
  {
    int bad = 0;
    for (auto& w : o.P) bad += w.empty() ? 0 : 1;
    for (auto& w : o.N) bad += w.empty() ? 1 : 0;
    if (bad <= o.max_err) {
      o.status = ST_OK;
      o.answer_cost = o.c1;
      o.answer_text = "\xCE\xB5";  // epsilon
      return;
    }
  }
  for (int c = o.c1; c <= o.max_cost; ++c)
    if (build_level(o, c)) return;
}

// ---- regular-expression parser, for checking single expressions ---------
// grammar: union := concat ('+' concat)* ; concat := post post* ;
// post := atom ('?' | '*')* ; atom := char | '(' union ')' | eps | emptyset

struct Parser {
  const Oracle& o;
  const std::string& s;
  size_t p = 0;
  bool ok = true;
  std::string parse_union() {
    std::string r = parse_concat();
    while (ok && p < s.size() && s[p] == '+') {
      ++p;
      std::string t = parse_concat();
      r = op_union(o, r, t);
    }
    return r;
  }
  bool atom_start() const {
    if (p >= s.size()) return false;
    char ch = s[p];
    return ch != '+' && ch != ')' && ch != '?' && ch != '*';
  }
  std::string parse_concat() {
    std::string r = parse_post();
    while (ok && atom_start()) {
      std::string t = parse_post();
      r = op_concat(o, r, t);
    }
    return r;
  }
  std::string parse_post() {
    std::string r = parse_atom();
    while (ok && p < s.size() && (s[p] == '?' || s[p] == '*')) {
      r = s[p] == '?' ? op_question(o, r) : op_star(o, r);
      ++p;
    }
    return r;
  }
  std::string parse_atom() {
    std::string r(o.ic.size(), 0);
    if (p >= s.size()) { ok = false; return r; }
    if (s[p] == '(') {
      ++p;
      r = parse_union();
      if (p >= s.size() || s[p] != ')') ok = false;
      ++p;
      return r;
    }
    if (s.compare(p, 2, "\xCE\xB5") == 0) { p += 2; if (o.eps >= 0) r[o.eps] = 1; return r; }
    if (s.compare(p, 3, "\xE2\x88\x85") == 0) { p += 3; return r; }
    char ch = s[p++];
    if (o.sigma.find(ch) == std::string::npos) { ok = false; return r; }
    auto it = o.index.find(std::string(1, ch));
    if (it != o.index.end()) r[it->second] = 1;
    return r;
  }
};

}  // namespace

extern "C" {

void* oracle_create(const char* alphabet, const char* const* pos, int npos, const char* const* neg,
                    int nneg, const int* costs, int max_cost, long long row_cap, int max_errors,
                    int threads, int* status) {
  Oracle* o = new Oracle();
  o->sigma = alphabet ? alphabet : "";
  for (int i = 0; i < npos; ++i) o->P.push_back(pos[i]);
  for (int i = 0; i < nneg; ++i) o->N.push_back(neg[i]);
  o->c1 = costs[0];
  o->c2 = costs[1];
  o->c3 = costs[2];
  o->c4 = costs[3];
  o->c5 = costs[4];
  o->max_cost = max_cost;
  o->row_cap = row_cap;
  o->max_err = max_errors;
  o->threads = threads;
  *status = validate_and_stage(*o);
  if (*status != ST_OK) {
    delete o;
    return nullptr;
  }
  return o;
}

void oracle_set_on_the_fly(void* h, int enable) { ((Oracle*)h)->otf = enable != 0; }

// Per-character costs, one per alphabet character in alphabet order (all at
// least 1); the smallest becomes c1.  Returns 0, or -1 on a bad argument.
int oracle_set_char_costs(void* h, const int* costs, int n) {
  Oracle* o = (Oracle*)h;
  if (n != (int)o->sigma.size()) return -1;
  int lo = 0;
  for (int i = 0; i < n; ++i) {
    if (costs[i] < 1) return -1;
    lo = i == 0 ? costs[i] : std::min(lo, costs[i]);
  }
  o->char_cost.assign(costs, costs + n);
  if (n) o->c1 = lo;
  return 0;
}

int oracle_solve(void* h) {
  Oracle* o = (Oracle*)h;
  solve(*o);
  return o->status;
}

void oracle_destroy(void* h) { delete (Oracle*)h; }
int oracle_status(void* h) { return ((Oracle*)h)->status; }
int oracle_cost(void* h) { return ((Oracle*)h)->answer_cost; }
const char* oracle_regex(void* h) { return ((Oracle*)h)->answer_text.c_str(); }
int oracle_ic_size(void* h) { return (int)((Oracle*)h)->ic.size(); }
const char* oracle_ic_word(void* h, int i) { return ((Oracle*)h)->ic[i].c_str(); }
int oracle_max_cost(void* h) { return ((Oracle*)h)->max_cost; }

void oracle_level_counts(void* h, unsigned long long* uniq, unsigned long long* cand) {
  Oracle* o = (Oracle*)h;
  for (int c = 0; c <= o->max_cost; ++c) {
    uniq[c] = c < (int)o->uniq.size() ? o->uniq[c] : 0;
    cand[c] = c < (int)o->cand.size() ? o->cand[c] : 0;
  }
}

long long oracle_num_rows(void* h) { return (long long)((Oracle*)h)->cs.size(); }
int oracle_row_level(void* h, long long r) { return ((Oracle*)h)->row_level[r]; }
long long oracle_level_size(void* h, int c) {
  Oracle* o = (Oracle*)h;
  return (c >= 0 && c < (int)o->level.size()) ? (long long)o->level[c].size() : 0;
}
long long oracle_level_row(void* h, int c, long long i) { return ((Oracle*)h)->level[c][i]; }

void oracle_row_cs(void* h, long long r, unsigned char* out) {
  Oracle* o = (Oracle*)h;
  std::memcpy(out, o->cs[r].data(), o->ic.size());
}

const char* oracle_row_regex(void* h, long long r) {
  Oracle* o = (Oracle*)h;
  o->scratch = print_row(*o, r);
  return o->scratch.c_str();
}

// Characteristic sequence (one byte per word of ic) of a regular expression
// written in the printed syntax.  Returns 0, or -1 on a syntax error.
int oracle_cs_of_regex(void* h, const char* text, unsigned char* out) {
  Oracle* o = (Oracle*)h;
  std::string s = text;
  Parser ps{*o, s};
  std::string r = ps.parse_union();
  if (!ps.ok || ps.p != s.size()) return -1;
  std::memcpy(out, r.data(), o->ic.size());
  return 0;
}

const char* oracle_last_error(void* h) { return ((Oracle*)h)->error.c_str(); }

}  // extern "C"
