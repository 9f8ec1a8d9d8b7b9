// Host staging: validation, infix closure, shortlex order, guide table and
// example masks (the precomputation the paper does once before the search:
// "Staging: guide table", Sec. 3; infix closure, Definition of infix power
// series).
#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "internal.h"

namespace rei {

namespace {

bool valid_alphabet(const char* a, std::string* err) {
  if (a == nullptr || a[0] == 0) {
    *err = "alphabet is empty";
    return false;
  }
  bool seen[256] = {false};
  for (const unsigned char* p = (const unsigned char*)a; *p; ++p) {
    if (*p >= 0x80 || std::strchr("()+*?", *p) != nullptr) {
      *err = "alphabet character not allowed";
      return false;
    }
    if (seen[*p]) {
      *err = "repeated alphabet character";
      return false;
    }
    seen[*p] = true;
  }
  return true;
}

}  // namespace

rei_status stage(const char* alphabet, const char* const* pos, size_t n_pos,
                 const char* const* neg, size_t n_neg, Staged* out, std::string* err) {
  if (!valid_alphabet(alphabet, err)) return REI_ERR_INVALID_ARG;
  if ((n_pos && !pos) || (n_neg && !neg)) {
    *err = "null example array";
    return REI_ERR_INVALID_ARG;
  }
  Staged& s = *out;
  s.sigma = alphabet;
  int rank[256];
  std::fill(rank, rank + 256, -1);
  for (size_t i = 0; i < s.sigma.size(); ++i) rank[(unsigned char)s.sigma[i]] = (int)i;

  auto take = [&](const char* const* src, size_t cnt, std::vector<std::string>* dst) -> rei_status {
    std::unordered_set<std::string> uniq;
    for (size_t i = 0; i < cnt; ++i) {
      if (!src[i]) {
        *err = "null example string";
        return REI_ERR_INVALID_ARG;
      }
      std::string w(src[i]);
      for (unsigned char ch : w)
        if (rank[ch] < 0) {
          *err = "example \"" + w + "\" uses a character outside the alphabet";
          return REI_ERR_BAD_CHAR;
        }
      if (uniq.insert(w).second) dst->push_back(w);
    }
    return REI_OK;
  };
  rei_status st = take(pos, n_pos, &s.P);
  if (st != REI_OK) return st;
  st = take(neg, n_neg, &s.N);
  if (st != REI_OK) return st;
  {
    std::unordered_set<std::string> pset(s.P.begin(), s.P.end());
    for (auto& w : s.N)
      if (pset.count(w)) {
        *err = "\"" + w + "\" is both positive and negative";
        return REI_ERR_INCONSISTENT;
      }
  }

  // infix closure
  std::unordered_set<std::string> inf;
  for (const auto* side : {&s.P, &s.N})
    for (const auto& w : *side)
      for (size_t a = 0; a <= w.size(); ++a)
        for (size_t len = 0; a + len <= w.size(); ++len) inf.insert(w.substr(a, len));
  if (inf.size() > kMaxIc) {
    *err = "infix closure has " + std::to_string(inf.size()) + " words; at most 2048 are supported";
    return REI_ERR_TOO_LARGE;
  }
  s.ic.assign(inf.begin(), inf.end());
  std::sort(s.ic.begin(), s.ic.end(), [&](const std::string& x, const std::string& y) {
    if (x.size() != y.size()) return x.size() < y.size();
    return std::lexicographical_compare(
        x.begin(), x.end(), y.begin(), y.end(),
        [&](char p, char q) { return rank[(unsigned char)p] < rank[(unsigned char)q]; });
  });
  s.n = (uint32_t)s.ic.size();
  s.W = 1;
  while ((uint32_t)(64 * s.W) < s.n) s.W *= 2;

  std::unordered_map<std::string, uint32_t> idx;
  idx.reserve(s.n * 2 + 1);
  for (uint32_t i = 0; i < s.n; ++i) idx.emplace(s.ic[i], i);

  // guide table: every cut of every word
  s.gt_off.assign(s.n + 1, 0);
  s.gt_pair.clear();
  for (uint32_t w = 0; w < s.n; ++w) {
    s.gt_off[w] = (uint32_t)s.gt_pair.size();
    const std::string& word = s.ic[w];
    for (size_t k = 0; k <= word.size(); ++k) {
      uint32_t u = idx.at(word.substr(0, k)), v = idx.at(word.substr(k));
      s.gt_pair.push_back((u << 16) | v);
    }
  }
  s.gt_off[s.n] = (uint32_t)s.gt_pair.size();

  s.max_len = s.n ? (uint32_t)s.ic.back().size() : 0;
  // len_off[l] = number of words shorter than l, l = 0 .. max_len + 1
  s.len_off.assign(s.max_len + 2, 0);
  for (uint32_t w = 0; w < s.n; ++w) s.len_off[s.ic[w].size() + 1] += 1;
  for (uint32_t l = 1; l < s.len_off.size(); ++l) s.len_off[l] += s.len_off[l - 1];

  s.pmask.assign(s.W, 0);
  s.nmask.assign(s.W, 0);
  for (auto& w : s.P) {
    uint32_t i = idx.at(w);
    s.pmask[i >> 6] |= 1ull << (i & 63);
  }
  for (auto& w : s.N) {
    uint32_t i = idx.at(w);
    s.nmask[i >> 6] |= 1ull << (i & 63);
  }
  s.char_index.clear();
  for (char ch : s.sigma) {
    auto it = idx.find(std::string(1, ch));
    s.char_index.push_back(it == idx.end() ? -1 : (int32_t)it->second);
  }
  return REI_OK;
}

}  // namespace rei
