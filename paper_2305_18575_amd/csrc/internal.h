// Internal declarations of the REI library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rei.h"

namespace rei {

constexpr int kMaxWords = 32;          // 2048 words of ic
constexpr uint32_t kMaxIc = 64 * kMaxWords;

enum Op : int { OP_CHAR = 0, OP_QUESTION = 1, OP_STAR = 2, OP_CONCAT = 3, OP_UNION = 4 };

// Host-side staging of one specification (infix closure, order, guide table).
struct Staged {
  std::string sigma;
  std::vector<std::string> P, N;       // deduplicated
  std::vector<std::string> ic;         // shortlex order, ic[0] = empty word
  uint32_t n = 0;                      // |ic|
  int W = 1;                           // words per language (power of two)
  // Guide table in CSR form: for word w, entries gt_off[w] .. gt_off[w+1]-1
  // are the cuts w = u v, cut position 0..|w|, packed (index(u) << 16) | index(v).
  std::vector<uint32_t> gt_off, gt_pair;
  // words of each length: len_off[l] .. len_off[l+1]-1
  std::vector<uint32_t> len_off;
  uint32_t max_len = 0;
  std::vector<uint64_t> pmask, nmask;  // W words each
  std::vector<int32_t> char_index;     // per alphabet char: its ic index or -1
};

// Validates and stages; returns REI_OK or an error status with *err set.
rei_status stage(const char* alphabet, const char* const* pos, size_t n_pos,
                 const char* const* neg, size_t n_neg, Staged* out, std::string* err);

// ---- slot encoding of the dedup table ------------------------------------
// EMPTY      all ones
// cached row bit63 = 0 | fingerprint (24 bits, 62..39) | row (39 bits)
// new entry  bit63 = 1 | chunk-relative enumeration index (31 bits) | survivor id (32 bits)
constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kRowBits = 39;
constexpr uint64_t kRowMask = (1ull << kRowBits) - 1;
constexpr uint64_t kNewFlag = 1ull << 63;
constexpr uint64_t kMaxChunk = (1ull << 28);  // chunk-relative indices stay far below 2^31 - 1

// Per-chunk control block in device memory.  The generator starts from
// n_surv = 0, answer_e = ~0; the chunk's last kernel puts them back.
struct Ctrl {
  uint32_t n_surv;          // survivors appended by the generator
  uint32_t answer_e;        // chunk-relative index of the first precise survivor (or ~0)
  uint32_t answer_rank;     // rank of the answer among the chunk's winners
  uint32_t winners;         // winners in the chunk
  uint32_t overflow_e;      // chunk-relative index of the winner that does not fit
  uint32_t pad[3];
};

// Search state in device memory, advanced by the last kernel of each chunk,
// so chunks are enqueued without waiting for the host.
enum StopCode : uint32_t { STOP_NONE = 0, STOP_ANSWER = 1, STOP_OOM = 2, STOP_CAPACITY = 3, STOP_HANDOFF = 4 };
// STOP_CAPACITY: the batched solver ran out of its preallocated rows; the
// instance is solved again, from the start, on the per-chunk path.
// STOP_HANDOFF: the batched solver reached a level of more than level_max
// candidates (resume_level) with every lower level stored;
// the per-chunk path continues from there.
struct DevState {
  uint64_t total_rows;      // rows stored (all levels)
  uint64_t row_cap;         // rows that fit the cache budget
  uint32_t stop;            // StopCode; kernels of later chunks return at once
  uint32_t answer_cost;
  uint64_t answer_e;        // level enumeration index of the answer
  uint64_t resume_level;    // STOP_HANDOFF: the first level not searched
  uint32_t otf_on;          // OnTheFly mode allowed when the cache fills
  uint32_t otf;             // OnTheFly mode active: no storage, precision only
  uint32_t done;            // batched solver: set last, once this state is final
  uint32_t chunks;          // per-chunk path: chunks accounted (the host mirror's is written last)
  uint64_t pad[1];
};

// Arguments shared by all generator kernels.
struct GenArgs {
  // language cache
  const uint64_t* rows;       // all rows, W words each
  // dedup table
  const uint64_t* slots;
  uint64_t slot_mask;
  // survivors
  uint64_t* skey;             // survivor keys, W words each
  uint32_t* se;               // survivor chunk-relative index
  uint64_t* spos;             // survivor slot records (hash until inserted)
  Ctrl* ctrl;
  // precision
  const uint64_t* pmask;
  const uint64_t* nmask;
  uint32_t max_err;
  // guide table
  const uint32_t* gt_off;
  const uint32_t* gt_pair;
  const uint32_t* len_off;
  uint32_t max_len;
  uint32_t n;                 // |ic|
  uint32_t n_pairs;           // guide-table entries
  // block / chunk
  uint64_t e0, e1;            // chunk range inside the block
  uint32_t rel0;              // chunk-relative index of the block's candidate e0
  uint64_t lstart, lcount;    // left operand level: first row, number of rows
  uint64_t rstart, rcount;    // right operand level
  const int32_t* char_index;  // base level only
  const DevState* st;
  uint32_t inl;               // inline-key table (one word per language, |ic| <= 63)
  // concatenation launch shape (0 = defaults): workgroups the grid aims at,
  // and the most left rows one workgroup takes
  uint32_t concat_wg, concat_xi;
};

// Tunable launch parameters of the per-chunk grid path (per word width):
// the first chunk of a level (each next one doubles), the largest chunk,
// and the concatenation kernel's grid target and left rows per workgroup.
// Results do not depend on them.
struct GridTune {
  uint64_t first_chunk = 1ull << 16;
  uint64_t chunk_max = 1ull << 24;
  uint32_t concat_wg = 2048;
  uint32_t concat_xi = 16;
};

struct ChunkArgs {
  const uint64_t* rows;
  uint64_t* rows_w;
  uint64_t* aux;
  uint64_t* slots;
  uint64_t* sref;             // inline-key table: smallest survivor per slot
  uint64_t slot_mask;
  uint32_t inl;
  uint64_t* skey;
  uint32_t* se;
  uint64_t* spos;             // slot of each survivor after insertion
  uint32_t* bitmap;           // one bit per chunk-relative index: winner
  uint32_t* word_prefix;      // exclusive prefix of popcounts
  uint32_t* block_sums;
  uint32_t n_bitmap_words;
  Ctrl* ctrl;
  DevState* st;
  uint64_t* uniq;             // per cost level: new languages
  uint64_t* cand;             // per cost level: candidates
  uint64_t* lcount;           // per cost level: stored rows
  uint32_t cost;              // level being built
  uint64_t chunk_e0;          // level enumeration index of chunk-relative 0
  uint64_t len;               // candidates in the chunk
  // host-visible mirrors of *st and of the three per-level counters (same
  // layout: lcount, uniq, cand, nlev each), written with them
  DevState* hst;
  uint64_t* hlev;
  uint64_t nlev;
  uint32_t clear_words;       // bitmap words insert_survivors clears (the grid finalize path)
};
// Whether a chunk is finalized by one workgroup (else by the grid kernels,
// which need the bitmap cleared by insert_survivors).
bool finalize_in_one_workgroup(int W, uint64_t len);

// Events of this thread's next timed kernel launch (set by the library's
// profiler).  launch_timed hands them to the launch itself, which records
// them at the kernel's own start and end, so the time excludes the dispatch
// gap that events recorded on the stream around the launch would include.
struct KernelTimer {
  hipEvent_t start, stop;
};
extern thread_local KernelTimer g_kernel_timer;

template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
  const KernelTimer t = g_kernel_timer;
  g_kernel_timer = KernelTimer{nullptr, nullptr};
  if (t.start)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, args...);
  else  // untimed: a plain launch (also what a stream capture records)
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Kernel launchers (kernels.hip).  Every launcher returns the hipError_t of
// the launch.
hipError_t launch_fill(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_rehash(int W, bool inl, const uint64_t* rows, uint64_t nrows, uint64_t* slots,
                         uint64_t slot_mask, hipStream_t s);
hipError_t launch_gen(int W, int op, const GenArgs& a, bool same_level, hipStream_t s);
hipError_t launch_insert(int W, const ChunkArgs& a, hipStream_t s);
// Winners, their ranks, the stored rows and the accounting of the chunk:
// one workgroup when the chunk is small (LDS bitmap), else a grid pipeline.
hipError_t launch_finalize(int W, const ChunkArgs& a, hipStream_t s);
// Accounting of a chunk without survivors (a level enumerated in OnTheFly
// mode): the answer, if any, and the candidate count.
hipError_t launch_account(const ChunkArgs& a, hipStream_t s);
// An empty kernel through launch_timed (calibrates the timing events).
hipError_t launch_noop_timed(hipStream_t s);

// The answer's expression tree of a per-chunk search, decoded on the device
// (one thread) from the stored back-pointers, so that the host reads a few
// hundred bytes instead of the back-pointer array.
constexpr uint32_t kTreeMaxLevels = 1024;  // max_cost + 2 at most
constexpr uint32_t kTreeMaxChars = 64;     // alphabet size at most
struct TreeArgs {
  const uint64_t* levels;  // stored rows per cost level (device)
  const uint64_t* aux;     // back-pointers (level index of each stored row)
  const DevState* st;      // answer cost and level index
  uint64_t* out;           // host-visible: [nodes k (0 = not decoded), then k x (row, op, a, b)];
                           // row ~0 is the answer, a of a character is its position in ccost
  uint32_t c1, c2, c3, c4, c5, nsigma, max_nodes, pad;
  uint32_t ccost[kTreeMaxChars];  // character costs in enumeration order
};
hipError_t launch_decode_tree(const TreeArgs& t, hipStream_t s);
hipError_t launch_state_reset(Ctrl* c, DevState* st, uint64_t row_cap, bool otf_on, hipStream_t s);
constexpr uint64_t kSmallChunk = 1ull << 14;   // candidates finalized by one workgroup


// The hash bits kept by the kernels of kernels.hip and of batch.hip.
hipError_t set_hash_mask_kernels(uint64_t mask);
hipError_t set_hash_mask_batch(uint64_t mask);

// Many small pieces of one chunk in one launch (gen_pieces): each wave takes
// one item of 64 candidates of one piece.  Items: CHAR, QUESTION, STAR,
// UNION: 64 consecutive candidates; CONCAT: one left row and a tile of 64
// right rows (or, with left_lanes, one right row and a tile of 64 left
// rows, when the right level is small).
constexpr int kMaxPieces = 32;
constexpr uint64_t kSmallPiece = 16384;  // pieces up to this size go to gen_pieces
constexpr int kPiecesMaxW = 32;          // widest languages gen_pieces handles
struct PieceD {
  uint32_t op, same, left_lanes, char_off;
  uint32_t rel0, pad;
  uint64_t e0, e1;                    // block-local candidate range
  uint64_t lstart, lcount, rstart, rcount;
  uint64_t item0;                     // first item of this piece
  uint64_t t0, nt;                    // CONCAT: first row of the uniform side's range, tiles per row
};
struct PieceArgs {
  uint32_t n, pad;
  uint64_t items;       // work items of all pieces
  uint64_t items_cand;  // candidates of all pieces (host bookkeeping)
  PieceD p[kMaxPieces];
};
hipError_t launch_gen_pieces(int W, const GenArgs& a, const PieceArgs& p, hipStream_t s);

// Several large concatenation blocks of one chunk in one gen_concat launch,
// so that blocks too small to fill the device run side by side: each part
// has its own operand levels and candidate range; the launcher gives each a
// tile shape and a range of workgroups.
constexpr int kMaxConcatParts = 16;
struct ConcatPart {
  uint64_t lstart, rstart, rcount;  // left level's first row; right level's first row and size
  uint64_t e0, e1;                  // block-local candidate range
  uint64_t i_lo, i_hi;              // left rows of the range (set by the launcher)
  uint32_t rel0;                    // chunk-relative index of candidate e0
  uint32_t yt, xi, gx;              // right tiles and left rows per workgroup, tile groups (launcher)
  uint32_t wg0, pad;                // first workgroup of this part (launcher)
};
struct ConcatSet {
  uint32_t n, pad;
  ConcatPart p[kMaxConcatParts];
};
hipError_t launch_concat_set(int W, const GenArgs& a, const ConcatSet& cs, hipStream_t s);

// Several large union blocks of one chunk in one gen_union launch (one
// thread per candidate; the launcher gives each part its workgroups).
constexpr int kMaxUnionParts = 16;
struct UnionPart {
  uint64_t lstart, lcount, rstart, rcount;  // operand levels: first row, number of rows
  uint64_t e0, e1;                          // block-local candidate range
  uint32_t rel0;                            // chunk-relative index of candidate e0
  uint32_t same;                            // both operands from one level: pairs x < y
  uint32_t wg0, pad;                        // first workgroup of this part (launcher)
};
struct UnionSet {
  uint32_t n, pad;
  UnionPart p[kMaxUnionParts];
};
hipError_t launch_union_set(int W, const GenArgs& a, const UnionSet& us, hipStream_t s);

// ---- batched solver: one workgroup runs the whole search of one instance --
constexpr uint32_t kBatchChunk = 8192;   // candidates per chunk
constexpr uint32_t kBatchMaxCost = 63;   // largest max_cost handled in a batch
constexpr int kBatchMaxW = 32;           // largest words per language
// The guide table sits in the workgroup's LDS: up to 512 infixes and 6144
// cuts for languages of at most 8 words, up to 64 W infixes and 12288 cuts
// for 16 and 32 words (the wider solvers run fewer threads, so their
// operand tiles leave room for it).
constexpr uint32_t batch_max_ic(int W) { return W <= 8 ? 512u : 64u * (uint32_t)W; }
constexpr uint32_t batch_max_pairs(int W) { return W <= 8 ? 6144u : 12288u; }
// Most threads per instance for W words: each wave holds a 64 x W-word
// operand tile in LDS.
constexpr uint32_t batch_max_threads(int W) { return W >= 32 ? 256u : W >= 8 ? 512u : 1024u; }
constexpr uint64_t kBatchTimeMinLevel = 4096;  // smaller levels stay on the workgroup whatever the time
constexpr uint32_t kBatchTimeUs = 500;         // default workgroup time before larger levels move
constexpr uint64_t kBatchLevelMax = 1ull << 16;  // default: candidates of one level a workgroup takes on
constexpr uint32_t kBatchTreeNodes = 64; // answer-tree nodes written back (cost <= 63 needs <= 63)

struct BatchDesc {
  // staged tables
  const uint32_t* gt_off;
  const uint32_t* gt_pair;
  const uint32_t* len_off;
  const uint64_t* pmask;
  const uint64_t* nmask;
  const int32_t* char_index;
  uint32_t n, n_pairs, max_len, nsigma;
  uint32_t c1, c2, c3, c4, c5, max_cost, max_err, pad;
  // buffers of the instance
  uint64_t* rows;
  uint64_t* aux;
  uint64_t rows_alloc;        // rows the buffers hold
  uint64_t row_cap;           // rows the cache budget allows
  uint64_t* slots;
  uint64_t* sref;
  uint64_t slot_mask;         // arena's table: rows_alloc + kBatchChunk entries at load <= 1/2
                              // (the kernel uses a growing prefix of it)
  uint32_t inl, pad2;
  uint64_t level_max;         // larger levels are handed to the per-chunk path
  uint64_t time_ticks;        // wall-clock ticks after which a level of more than
                              // kBatchTimeMinLevel candidates is handed over too (0: never)
  uint64_t* skey;             // kBatchChunk survivors
  uint32_t* se;
  uint64_t* spos;
  // results, in host-visible (pinned) memory, written once at the end:
  DevState* hst;              // final search state
  uint64_t* hlev;             // per cost: rows, unique, candidates (max_cost + 2 each)
  uint64_t* htree;            // [node count, then per node: row (~0 = the answer), op, a, b]
};

// Host-written control block of a queue launch of the batched solver (in
// coherent pinned memory): ring slots published so far, a request to leave,
// and how long a workgroup waits without work before it leaves (wall-clock
// ticks).
struct QueueCtl {
  uint32_t tail;
  uint32_t closing;
  uint64_t idle_ticks;
};

// Launches the batched solver with `threads` per workgroup (256, 512 or
// 1024, at most batch_max_threads(W)) over n descriptors (all with the same
// W).
// next == nullptr: one workgroup per descriptor (grid ignored).  Else a
// persistent grid of `grid` workgroups (1..n) that take items from the
// device counter *next (zero at launch) and solve descriptor order[item]
// (item itself when order is null).
// qc != nullptr (with next): queue form over a ring of n slots (see
// solve_batch); grid may exceed n.
hipError_t launch_solve_batch(int W, bool inl, uint32_t threads, const BatchDesc* d_descs, uint32_t n,
                              hipStream_t s, const uint32_t* order = nullptr, uint32_t* next = nullptr,
                              uint32_t grid = 0, const QueueCtl* qc = nullptr);
// Workgroups of the batched solver that fit one compute unit at once.
hipError_t batch_resident(int W, bool inl, uint32_t threads, uint32_t* per_cu);
// Zeroes n (<= 64) work counters with a kernel (graph-capturable).
hipError_t launch_reset_counters(uint32_t* c, uint32_t n, hipStream_t s);

// ---- the allocation-free batched entry point ------------------------------
// A static device array (one per GPU, held until the process ends) carries
// the per-instance arenas and descriptors of rei_solve_batch_noalloc.
constexpr uint64_t kStaticScratchBytes = 128ull << 20;
constexpr uint32_t kStaticMaxInstances = 64;        // instances per call
constexpr uint64_t kStaticHeaderBytes = 64ull << 10;  // descriptors at the front
// Device address of that array on the current device (looked up once per
// device with hipGetSymbolAddress, then kept).
hipError_t static_scratch(void** out);
static_assert(kStaticMaxInstances * sizeof(BatchDesc) <= kStaticHeaderBytes, "descriptors fit the header");
// Writes n descriptors from host memory to dst with kernels that take them
// as arguments (kDescPack per launch), on stream s.
constexpr uint32_t kDescPack = 8;
hipError_t launch_put_descs(BatchDesc* dst, const BatchDesc* src, uint32_t n, hipStream_t s);

// Achievable peak of one operation class on the current device (peaks.hip):
// kind 0 stream copy (rate = bytes read + written per second), 1 random
// table reads, 2 random reads plus atomicMin (rate = probes per second),
// 3 bitwise AND-OR loop (rate = 32-bit bitwise lane operations per second).
hipError_t measure_peak(int kind, uint64_t size, double* rate, double* seconds);

}  // namespace rei
