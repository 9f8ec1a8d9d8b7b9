/* rei.h -- C ABI of the MI355X regular-expression-inference library.
 *
 * Search-based regular expression inference (Valizadeh & Berger, PLDI 2023):
 * given positive examples P, negative examples N and a cost homomorphism,
 * return a regular expression of minimal cost whose language contains every
 * string of P and none of N (Sec. 3, Definition of specification, Definition
 * of cost homomorphism, Algorithm 1).
 *
 * Languages are characteristic sequences over the infix closure ic(P u N),
 * ordered shortlex (Definition of infix power series, Example 1); the search
 * builds them bottom-up by cost (Lemma "build up", Algorithm 1) with the
 * constructors ?, *, concatenation (guide-table fold, Algorithm 2) and union,
 * keeps each language once (global uniqueness check) and stops at the first
 * one that satisfies (P, N).
 *
 * Conventions
 *   - Every function returns a status; no C++ exception crosses the ABI.
 *   - Strings are NUL-terminated byte strings.  Inputs are copied; the caller
 *     keeps ownership of everything it passes in.
 *   - Results (strings, arrays) are owned by the instance and stay valid
 *     until the next rei_solve on it or rei_destroy.
 *   - An instance is used by one host thread at a time.  Different instances
 *     may be solved concurrently on different streams.
 *   - Device memory is allocated by the library (hipMalloc) on the device
 *     that is current when rei_create is called, and freed by rei_destroy.
 *
 * Enumeration order inside a cost level (the paper leaves it open; this is
 * the order the returned expression and per-level counts refer to):
 *   level c_char: one candidate per alphabet character, in argument order;
 *   level c > c_char: Q (r? over level c-c_question), S (r* over level
 *   c-c_star), C (for left cost L = c_char, c_char+1, ... with right cost
 *   R = c-c_concat-L: x in level L outer, y in level R inner: x.y), U (for
 *   L <= R = c-c_union-L ascending: all pairs if L < R, pairs x before y if
 *   L == R: x+y).  The enumeration index e of a candidate is its position in
 *   that sequence.  New languages are appended to their level in order of
 *   first occurrence; the answer is the first precise candidate.
 */
#ifndef REI_H
#define REI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  REI_OK = 0,                /* a minimal precise expression was found          */
  REI_NOT_FOUND = 1,         /* none of cost <= max_cost (Algorithm 1 output)   */
  REI_OUT_OF_MEMORY = 2,     /* the language cache row cap was reached          */
  REI_ERR_INVALID_ARG = -1,  /* null pointer, cost < 1, bad alphabet, ...       */
  REI_ERR_INCONSISTENT = -2, /* a string is both in P and in N                  */
  REI_ERR_BAD_CHAR = -3,     /* an example uses a character outside the alphabet*/
  REI_ERR_TOO_LARGE = -4,    /* |ic(P u N)| > 2048 (more than 32 words per row) */
  REI_ERR_DEVICE = -5,       /* a HIP call failed (message in rei_last_error)   */
  REI_ERR_HOST_ALLOC = -6    /* host allocation failed                          */
} rei_status;

/* Cost homomorphism (c1..c5) = (character, ?, *, concatenation, union), all
 * at least 1 (Definition of cost homomorphism).  cost(eps) = cost(empty set)
 * = c_char. */
typedef struct {
  uint32_t c_char, c_question, c_star, c_concat, c_union;
} rei_costs;

typedef struct rei_instance rei_instance;

/* Stage one specification (Sec. 3, Definition of specification: a pair of
 * finite sets of positive and negative strings; Definition of cost
 * homomorphism; the staging of Sec. 3: infix closure, shortlex order, guide
 * table of all cuts of each infix, P/N masks).
 *   alphabet    distinct bytes in 0x01..0x7f, none of ( ) + * ? ; its order
 *               is the shortlex character order and the level-c_char order.
 *   pos, neg    n_pos / n_neg NUL-terminated strings ("" is the empty word);
 *               duplicates are ignored (a specification is a pair of sets).
 *   costs       the cost homomorphism.
 *   max_cost    largest cost searched, inclusive.
 *   cache_bytes language-cache budget: at most floor(cache_bytes / (8W + 8))
 *               languages are kept (W = 64-bit words per language, the
 *               smallest power of two with 64W >= |ic|); beyond that the
 *               search stops with REI_OUT_OF_MEMORY.  The dedup table and
 *               per-chunk staging buffers are allocated beside it.
 * Staging (infix closure, shortlex order, guide table, P/N masks) runs on the
 * host and is copied to the device once.  On success *out owns the instance;
 * on failure *out is NULL and the status says why. */
rei_status rei_create(const char *alphabet, const char *const *pos, size_t n_pos,
                      const char *const *neg, size_t n_neg, rei_costs costs,
                      uint32_t max_cost, uint64_t cache_bytes, rei_instance **out);

typedef struct {
  rei_status status;         /* REI_OK, REI_NOT_FOUND or REI_OUT_OF_MEMORY      */
  uint32_t cost;             /* minimal cost when REI_OK                        */
  const char *regex;         /* UTF-8; "∅" / "ε" only for the trivial
                                specifications P = {} and P = {eps}             */
  uint32_t first_level;      /* = c_char (the smallest character cost)          */
  uint32_t n_levels;         /* levels first_level .. first_level+n_levels-1    */
  const uint64_t *unique_per_level;     /* new languages per level; the last
                                           level counts those up to the answer */
  const uint64_t *candidates_per_level; /* candidates generated per level      */
  uint64_t total_unique;     /* sum of unique_per_level                         */
  uint32_t ic_size;          /* |ic(P u N)|                                     */
  uint32_t cs_words;         /* W                                               */
  double seconds_stage;      /* rei_create wall time                            */
  double seconds_solve;      /* rei_solve wall time                             */
} rei_result;

/* Run the search (Algorithm 1: levels by increasing cost, each built from
 * the cached lower levels with ?, *, concatenation (Algorithm 2) and union,
 * new languages kept once, stop at the first precise one; Sec. 3, "GPU
 * language cache implementation", "Uniqueness checking") on `hip_stream`
 * (a hipStream_t; NULL = the null stream).
 * Blocks until the search ends.  Repeated calls restart from scratch and give
 * identical results. */
rei_status rei_solve(rei_instance *inst, void *hip_stream, rei_result *out);

/* Solve n independent specifications together, each by Algorithm 1 as in
 * rei_solve (the batched configuration: many small uneven instances in one
 * call).  Instances with at most 32 words per language (and a guide table
 * of at most 6144 cuts up to 8 words, 12288 beyond), equal character costs,
 * OnTheFly mode off and max_cost <= 63 run in one launch per word width
 * (the launches run side
 * by side), one workgroup per instance executing the whole level loop on the
 * device (no host round trip per level or chunk; the answer's expression
 * tree is decoded there too).  An instance whose next level has more
 * candidates than the hand-off size (rei_set_batch_level; 2^16 by default),
 * or more than 4096 after its workgroup has run for the hand-off time
 * (rei_set_batch_time; 500 us by default),
 * continues from that level on rei_solve's path with its lower levels kept;
 * one that outgrows its preallocated rows starts again there; the others
 * run there from the start.  Up to 8 such instances run at once, each on
 * its own stream.  Every result equals what rei_solve returns for that
 * instance.
 *   insts        n distinct instances (each used by this call only).
 *   arena_bytes  device bytes preallocated per batched instance for rows,
 *                back-pointers and table (0 = 16 MiB); capped by the
 *                instance's cache budget.
 *   out          n results; out[i] belongs to insts[i] (owned by it, as for
 *                rei_solve).  seconds_solve is the time from the start
 *                of the call until that result was known (the launch's
 *                completion flag, or the end of its per-chunk levels).
 * Returns REI_OK when every instance was searched (each out[i].status tells
 * its outcome), or the first error. */
rei_status rei_solve_batch(rei_instance *const *insts, size_t n, void *hip_stream, uint64_t arena_bytes,
                           rei_result *out);

/* ---- batched solving without allocation --------------------------------------
 * For callers that cannot allocate device memory during a solve: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same search as rei_solve_batch, with every batchable instance's whole
 * search kept in the one-workgroup solver (no hand-off to rei_solve's path).
 * Rows, back-pointers, dedup table and survivor buffers live in a static
 * device array of 128 MiB (one per GPU, part of the library's device code,
 * held until the process ends), split in equal shares
 * among the call's searches; descriptors are written by kernels.  The call
 * makes no hipMalloc, hipFree, hipHostMalloc or other allocating call.
 *   insts   n <= 64 distinct instances on the current device, created
 *           beforehand (rei_create allocates their staged tables and pinned
 *           result buffers); trivial specifications are answered at once.
 *   out     n results, as for rei_solve_batch; out[i] equals what
 *           rei_solve_batch and rei_solve return for insts[i].
 * The rows of these searches are not kept: rei_row_bits and rei_row_regex
 * return REI_ERR_INVALID_ARG until the instance is solved another way.
 * Errors: REI_ERR_TOO_LARGE when n > 64, when an instance cannot run in the
 * one-workgroup solver (see rei_solve_batch), or when a search outgrows its
 * share (128 MiB / number of searches; call again with fewer instances);
 * rei_last_error of the instance concerned says which.  Calls on one GPU
 * share the array: calls that overlap in time on one GPU race and give
 * undefined results.  Every call writes what it reads before reading it, so
 * no state carries over from the previous call. */
rei_status rei_solve_batch_noalloc(rei_instance *const *insts, size_t n, void *hip_stream, rei_result *out);

/* ---- the batched configuration as one captured graph -------------------------
 * For a fixed set of instances solved again and again (a workload replayed
 * step after step): the batched solver's launches are captured once in a
 * hipGraph and each step is one graph launch.  Every batchable instance
 * (as for rei_solve_batch) keeps its whole search inside the launch: a
 * persistent grid per word width, its workgroups taking instances from a
 * device counter, longest first (their work measured by one eager run at
 * creation), the device's resident workgroups shared between the widths in
 * proportion to their work.  Results equal rei_solve's for every instance.
 *
 * rei_batch_graph_create   prepares every instance's arena (arena_bytes as
 *                          for rei_solve_batch, 0 = 16 MiB), runs the
 *                          launches once to measure, captures the graph.
 *                          The instances (all on the current device) belong
 *                          to the graph until it is destroyed: do not solve
 *                          them otherwise meanwhile.  Trivial
 *                          specifications are answered at results time;
 *                          instances that cannot be batched, and those
 *                          too heavy for one workgroup (see
 *                          rei_batch_graph_outside), run rei_solve's path
 *                          on the worker threads, started by each launch
 *                          beside the replay.
 * rei_batch_graph_launch   enqueues one replay on hip_stream (NULL = the
 *                          null stream) and returns; the previous replay's
 *                          results must have been collected.
 * rei_batch_graph_results  waits for the replay and writes n results (owned
 *                          by the instances, as for rei_solve; seconds_solve
 *                          = time from the launch call until the instance's
 *                          completion flag showed).  An instance that
 *                          outgrew its preallocated rows is solved again on
 *                          rei_solve's path and gets an arena that holds its
 *                          rows for the next replays.
 * rei_batch_graph_error    the message of the last failure ("" if none).
 * rei_batch_graph_destroy  waits for a replay in flight, frees the graph. */
typedef struct rei_batch_graph rei_batch_graph;
rei_status rei_batch_graph_create(rei_instance *const *insts, size_t n, uint64_t arena_bytes,
                                  rei_batch_graph **out);
rei_status rei_batch_graph_launch(rei_batch_graph *g, void *hip_stream);
rei_status rei_batch_graph_results(rei_batch_graph *g, rei_result *out);
const char *rei_batch_graph_error(const rei_batch_graph *g);
void rei_batch_graph_destroy(rei_batch_graph *g);
/* Instances of the graph that run rei_solve's path on worker threads beside
 * each replay instead of inside it: those that cannot be batched, those
 * whose measured work (candidates, weighted by words per language) exceeds
 * twice the average per resident workgroup (and 10^5), which would decide a
 * replay's length alone on one workgroup, and those with a level larger
 * than rei_solve_batch's hand-off size (tuned per word width, else 2^16
 * candidates). */
size_t rei_batch_graph_outside(const rei_batch_graph *g);

/* Autotuner of rei_solve_batch, by whole calls (what the caller waits for,
 * hand-offs included), each setting timed as the shortest of five calls.
 * First the launch shape: every word-width group at 256, 512 and 1024
 * threads per instance (at most 512 with 8 or 16 words per language, 256
 * with 32), the three taking turns, one call each per round; the fastest
 * is kept, for each group present, for groups of its size (by power-of-two
 * size class) in a table of the process that later rei_solve_batch calls on
 * any thread use.  Without an entry, a group gets enough waves per instance
 * to fill the device's wave slots.  Then the hand-off level size (for
 * instances that did not set rei_set_batch_level): one size for every group
 * present, 2^8, 2^10, 2^12, then 2^13 .. 2^19 candidates, the fastest kept;
 * then, widest first, each group of at most 8 instances (as many as run on
 * rei_solve's path at once) tries 0, its instances taking rei_solve's path
 * from the start, kept only if at least 3 % faster.  The sizes become the
 * process defaults per word width (2^16 until tuned).  Other
 * rei_solve_batch calls running meanwhile also take the setting being
 * timed.  Results do not depend on either choice.
 * threads_out (NULL or 7 entries, for W = 1 with keys in the table slots,
 * then W = 1, 2, 4, 8, 16, 32) receives the chosen sizes, 0 for groups
 * without instances; level_max_out (NULL or 7 entries, same order) the
 * chosen level sizes, UINT64_MAX for groups without instances.  The
 * instances end up solved, as by rei_solve_batch. */
rei_status rei_tune_batch(rei_instance *const *insts, size_t n, void *hip_stream, uint64_t arena_bytes,
                          uint32_t *threads_out, uint64_t *level_max_out);

/* Autotuner of rei_solve's per-chunk path, by whole solves: for the
 * instances of each word width present, the first chunk of a level
 * (2^14 .. 2^19 candidates; each next chunk doubles), the largest chunk
 * (2^20 .. 2^24), and the concatenation kernel's grid target (512 .. 8192
 * workgroups) and left rows per workgroup (4 .. 64), one parameter after
 * the other, each value timed as the best of three passes of rei_solve over
 * the width's instances on hip_stream.  The fastest set is kept per word
 * width in a table of the process that later solves of any instance of that
 * width use.  Results do not depend on these parameters.  params_out (NULL
 * or 24 entries: W = 1, 2, 4, 8, 16, 32, each first_chunk, chunk_max,
 * concat_wg, concat_xi; 0 for widths absent) receives the choice.  The
 * instances end up solved, as by rei_solve. */
rei_status rei_tune_grid(rei_instance *const *insts, size_t n, void *hip_stream, uint64_t *params_out);
/* The per-chunk path's launch parameters for one instance, overriding the
 * tuned table for its width (0 = keep the table's or the default value for
 * that field; defaults 2^16, 2^24, 2048, 16).  concat_xi at most 64.
 * Results do not depend on them; tests vary them to check that. */
rei_status rei_set_grid_tuning(rei_instance *inst, uint64_t first_chunk, uint64_t chunk_max,
                               uint32_t concat_wg, uint32_t concat_xi);
/* The process's tuning tables (rei_tune_batch's launch shapes and hand-off
 * size, rei_tune_grid's parameters) written to a JSON file, or read back
 * from one (entries read replace those of the same key; a file with an
 * entry out of range is rejected whole).  A process whose environment sets
 * REI_TUNE_FILE loads that file when its first instance is created.
 * REI_ERR_INVALID_ARG when the file cannot be written or read or parsed. */
rei_status rei_tune_save(const char *path);
rei_status rei_tune_load(const char *path);

/* ---- serving: continuous batching ------------------------------------------
 * A server solves submitted instances asynchronously.  Requests are admitted
 * in arrival order while the device bytes they need fit hbm_budget (0 = the
 * device's free memory when the server is created, less 8 GB kept for
 * everything else), and their device buffers are allocated at admission.
 * Admitted requests that can be batched (as in rei_solve_batch) reach the
 * device in one of two modes (rei_server_set_queue_mode):
 *  - queue mode (default): per word-width group a persistent launch of the
 *    batched solver takes requests from a ring in pinned host memory while
 *    it runs; each admitted request is written into the ring and published,
 *    and the next free workgroup starts it, with no launch in between.  A
 *    launch (one workgroup per eight compute units) ends after its
 *    workgroups found no work for 150 us; the next admitted request of the
 *    group starts another.
 *  - launch mode: admitted requests are launched together on a free stream
 *    from a pool of n_streams (at most max_batch per launch), so requests
 *    arriving while others run are started at once and their work overlaps
 *    on the device.
 * The others (and batched ones that hand off or outgrow their preallocated
 * rows) run rei_solve's path on one of n_workers worker threads, each with
 * its own stream (0 = defaults: 64 per batch, 4 streams, 4 workers).  Each
 * result equals rei_solve's for that instance.  The budget counts the device bytes
 * of requests in flight (an estimate made at submit: the batched arena, or
 * the cache budget plus its table for the per-chunk path); a finished
 * instance keeps its buffers until rei_destroy, so that nothing on the
 * serving path frees device memory (a free waits for the whole device).
 * A submitted instance must not be used by the caller until its ticket
 * reports done.  Calls may come from any host thread. */
typedef struct rei_server rei_server;
rei_status rei_server_create(uint64_t hbm_budget, uint32_t max_batch, uint32_t n_streams,
                             uint32_t n_workers, rei_server **out);
rei_status rei_server_submit(rei_server *srv, rei_instance *inst, uint64_t *ticket);
/* *done = 1 when the ticket's search has ended: then *out (if not NULL) gets
 * its result, *latency_s (if not NULL) the time from submit to completion,
 * the ticket is retired and the return value is the search's status (REI_OK
 * also for REI_NOT_FOUND / REI_OUT_OF_MEMORY outcomes, see out->status).
 * With wait != 0 the call blocks until done. */
rei_status rei_server_poll(rei_server *srv, uint64_t ticket, int wait, int *done, rei_result *out,
                           double *latency_s);
/* Finishes every submitted request, then frees the server. */
void rei_server_destroy(rei_server *srv);
/* Queue mode (enable != 0, the default) or launch mode, as described above.
 * REI_ERR_INVALID_ARG once a request has been submitted. */
rei_status rei_server_set_queue_mode(rei_server *srv, int enable);

/* Free the device memory of the instance's last search (language cache,
 * dedup table, chunk buffers) but keep the staged specification and the
 * last result (its regex and counts).  The next rei_solve allocates again.
 * After it, the inspection calls below have no rows to read.  Waits for the
 * device.  For callers that solve many large instances in turn. */
rei_status rei_trim(rei_instance *inst);

/* Route the device memory of instances created from now on through the
 * caller's allocator, for a framework that owns the device memory (a caching
 * allocator, say) and hands it out.  alloc(bytes,
 * ctx) returns device memory of the current device or NULL on failure (the
 * call then fails with REI_ERR_DEVICE); free_(ptr, ctx) takes back a pointer
 * alloc returned.  An instance keeps the pair it was created with for all its
 * allocations and frees, so the pair and ctx must stay valid until every such
 * instance is destroyed.  The library drains the device after each alloc and
 * before each free_, so the allocator may reuse memory in the order of any
 * stream.  Both NULL restores hipMalloc / hipFree; exactly one NULL is
 * REI_ERR_INVALID_ARG.  Process-wide; thread-safe. */
rei_status rei_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                             void (*free_)(void *ptr, void *ctx), void *ctx);

/* Free the instance and its device memory.  NULL is ignored. */
void rei_destroy(rei_instance *inst);

const char *rei_status_str(rei_status s);
/* Last error message of the instance (empty string if none). */
const char *rei_last_error(const rei_instance *inst);
/* Last error of a failed rei_create on this thread. */
const char *rei_create_error(void);

/* ---- inspection, valid after rei_solve (used by the tests) ---------------- */

/* Word i of ic(P u N) in shortlex order, copied into buf (cap bytes). */
rei_status rei_ic_word(const rei_instance *inst, uint32_t i, char *buf, size_t cap);
/* Number of languages stored in level `cost`. */
rei_status rei_level_size(const rei_instance *inst, uint32_t cost, uint64_t *out);
/* The W words of row i of level `cost` (bit k of word k/64 = membership of
 * ic word k), copied to host memory words_out[W]. */
rei_status rei_row_bits(rei_instance *inst, uint32_t cost, uint64_t i, uint64_t *words_out);
/* A minimal expression for row i of level `cost`, printed as the answer is. */
rei_status rei_row_regex(rei_instance *inst, uint32_t cost, uint64_t i, char *buf, size_t cap);

/* ---- tuning and measurement ------------------------------------------------ */

/* Largest number of candidates processed per chunk (0 = default).  Results
 * do not depend on it; tests vary it to check that. */
rei_status rei_set_chunk(rei_instance *inst, uint64_t max_candidates);
/* Largest level, in candidates, that rei_solve_batch searches inside its
 * one-workgroup solver (0 = the process default for the instance's word
 * width: 2^16, or what rei_tune_batch chose, where 0 means rei_solve's path
 * from the start).  At a larger level the instance,
 * with every lower level kept, continues on rei_solve's path.  Results do not
 * depend on it. */
rei_status rei_set_batch_level(rei_instance *inst, uint64_t max_candidates);
/* Hand-off time of rei_solve_batch: once the instance's workgroup has run
 * this many microseconds, its next level moves to rei_solve's path if it has
 * more than 4096 candidates, so that the deep searches of a batch use the
 * device beside the workgroups of the others; only in batches with fewer
 * instances than the device has compute units (a larger batch leaves none
 * idle).  -1 = the default (500), 0 = never on time (only
 * rei_set_batch_level's size).  The hand-off level then depends on timing;
 * results do not. */
rei_status rei_set_batch_time(rei_instance *inst, int64_t microseconds);
/* Per-character costs (the cost-homomorphism definition allows a different
 * cost for each alphabet character).  costs[a] >= 1 is the cost of the a-th
 * character of the alphabet given to rei_create; n must equal the alphabet
 * size.  Character a enters at level costs[a], before the other blocks of
 * that level, in alphabet order; the smallest of them replaces c_char (the
 * first level, and the cost of the trivial answers ∅ and ε).  Instances with
 * unequal character costs are solved on rei_solve's path by
 * rei_solve_batch.  REI_ERR_INVALID_ARG on a wrong n or a zero cost. */
rei_status rei_set_char_costs(rei_instance *inst, const uint32_t *costs, size_t n);
/* OnTheFly mode (Sec. 3, "OnTheFly mode"), off by default.  When on, the
 * first new language that does not fit the cache budget does not stop the
 * search: from there on candidates are neither stored nor checked for
 * uniqueness, only for precision, while every constructor block drawn on
 * lies in complete (fully stored) levels.  The first block that needs the
 * level where the cache filled, or a later one, ends the search with
 * REI_OUT_OF_MEMORY (a block with a complete, empty operand level has no
 * candidates and is skipped).  An answer found this way is the answer of a
 * search without a cap.  unique_per_level counts stored languages only.
 * Instances with it on are solved on rei_solve's path by rei_solve_batch. */
rei_status rei_set_on_the_fly(rei_instance *inst, int enable);
/* Misclassified examples allowed (REI with error: Sec. 5.2, Future Work,
 * where an expression may misclassify a given share of the examples and
 * the allowed-error table shows the effect on the Table 1 row 1
 * specification); 0 = precise.  An expression is then accepted when it
 * misclassifies at most max_errors examples of P u N. */
rei_status rei_set_max_errors(rei_instance *inst, uint32_t max_errors);

/* Kernel classes timed with HIP events when profiling is on. */
typedef enum {
  REI_K_GEN_CHAR = 0,
  REI_K_GEN_QUESTION,
  REI_K_GEN_STAR,
  REI_K_GEN_CONCAT,
  REI_K_GEN_UNION,
  REI_K_INSERT,
  REI_K_COMPACT,
  REI_K_OTHER,
  REI_K_BATCH,          /* the batched solver (rei_solve_batch), per word width */
  REI_K_GEN_MIXED,      /* small blocks of several constructors in one launch */
  REI_K_COUNT
} rei_kernel_class;

/* Time kernel launches of the next solves with HIP event pairs.  enable = 1:
 * the generator classes and the batched solver, whose launches record the
 * pair at the kernel's own start and end (for rei_solve_batch: each batched
 * launch, counted on insts[0]); enable = 2: every class (the others with
 * events on the stream around the launch); 0: off.  Turning profiling on
 * clears the statistics; turning it off keeps them. */
rei_status rei_set_profiling(rei_instance *inst, int enable);
/* As rei_set_profiling, for the launches of one kernel class only: a caller
 * that needs one class's average launch time leaves every other launch
 * untouched by events.  Clears the statistics; rei_set_profiling(inst, 0)
 * turns it off. */
rei_status rei_set_profiling_class(rei_instance *inst, rei_kernel_class k);
/* Launch count, total device milliseconds and work units (candidates for the
 * generator classes, survivors for REI_K_INSERT) of one kernel class,
 * accumulated over the solves since profiling was enabled. */
rei_status rei_kernel_stats(const rei_instance *inst, rei_kernel_class k, uint64_t *launches,
                            double *ms, uint64_t *units);
/* Testing: keep only the low `bits` bits of every language hash (0 = all 64)
 * on the current device.  Forces table collisions, equal fingerprints (so
 * every probe compares whole languages) and long probe sequences; results
 * do not change, searches get slower.  Process-wide: call only while no
 * search runs. */
rei_status rei_set_hash_bits(uint32_t bits);
/* Shortest time the timing events read for an empty kernel launched the same
 * way (the events a launch records include the dispatch and completion of
 * the launch, which an external kernel trace leaves out), in microseconds.
 * Creates and destroys a stream of its own.  For reading the statistics. */
rei_status rei_timing_overhead(double *us);
/* Achievable peaks on the current device, for reading the roofline figures
 * of the kernels against measured rates as well as published ones.  Each is
 * the best of five timed launches (after one warm-up) of a kernel built for
 * the purpose, on a stream of its own; buffers are allocated and freed
 * inside the call.
 *   REI_PEAK_COPY         copy `size` bytes with 16-byte loads and stores:
 *                         *rate = bytes read + bytes written per second;
 *   REI_PEAK_PROBE        2^27 reads of 8-byte slots at pseudo-random
 *                         positions of a table of `size` bytes (rounded down
 *                         to a power of two; a table larger than the
 *                         device's caches makes every probe an HBM access,
 *                         as a dedup-table probe is): *rate = probes per
 *                         second;
 *   REI_PEAK_PROBE_ATOMIC as REI_PEAK_PROBE, each probe followed by a 64-bit
 *                         atomicMin on another pseudo-random slot (the claim
 *                         of a new language): *rate = probes per second;
 *   REI_PEAK_BITWISE      a loop of fused 32-bit AND-OR operations on every
 *                         lane of a full device (size ignored): *rate =
 *                         32-bit bitwise operations per second (each fused
 *                         instruction counts two).
 * *seconds = the best launch's duration.  REI_ERR_INVALID_ARG for an
 * unknown kind or a size under 4096 bytes; REI_ERR_DEVICE when a HIP call
 * fails (for example a table that does not fit the device). */
typedef enum {
  REI_PEAK_COPY = 0,
  REI_PEAK_PROBE = 1,
  REI_PEAK_PROBE_ATOMIC = 2,
  REI_PEAK_BITWISE = 3
} rei_peak_kind;
rei_status rei_measure_peak(rei_peak_kind kind, uint64_t size, double *rate, double *seconds);
/* Kernel symbol name of a class (for matching profiler output). */
const char *rei_kernel_name(rei_kernel_class k);

#ifdef __cplusplus
}
#endif

#endif /* REI_H */
