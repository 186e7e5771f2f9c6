/*
 * fbg.h -- evaluation of Boolean terms on free Boolean generators, MI355X.
 *
 * Problem (Section 2.3, Proposition "prop22"): for a Boolean term
 * t(x0..x{n-1}) and the free generators b_0..b_{n-1} of the algebra 2^(2^n)
 * (Section 2.2: generator k is row k of the matrix whose columns are the
 * binary expansions of 0..2^n-1), the vector d = t(b_0..b_{n-1}) codes the
 * full DNF of t: bit mu of d is t at the valuation mu.  The number of 1-bits
 * of d is the number of models of t (Section 3.2, l_{T,n}), and the positions
 * of the 1-bits are the models themselves (a system of equations phi_i = 1
 * has exactly those solutions, Section 5.1).  The method computes d block by
 * block on wide bitwise processors (Section 2.3, time T = 2^(l+n-k-r) delta).
 *
 * Conventions used by every call:
 *  - variable xk is bit k of the valuation index mu (least significant first);
 *  - the DNF vector is an array of uint64 words; word w holds valuations
 *    64w .. 64w+63, valuation mu at bit (mu & 63).  It has max(1, 2^(n-6))
 *    words; bits at or above 2^n are zero;
 *  - formula text: statements separated by newlines or ';', '#' comments.
 *    "name = expr" defines a temporary; a bare "expr" is an assertion and the
 *    formula is the conjunction of all assertions (at least one).  Operators
 *    are the Python ones of the paper's scripts (Section 4.2): '~' not, '&'
 *    and, '^' symmetric difference (the paper's '+'), '|' or, with Python
 *    precedence ~ > & > ^ > |; parentheses; constants 0 and 1 (removed by
 *    constant folding, the paper's Reduction of Section 4.1); variables
 *    x0 .. x{n-1}.
 *
 * Memory and streams: device pointers are caller-owned device memory (for
 * example torch tensors' data_ptr()); `stream` is a hipStream_t (NULL = the
 * legacy default stream).  Every compute call is asynchronous on `stream`:
 * results are valid once the stream is synchronised.  Argument errors are
 * reported synchronously and nothing is launched.  A program is immutable
 * after fbg_compile and may be used from several streams at once.
 *
 * Errors: every call returns an fbg_status; on failure fbg_last_error() (per
 * thread) describes it and fbg_last_error_offset() gives the byte offset of a
 * parse error (-1 otherwise).
 */
#ifndef FBG_H
#define FBG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FBG_OK = 0,
  FBG_E_INVAL = -1,   /* bad argument (null pointer, too-small buffer, ...) */
  FBG_E_PARSE = -2,   /* malformed formula text */
  FBG_E_RANGE = -3,   /* n out of range, variable >= n, program too large */
  FBG_E_NOMEM = -4,   /* host or device allocation failed */
  FBG_E_DEVICE = -5   /* HIP error (launch, copy, no device) */
} fbg_status;

/* Largest n accepted by fbg_count / fbg_enumerate / batches, and by
   fbg_eval_dnf (whose output has 2^(n-6) words). */
#define FBG_MAX_VARS 48
#define FBG_MAX_DNF_VARS 40

/* Largest number of variables in the text given to fbg_compile_assume (the
   free ones must still number at most FBG_MAX_VARS). */
#define FBG_MAX_TEXT_VARS 65536

/* Largest number of words (32-bit slices) one lane evaluates per tile. */
#define FBG_MAX_WORDS_PER_LANE 32

typedef struct fbg_program fbg_program; /* opaque, library-owned */
typedef struct fbg_batch fbg_batch;     /* opaque, library-owned */

/* Metadata of a compiled program (Section 2.3 time model: the node count l
   and the work per valuation).  Used as `struct fbg_program_info`: the tag
   shares its name with the call fbg_program_info below. */
struct fbg_program_info {
  int32_t n_vars;        /* n: the valuation space is 2^n */
  int32_t const_value;   /* -1, or 0/1 when the formula folds to a constant */
  uint64_t l2in;         /* 2-input AND/OR/XOR operations of the term after
                            constant folding, hashing and dead-code removal
                            (NOT is not counted): the node count of the time
                            model of Section 2.3 */
  int32_t n_instr;       /* clauses plus the instructions after them */
  int32_t n_regs;        /* registers the general part needs (the first four
                            live in VGPRs, the rest in LDS) */
  int32_t n_clause_instr;/* leading clauses (OR-sets conjoined directly; they
                            form the clause block of the encoding) */
  int32_t words_per_lane;/* tuning the library picked for this program */
  uint64_t dnf_words;    /* max(1, 2^(n-6)) */
  uint64_t code_bytes;   /* device memory the program holds (0 without a
                            device): all tilings' encodings and tables */
  double l_valu;         /* VALU instructions the evaluator issues per 32-bit
                            slice (one lane, one word) for this program at
                            words_per_lane: a static count over the encoded
                            program (clause block, product tree, general
                            instructions), per tile divided by the words per
                            lane; the popcount and store epilogue excluded */
};

/* Launch tuning.  Zero fields mean "let the library choose". */
typedef struct {
  int32_t words_per_lane;  /* 1, 2, 4, 8, 16 or 32 (32-bit words per lane per tile) */
  int32_t grid_blocks;     /* grid size in blocks (capped at one wave per tile or
                              item); 0: as many as stay resident, except for
                              fbg_eval_dnf without the cofactor: one wave per tile */
  int32_t flags;           /* FBG_TUNE_* */
  int32_t direct_run;      /* fbg_batch_eval_dnf of clause-only programs (one
                              wave per run of tiles on fresh blocks): tiles
                              per run, 1..64; 0: the library's choice (1 when
                              a program takes the XCD-local layout, else 4) */
} fbg_tune;

/* Uniform-cofactor evaluation: the index bits above the lane and word bits
   are constant on a tile, so clauses with a true tile literal are skipped and
   a clause made only of false tile literals ends the tile.  Same results;
   data-dependent (usually much smaller) work. */
#define FBG_TUNE_COFACTOR 1

/* Compile flags: the tilings to encode.  A program is encoded once per
   tiling (1, 2, 4, 8, 16 and 32 words per lane), which is most of a short
   program's compile time; a caller that only ever runs it at known tilings
   (a server at a fixed tiling) asks for those alone.  flags = 0 encodes
   every tiling.  A call at a tiling the program was not encoded for
   (words_per_lane of fbg_tune, a batch, a server, fbg_program_emulate,
   fbg_program_disasm) fails with FBG_E_INVAL; the library's own default
   tiling is always one that was encoded. */
#define FBG_COMPILE_WPL(words_per_lane_log2) (1u << (words_per_lane_log2))
#define FBG_COMPILE_WPL_MASK 0x3Fu

/*
 * fbg_compile -- turn formula text into a straight-line bitwise program and
 * upload it to the current HIP device (Section 4.1: the engine builds a
 * computing tree for the formula; Reduction removes constants).
 *   src     NUL-terminated formula text (format above).
 *   n_vars  n, 0 <= n <= FBG_MAX_VARS; every variable used must be < n.
 *           Variables below n that do not occur still index valuations.
 *   flags   0, or an OR of FBG_COMPILE_WPL(k): encode only those tilings.
 *           Other bits: FBG_E_INVAL.
 *   out     receives the program; free it with fbg_program_free.
 * Errors: FBG_E_PARSE (with offset), FBG_E_RANGE, FBG_E_INVAL, FBG_E_NOMEM,
 * FBG_E_DEVICE.  Synchronous.
 */
fbg_status fbg_compile(const char *src, int32_t n_vars, uint32_t flags, fbg_program **out);

/*
 * fbg_compile_assume -- fbg_compile with killed variables (Section 3.3: a
 * theory that fixes the value of a letter removes it from the search space;
 * Section 3.4, step 3 of the counting procedure: each c-partition kills a set
 * of letters; the reduced theory follows by substitution and Reduction,
 * Section 4.1).
 *   src     formula text over x0..x{n_vars-1}.
 *   n_vars  0 <= n_vars <= FBG_MAX_TEXT_VARS.
 *   assume  host array of n_vars entries (caller-owned, read during the
 *           call): 0 or 1 kills xk to that constant, -1 leaves it free.  May
 *           be NULL only when n_vars = 0.
 *   flags   as fbg_compile.
 *   out     the program over the f free variables, renumbered in increasing
 *           order: bit j of a valuation index is the j-th free variable.
 * FBG_E_INVAL for an entry outside {-1, 0, 1}, FBG_E_RANGE if f exceeds
 * FBG_MAX_VARS; otherwise as fbg_compile.  Synchronous.
 */
fbg_status fbg_compile_assume(const char *src, int32_t n_vars, const int8_t *assume, uint32_t flags,
                              fbg_program **out);

/* Entries of the substitution of fbg_compile_subst besides variable indices. */
#define FBG_SUBST_ZERO (-1)
#define FBG_SUBST_ONE (-2)

/*
 * fbg_compile_subst -- fbg_compile after a substitution of the variables:
 * letters replaced by constants (killing, Section 3.3) or identified with
 * one another.  Identifying the letters of each orbit of a permutation of the
 * domain gives the theory of the models that the permutation fixes, which
 * the Frobenius-Burnside counting lemma of Section 3.2 sums over.
 *   src     formula text over x0..x{n_vars-1}.
 *   n_vars  0 <= n_vars <= FBG_MAX_TEXT_VARS.
 *   subst   host array of n_vars entries (read during the call):
 *           FBG_SUBST_ZERO / FBG_SUBST_ONE put the constant in place of xk,
 *           j in [0, n_free) puts the program's variable j (several letters
 *           may map to one j).  May be NULL only when n_vars = 0.
 *   n_free  the program's variables, 0 <= n_free <= FBG_MAX_VARS; a j that
 *           no letter maps to still indexes valuations (and doubles counts).
 *   flags   as fbg_compile.
 * FBG_E_INVAL for an entry outside [-2, n_free); otherwise as fbg_compile.
 * Synchronous.
 */
fbg_status fbg_compile_subst(const char *src, int32_t n_vars, const int32_t *subst, int32_t n_free, uint32_t flags,
                             fbg_program **out);

/* Release a program and its device copy.  NULL is a no-op.  The caller must
   make sure no launch that uses it is still pending. */
void fbg_program_free(fbg_program *p);

/*
 * fbg_program_info -- metadata of a compiled program: n, the node count
 * L_2in of the time model (Section 2.3), L_valu, registers, tiling, sizes.
 *   out  host memory, written in full.
 * FBG_E_INVAL for a NULL argument.  Synchronous; no device work.
 * fbg_program_get_info is the same call under its earlier name.
 */
fbg_status fbg_program_info(const fbg_program *p, struct fbg_program_info *out);
fbg_status fbg_program_get_info(const fbg_program *p, struct fbg_program_info *out);

/* Make tune->words_per_lane (non-zero) the program's default tiling, and
   tune->flags (FBG_TUNE_COFACTOR) its default evaluation variant, for
   fbg_count, fbg_eval_dnf, fbg_enumerate and new batches (the autotuner's
   hook).  FBG_E_RANGE if the program's registers do not fit in LDS at that
   tiling.  Not synchronised with launches in flight on other threads. */
fbg_status fbg_program_set_tuning(fbg_program *p, const fbg_tune *tune);

/*
 * fbg_eval_dnf -- write d = t(b_0..b_{n-1}) (Proposition "prop22") into
 * d_out[0 .. max(1, 2^(n-6))), layout above.
 *   d_out      device pointer, caller-owned, 8-byte aligned.
 *   out_words  capacity of d_out in words; must be >= max(1, 2^(n-6)).
 * n <= FBG_MAX_DNF_VARS.  A program made only of clauses with n >= 21, at 32
 * words per lane without the cofactor, into a d_out 16 bytes aligned, is
 * evaluated in a second encoding whose tiles are pairs of 4 KiB pieces of d
 * written as 16-byte groups, each block of waves writing the pieces of one
 * residue class modulo 8 (one per XCD); the result is the same vector, and
 * it is written fastest when d_out is 32 KiB aligned.
 */
fbg_status fbg_eval_dnf(const fbg_program *p, uint64_t *d_out, uint64_t out_words, void *stream);

/*
 * fbg_count -- *d_count = number of 1-bits of d, i.e. the number of models
 * (Section 3.2: l_{T,n} is the number of 1-bits of b).  Overwrites *d_count
 * (device pointer to one uint64).  No device memory is allocated.
 */
fbg_status fbg_count(const fbg_program *p, uint64_t *d_count, void *stream);

/*
 * fbg_enumerate -- the models, i.e. the positions mu of the 1-bits of d in
 * ascending order (Section 3.2: every model of T* is read off b; the paper
 * writes all solutions to out.txt, Section 4.2).
 *   d_idx     device array of `capacity` uint64; receives the first
 *             min(total, capacity) model indices, ascending.  May be NULL
 *             when capacity is 0.
 *   d_total   device pointer to one uint64; receives the total number of
 *             models (also when it exceeds capacity).
 * Allocates temporary device memory on `stream` (stream-ordered) for the
 * per-tile counts and offsets.
 */
fbg_status fbg_enumerate(const fbg_program *p, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total,
                         void *stream);

/*
 * Batches (Section 2.3: 2^r processors act as one wide processor; Section
 * 4.1: the search space is sliced into blocks by the available processors).
 * A batch packs the tiles of many programs into one work queue served by one
 * persistent launch, largest work first.
 *
 * fbg_batch_create -- build and upload the work plan for `np` programs.
 *   ps     array of np program pointers (the programs must outlive the batch).
 *   tune   NULL for automatic tuning, else fixed words_per_lane / grid.
 * fbg_batch_count -- d_counts[i] = number of models of ps[i], i < np
 *   (overwritten).  One zero-fill kernel and one persistent kernel on
 *   `stream`; allocates nothing, so it may be captured into a HIP graph.
 *   Concurrent fbg_batch_count calls on one batch object race (it holds the
 *   queue head); use one batch object per stream.
 * fbg_count_batch -- create, count and free in one call (allocates).
 */
fbg_status fbg_batch_create(const fbg_program *const *ps, int32_t np, const fbg_tune *tune, fbg_batch **out);
fbg_status fbg_batch_count(fbg_batch *b, uint64_t *d_counts, void *stream);
void fbg_batch_free(fbg_batch *b);

/*
 * fbg_batch_count_graph -- as fbg_batch_count, replayed from a HIP graph:
 * the first call for a given d_counts captures the two launches (on a
 * private stream) and instantiates the graph; later calls launch the graph on
 * `stream`.  A different d_counts re-captures.  Same ordering rules as
 * fbg_batch_count (one batch object per stream).
 */
fbg_status fbg_batch_count_graph(fbg_batch *b, uint64_t *d_counts, void *stream);

/*
 * fbg_batch_set_dnf_outputs -- fix, for every program of the batch, the
 * device buffer that fbg_batch_eval_dnf writes its DNF vector into (Section
 * 2.3: one pass evaluates all blocks of every formula of the batch).
 *   d_outs     host array of np device pointers (caller-owned buffers; the
 *              array itself is read during the call only).
 *   out_words  host array of np sizes in uint64 words; out_words[i] must be
 *              at least max(1, 2^(n_i - 6)), and n_i <= FBG_MAX_DNF_VARS.
 * Synchronous (uploads a table); must not run while a launch of this batch
 * is pending.  May be called again to change the buffers.
 * fbg_batch_eval_dnf -- for every program i: its DNF vector into d_outs[i]
 *   (layout as fbg_eval_dnf) and d_counts[i] = its number of models
 *   (overwritten), computing each word once: one launch per plan.  Once the
 *   tile counts exist (fbg_batch_set_enum_outputs), a plan of clause-only
 *   programs without the cofactor runs on a grid of fresh blocks, one run of
 *   tiles per wave (programs with n >= 21 in the XCD-local layout described
 *   at fbg_eval_dnf, one tile per wave), and its counts are summed from the
 *   tile counts by a second small launch; other plans run persistent waves
 *   over work queues.  FBG_E_INVAL if no outputs were set.  Allocates
 *   nothing.
 */
fbg_status fbg_batch_set_dnf_outputs(fbg_batch *b, uint64_t *const *d_outs, const uint64_t *out_words);
fbg_status fbg_batch_eval_dnf(fbg_batch *b, uint64_t *d_counts, void *stream);

/*
 * fbg_batch_set_enum_outputs -- where fbg_batch_enumerate writes the models
 * of every program (Section 3.2: the models are the set bits of the DNF
 * vector, read here in ascending order).  Call after
 * fbg_batch_set_dnf_outputs; from then on fbg_batch_eval_dnf also records
 * the number of models of every tile.
 *   d_idx     host array of np device pointers (caller-owned), program i
 *             receives at most capacity[i] uint64 indices; NULL allowed
 *             when capacity[i] = 0.
 *   capacity  host array of np capacities.
 * Synchronous (allocates the tile-count, offset and piece-count buffers once
 * and uploads a table); must not run while a launch of this batch is
 * pending.
 * fbg_batch_enumerate -- after fbg_batch_eval_dnf on the same stream: the
 *   first min(count_i, capacity_i) models of every program i, ascending,
 *   into d_idx[i] (count_i is d_counts[i] of that call).  One scan over the
 *   tile counts of all programs, then one compaction launch per plan that
 *   reads only the tiles holding models.  Allocates nothing.
 */
fbg_status fbg_batch_set_enum_outputs(fbg_batch *b, uint64_t *const *d_idx, const uint64_t *capacity);
fbg_status fbg_batch_enumerate(fbg_batch *b, void *stream);
fbg_status fbg_count_batch(const fbg_program *const *ps, int32_t np, uint64_t *d_counts, const fbg_tune *tune,
                           void *stream);

/*
 * fbg_enumerate_noalloc -- fbg_enumerate for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Same arguments, outputs, order and errors as
 * fbg_enumerate, same kernels; the temporaries (per-tile model counts, their
 * exclusive scan, block sums) live in a static device array of
 * FBG_NOALLOC_SCRATCH_BYTES on each device (held until the process ends)
 * instead of a stream-ordered allocation, so the call allocates nothing.
 * FBG_E_RANGE when the program has more than FBG_NOALLOC_MAX_TILES tiles at
 * its tiling (64 * words_per_lane 32-bit words per tile: n <= 36 at 32 words
 * per lane).  Every call on one device shares that device's array: calls
 * that overlap on one device, on any streams, race and must be serialised
 * by the caller.  Nothing in the array needs clearing between calls (every
 * word is written before it is read).
 */
#define FBG_NOALLOC_MAX_TILES (1ull << 20)
#define FBG_NOALLOC_SCRATCH_BYTES ((12ull << 20) + (64ull << 10))
fbg_status fbg_enumerate_noalloc(const fbg_program *p, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total,
                                 void *stream);

/*
 * fbg_enumerate_dnf -- the models read off a stored DNF vector (Section 3.2:
 * all models of T* come from b), in ascending order: the same outputs and
 * conventions as fbg_enumerate, for a vector d_dnf of max(1, 2^(n-6)) words
 * that a previous fbg_eval_dnf wrote (bits at or above 2^n must be zero).
 * Reads 2^n/8 bytes instead of evaluating the program again.  n <=
 * FBG_MAX_DNF_VARS.  Allocates temporary device memory on `stream`.
 */
fbg_status fbg_enumerate_dnf(const uint64_t *d_dnf, int32_t n_vars, uint64_t *d_idx, uint64_t capacity,
                             uint64_t *d_total, void *stream);

/*
 * Serving (continuous batching of many requests on one GPU; the slicing of
 * the search space into blocks of Section 4.1 applied across requests).
 *
 * A request's valuation space is cut into tiles of 64 * words_per_lane
 * 32-bit words; fbg_program_tiles gives their number (0 for a bad argument).
 * A work item names a program of the launch (`prog`, index into ps), a
 * counter (`slot`, index into d_counts) and a tile range [tile_begin,
 * tile_end).  fbg_server_launch adds the models found in every item to
 * d_counts[slot] (it does not clear them), so one request may be spread over
 * many launches and many requests share one launch.
 *
 * fbg_server_create -- staging for up to max_programs programs and max_items
 *   items per launch, nbuf launches in flight (pinned host and device buffers
 *   allocated here, once).  words_per_lane fixes the tile size; flags takes
 *   FBG_TUNE_COFACTOR.
 * fbg_server_launch -- upload the cleared queue heads, the program table and
 *   the items (one asynchronous copy from pinned memory) and launch one
 *   persistent batched kernel on `stream`.
 *   Items are cut into pieces of about equal estimated cost (at most
 *   max_items pieces in all) so that a few large requests still occupy
 *   every compute unit.
 *   Items are validated on the host (FBG_E_INVAL on a bad index or range).
 *   A staging buffer is reused only after its previous launch has finished.
 *   Not thread-safe: one server object per host thread.
 * fbg_server_free -- waits for the launches in flight, then releases.
 */
typedef struct {
  int32_t prog;
  int32_t slot;
  uint64_t tile_begin;
  uint64_t tile_end;
} fbg_item;

typedef struct fbg_server fbg_server; /* opaque, library-owned */

uint64_t fbg_program_tiles(const fbg_program *p, int32_t words_per_lane);
fbg_status fbg_server_create(int32_t max_programs, int32_t max_items, int32_t words_per_lane, int32_t nbuf,
                             int32_t flags, fbg_server **out);
fbg_status fbg_server_launch(fbg_server *s, const fbg_program *const *ps, int32_t np, const fbg_item *items,
                             int32_t nitems, uint64_t *d_counts, int32_t ncounts, void *stream);
void fbg_server_free(fbg_server *s);

/*
 * Tuned single-program variants: as fbg_count / fbg_eval_dnf but with an
 * explicit tuning (used by the autotuner and by tests that sweep tilings).
 */
fbg_status fbg_count_tuned(const fbg_program *p, uint64_t *d_count, const fbg_tune *tune, void *stream);
fbg_status fbg_eval_dnf_tuned(const fbg_program *p, uint64_t *d_out, uint64_t out_words, const fbg_tune *tune,
                              void *stream);

/*
 * fbg_program_emulate -- run the encoded device program of `p` for the given
 * words_per_lane on the host, slice by slice, exactly as the kernels
 * interpret it (the uniform-cofactor reading when the program's default
 * tuning selects it, fbg_program_set_tuning), and write the DNF words
 * (h_dnf, host memory, >= dnf_words) and/or the count (h_count).  The result
 * does not depend on the words per lane or the reading; comparing them
 * checks the encoder.  A debugging aid for the compiler and encoder,
 * never used by the calls above.  n <= 30.
 */
fbg_status fbg_program_emulate(const fbg_program *p, int32_t words_per_lane, uint64_t *h_dnf, uint64_t out_words,
                               uint64_t *h_count);

/* Human-readable listing of the encoded program (host memory, NUL-terminated,
   truncated to `cap` bytes).  Returns the full length. */
int64_t fbg_program_disasm(const fbg_program *p, int32_t words_per_lane, char *buf, int64_t cap);

const char *fbg_last_error(void);
int64_t fbg_last_error_offset(void);

/* Library version string. */
const char *fbg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FBG_H */
