// fbg_kernels.h -- kernel argument blocks and launch wrappers (host side).
#ifndef FBG_KERNELS_H
#define FBG_KERNELS_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/fbg.h"
#include "fbg_isa.h"

namespace fbg {

// Registers of the general part held in VGPRs; the rest live in LDS.  The
// jump-table interpreter at 16 words per lane keeps three (its fixed register
// map leaves room for no more without spilling).
constexpr uint32_t kVgprRegs = 4;
constexpr uint32_t kJ16VgprRegs = FBG_J16_VGPR_REGS;
inline uint32_t vgpr_regs_of(int log2w) { return log2w == FBG_J16_LOG2W ? kJ16VgprRegs : kVgprRegs; }

struct EvalArgs {
  const uint32_t *code;   // encoded program: clause block, instructions, pattern table
  uint32_t nins;          // instructions after the clause block (16 words per lane: 2-word units)
  uint32_t nregs;         // registers held in LDS (beyond vgpr_regs_of(log2w))
  int32_t n;              // variables
  uint64_t nslices;       // 2^max(n-5, 0) valid 32-bit words
  uint64_t ntiles;        // ceil(nslices / (64 W))
  uint64_t *out_count;    // MODE_COUNT
  uint32_t *out32;        // MODE_DNF (written); stored-DNF scans (read)
  uint64_t out_slices;    // MODE_DNF: words written (>= nslices, >= 2)
  const uint32_t *xcd_code;  // MODE_DNF at 32 words per lane: the XCD-local encoding, or null
  uint32_t *tile_counts;  // MODE_TILECNT (out), MODE_ENUM (in)
  const uint64_t *tile_offsets;  // MODE_ENUM
  uint64_t *out_idx;      // MODE_ENUM
  uint64_t capacity;      // MODE_ENUM
  // non-zero: the jump-table interpreter (16 words per lane) runs the copy of
  // its table for code off a 64 KiB boundary (same results; for tests)
  uint32_t j16_any = 0;
};

// The XCD-local layout of the batched DNF write-out (32 words per lane, a
// program made of clauses alone, n >= kXcdMinVars, an output 16 bytes
// aligned).  The write-out kernel evaluates a second encoding of the
// program with its variables renamed (xcd_write_out_permutation), so that
// its tile t (64 lanes x 32 words) holds two whole 4 KiB pieces of the DNF
// vector, pieces p and p + 8 (32 KiB apart), p = ((t >> 2) & 7) + 16 (t & 3)
// + 64 (t >> 5), and each lane's words 4g .. 4g+3 are adjacent in memory:
// eight 16-byte stores per lane, each a whole 1 KiB of a piece.  With one
// tile per wave and four waves per block, every block writes 4 KiB pieces of
// one residue class modulo 8 (blocks go to the eight XCDs in turn), so that
// the XCDs write interleaved 4 KiB pieces of one region of the vector at a
// time; HBM takes that faster than the same bytes in plain order or in
// larger pieces per XCD.  The model counts of a tile's two pieces go to
// chunk_counts[2t], [2t + 1]; k_sum_tile_counts adds the two pieces of each
// 8 KiB tile of the vector into the tile counts the batched enumeration
// reads.
constexpr int kXcdMinVars = 21;

struct BatchProg {
  const uint32_t *code;
  uint32_t nins;
  uint32_t nregs;
  int32_t n;
  uint64_t nslices;
  uint64_t ntiles;
  uint32_t *out32;      // MODE_DNF: the program's DNF vector
  uint64_t out_slices;  // MODE_DNF: 32-bit words of out32
  uint32_t *tile_counts;  // MODE_DNF: per-tile model counts (or null)
  // the batched DNF write-out in the XCD-local layout (or null): the program
  // with variables renamed, and the per-piece model counts it writes
  const uint32_t *xcd_code;
  uint32_t *chunk_counts;
};

// One program of a batched enumeration over stored DNF vectors.
struct EnumProg {
  const uint32_t *dnf;  // the DNF vector as 32-bit words
  uint64_t nslices;     // valid 32-bit words
  uint64_t tile0;       // first global tile of the program
  uint64_t *out;        // model indices (capacity entries)
  uint64_t capacity;
  uint32_t log2w;       // tiling of the program's plan
  uint32_t pad;
};

struct BatchEnumArgs {
  const EnumProg *progs;
  uint32_t np;
  uint64_t total_tiles;
  const uint32_t *tile_counts;  // all programs, concatenated
  const uint64_t *offsets;      // exclusive scan of tile_counts
  uint32_t *list;               // tiles holding models (k_list_tiles)
  uint32_t *nlist;              // their number (zeroed before k_list_tiles)
};

struct BatchItem {
  uint32_t prog;    // index into the program table
  uint32_t slot;    // index into the counts array
  uint64_t t0, t1;  // tiles t0, t0 + step, t0 + 2 step, ... below t1
  uint64_t step;
};

// A plan's work items are split over kQueues queues (item i in queue
// i mod kQueues), one per XCD, each with its own head counter kQueueStride
// words (64 bytes) from the next, so that the queue atomics of the eight
// XCDs do not all meet at one address.
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStride = 16;
constexpr uint32_t kHeadWords = kQueues * kQueueStride;

struct BatchArgs {
  const BatchProg *progs;
  const BatchItem *items;
  uint32_t nitems;
  uint32_t max_regs;      // LDS registers per wave (beyond vgpr_regs_of(log2w))
  uint32_t *head;     // kHeadWords words of queue heads, zeroed before the launch
  uint64_t *counts;   // per slot; the kernel adds to it
  uint32_t run = 1;   // k_batch_direct: consecutive tiles per wave
  // registers beyond the max_regs LDS registers (jump-table form only):
  // gstride words of global scratch per wave of the grid, or none
  uint32_t *gscratch = nullptr;
  uint64_t gstride = 0;
  uint32_t j16_any = 0;   // as in EvalArgs
};

enum { EVAL_COUNT = 0, EVAL_DNF = 1, EVAL_TILECNT = 2, EVAL_ENUM = 3 };

hipError_t launch_eval(int mode, int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds,
                       hipStream_t s);
hipError_t launch_dnf_scan(int mode, const EvalArgs &a, int grid, int block, hipStream_t s);
hipError_t launch_batch(int mode, int log2w, int var, const BatchArgs &a, int grid, int block, size_t lds,
                        hipStream_t s);
// The DNF write-out of a plan of clause-only programs without the cofactor,
// a.run consecutive tiles per wave (a.items: one entry per program, [t0, t1) its tiles in the
// plan, ascending; every program has tile counts), then the per-program sums
// of those tile counts into a.counts (sum_blocks blocks per program).
hipError_t launch_batch_direct(int log2w, const BatchArgs &a, int grid, int block, int sum_blocks, hipStream_t s);
// Resident blocks per compute unit of an evaluator or batch launch.
int eval_blocks_per_cu(int mode, int log2w, int var, int block, size_t lds);
int batch_blocks_per_cu(int mode, int log2w, int var, int block, size_t lds);
hipError_t launch_list_tiles(const BatchEnumArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_compact(int log2w, const BatchEnumArgs &a, int grid, int block, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *block_sums, uint64_t *total,
                       hipStream_t s);
uint64_t scan_block_count(uint64_t n);
// p[0..n) = 0 and head[0..nhead) = 0.
hipError_t launch_zero(uint64_t *p, uint64_t n, uint32_t *head, uint32_t nhead, hipStream_t s);
hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s);

// The scratch of fbg_enumerate_noalloc (noalloc.hip): a static device array
// of kNoallocScratchBytes per device, enough for the temporaries of an
// enumeration over at most kNoallocMaxTiles tiles (4-byte tile counts,
// 8-byte offsets, block sums).
constexpr uint64_t kNoallocMaxTiles = FBG_NOALLOC_MAX_TILES;
constexpr uint64_t kNoallocScratchBytes = FBG_NOALLOC_SCRATCH_BYTES;
// Its device address on the current device (looked up once per device).
hipError_t noalloc_scratch(void **out);

}  // namespace fbg

#endif
