// capi.cpp -- the C ABI of include/fbg.h: program residency, launch
// geometry, work plans for batches and serving, and argument checking.
#include <hip/hip_runtime_api.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fbg.h"
#include "fbg_internal.h"
#include "fbg_kernels.h"

namespace {

thread_local std::string g_err;
thread_local int64_t g_err_off = -1;

fbg_status fail(fbg_status st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  g_err_off = -1;
  return st;
}

fbg_status hip_fail(hipError_t e, const char *what) {
  return fail(FBG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kMaxLog2W = 5;
constexpr int kWavesPerBlock = 4;
constexpr size_t kMaxLdsPerBlock = 64 * 1024;
// Consecutive tiles per wave of the one-wave-per-tile DNF write-out of a batch
// plan (C1, 16 x 2^32 bits at W = 32: 1.45-1.46 ms at 4, 1.48 at 1, 1.58 at 2
// and 1.59 at 8).
constexpr uint32_t kDirectRun = 4;
// LDS registers a wave of a batch plan keeps at 16 words per lane (4 KiB
// each): four waves a block then take 32 KiB, so LDS allows the four blocks
// per CU that the registers of the jump-table interpreter allow.
constexpr uint32_t kJ16LdsRegs = 2;

int g_cu_count[64];
std::once_flag g_cu_once[64];

int cu_count(int dev) {
  if (dev < 0 || dev >= 64) return 256;
  std::call_once(g_cu_once[dev], [dev] {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    g_cu_count[dev] = v;
  });
  return g_cu_count[dev];
}

uint64_t slices_of(int n) { return n >= FBG_SLICE_BITS ? (1ull << (n - FBG_SLICE_BITS)) : 1ull; }
uint64_t dnf_words_of(int n) { return n >= 6 ? (1ull << (n - 6)) : 1ull; }
uint64_t tiles_of(uint64_t nslices, int log2w) {
  const uint64_t per = 64ull << log2w;
  return (nslices + per - 1) / per;
}

// Registers beyond the first kVgprRegs live in LDS: W*64 words each per wave.
uint32_t lds_regs(uint32_t nregs, int log2w) {
  const uint32_t v = fbg::vgpr_regs_of(log2w);
  return nregs > v ? nregs - v : 0u;
}
size_t lds_per_wave(uint32_t nregs, int log2w) { return (size_t)lds_regs(nregs, log2w) * (64u << log2w) * 4u; }

// Device memory for programs: size classes of powers of two (>= 4 KiB) carved
// out of 64 MiB chunks and recycled through free lists, so that compiling a
// request costs one small copy and no hipMalloc.  One arena per device.
class CodeArena {
 public:
  static CodeArena &of(int dev) {
    static std::mutex m;
    static std::vector<CodeArena *> arenas;
    std::lock_guard<std::mutex> g(m);
    if ((size_t)dev >= arenas.size()) arenas.resize((size_t)dev + 1, nullptr);
    if (!arenas[(size_t)dev]) arenas[(size_t)dev] = new CodeArena();
    return *arenas[(size_t)dev];
  }

  hipError_t alloc(size_t bytes, void **out, int &cls) {
    std::lock_guard<std::mutex> g(mu_);
    cls = 12;
    while (((size_t)1 << cls) < bytes) cls++;
    const size_t sz = (size_t)1 << cls;
    if (sz > kChunk) {  // very large programs get their own allocation
      cls = -1;
      return hipMalloc(out, bytes);
    }
    auto &fl = free_[(size_t)cls];
    if (!fl.empty()) {
      *out = fl.back();
      fl.pop_back();
      return hipSuccess;
    }
    if (!cur_ || used_ + sz > kChunk) {
      void *c = nullptr;
      hipError_t e = hipMalloc(&c, kChunk);
      if (e != hipSuccess) return e;
      cur_ = (char *)c;
      used_ = 0;
    }
    *out = cur_ + used_;
    used_ += sz;
    return hipSuccess;
  }

  void release(void *p, int cls) {
    if (!p) return;
    if (cls < 0) {
      (void)hipFree(p);
      return;
    }
    std::lock_guard<std::mutex> g(mu_);
    free_[(size_t)cls].push_back(p);
  }

 private:
  static constexpr size_t kChunk = (size_t)64 << 20;
  std::mutex mu_;
  char *cur_ = nullptr;
  size_t used_ = 0;
  std::vector<void *> free_[64];
};

fbg_status parse_wpl(int w, int &log2w) {
  if (w < 1 || w > FBG_MAX_WORDS_PER_LANE || (w & (w - 1)))
    return fail(FBG_E_INVAL, "words_per_lane must be 1, 2, 4, 8, 16 or 32 (got %d)", w);
  log2w = __builtin_ctz((unsigned)w);
  return FBG_OK;
}

}  // namespace

struct fbg_program {
  fbg::Compiled c;
  int device = -1;  // -1: compiled without a device (host only)
  uint32_t *d_code = nullptr;
  int code_class = 0;  // size class in the device's code arena
  uint64_t code_bytes = 0;  // bytes held on the device
  std::vector<uint32_t> words[kMaxLog2W + 1];
  uint64_t dev_off[kMaxLog2W + 1] = {0, 0, 0, 0, 0, 0};
  uint32_t nins[kMaxLog2W + 1] = {0, 0, 0, 0, 0, 0};
  uint32_t tilings = FBG_COMPILE_WPL_MASK;  // bit l: encoded for 2^l words per lane
  bool has_tiling(int l) const { return (tilings >> l) & 1u; }
  // programs of clauses alone with n >= kXcdMinVars: the 32-words-per-lane
  // encoding with variables renamed for the XCD-local DNF write-out
  std::vector<uint32_t> words_xcd;
  uint64_t dev_off_xcd = 0;
  bool has_xcd = false;
  double j16_cost = 0;  // per tile at 16 words per lane, from the jump-table form (0: none)
  uint32_t ncl = 0;  // leading clause instructions
  int auto_log2w = 0;
  uint64_t nslices = 1;
  bool cofactor = false;  // default evaluation variant (fbg_program_set_tuning)
  bool general() const { return c.code.size() > ncl; }
  // kernel variant: bit 0 = general code after the clauses, bit 1 = cofactor
  int variant(const fbg_tune *tune) const {
    const bool cof = cofactor || (tune && (tune->flags & FBG_TUNE_COFACTOR));
    return (general() ? 1 : 0) | (cof ? 2 : 0);
  }
};

struct fbg_batch {
  // One persistent launch per plan: programs made only of clauses run at
  // their own (wide) tiling, general programs at a narrower one whose
  // registers fit; a batch holds one or two plans.
  struct Plan {
    int log2w = 0;
    int var = 0;
    int grid = 1, grid_dnf = 1;
    int block = 256;
    size_t lds = 0;
    uint32_t nitems = 0;
    uint32_t max_regs = 0;  // LDS registers per wave
    fbg::BatchItem *d_items = nullptr;
    // clause-only programs without the cofactor: the DNF write-out runs one
    // wave per tile over this table (one entry per program, its tiles in the
    // plan's order) once the tile counts exist (fbg_batch_set_enum_outputs)
    fbg::BatchItem *d_direct = nullptr;
    uint32_t ndirect = 0;
    uint64_t ntiles = 0, max_prog_tiles = 0;
    uint32_t direct_run = kDirectRun;  // tiles per wave of the direct write-out
    // jump-table form (16 words per lane): registers beyond the plan's LDS
    // registers, gstride words per wave of the grid
    uint32_t *d_gscratch = nullptr;
    uint64_t gstride = 0;
  };
  int device = -1;
  int32_t np = 0;
  std::vector<Plan> plans;
  fbg::BatchProg *d_progs = nullptr;
  fbg::BatchProg *d_progs_dnf = nullptr;  // with DNF outputs (fbg_batch_set_dnf_outputs)
  std::vector<fbg::BatchProg> host_progs;
  std::vector<fbg::BatchProg> host_dnf;   // host copy of d_progs_dnf
  // batched enumeration (fbg_batch_set_enum_outputs): per-tile counts written
  // by fbg_batch_eval_dnf, their scan, and the per-program output table
  std::vector<int> plan_of;               // plan index of every program
  uint64_t total_tiles = 0;
  uint32_t *d_tile_counts = nullptr;
  uint32_t *d_chunk_counts = nullptr;     // XCD-local write-out: counts per 4 KiB piece
  uint64_t *d_offsets = nullptr;
  uint64_t *d_scan_blk = nullptr;
  uint32_t *d_tile_list = nullptr;        // tiles holding models, then their number
  fbg::EnumProg *d_enum = nullptr;
  uint32_t *d_head = nullptr;             // kHeadWords of queue heads per plan (at most 4 plans)
  // captured graph of (zero fill, persistent kernels) for one counts pointer
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t *graph_counts = nullptr;
};

// Bytes of queue heads at the start of a server slot: kHeadWords words,
// rounded to whole 256-byte blocks so that the program table that follows
// starts on its own cache lines.
constexpr size_t kServerHeadBytes = (fbg::kHeadWords * sizeof(uint32_t) + 255) / 256 * 256;

struct fbg_server {
  int device = -1;
  int log2w = 0;
  int32_t max_programs = 0, max_items = 0, nbuf = 0, next = 0;
  bool cofactor = false;
  // A slot's staging (pinned) and device buffers hold, in this order, the
  // kHeadWords queue heads (zero in the staging copy), the slice's program
  // table and its pieces, so that one copy uploads the slice and clears its
  // heads.
  struct Slot {
    char *h = nullptr;  // pinned staging
    char *d = nullptr;  // device copy
    hipEvent_t done = nullptr;
    bool used = false;
  };
  std::vector<Slot> slots;
};

namespace {

// Largest words-per-lane that still gives every wave of a full grid a tile,
// within the LDS budget of the program's registers.
int pick_log2w(uint64_t nslices, uint32_t nregs, bool general, int dev) {
  const uint64_t waves = (uint64_t)cu_count(dev) * 32;  // 8 waves per SIMD
  int best = 0;
  // Programs with a general part: the jump-table interpreter at 16 words per
  // lane (four waves per SIMD) whenever every compute unit gets a few tiles;
  // below that the plain interpreter, which beyond 8 words per lane loses
  // more occupancy than it gains.
  if (general && lds_per_wave(nregs, FBG_J16_LOG2W) <= kMaxLdsPerBlock &&
      tiles_of(nslices, FBG_J16_LOG2W) >= (uint64_t)cu_count(dev) * 4)
    return FBG_J16_LOG2W;
  for (int l = general ? 3 : kMaxLog2W; l >= 0; l--) {
    if (lds_per_wave(nregs, l) > kMaxLdsPerBlock) continue;
    if (tiles_of(nslices, l) >= waves || l == 0) {
      best = l;
      break;
    }
  }
  while (best > 0 && lds_per_wave(nregs, best) > kMaxLdsPerBlock) best--;
  return best;
}

struct Geometry {
  int log2w, grid, block;
  size_t lds;
};

fbg_status block_shape(uint32_t nregs, int l, int &wpb, size_t &lds) {
  const size_t lw = lds_per_wave(nregs, l);
  wpb = kWavesPerBlock;
  if (lw * wpb > kMaxLdsPerBlock) wpb = 1;
  if (lw * wpb > kMaxLdsPerBlock)
    return fail(FBG_E_RANGE, "program needs %u registers x %d words per lane: %zu bytes of LDS per wave (max %zu)",
                nregs, 1 << l, lw, kMaxLdsPerBlock);
  lds = lw * wpb;
  return FBG_OK;
}

// FBG_E_INVAL unless the program was encoded for 2^l words per lane.
fbg_status check_tiling(const fbg_program *p, int l) {
  if (!p->has_tiling(l))
    return fail(FBG_E_INVAL, "the program was compiled without %d words per lane (FBG_COMPILE_WPL)", 1 << l);
  return FBG_OK;
}

// Launch shape of an evaluator kernel: a persistent grid of exactly the
// blocks that can be resident at once (more would only queue behind them and
// finish in a tail), each wave striding over the tiles.
fbg_status geometry(const fbg_program *p, const fbg_tune *tune, int mode, Geometry &g) {
  int l = p->auto_log2w;
  fbg_status st;
  if (tune && tune->words_per_lane && (st = parse_wpl(tune->words_per_lane, l))) return st;
  if ((st = check_tiling(p, l))) return st;
  int wpb;
  if ((st = block_shape((uint32_t)p->c.nregs, l, wpb, g.lds))) return st;
  const uint64_t ntiles = tiles_of(p->nslices, l);
  const uint64_t blocks = (ntiles + wpb - 1) / wpb;
  const int occ = fbg::eval_blocks_per_cu(mode, l, p->variant(tune), 64 * wpb, g.lds);
  uint64_t maxb = (uint64_t)cu_count(p->device) * (uint64_t)occ;
  // A DNF write-out without the cofactor runs one tile per wave on a grid of
  // fresh blocks: the blocks start in order, so the writes advance through
  // the vector together (a 2^32-bit vector at W = 32: 0.101 ms against 0.109
  // on a resident grid).  Counting keeps the resident grid, whose waves add
  // their counts once each; the cofactor filters 64 tiles per wave at once.
  if (mode == fbg::EVAL_DNF && !(p->variant(tune) & 2)) maxb = blocks;
  if (tune && tune->grid_blocks > 0) maxb = (uint64_t)tune->grid_blocks;
  g.log2w = l;
  g.block = 64 * wpb;
  g.grid = (int)std::max<uint64_t>(1, std::min(blocks, maxb));
  return FBG_OK;
}

// FBG_J16_TABLE=any in the environment makes the jump-table interpreter run
// the copy of its table meant for code loaded off a 64 KiB boundary, so that
// tests cover it (both copies compute the same).  Read at every launch.
uint32_t j16_any() {
  const char *v = getenv("FBG_J16_TABLE");
  return (v && strcmp(v, "any") == 0) ? 1u : 0u;
}

fbg_status check_device(int want) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != want) return fail(FBG_E_INVAL, "object lives on device %d but the current device is %d", want, dev);
  return FBG_OK;
}

fbg_status check_program(const fbg_program *p) {
  if (!p) return fail(FBG_E_INVAL, "program is NULL");
  if (p->device < 0 || !p->d_code) return fail(FBG_E_DEVICE, "program was compiled without a HIP device");
  return check_device(p->device);
}

fbg::EvalArgs base_args(const fbg_program *p, int log2w) {
  fbg::EvalArgs a;
  memset(&a, 0, sizeof a);
  a.code = p->d_code + p->dev_off[log2w];
  a.nins = p->nins[log2w];
  a.nregs = lds_regs((uint32_t)p->c.nregs, log2w);
  a.n = p->c.n;
  a.nslices = p->nslices;
  a.ntiles = tiles_of(p->nslices, log2w);
  a.j16_any = j16_any();
  return a;
}

// Estimated cost of one tile of a program in a batch or a server slice at 2^l
// words per lane, in steps of the interpreter: at 16 words per lane the
// general part's VALU instructions per word and half a step per dispatch of
// its jump-table form (j16_general_cost), elsewhere one step per instruction
// after the clause block in the plain form; a few more per tile; a clause
// block adds its setup, product tree and count, and one step per clause.  (On
// the C3 programs made of one to four clauses a tile takes about 12 steps.)
double tile_cost(const fbg_program *p, int l) {
  const double general = l == FBG_J16_LOG2W && p->j16_cost > 0 ? p->j16_cost : (double)(p->c.code.size() - p->ncl);
  return general + 4.0 + (p->ncl ? 8.0 + (double)p->ncl : 0.0);
}

fbg::BatchProg batch_prog(const fbg_program *p, int l) {
  fbg::BatchProg b;
  memset(&b, 0, sizeof b);
  b.code = p->d_code + p->dev_off[l];
  b.nins = p->nins[l];
  b.nregs = lds_regs((uint32_t)p->c.nregs, l);
  b.n = p->c.n;
  b.nslices = p->nslices;
  b.ntiles = tiles_of(p->nslices, l);
  if (l == 5 && p->has_xcd && p->d_code) b.xcd_code = p->d_code + p->dev_off_xcd;
  return b;
}

// Bytes of the enumeration temporaries for nt tiles: per-tile uint32 counts,
// their uint64 exclusive scan and the scan's block sums (each part 256-byte
// aligned).
size_t enum_temp_bytes(uint64_t nt, size_t *bytes_cnt, size_t *bytes_off) {
  *bytes_cnt = ((nt * 4 + 255) / 256) * 256;
  *bytes_off = ((nt * 8 + 255) / 256) * 256;
  return *bytes_cnt + *bytes_off + (fbg::scan_block_count(nt) + 1) * 8;
}

// Two-pass enumeration given the pass launcher and the temporaries `tmp`
// (enum_temp_bytes(a.ntiles) bytes of device memory): counts -> scan ->
// compaction.  Every temporary word is written before it is read.  With
// zero_counts (the uniform-cofactor passes, which write the counts of live
// tiles only) a fill kernel clears the tile counts first, in one coalesced
// sweep instead of a scattered write per dead tile.
template <typename Pass>
hipError_t enumerate_passes(fbg::EvalArgs a, char *tmp, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total,
                            hipStream_t s, bool zero_counts, Pass pass) {
  const uint64_t nt = a.ntiles;
  size_t bytes_cnt, bytes_off;
  enum_temp_bytes(nt, &bytes_cnt, &bytes_off);
  uint32_t *cnt = (uint32_t *)tmp;
  uint64_t *off = (uint64_t *)(tmp + bytes_cnt);
  uint64_t *blk = (uint64_t *)(tmp + bytes_cnt + bytes_off);
  a.tile_counts = cnt;
  hipError_t e = zero_counts ? fbg::launch_zero((uint64_t *)cnt, bytes_cnt / 8, nullptr, 0, s) : hipSuccess;
  if (e == hipSuccess) e = pass(fbg::EVAL_TILECNT, a);
  if (e == hipSuccess) e = fbg::launch_scan(cnt, nt, off, blk, d_total, s);
  if (e == hipSuccess && capacity > 0) {
    a.tile_offsets = off;
    a.out_idx = d_idx;
    a.capacity = capacity;
    e = pass(fbg::EVAL_ENUM, a);
  }
  return e;
}

// The same with the temporaries allocated on the stream and freed after.
template <typename Pass>
fbg_status enumerate_with(fbg::EvalArgs a, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total, hipStream_t s,
                          bool zero_counts, Pass pass) {
  size_t bytes_cnt, bytes_off;
  const size_t bytes = enum_temp_bytes(a.ntiles, &bytes_cnt, &bytes_off);
  char *tmp = nullptr;
  hipError_t e = hipMallocAsync((void **)&tmp, bytes, s);
  if (e != hipSuccess) return fail(FBG_E_NOMEM, "hipMallocAsync of %zu bytes: %s", bytes, hipGetErrorString(e));
  e = enumerate_passes(a, tmp, d_idx, capacity, d_total, s, zero_counts, pass);
  hipError_t e2 = hipFreeAsync(tmp, s);
  if (e != hipSuccess) return hip_fail(e, "launch of an enumeration kernel");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return FBG_OK;
}

}  // namespace

extern "C" {

const char *fbg_version(void) { return "fbg 0.2 (gfx950)"; }
const char *fbg_last_error(void) { return g_err.c_str(); }
int64_t fbg_last_error_offset(void) { return g_err_off; }

}  // extern "C"

namespace {

// The tiling that pick_log2w prefers, or the nearest one the program is
// encoded for (the larger of two equally near).
int nearest_tiling(uint32_t tilings, int l) {
  for (int d = 0; d <= kMaxLog2W; d++) {
    if (l + d <= kMaxLog2W && ((tilings >> (l + d)) & 1u)) return l + d;
    if (l - d >= 0 && ((tilings >> (l - d)) & 1u)) return l - d;
  }
  return l;
}

fbg_status check_flags(uint32_t flags) {
  if (flags & ~FBG_COMPILE_WPL_MASK)
    return fail(FBG_E_INVAL, "flags 0x%x: only FBG_COMPILE_WPL(0..5) bits are defined", flags);
  return FBG_OK;
}

fbg_status compile_common(const char *src, int32_t n_vars, const int32_t *subst, int32_t n_free, uint32_t flags,
                          fbg_program **out) {
  fbg_program *p = new (std::nothrow) fbg_program();
  if (!p) return fail(FBG_E_NOMEM, "out of host memory");
  p->tilings = flags & FBG_COMPILE_WPL_MASK ? flags & FBG_COMPILE_WPL_MASK : FBG_COMPILE_WPL_MASK;
  std::string msg;
  int64_t off = -1;
  int st = fbg::compile_formula(src, n_vars, p->c, msg, off, subst, n_free);
  if (st != FBG_OK) {
    delete p;
    g_err = msg;
    g_err_off = off;
    if (off >= 0) g_err += " (offset " + std::to_string(off) + ")";
    return (fbg_status)st;
  }
  p->nslices = slices_of(p->c.n);
  p->ncl = fbg::leading_clauses(p->c);
  size_t total = 0;
  std::string enc_err;
  for (int l = 0; l <= kMaxLog2W; l++) {
    if (!p->has_tiling(l)) continue;  // not asked for: left empty
    p->nins[l] = fbg::encode_program(p->c, l, p->words[l], &enc_err);
    p->dev_off[l] = total;
    total += p->words[l].size();
  }
  if (!p->general() && p->c.n >= fbg::kXcdMinVars && p->has_tiling(5)) {
    const fbg::Compiled x = fbg::permute_variables(p->c, fbg::xcd_write_out_permutation(p->c.n));
    const uint32_t nx = fbg::encode_program(x, 5, p->words_xcd, &enc_err);
    if (nx != p->nins[5] && enc_err.empty()) enc_err = "internal: renamed encoding differs in length";
    p->dev_off_xcd = total;
    total += p->words_xcd.size();
    p->has_xcd = true;
  }
  if (!enc_err.empty()) {
    delete p;
    return fail(FBG_E_RANGE, "%s", enc_err.c_str());
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "hipGetDevice");
    }
    p->device = dev;
    std::vector<uint32_t> all;
    all.reserve(total + 64);
    for (int l = 0; l <= kMaxLog2W; l++) all.insert(all.end(), p->words[l].begin(), p->words[l].end());
    all.insert(all.end(), p->words_xcd.begin(), p->words_xcd.end());
    all.resize(all.size() + 64, 0);  // padding: scalar loads never run past the allocation
    e = CodeArena::of(dev).alloc(all.size() * sizeof(uint32_t), (void **)&p->d_code, p->code_class);
    p->code_bytes = p->code_class >= 0 ? (1ull << p->code_class) : all.size() * sizeof(uint32_t);
    if (e != hipSuccess) {
      delete p;
      return fail(FBG_E_NOMEM, "device memory for the program: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_code, all.data(), all.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      CodeArena::of(dev).release(p->d_code, p->code_class);
      delete p;
      return hip_fail(e, "hipMemcpy of the program");
    }
    p->auto_log2w = pick_log2w(p->nslices, (uint32_t)p->c.nregs, p->general(), dev);
  } else {
    p->auto_log2w = pick_log2w(p->nslices, (uint32_t)p->c.nregs, p->general(), -1);
  }
  p->auto_log2w = nearest_tiling(p->tilings, p->auto_log2w);
  if (p->general() && p->has_tiling(FBG_J16_LOG2W))
    p->j16_cost = fbg::j16_general_cost(p->words[FBG_J16_LOG2W], p->nins[FBG_J16_LOG2W]);
  *out = p;
  return FBG_OK;
}

}  // namespace

extern "C" {

fbg_status fbg_compile(const char *src, int32_t n_vars, uint32_t flags, fbg_program **out) {
  if (!out) return fail(FBG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!src) return fail(FBG_E_INVAL, "src is NULL");
  fbg_status st = check_flags(flags);
  if (st) return st;
  if (n_vars < 0 || n_vars > FBG_MAX_VARS) return fail(FBG_E_RANGE, "n=%d out of range [0,%d]", n_vars, FBG_MAX_VARS);
  return compile_common(src, n_vars, nullptr, 0, flags, out);
}

fbg_status fbg_compile_assume(const char *src, int32_t n_vars, const int8_t *assume, uint32_t flags,
                              fbg_program **out) {
  if (!out) return fail(FBG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!src) return fail(FBG_E_INVAL, "src is NULL");
  fbg_status st = check_flags(flags);
  if (st) return st;
  if (n_vars < 0 || n_vars > FBG_MAX_TEXT_VARS)
    return fail(FBG_E_RANGE, "n=%d out of range [0,%d]", n_vars, FBG_MAX_TEXT_VARS);
  if (n_vars > 0 && !assume) return fail(FBG_E_INVAL, "assume is NULL");
  std::vector<int32_t> subst((size_t)n_vars);
  int32_t nfree = 0;
  for (int32_t k = 0; k < n_vars; k++) {
    if (assume[k] < -1 || assume[k] > 1)
      return fail(FBG_E_INVAL, "assume[%d] = %d (must be -1, 0 or 1)", k, (int)assume[k]);
    subst[(size_t)k] = assume[k] < 0 ? nfree++ : (assume[k] ? FBG_SUBST_ONE : FBG_SUBST_ZERO);
  }
  if (nfree > FBG_MAX_VARS) return fail(FBG_E_RANGE, "%d free variables (max %d)", nfree, FBG_MAX_VARS);
  return compile_common(src, n_vars, subst.data(), nfree, flags, out);
}

fbg_status fbg_compile_subst(const char *src, int32_t n_vars, const int32_t *subst, int32_t n_free, uint32_t flags,
                             fbg_program **out) {
  if (!out) return fail(FBG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!src) return fail(FBG_E_INVAL, "src is NULL");
  fbg_status st = check_flags(flags);
  if (st) return st;
  if (n_vars < 0 || n_vars > FBG_MAX_TEXT_VARS)
    return fail(FBG_E_RANGE, "n=%d out of range [0,%d]", n_vars, FBG_MAX_TEXT_VARS);
  if (n_free < 0 || n_free > FBG_MAX_VARS) return fail(FBG_E_RANGE, "n_free=%d out of range [0,%d]", n_free,
                                                       FBG_MAX_VARS);
  if (n_vars > 0 && !subst) return fail(FBG_E_INVAL, "subst is NULL");
  for (int32_t k = 0; k < n_vars; k++)
    if (subst[k] < FBG_SUBST_ONE || subst[k] >= n_free)
      return fail(FBG_E_INVAL, "subst[%d] = %d (must be -1, -2 or in [0, %d))", k, subst[k], n_free);
  return compile_common(src, n_vars, subst, n_free, flags, out);
}

void fbg_program_free(fbg_program *p) {
  if (!p) return;
  if (p->d_code) CodeArena::of(p->device).release(p->d_code, p->code_class);
  delete p;
}

fbg_status fbg_program_info(const fbg_program *p, struct fbg_program_info *out) {
  if (!p || !out) return fail(FBG_E_INVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  out->n_vars = p->c.n;
  out->const_value = p->c.const_value;
  out->l2in = p->c.l2in;
  // clauses + instructions after them, in the plain form
  out->n_instr = (int32_t)p->c.code.size();
  out->n_regs = p->c.nregs;
  out->n_clause_instr = (int32_t)p->ncl;
  out->words_per_lane = 1 << p->auto_log2w;
  out->dnf_words = dnf_words_of(p->c.n);
  out->code_bytes = p->code_bytes;
  const int l = p->auto_log2w;
  out->l_valu = fbg::valu_per_slice(p->words[l], p->nins[l], l, (uint32_t)p->c.nregs);
  return FBG_OK;
}

fbg_status fbg_program_get_info(const fbg_program *p, struct fbg_program_info *out) {
  return fbg_program_info(p, out);
}

fbg_status fbg_program_set_tuning(fbg_program *p, const fbg_tune *tune) {
  if (!p || !tune) return fail(FBG_E_INVAL, "NULL argument");
  int l = p->auto_log2w;
  fbg_status st;
  if (tune->words_per_lane && (st = parse_wpl(tune->words_per_lane, l))) return st;
  if ((st = check_tiling(p, l))) return st;
  int wpb;
  size_t lds;
  if ((st = block_shape((uint32_t)p->c.nregs, l, wpb, lds))) return st;
  p->auto_log2w = l;
  p->cofactor = (tune->flags & FBG_TUNE_COFACTOR) != 0;
  return FBG_OK;
}

uint64_t fbg_program_tiles(const fbg_program *p, int32_t words_per_lane) {
  int l;
  if (!p || parse_wpl(words_per_lane, l)) return 0;
  return tiles_of(p->nslices, l);
}

fbg_status fbg_count_tuned(const fbg_program *p, uint64_t *d_count, const fbg_tune *tune, void *stream) {
  fbg_status st = check_program(p);
  if (st) return st;
  if (!d_count) return fail(FBG_E_INVAL, "d_count is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (p->c.const_value >= 0) {
    e = fbg::launch_set_u64(d_count, p->c.const_value ? (1ull << p->c.n) : 0ull, s);
    return e == hipSuccess ? FBG_OK : hip_fail(e, "launch");
  }
  Geometry g;
  if ((st = geometry(p, tune, fbg::EVAL_COUNT, g))) return st;
  fbg::EvalArgs a = base_args(p, g.log2w);
  a.out_count = d_count;
  e = fbg::launch_set_u64(d_count, 0, s);
  if (e != hipSuccess) return hip_fail(e, "launch");
  e = fbg::launch_eval(fbg::EVAL_COUNT, g.log2w, p->variant(tune), a, g.grid, g.block, g.lds, s);
  return e == hipSuccess ? FBG_OK : hip_fail(e, "launch of the count kernel");
}

fbg_status fbg_count(const fbg_program *p, uint64_t *d_count, void *stream) {
  return fbg_count_tuned(p, d_count, nullptr, stream);
}

fbg_status fbg_eval_dnf_tuned(const fbg_program *p, uint64_t *d_out, uint64_t out_words, const fbg_tune *tune,
                              void *stream) {
  fbg_status st = check_program(p);
  if (st) return st;
  if (!d_out) return fail(FBG_E_INVAL, "d_out is NULL");
  if (p->c.n > FBG_MAX_DNF_VARS) return fail(FBG_E_RANGE, "n=%d above %d for a DNF vector", p->c.n, FBG_MAX_DNF_VARS);
  const uint64_t need = dnf_words_of(p->c.n);
  if (out_words < need)
    return fail(FBG_E_INVAL, "out_words=%llu < %llu", (unsigned long long)out_words, (unsigned long long)need);
  Geometry g;
  if ((st = geometry(p, tune, fbg::EVAL_DNF, g))) return st;
  fbg::EvalArgs a = base_args(p, g.log2w);
  a.out32 = (uint32_t *)d_out;
  a.out_slices = 2 * need;
  // the XCD-local layout (fbg_kernels.h) on the grid of one tile per wave
  if (g.log2w == 5 && p->has_xcd && p->variant(tune) == 0 && ((uintptr_t)d_out & 15) == 0)
    a.xcd_code = p->d_code + p->dev_off_xcd;
  hipError_t e =
      fbg::launch_eval(fbg::EVAL_DNF, g.log2w, p->variant(tune), a, g.grid, g.block, g.lds, (hipStream_t)stream);
  return e == hipSuccess ? FBG_OK : hip_fail(e, "launch of the DNF kernel");
}

fbg_status fbg_eval_dnf(const fbg_program *p, uint64_t *d_out, uint64_t out_words, void *stream) {
  return fbg_eval_dnf_tuned(p, d_out, out_words, nullptr, stream);
}

fbg_status fbg_enumerate(const fbg_program *p, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total,
                         void *stream) {
  fbg_status st = check_program(p);
  if (st) return st;
  if (!d_total) return fail(FBG_E_INVAL, "d_total is NULL");
  if (capacity > 0 && !d_idx)
    return fail(FBG_E_INVAL, "d_idx is NULL with capacity %llu", (unsigned long long)capacity);
  Geometry g;
  if ((st = geometry(p, nullptr, fbg::EVAL_TILECNT, g))) return st;
  hipStream_t s = (hipStream_t)stream;
  const int var = p->variant(nullptr);
  return enumerate_with(base_args(p, g.log2w), d_idx, capacity, d_total, s, (var & 2) != 0,
                        [&](int mode, const fbg::EvalArgs &a) {
                          return fbg::launch_eval(mode, g.log2w, var, a, g.grid, g.block, g.lds, s);
                        });
}

fbg_status fbg_enumerate_noalloc(const fbg_program *p, uint64_t *d_idx, uint64_t capacity, uint64_t *d_total,
                                 void *stream) {
  fbg_status st = check_program(p);
  if (st) return st;
  if (!d_total) return fail(FBG_E_INVAL, "d_total is NULL");
  if (capacity > 0 && !d_idx)
    return fail(FBG_E_INVAL, "d_idx is NULL with capacity %llu", (unsigned long long)capacity);
  Geometry g;
  if ((st = geometry(p, nullptr, fbg::EVAL_TILECNT, g))) return st;
  const fbg::EvalArgs a = base_args(p, g.log2w);
  size_t bytes_cnt, bytes_off;
  const size_t bytes = enum_temp_bytes(a.ntiles, &bytes_cnt, &bytes_off);
  if (a.ntiles > fbg::kNoallocMaxTiles || bytes > fbg::kNoallocScratchBytes)
    return fail(FBG_E_RANGE,
                "fbg_enumerate_noalloc: %llu tiles at %d words per lane need %zu bytes of scratch; the static "
                "scratch holds %llu tiles (%llu bytes)",
                (unsigned long long)a.ntiles, 1 << g.log2w, bytes, (unsigned long long)fbg::kNoallocMaxTiles,
                (unsigned long long)fbg::kNoallocScratchBytes);
  void *scratch = nullptr;
  hipError_t e = fbg::noalloc_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
  hipStream_t s = (hipStream_t)stream;
  const int var = p->variant(nullptr);
  e = enumerate_passes(a, (char *)scratch, d_idx, capacity, d_total, s, (var & 2) != 0,
                       [&](int mode, const fbg::EvalArgs &aa) {
    return fbg::launch_eval(mode, g.log2w, var, aa, g.grid, g.block, g.lds, s);
  });
  return e == hipSuccess ? FBG_OK : hip_fail(e, "launch of an enumeration kernel");
}

fbg_status fbg_enumerate_dnf(const uint64_t *d_dnf, int32_t n_vars, uint64_t *d_idx, uint64_t capacity,
                             uint64_t *d_total, void *stream) {
  if (!d_dnf || !d_total) return fail(FBG_E_INVAL, "NULL device pointer");
  if (capacity > 0 && !d_idx)
    return fail(FBG_E_INVAL, "d_idx is NULL with capacity %llu", (unsigned long long)capacity);
  if (n_vars < 0 || n_vars > FBG_MAX_DNF_VARS) return fail(FBG_E_RANGE, "n=%d out of range", n_vars);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  fbg::EvalArgs a;
  memset(&a, 0, sizeof a);
  a.n = n_vars;
  a.nslices = 2 * dnf_words_of(n_vars);  // bits at or above 2^n are zero in a DNF vector
  a.ntiles = tiles_of(a.nslices, 5);
  a.out32 = (uint32_t *)d_dnf;
  const uint64_t blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (uint64_t)cu_count(dev) * 8));
  hipStream_t s = (hipStream_t)stream;
  return enumerate_with(a, d_idx, capacity, d_total, s, false, [&](int mode, const fbg::EvalArgs &aa) {
    return fbg::launch_dnf_scan(mode, aa, grid, 64 * kWavesPerBlock, s);
  });
}

// ------------------------------------------------------------------ batches

fbg_status fbg_batch_create(const fbg_program *const *ps, int32_t np, const fbg_tune *tune, fbg_batch **out) {
  if (!out) return fail(FBG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (np <= 0 || !ps) return fail(FBG_E_INVAL, "empty batch");
  int dev = -1;
  for (int32_t i = 0; i < np; i++) {
    fbg_status st = check_program(ps[i]);
    if (st) return st;
    dev = ps[i]->device;
  }
  fbg_status st;
  int fixed_l = -1;
  if (tune && tune->words_per_lane && (st = parse_wpl(tune->words_per_lane, fixed_l))) return st;
  if (tune && (tune->direct_run < 0 || tune->direct_run > 64))
    return fail(FBG_E_INVAL, "direct_run must be 0..64 (got %d)", tune->direct_run);
  const int cus = cu_count(dev);
  const uint64_t waves = (uint64_t)cus * 32;

  fbg_batch *b = new (std::nothrow) fbg_batch();
  if (!b) return fail(FBG_E_NOMEM, "out of host memory");
  b->device = dev;
  b->np = np;
  b->host_progs.resize((size_t)np);
  b->plan_of.assign((size_t)np, 0);
  std::vector<std::vector<fbg::BatchItem>> plan_items;
  std::vector<std::vector<fbg::BatchItem>> plan_direct;  // per plan: one entry per program (clause-only plans)
  // 0: clause-only programs; 1: general programs whose registers all fit in
  // VGPRs (at every tiling); 2: up to four registers in LDS; 3: more.  The LDS a plan's widest
  // program needs per wave sets the occupancy of the whole plan, so the few
  // register-hungry programs do not slow down the rest.
  // At 16 words per lane (the jump-table form) a plan keeps at most
  // kJ16LdsRegs registers of a wave in LDS and the rest in global scratch,
  // so the register count no longer limits occupancy: when the tuning fixes
  // that tiling and some program has a general part, every program goes into
  // one plan, one persistent launch.
  bool any_general = false;
  for (int32_t i = 0; i < np; i++) any_general = any_general || ps[i]->general();
  // (the library's own choice for a batch with general programs when the
  // tuning does not fix the tiling)
  if (fixed_l < 0 && any_general) fixed_l = FBG_J16_LOG2W;
  const bool one_plan = fixed_l == FBG_J16_LOG2W && any_general;
  auto group_of = [one_plan](const fbg_program *q) {
    if (one_plan) return 1;
    if (!q->general()) return 0;
    const uint32_t r = lds_regs((uint32_t)q->c.nregs, FBG_J16_LOG2W);
    return r == 0 ? 1 : (r <= 4 ? 2 : 3);
  };
  for (int group = 0; group < 4; group++) {
    std::vector<int32_t> members;
    for (int32_t i = 0; i < np; i++)
      if (group_of(ps[i]) == group) members.push_back(i);
    if (members.empty()) continue;
    // words per lane: the tuning, else the choice for the largest program
    int l = fixed_l;
    if (l < 0) {
      uint64_t best = 0;
      l = 0;
      for (int32_t i : members) {
        const uint64_t cost = ps[i]->nslices * (uint64_t)std::max<size_t>(1, ps[i]->c.code.size());
        if (cost >= best) {
          best = cost;
          l = ps[i]->auto_log2w;
        }
      }
    }
    uint32_t max_regs = 0;
    int var = 0;
    for (int32_t i : members) {
      if (!ps[i]->has_tiling(l)) {
        fbg_batch_free(b);
        return fail(FBG_E_INVAL, "program %d was compiled without %d words per lane (FBG_COMPILE_WPL)", i, 1 << l);
      }
      max_regs = std::max<uint32_t>(max_regs, (uint32_t)ps[i]->c.nregs);
      var |= ps[i]->variant(tune);
    }
    if (one_plan) var |= 1;  // clause-only programs run in the general kernel too
    // registers that stay in LDS, the rest (jump-table form only) in global
    // scratch, gstride words per wave
    uint32_t lds_keep = lds_regs(max_regs, l < 0 ? 0 : l);
    uint64_t gstride = 0;
    if (l == FBG_J16_LOG2W && lds_keep > kJ16LdsRegs) {
      gstride = (uint64_t)(lds_keep - kJ16LdsRegs) * (64u << l);
      lds_keep = kJ16LdsRegs;
    }
    if (gstride == 0) {
      while (l > 0 && lds_per_wave(max_regs, l) > kMaxLdsPerBlock) l--;
      // LDS registers: keep a block of 4 waves within 32 KiB (5 blocks per CU)
      if (fixed_l < 0)
        while (l > 0 && lds_per_wave(max_regs, l) * kWavesPerBlock > kMaxLdsPerBlock / 2) l--;
      lds_keep = lds_regs(max_regs, l);
    }
    int wpb;
    size_t lds;
    if ((st = block_shape(lds_keep + fbg::vgpr_regs_of(l), l, wpb, lds))) {
      fbg_batch_free(b);
      return st;
    }
    double total_cost = 0;
    for (int32_t i : members) {
      fbg::BatchProg &q = b->host_progs[(size_t)i];
      q = batch_prog(ps[i], l);
      total_cost += (double)q.ntiles * tile_cost(ps[i], l);
      b->plan_of[(size_t)i] = (int)b->plans.size();
    }
    // about eight items per wave (on C3, 2.1 % faster than four and 0.9 %
    // than sixteen: finer items even out the end of the queues, more of them
    // cost pops); never split below one tile.  A program's K items
    // interleave: item k takes tiles k, k + K, k + 2K, ..., so the waves
    // working on neighbouring items at the same time write neighbouring tiles
    // (DNF vectors), which keeps the HBM writes close together.
    const double target = std::max(1.0, total_cost / (double)(waves * 8));
    std::vector<fbg::BatchItem> items;
    std::vector<double> cost;
    for (int32_t i : members) {
      const fbg::BatchProg &q = b->host_progs[(size_t)i];
      const double per_tile = tile_cost(ps[i], l);
      const uint64_t chunk = (uint64_t)std::max(1.0, target / per_tile);
      uint64_t K = (q.ntiles + chunk - 1) / chunk;
      // with the uniform cofactor an odd K: the tiles that survive its test
      // often share their low index bits, and an even (above all a
      // power-of-two) K would give them to a few items
      if ((var & 2) && K > 1 && K < q.ntiles && !(K & 1)) K++;
      for (uint64_t k = 0; k < K; k++) {
        fbg::BatchItem it;
        it.prog = (uint32_t)i;
        it.slot = (uint32_t)i;
        it.t0 = k;
        it.t1 = q.ntiles;
        it.step = K;
        items.push_back(it);
        cost.push_back((double)((q.ntiles - k + K - 1) / K) * per_tile);
      }
    }
    if (items.size() > 0xFFFFFFF0ull) {
      fbg_batch_free(b);
      return fail(FBG_E_RANGE, "too many work items");
    }
    // largest first, so that the queue ends on small items
    std::vector<size_t> order(items.size());
    for (size_t k = 0; k < order.size(); k++) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<fbg::BatchItem> sorted;
    sorted.reserve(items.size());
    for (size_t k : order) sorted.push_back(items[k]);

    fbg_batch::Plan pl;
    pl.log2w = l;
    pl.var = var;
    pl.block = 64 * wpb;
    pl.lds = lds;
    pl.nitems = (uint32_t)sorted.size();
    if (tune && tune->direct_run > 0) pl.direct_run = (uint32_t)tune->direct_run;
    pl.max_regs = lds_keep;
    pl.gstride = gstride;
    const uint64_t want = (pl.nitems + wpb - 1) / wpb;
    for (int mode : {fbg::EVAL_COUNT, fbg::EVAL_DNF}) {
      uint64_t maxb = (uint64_t)cus * (uint64_t)fbg::batch_blocks_per_cu(mode, l, var, pl.block, lds);
      if (tune && tune->grid_blocks > 0) maxb = (uint64_t)tune->grid_blocks;
      (mode == fbg::EVAL_COUNT ? pl.grid : pl.grid_dnf) = (int)std::max<uint64_t>(1, std::min<uint64_t>(want, maxb));
    }
    std::vector<fbg::BatchItem> direct;
    if (var == 0 && !(tune && tune->grid_blocks > 0)) {
      bool any_xcd = false;
      for (int32_t i : members) {
        const fbg::BatchProg &q = b->host_progs[(size_t)i];
        if (q.xcd_code) {
          // the XCD-local layout: the program starts at a multiple of 32
          // tiles, so that block k of its waves runs on XCD k mod 8 (the
          // tiles in between belong to no program and are skipped)
          pl.ntiles = (pl.ntiles + 31) & ~(uint64_t)31;
          any_xcd = true;
        }
        fbg::BatchItem it;
        it.prog = (uint32_t)i;
        it.slot = (uint32_t)i;
        it.t0 = pl.ntiles;
        it.t1 = pl.ntiles + q.ntiles;
        it.step = 1;
        direct.push_back(it);
        pl.ntiles += q.ntiles;
        pl.max_prog_tiles = std::max<uint64_t>(pl.max_prog_tiles, q.ntiles);
      }
      pl.ndirect = (uint32_t)direct.size();
      // one tile per wave, four waves per block: a block's tiles share bits
      // 2..4 of their tile index, i.e. one residue class of 4 KiB pieces
      if (any_xcd && !(tune && tune->direct_run > 0)) pl.direct_run = 1;
    }
    b->plans.push_back(pl);
    plan_items.push_back(std::move(sorted));
    plan_direct.push_back(std::move(direct));
  }
  hipError_t e = hipMalloc((void **)&b->d_progs, (size_t)np * sizeof(fbg::BatchProg));
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_head, 4 * fbg::kHeadWords * sizeof(uint32_t));
  for (size_t k = 0; k < b->plans.size() && e == hipSuccess; k++) {
    fbg_batch::Plan &pl = b->plans[k];
    if (pl.gstride == 0) continue;
    const uint64_t waves_max = (uint64_t)std::max(pl.grid, pl.grid_dnf) * (uint64_t)(pl.block / 64);
    e = hipMalloc((void **)&pl.d_gscratch, waves_max * pl.gstride * sizeof(uint32_t));
  }
  for (size_t k = 0; k < b->plans.size() && e == hipSuccess; k++) {
    e = hipMalloc((void **)&b->plans[k].d_items, plan_items[k].size() * sizeof(fbg::BatchItem));
    if (e == hipSuccess)
      e = hipMemcpy(b->plans[k].d_items, plan_items[k].data(), plan_items[k].size() * sizeof(fbg::BatchItem),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess && !plan_direct[k].empty()) {
      e = hipMalloc((void **)&b->plans[k].d_direct, plan_direct[k].size() * sizeof(fbg::BatchItem));
      if (e == hipSuccess)
        e = hipMemcpy(b->plans[k].d_direct, plan_direct[k].data(), plan_direct[k].size() * sizeof(fbg::BatchItem),
                      hipMemcpyHostToDevice);
    }
  }
  if (e == hipSuccess)
    e = hipMemcpy(b->d_progs, b->host_progs.data(), (size_t)np * sizeof(fbg::BatchProg), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    fbg_batch_free(b);
    return fail(FBG_E_NOMEM, "batch upload: %s", hipGetErrorString(e));
  }
  *out = b;
  return FBG_OK;
}

}  // extern "C"

namespace {

fbg_status batch_launch(fbg_batch *b, int mode, const fbg::BatchProg *d_progs, uint64_t *d_counts, hipStream_t s) {
  // zero the counts and every plan's queue head, then one persistent kernel per plan
  hipError_t e = fbg::launch_zero(d_counts, (uint64_t)b->np, b->d_head, (uint32_t)b->plans.size() * fbg::kHeadWords, s);
  if (e != hipSuccess) return hip_fail(e, "launch of the zero fill");
  for (size_t k = 0; k < b->plans.size(); k++) {
    const fbg_batch::Plan &pl = b->plans[k];
    fbg::BatchArgs a;
    a.progs = d_progs;
    a.items = pl.d_items;
    a.nitems = pl.nitems;
    a.max_regs = pl.max_regs;
    a.head = b->d_head + k * fbg::kHeadWords;
    a.counts = d_counts;
    a.gscratch = pl.d_gscratch;
    a.gstride = pl.gstride;
    a.j16_any = j16_any();
    if (mode == fbg::EVAL_DNF && pl.d_direct && b->d_tile_counts) {
      // one wave per tile over the plan's programs in order; counts from the
      // tile counts
      a.items = pl.d_direct;
      a.nitems = pl.ndirect;
      a.run = pl.direct_run;
      const uint64_t wpb = (uint64_t)(pl.block / 64);
      const uint64_t waves = (pl.ntiles + a.run - 1) / a.run;
      const uint64_t grid = (waves + wpb - 1) / wpb;
      // about 1024 tiles per block of the count sums (C1: 64 per program)
      const int sum_blocks = (int)std::min<uint64_t>(256, std::max<uint64_t>(1, pl.max_prog_tiles / 1024));
      e = fbg::launch_batch_direct(pl.log2w, a, (int)grid, pl.block, sum_blocks, s);
      if (e != hipSuccess) return hip_fail(e, "launch of the batch kernel");
      continue;
    }
    e = fbg::launch_batch(mode, pl.log2w, pl.var, a, mode == fbg::EVAL_DNF ? pl.grid_dnf : pl.grid, pl.block, pl.lds,
                          s);
    if (e != hipSuccess) return hip_fail(e, "launch of the batch kernel");
  }
  return FBG_OK;
}

}  // namespace

extern "C" {

fbg_status fbg_batch_count(fbg_batch *b, uint64_t *d_counts, void *stream) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!d_counts) return fail(FBG_E_INVAL, "d_counts is NULL");
  fbg_status st = check_device(b->device);
  if (st) return st;
  return batch_launch(b, fbg::EVAL_COUNT, b->d_progs, d_counts, (hipStream_t)stream);
}

fbg_status fbg_batch_set_dnf_outputs(fbg_batch *b, uint64_t *const *d_outs, const uint64_t *out_words) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!d_outs || !out_words) return fail(FBG_E_INVAL, "NULL argument");
  fbg_status st = check_device(b->device);
  if (st) return st;
  std::vector<fbg::BatchProg> t = b->host_progs;
  for (int32_t i = 0; i < b->np; i++) {
    fbg::BatchProg &q = t[(size_t)i];
    if (q.n > FBG_MAX_DNF_VARS) return fail(FBG_E_RANGE, "program %d: n=%d above %d for a DNF vector", i, q.n,
                                            FBG_MAX_DNF_VARS);
    const uint64_t need = dnf_words_of(q.n);
    if (!d_outs[i]) return fail(FBG_E_INVAL, "d_outs[%d] is NULL", i);
    if (out_words[i] < need)
      return fail(FBG_E_INVAL, "out_words[%d]=%llu < %llu", i, (unsigned long long)out_words[i],
                  (unsigned long long)need);
    q.out32 = (uint32_t *)d_outs[i];
    q.out_slices = 2 * need;
    // the XCD-local layout writes 16-byte groups: other outputs take the
    // plain one
    if ((uintptr_t)q.out32 & 15) q.xcd_code = nullptr;
    if (!b->host_dnf.empty()) {
      q.tile_counts = b->host_dnf[(size_t)i].tile_counts;
      q.chunk_counts = b->host_dnf[(size_t)i].chunk_counts;
    }
  }
  hipError_t e = hipSuccess;
  if (!b->d_progs_dnf) e = hipMalloc((void **)&b->d_progs_dnf, t.size() * sizeof(fbg::BatchProg));
  if (e == hipSuccess) e = hipMemcpy(b->d_progs_dnf, t.data(), t.size() * sizeof(fbg::BatchProg), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload of the DNF output table");
  b->host_dnf = t;
  return FBG_OK;
}

fbg_status fbg_batch_set_enum_outputs(fbg_batch *b, uint64_t *const *d_idx, const uint64_t *capacity) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!d_idx || !capacity) return fail(FBG_E_INVAL, "NULL argument");
  if (b->host_dnf.empty()) return fail(FBG_E_INVAL, "set the DNF outputs first (fbg_batch_set_dnf_outputs)");
  fbg_status st = check_device(b->device);
  if (st) return st;
  for (int32_t i = 0; i < b->np; i++)
    if (capacity[i] > 0 && !d_idx[i]) return fail(FBG_E_INVAL, "d_idx[%d] is NULL with capacity %llu", i,
                                                  (unsigned long long)capacity[i]);
  // programs whose DNF write-out takes the XCD-local layout: two piece
  // counts per tile
  auto xcd_direct = [&](int32_t i) {
    return b->host_progs[(size_t)i].xcd_code && b->plans[(size_t)b->plan_of[(size_t)i]].d_direct;
  };
  hipError_t e = hipSuccess;
  if (!b->d_tile_counts) {
    uint64_t total = 0, chunks = 0;
    for (int32_t i = 0; i < b->np; i++) {
      total += b->host_progs[(size_t)i].ntiles;
      if (xcd_direct(i)) chunks += 2 * b->host_progs[(size_t)i].ntiles;
    }
    if (total >= (1ull << 32)) return fail(FBG_E_RANGE, "%llu tiles: batched enumeration lists tiles in 32 bits",
                                           (unsigned long long)total);
    b->total_tiles = total;
    const uint64_t nb = fbg::scan_block_count(total);
    e = hipMalloc((void **)&b->d_tile_counts, std::max<uint64_t>(total, 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_offsets, std::max<uint64_t>(total, 1) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_scan_blk, (nb + 2) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_enum, (size_t)b->np * sizeof(fbg::EnumProg));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_tile_list, (std::max<uint64_t>(total, 1) + 64) * sizeof(uint32_t));
    if (e == hipSuccess && chunks) e = hipMalloc((void **)&b->d_chunk_counts, chunks * sizeof(uint32_t));
    if (e != hipSuccess) return fail(FBG_E_NOMEM, "enumeration buffers: %s", hipGetErrorString(e));
  }
  std::vector<fbg::EnumProg> ep((size_t)b->np);
  uint64_t tile0 = 0, chunk0 = 0;
  for (int32_t i = 0; i < b->np; i++) {
    fbg::BatchProg &q = b->host_dnf[(size_t)i];
    q.tile_counts = b->d_tile_counts + tile0;
    q.chunk_counts = nullptr;
    if (xcd_direct(i)) {
      q.chunk_counts = b->d_chunk_counts + chunk0;
      chunk0 += 2 * q.ntiles;
    }
    fbg::EnumProg &x = ep[(size_t)i];
    memset(&x, 0, sizeof x);
    x.dnf = q.out32;
    x.nslices = q.nslices;
    x.tile0 = tile0;
    x.out = d_idx[i];
    x.capacity = capacity[i];
    x.log2w = (uint32_t)b->plans[(size_t)b->plan_of[(size_t)i]].log2w;
    tile0 += q.ntiles;
  }
  e = hipMemcpy(b->d_enum, ep.data(), ep.size() * sizeof(fbg::EnumProg), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_progs_dnf, b->host_dnf.data(), b->host_dnf.size() * sizeof(fbg::BatchProg),
                  hipMemcpyHostToDevice);
  return e == hipSuccess ? FBG_OK : hip_fail(e, "upload of the enumeration tables");
}

fbg_status fbg_batch_enumerate(fbg_batch *b, void *stream) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!b->d_enum) return fail(FBG_E_INVAL, "no enumeration outputs set (fbg_batch_set_enum_outputs)");
  fbg_status st = check_device(b->device);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t nb = fbg::scan_block_count(b->total_tiles);
  hipError_t e = fbg::launch_scan(b->d_tile_counts, b->total_tiles, b->d_offsets, b->d_scan_blk,
                                  b->d_scan_blk + nb + 1, s);
  if (e != hipSuccess) return hip_fail(e, "launch of the tile-count scan");
  fbg::BatchEnumArgs a;
  a.progs = b->d_enum;
  a.np = (uint32_t)b->np;
  a.total_tiles = b->total_tiles;
  a.tile_counts = b->d_tile_counts;
  a.offsets = b->d_offsets;
  a.list = b->d_tile_list;
  a.nlist = b->d_tile_list + std::max<uint64_t>(b->total_tiles, 1);
  const int grid = cu_count(b->device) * 8;
  e = fbg::launch_zero(nullptr, 0, a.nlist, 1, s);
  if (e == hipSuccess) e = fbg::launch_list_tiles(a, grid, s);
  if (e != hipSuccess) return hip_fail(e, "launch of the tile listing");
  for (const auto &pl : b->plans) {
    e = fbg::launch_batch_compact(pl.log2w, a, grid, 256, s);
    if (e != hipSuccess) return hip_fail(e, "launch of the compaction kernel");
  }
  return FBG_OK;
}

fbg_status fbg_batch_eval_dnf(fbg_batch *b, uint64_t *d_counts, void *stream) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!d_counts) return fail(FBG_E_INVAL, "d_counts is NULL");
  if (!b->d_progs_dnf) return fail(FBG_E_INVAL, "no DNF outputs set (fbg_batch_set_dnf_outputs)");
  fbg_status st = check_device(b->device);
  if (st) return st;
  return batch_launch(b, fbg::EVAL_DNF, b->d_progs_dnf, d_counts, (hipStream_t)stream);
}

fbg_status fbg_batch_count_graph(fbg_batch *b, uint64_t *d_counts, void *stream) {
  if (!b) return fail(FBG_E_INVAL, "batch is NULL");
  if (!d_counts) return fail(FBG_E_INVAL, "d_counts is NULL");
  fbg_status st = check_device(b->device);
  if (st) return st;
  hipError_t e;
  if (!b->graph_exec || b->graph_counts != d_counts) {
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
    hipStream_t cs;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      st = fbg_batch_count(b, d_counts, cs);  // kernels only: no memset node, no allocation
      hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
      if (st == FBG_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
      if (st == FBG_OK && (e2 = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        st = hip_fail(e2, "hipGraphInstantiate");
    } else {
      st = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (st) return st;
    b->graph_counts = d_counts;
  }
  e = hipGraphLaunch(b->graph_exec, (hipStream_t)stream);
  return e == hipSuccess ? FBG_OK : hip_fail(e, "hipGraphLaunch");
}

void fbg_batch_free(fbg_batch *b) {
  if (!b) return;
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_progs) (void)hipFree(b->d_progs);
  if (b->d_progs_dnf) (void)hipFree(b->d_progs_dnf);
  if (b->d_tile_counts) (void)hipFree(b->d_tile_counts);
  if (b->d_chunk_counts) (void)hipFree(b->d_chunk_counts);
  if (b->d_offsets) (void)hipFree(b->d_offsets);
  if (b->d_scan_blk) (void)hipFree(b->d_scan_blk);
  if (b->d_enum) (void)hipFree(b->d_enum);
  if (b->d_tile_list) (void)hipFree(b->d_tile_list);
  for (auto &pl : b->plans) {
    if (pl.d_items) (void)hipFree(pl.d_items);
    if (pl.d_direct) (void)hipFree(pl.d_direct);
    if (pl.d_gscratch) (void)hipFree(pl.d_gscratch);
  }
  if (b->d_head) (void)hipFree(b->d_head);
  delete b;
}

fbg_status fbg_count_batch(const fbg_program *const *ps, int32_t np, uint64_t *d_counts, const fbg_tune *tune,
                           void *stream) {
  fbg_batch *b = nullptr;
  fbg_status st = fbg_batch_create(ps, np, tune, &b);
  if (st) return st;
  st = fbg_batch_count(b, d_counts, stream);
  // the plan must outlive the launch
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  fbg_batch_free(b);
  if (st) return st;
  return e == hipSuccess ? FBG_OK : hip_fail(e, "hipStreamSynchronize");
}

// ------------------------------------------------------------------ serving

fbg_status fbg_server_create(int32_t max_programs, int32_t max_items, int32_t words_per_lane, int32_t nbuf,
                             int32_t flags, fbg_server **out) {
  if (!out) return fail(FBG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (max_programs <= 0 || max_items <= 0 || nbuf <= 0 || nbuf > 64) return fail(FBG_E_INVAL, "bad server sizes");
  int l;
  fbg_status st = parse_wpl(words_per_lane, l);
  if (st) return st;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  fbg_server *sv = new (std::nothrow) fbg_server();
  if (!sv) return fail(FBG_E_NOMEM, "out of host memory");
  sv->device = dev;
  sv->log2w = l;
  sv->max_programs = max_programs;
  sv->max_items = max_items;
  sv->nbuf = nbuf;
  sv->cofactor = (flags & FBG_TUNE_COFACTOR) != 0;
  sv->slots.resize((size_t)nbuf);
  const size_t bytes = kServerHeadBytes + (size_t)max_programs * sizeof(fbg::BatchProg) +
                       (size_t)max_items * sizeof(fbg::BatchItem);
  for (auto &sl : sv->slots) {
    e = hipHostMalloc((void **)&sl.h, bytes, hipHostMallocDefault);
    if (e == hipSuccess) memset(sl.h, 0, kServerHeadBytes);
    if (e == hipSuccess) e = hipMalloc((void **)&sl.d, bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      fbg_server_free(sv);
      return fail(FBG_E_NOMEM, "server buffers: %s", hipGetErrorString(e));
    }
  }
  *out = sv;
  return FBG_OK;
}

fbg_status fbg_server_launch(fbg_server *sv, const fbg_program *const *ps, int32_t np, const fbg_item *items,
                             int32_t nitems, uint64_t *d_counts, int32_t ncounts, void *stream) {
  if (!sv) return fail(FBG_E_INVAL, "server is NULL");
  if (np <= 0 || np > sv->max_programs || !ps) return fail(FBG_E_INVAL, "np=%d out of range", np);
  if (nitems <= 0 || nitems > sv->max_items || !items) return fail(FBG_E_INVAL, "nitems=%d out of range", nitems);
  if (!d_counts || ncounts <= 0) return fail(FBG_E_INVAL, "no counts array");
  fbg_status st = check_device(sv->device);
  if (st) return st;
  const int l = sv->log2w;
  uint32_t max_regs = 0;
  int var = sv->cofactor ? 2 : 0;
  for (int32_t i = 0; i < np; i++) {
    if ((st = check_program(ps[i]))) return st;
    if ((st = check_tiling(ps[i], l))) return st;
    max_regs = std::max<uint32_t>(max_regs, (uint32_t)ps[i]->c.nregs);
    var |= ps[i]->variant(nullptr);
  }
  // validate every item on the host: the kernel trusts them
  for (int32_t k = 0; k < nitems; k++) {
    const fbg_item &it = items[k];
    if (it.prog < 0 || it.prog >= np) return fail(FBG_E_INVAL, "item %d: program %d out of range", k, it.prog);
    if (it.slot < 0 || it.slot >= ncounts) return fail(FBG_E_INVAL, "item %d: slot %d out of range", k, it.slot);
    const uint64_t nt = tiles_of(ps[it.prog]->nslices, l);
    if (it.tile_begin > it.tile_end || it.tile_end > nt)
      return fail(FBG_E_INVAL, "item %d: tiles [%llu,%llu) outside [0,%llu)", k, (unsigned long long)it.tile_begin,
                  (unsigned long long)it.tile_end, (unsigned long long)nt);
  }
  int wpb;
  size_t lds;
  if ((st = block_shape(max_regs, l, wpb, lds))) return st;
  const int cus = cu_count(sv->device);
  const int occ = fbg::batch_blocks_per_cu(fbg::EVAL_COUNT, l, var, 64 * wpb, lds);
  fbg_server::Slot &sl = sv->slots[(size_t)sv->next];
  sv->next = (sv->next + 1) % sv->nbuf;
  hipError_t e;
  if (sl.used && (e = hipEventSynchronize(sl.done)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  const size_t items_at = kServerHeadBytes + (size_t)np * sizeof(fbg::BatchProg);
  fbg::BatchProg *hp = (fbg::BatchProg *)(sl.h + kServerHeadBytes);
  fbg::BatchItem *hi = (fbg::BatchItem *)(sl.h + items_at);
  for (int32_t i = 0; i < np; i++) hp[i] = batch_prog(ps[i], l);  // tilings checked above
  // Cut the items into pieces of about equal estimated cost (tile_cost per
  // tile) so that every resident wave gets about four, within the staging
  // capacity: an item of c tiles at cost w each gives ceil(c / ceil(T / w)) <=
  // c w / T + 1 pieces for a target T (one more with the uniform cofactor,
  // below), so want + 2 nitems <= max_items in all (checked below all the
  // same).  (Sorting the pieces by cost as the batch plans do cost more host
  // time per slice than it saved.)
  double total = 0;
  for (int32_t k = 0; k < nitems; k++)
    total += (double)(items[k].tile_end - items[k].tile_begin) * tile_cost(ps[items[k].prog], l);
  const int64_t spare = (int64_t)sv->max_items - (sv->cofactor ? 2 : 1) * (int64_t)nitems;
  const uint64_t room = (uint64_t)std::max<int64_t>(0, spare);
  const uint64_t want = std::min<uint64_t>(room, (uint64_t)cus * occ * wpb * 4);
  const double target = want > 0 ? total / (double)want * (1.0 + 1e-9) : 0.0;
  // With the uniform cofactor an item's P pieces interleave (piece j takes
  // tiles j, j + P, ... of it) with P odd: the tiles that survive the test
  // often share index bits, and contiguous pieces, or an even stride, would
  // give them to a few pieces.
  int32_t npieces = 0;
  for (int32_t k = 0; k < nitems; k++) {
    const double w = tile_cost(ps[items[k].prog], l);
    const uint64_t chunk = want > 0 ? std::max<uint64_t>(1, (uint64_t)std::ceil(target / w)) : ~0ull;
    const uint64_t b = items[k].tile_begin, e = items[k].tile_end;
    if (sv->cofactor && e - b > chunk) {
      uint64_t P = (e - b + chunk - 1) / chunk;
      if (!(P & 1) && P < e - b) P++;
      for (uint64_t j = 0; j < P; j++) {
        if (npieces >= sv->max_items) return fail(FBG_E_INVAL, "internal: more pieces than staging room");
        fbg::BatchItem &q = hi[npieces++];
        q.prog = (uint32_t)items[k].prog;
        q.slot = (uint32_t)items[k].slot;
        q.t0 = b + j;
        q.t1 = e;
        q.step = P;
      }
      continue;
    }
    for (uint64_t t = b; t < e; t += std::min(chunk, e - t)) {
      if (npieces >= sv->max_items) return fail(FBG_E_INVAL, "internal: more pieces than staging room");
      fbg::BatchItem &q = hi[npieces++];
      q.prog = (uint32_t)items[k].prog;
      q.slot = (uint32_t)items[k].slot;
      q.t0 = t;
      q.t1 = t + std::min(chunk, e - t);
      q.step = 1;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  e = hipMemcpyAsync(sl.d, sl.h, items_at + (size_t)npieces * sizeof(fbg::BatchItem), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "server upload");
  fbg::BatchArgs a;
  a.progs = (const fbg::BatchProg *)(sl.d + kServerHeadBytes);
  a.items = (const fbg::BatchItem *)(sl.d + items_at);
  a.nitems = (uint32_t)npieces;
  a.max_regs = lds_regs(max_regs, l);
  a.head = (uint32_t *)sl.d;
  a.counts = d_counts;
  a.j16_any = j16_any();
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((npieces + wpb - 1) / wpb, (int64_t)cus * occ));
  e = fbg::launch_batch(fbg::EVAL_COUNT, l, var, a, grid, 64 * wpb, lds, s);
  if (e == hipSuccess) e = hipEventRecord(sl.done, s);
  sl.used = true;
  return e == hipSuccess ? FBG_OK : hip_fail(e, "launch of the server slice");
}

void fbg_server_free(fbg_server *sv) {
  if (!sv) return;
  for (auto &sl : sv->slots) {
    if (sl.used && sl.done) (void)hipEventSynchronize(sl.done);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.h) (void)hipHostFree(sl.h);
    if (sl.d) (void)hipFree(sl.d);
  }
  delete sv;
}

// --------------------------------------------------------------- debugging

fbg_status fbg_program_emulate(const fbg_program *p, int32_t words_per_lane, uint64_t *h_dnf, uint64_t out_words,
                               uint64_t *h_count) {
  if (!p) return fail(FBG_E_INVAL, "program is NULL");
  if (p->c.n > 30) return fail(FBG_E_RANGE, "emulation is limited to n <= 30");
  int l;
  fbg_status st = parse_wpl(words_per_lane, l);
  if (st) return st;
  if ((st = check_tiling(p, l))) return st;
  const uint64_t need = dnf_words_of(p->c.n);
  if (h_dnf && out_words < need) return fail(FBG_E_INVAL, "out_words too small");
  std::vector<uint32_t> s32((size_t)std::max<uint64_t>(2, p->nslices), 0u);
  fbg::emulate_program(p->words[l], p->nins[l], p->c.nregs, p->c.n, l, p->cofactor, s32.data());
  if (h_dnf) memcpy(h_dnf, s32.data(), need * 8);
  if (h_count) {
    uint64_t c = 0;
    for (uint64_t i = 0; i < p->nslices; i++) c += (uint64_t)__builtin_popcount(s32[i]);
    *h_count = c;
  }
  return FBG_OK;
}

int64_t fbg_program_disasm(const fbg_program *p, int32_t words_per_lane, char *buf, int64_t cap) {
  if (!p) return -1;
  int l = p->auto_log2w;
  if (words_per_lane > 0 && parse_wpl(words_per_lane, l)) return -1;
  if (check_tiling(p, l)) return -1;
  std::string s = fbg::disasm_program(p->words[l], p->nins[l], l);
  if (buf && cap > 0) {
    size_t k = std::min<size_t>((size_t)cap - 1, s.size());
    memcpy(buf, s.data(), k);
    buf[k] = 0;
  }
  return (int64_t)s.size();
}

}  // extern "C"
