// kernels.hip -- gfx950 kernels for evaluating Boolean terms on the free
// generators (Section 2.3: d_j = t(b_1j .. b_nj) for every block j, each block
// computed bitwise; 2^r processors act as one 2^(k+r)-bit processor).
//
// One wave (64 lanes) evaluates one tile of 64*W 32-bit words per step; the
// index layout and the instruction format are described in fbg_isa.h.  The
// program is read with scalar loads (it is wave-uniform), generator words are
// synthesised in registers, and all bitwise work is VALU integer logic.
//
// Kernels:
//   k_eval<LOG2W, MODE, VAR>  one program, persistent grid-stride over tiles;
//                         MODE_COUNT   popcount -> wave sum -> 64-bit atomic
//                         MODE_DNF     store the words (coalesced)
//                         MODE_TILECNT per-tile model counts (enumeration 1)
//                         MODE_ENUM    ascending model indices (enumeration 2)
//                         VAR bit 0 (GEN): programs with more than clauses
//                         VAR bit 1 (COF): the uniform-cofactor variant
//   k_dnf_scan<MODE>      the two enumeration passes over a stored DNF vector
//   k_batch<LOG2W, VAR>   many programs, persistent waves popping work items
//                         (program, tile range) from a device queue
//   k_scan_*              exclusive scan of per-tile counts
//   k_zero_*, k_set_u64   fills (used instead of memset so that a caller may
//                         capture the launches into a graph)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbg_isa.h"
#include "fbg_kernels.h"

namespace fbg {
namespace dev {

enum { MODE_COUNT = 0, MODE_DNF = 1, MODE_TILECNT = 2, MODE_ENUM = 3 };

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint32_t fapply(uint32_t f, uint32_t a, uint32_t b) {
  return f == FBG_F_AND ? (a & b) : (f == FBG_F_OR ? (a | b) : (a ^ b));
}

// Truth table of v_bitop3_b32(a, b, c): the function applied to the masks
// a = 0xF0, b = 0xCC, c = 0xAA.  kTT_AND_OR(T, acc, P) = acc & (T | P).
constexpr uint32_t kTT_AND_OR = 0xCCu & (0xF0u | 0xAAu);

// Program words are wave-uniform and never written by a kernel: reading them
// through the constant address space makes every fetch a scalar load.
typedef const __attribute__((address_space(4))) uint32_t *code_ptr;
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

// Lane part of a literal set: all-ones on the lanes whose bit is set in the
// 64-bit lane mask (a VCC-style mask, so this is one v_cndmask).
__device__ __forceinline__ uint32_t lane_part(uint64_t lanemask) {
  return __builtin_amdgcn_inverse_ballot_w64(lanemask) ? ~0u : 0u;
}

// Interpret one program over the W words of this lane in tile group U0.
// The first ncl instructions are clauses (the code generator emits them
// first); GEN = false means there is nothing else.
//
// COF = true is the uniform-cofactor variant: the tile bits of the index are
// constants on the whole tile, so a clause with a true tile literal holds on
// the tile and is skipped, and a clause whose only literals are false tile
// literals is false on the whole tile, which ends the tile (acc = 0).  The
// result is the same; the work depends on the data.  The encoder puts the
// clauses made only of tile literals first.
template <int LOG2W, bool GEN, bool COF>
__device__ __forceinline__ void run_program(const uint32_t *__restrict__ code_g, uint32_t nins, uint32_t ncl,
                                            uint64_t U0, uint32_t lane, uint32_t (&acc)[1 << LOG2W],
                                            uint32_t *__restrict__ regs) {
  constexpr int W = 1 << LOG2W;
  const code_ptr code = (code_ptr)code_g;
  const code_ptr table = code + (size_t)nins * FBG_INS_WORDS;
#pragma unroll
  for (int i = 0; i < W; i++) acc[i] = ~0u;

  // ---- clauses: acc &= mconst | V(lane) | P(i) | Q(U0), one v_bitop3 per
  // word.  Branch-free, so acc stays in place across iterations.
  code_ptr w = code;
  if (COF) {
    for (uint32_t k = 0; k < ncl; ++k, w += FBG_INS_WORDS) {
      const u32x8 ins = *(const __attribute__((address_space(4))) u32x8 *)w;
      const uint64_t sel = (uint64_t)ins[4] | ((uint64_t)ins[5] << 32);
      const uint64_t neg = (uint64_t)ins[6] | ((uint64_t)ins[7] << 32);
      if ((U0 & sel) != neg) continue;  // a true tile literal: the clause holds on the tile
      const uint64_t lm = (uint64_t)ins[2] | ((uint64_t)ins[3] << 32);
      const uint32_t poff = ins[0] >> FBG_ARG_SHIFT;  // entry 0 is the all-zero pattern
      if (lm == 0 && ins[1] == 0u && poff == 0u) {    // only false tile literals: the tile is dead
#pragma unroll
        for (int i = 0; i < W; i++) acc[i] = 0u;
        return;
      }
      const uint32_t T = __builtin_amdgcn_inverse_ballot_w64(lm) ? ~0u : ins[1];
      const code_ptr P = table + poff;
#pragma unroll
      for (int i = 0; i < W; i++) acc[i] = __builtin_amdgcn_bitop3_b32(T, acc[i], P[i], kTT_AND_OR);
    }
  } else if (LOG2W <= 4 && ncl > 0) {
    // Software-pipelined: while clause k runs on the VALU, the scalar unit
    // already fetches clause k+1 and its pattern entry (whose index clause k
    // carries in w0 bits 8..15), so neither load latency is exposed.  Reads
    // one instruction past the clauses, which stays inside the program.
    u32x8 a = *(const __attribute__((address_space(4))) u32x8 *)w;
    uint32_t pa[W], pb[W];
    u32x8 b;
    {
      const code_ptr P = table + (a[0] >> FBG_ARG_SHIFT);
#pragma unroll
      for (int i = 0; i < W; i++) pa[i] = P[i];
    }
    // one clause with (cur, pcur) while (nxt, pnxt) is fetched; the two
    // halves of the loop swap the roles, so no register is ever copied
    auto step = [&](const u32x8 &cur, const uint32_t (&pcur)[W], u32x8 &nxt, uint32_t (&pnxt)[W]) {
      const uint64_t lm = (uint64_t)cur[2] | ((uint64_t)cur[3] << 32);
      const uint64_t sel = (uint64_t)cur[4] | ((uint64_t)cur[5] << 32);
      const uint64_t neg = (uint64_t)cur[6] | ((uint64_t)cur[7] << 32);
      const uint64_t lmq = lm | (((U0 & sel) != neg) ? ~0ull : 0ull);
      const uint32_t mconst = cur[1];
      const code_ptr Pn = table + ((cur[0] >> FBG_F_SHIFT) & 0xFFu) * (uint32_t)W;
      // keep the prefetch below the (waited) uses of the current clause
      __builtin_amdgcn_sched_barrier(0);
      w += FBG_INS_WORDS;
      nxt = *(const __attribute__((address_space(4))) u32x8 *)w;
#pragma unroll
      for (int i = 0; i < W; i++) pnxt[i] = Pn[i];
      const uint32_t T = __builtin_amdgcn_inverse_ballot_w64(lmq) ? ~0u : mconst;
#pragma unroll
      for (int i = 0; i < W; i++) acc[i] = __builtin_amdgcn_bitop3_b32(T, acc[i], pcur[i], kTT_AND_OR);
    };
    uint32_t k = 0;
    for (;;) {
      step(a, pa, b, pb);
      if (++k >= ncl) break;
      step(b, pb, a, pa);
      if (++k >= ncl) break;
    }
  } else {
  for (uint32_t k = 0; k < ncl; ++k, w += FBG_INS_WORDS) {
    // the whole instruction in one s_load_dwordx8
    const u32x8 ins = *(const __attribute__((address_space(4))) u32x8 *)w;
    const uint32_t w0 = ins[0];
    const uint64_t lm = (uint64_t)ins[2] | ((uint64_t)ins[3] << 32);
    const uint64_t sel = (uint64_t)ins[4] | ((uint64_t)ins[5] << 32);
    const uint64_t neg = (uint64_t)ins[6] | ((uint64_t)ins[7] << 32);
    // a true tile literal makes the clause all-ones on every lane: fold it
    // into the 64-bit lane mask (scalar logic), then one v_cndmask gives
    // T = V(lane) | Q ? all-ones : mconst
    const uint64_t lmq = lm | (((U0 & sel) != neg) ? ~0ull : 0ull);
    const uint32_t T = __builtin_amdgcn_inverse_ballot_w64(lmq) ? ~0u : ins[1];
    const code_ptr P = table + (w0 >> FBG_ARG_SHIFT);
#pragma unroll
    for (int i = 0; i < W; i++) acc[i] = __builtin_amdgcn_bitop3_b32(T, acc[i], P[i], kTT_AND_OR);
  }
  }
  if (!GEN) return;

  // ---- general structure through cur and the LDS registers
  uint32_t cur[W];
#pragma unroll
  for (int i = 0; i < W; i++) cur[i] = 0u;
  for (uint32_t pc = ncl; pc < nins; ++pc, w += FBG_INS_WORDS) {
    const uint32_t w0 = w[0];
    const uint32_t op = w0 & 15u;
    const uint32_t invm = (w0 & FBG_INV) ? ~0u : 0u;
    if (op <= FBG_OP_OPL) {
      // literal set L = mconst OP V(lane) OP P(i) OP Q(U0), then cur = f(cur, L)
      const uint64_t lm = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
      const uint64_t sel = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
      const bool isx = (w0 & FBG_XORSET) != 0;
      uint32_t S;
      if (!isx) {
        const uint64_t neg = (uint64_t)w[6] | ((uint64_t)w[7] << 32);
        S = ((U0 & sel) != neg) ? ~0u : w[1];
      } else {
        S = w[1] ^ ((__popcll(U0 & sel) & 1) ? ~0u : 0u);
      }
      const uint32_t V = lane_part(lm);
      const code_ptr P = table + (w0 >> FBG_ARG_SHIFT);
      if (op == FBG_OP_CL) {  // a clause outside the prefix (the compiler emits none)
#pragma unroll
        for (int i = 0; i < W; i++) acc[i] &= V | (S | P[i]);
        continue;
      }
      const uint32_t f = (op == FBG_OP_LDL) ? 3u : ((w0 >> FBG_F_SHIFT) & 3u);
#pragma unroll
      for (int i = 0; i < W; i++) {
        const uint32_t L = (isx ? (V ^ (S ^ P[i])) : (V | (S | P[i]))) ^ invm;
        cur[i] = (f == 3u) ? L : fapply(f, cur[i], L);
      }
    } else {
      const uint32_t r = w0 >> FBG_ARG_SHIFT;
      uint32_t *R = regs + (size_t)r * (W * 64) + lane;
      switch (op) {
        case FBG_OP_ST:
#pragma unroll
          for (int i = 0; i < W; i++) R[i * 64] = cur[i];
          break;
        case FBG_OP_OPR: {
          const uint32_t f = (w0 >> FBG_F_SHIFT) & 3u;
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = fapply(f, cur[i], R[i * 64] ^ invm);
          break;
        }
        case FBG_OP_ACC:
#pragma unroll
          for (int i = 0; i < W; i++) acc[i] &= cur[i] ^ invm;
          break;
        case FBG_OP_LDR:
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = R[i * 64] ^ invm;
          break;
        default:  // FBG_OP_NOT
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = ~cur[i];
          break;
      }
    }
    if (w0 & FBG_INVOUT) {
#pragma unroll
      for (int i = 0; i < W; i++) cur[i] = ~cur[i];
    }
  }
}

// Zero the words of this lane that lie beyond the valuation space.
template <int LOG2W>
__device__ __forceinline__ void mask_tail(uint32_t (&acc)[1 << LOG2W], uint64_t U0, uint32_t lane,
                                          uint64_t nslices, int n) {
  constexpr int W = 1 << LOG2W;
  if ((U0 + W) * 64 > nslices) {  // wave-uniform
#pragma unroll
    for (int i = 0; i < W; i++) {
      const uint64_t s = (U0 + i) * 64 + lane;
      if (s >= nslices) acc[i] = 0u;
    }
    if (n < FBG_SLICE_BITS) acc[0] &= (uint32_t)((1ull << (1u << n)) - 1u);
  }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t olo = __shfl_xor(lo, off, 64), ohi = __shfl_xor(hi, off, 64);
    const uint64_t t = ((uint64_t)hi << 32 | lo) + ((uint64_t)ohi << 32 | olo);
    lo = (uint32_t)t;
    hi = (uint32_t)(t >> 32);
  }
  return (uint64_t)hi << 32 | lo;
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= (uint32_t)off) v += o;
  }
  return v;
}

// Enumeration epilogues shared by the evaluator and the stored-DNF path.
template <int LOG2W>
__device__ __forceinline__ void tile_count_out(const uint32_t (&acc)[1 << LOG2W], uint32_t lane, uint32_t *dst) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < (1 << LOG2W); i++) c += __popc(acc[i]);
  c = wave_sum_u32(c);
  if (lane == 0) *dst = c;
}

// Words of a tile ascend with (i, lane): word (U0 + i) * 64 + lane.
template <int LOG2W>
__device__ __forceinline__ void tile_compact(const uint32_t (&acc)[1 << LOG2W], uint64_t U0, uint32_t lane,
                                             uint64_t base, uint64_t *out, uint64_t capacity) {
#pragma unroll
  for (int i = 0; i < (1 << LOG2W); i++) {
    uint32_t x = acc[i];
    const uint32_t c = __popc(x);
    const uint32_t incl = wave_inclusive_scan(c, lane);
    const uint32_t tot = __shfl(incl, 63, 64);
    uint64_t pos = base + (incl - c);
    const uint64_t vbase = ((U0 + i) * 64 + lane) * 32;
    while (x) {
      const uint32_t j = (uint32_t)__builtin_ctz(x);
      if (pos < capacity) out[pos] = vbase + j;
      pos++;
      x &= x - 1u;
    }
    base += tot;
  }
}

template <int LOG2W, int MODE, int VAR>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
  constexpr int W = 1 << LOG2W;
  extern __shared__ uint32_t lds[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  uint32_t *regs = lds + (size_t)wib * a.nregs * (W * 64);
  const uint64_t wave = (uint64_t)blockIdx.x * wpb + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
  uint64_t total = 0;
  for (uint64_t t = wave; t < a.ntiles; t += nwaves) {
    const uint64_t U0 = t << LOG2W;
    if (MODE == MODE_ENUM) {
      if (a.tile_counts[t] == 0u) continue;  // no model in this tile
    }
    uint32_t acc[W];
    run_program<LOG2W, (VAR & 1) != 0, (VAR & 2) != 0>(a.code, a.nins, a.ncl, U0, lane, acc, regs);
    mask_tail<LOG2W>(acc, U0, lane, a.nslices, a.n);
    if (MODE == MODE_COUNT) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < W; i++) c += __popc(acc[i]);
      total += c;
    } else if (MODE == MODE_DNF) {
#pragma unroll
      for (int i = 0; i < W; i++) {
        const uint64_t s = (U0 + i) * 64 + lane;
        if (s < a.out_slices) a.out32[s] = acc[i];
      }
    } else if (MODE == MODE_TILECNT) {
      tile_count_out<LOG2W>(acc, lane, a.tile_counts + t);
    } else {
      tile_compact<LOG2W>(acc, U0, lane, a.tile_offsets[t], a.out_idx, a.capacity);
    }
  }
  if (MODE == MODE_COUNT) {
    const uint64_t s = wave_sum_u64(total);
    if (lane == 0 && s) atomicAdd((unsigned long long *)a.out_count, (unsigned long long)s);
  }
}

// Enumeration over a stored DNF vector: chunks of 64 x 32 words laid out as
// the evaluator's tiles with W = 32; a.out32 is the DNF (read only here).
template <int MODE>
__global__ __launch_bounds__(256) void k_dnf_scan(EvalArgs a) {
  constexpr int LOG2W = 5, W = 32;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * wpb + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
  for (uint64_t t = wave; t < a.ntiles; t += nwaves) {
    const uint64_t U0 = t << LOG2W;
    if (MODE == MODE_ENUM) {
      if (a.tile_counts[t] == 0u) continue;
    }
    uint32_t acc[W];
#pragma unroll
    for (int i = 0; i < W; i++) {
      const uint64_t s = (U0 + i) * 64 + lane;
      acc[i] = s < a.nslices ? a.out32[s] : 0u;
    }
    if (MODE == MODE_TILECNT)
      tile_count_out<LOG2W>(acc, lane, a.tile_counts + t);
    else
      tile_compact<LOG2W>(acc, U0, lane, a.tile_offsets[t], a.out_idx, a.capacity);
  }
}

// ---------------------------------------------------------------- batches

template <int LOG2W, int VAR>
__global__ __launch_bounds__(256) void k_batch(BatchArgs a) {
  constexpr int W = 1 << LOG2W;
  extern __shared__ uint32_t lds[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  uint32_t *regs = lds + (size_t)wib * a.max_regs * (W * 64);
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(a.head, 1u);
    item = uni(__shfl(item, 0, 64));
    if (item >= a.nitems) break;  // every wave leaves once the queue is drained
    const BatchItem it = a.items[item];
    const BatchProg p = a.progs[it.prog];
    uint64_t total = 0;
    for (uint64_t t = it.t0; t < it.t1; ++t) {
      const uint64_t U0 = t << LOG2W;
      uint32_t acc[W];
      run_program<LOG2W, (VAR & 1) != 0, (VAR & 2) != 0>(p.code, p.nins, p.ncl, U0, lane, acc, regs);
      mask_tail<LOG2W>(acc, U0, lane, p.nslices, p.n);
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < W; i++) c += __popc(acc[i]);
      total += c;
    }
    const uint64_t s = wave_sum_u64(total);
    if (lane == 0 && s) atomicAdd((unsigned long long *)(a.counts + it.slot), (unsigned long long)s);
  }
}

// ------------------------------------------------------------------ scans

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t &block_total) {
  const uint32_t tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    const uint64_t o = tid >= (uint32_t)off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += o;
    __syncthreads();
  }
  block_total = sh[SCAN_THREADS - 1];
  const uint64_t excl = sh[tid] - v;
  __syncthreads();
  return excl;
}

// Per block of SCAN_BLOCK elements: the block's sum.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *in, uint64_t n, uint64_t *block_sums) {
  __shared__ uint64_t sh[SCAN_THREADS];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
  uint64_t s = 0;
  for (int k = 0; k < SCAN_PER_THREAD; k++)
    if (base + k < n) s += in[base + k];
  uint64_t tot;
  block_exclusive_scan(s, sh, tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the block sums in place; *total = grand total.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(uint64_t *sums, uint64_t nb, uint64_t *total) {
  __shared__ uint64_t sh[SCAN_THREADS];
  uint64_t carry = 0;
  for (uint64_t st = 0; st < nb; st += SCAN_THREADS) {
    const uint64_t i = st + threadIdx.x;
    const uint64_t v = i < nb ? sums[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan(v, sh, tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const uint32_t *in, uint64_t n,
                                                             const uint64_t *block_prefix, uint64_t *out) {
  __shared__ uint64_t sh[SCAN_THREADS];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
  uint64_t s = 0;
  for (int k = 0; k < SCAN_PER_THREAD; k++)
    if (base + k < n) s += in[base + k];
  uint64_t tot;
  uint64_t ex = block_exclusive_scan(s, sh, tot) + block_prefix[blockIdx.x];
  for (int k = 0; k < SCAN_PER_THREAD; k++)
    if (base + k < n) {
      out[base + k] = ex;
      ex += in[base + k];
    }
}

// ------------------------------------------------------------------ fills

__global__ void k_zero_u64(uint64_t *p, uint64_t n, uint32_t *head) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (head && i == 0) *head = 0;
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace dev

// ------------------------------------------------------- host-side launches

namespace {

template <int MODE, int VAR>
hipError_t launch_eval_w(int log2w, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_eval<0, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_eval<1, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_eval<2, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_eval<3, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_eval<4, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_eval<5, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_eval_mode(int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds,
                            hipStream_t s) {
  switch (var) {
    case 0: return launch_eval_w<MODE, 0>(log2w, a, grid, block, lds, s);
    case 1: return launch_eval_w<MODE, 1>(log2w, a, grid, block, lds, s);
    case 2: return launch_eval_w<MODE, 2>(log2w, a, grid, block, lds, s);
    case 3: return launch_eval_w<MODE, 3>(log2w, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int VAR>
hipError_t launch_batch_w(int log2w, const BatchArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_batch<0, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_batch<1, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_batch<2, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_batch<3, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_batch<4, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_batch<5, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(int mode, int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds,
                       hipStream_t s) {
  switch (mode) {
    case dev::MODE_COUNT: return launch_eval_mode<dev::MODE_COUNT>(log2w, var, a, grid, block, lds, s);
    case dev::MODE_DNF: return launch_eval_mode<dev::MODE_DNF>(log2w, var, a, grid, block, lds, s);
    case dev::MODE_TILECNT: return launch_eval_mode<dev::MODE_TILECNT>(log2w, var, a, grid, block, lds, s);
    case dev::MODE_ENUM: return launch_eval_mode<dev::MODE_ENUM>(log2w, var, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dnf_scan(int mode, const EvalArgs &a, int grid, int block, hipStream_t s) {
  if (mode == dev::MODE_TILECNT)
    hipLaunchKernelGGL((dev::k_dnf_scan<dev::MODE_TILECNT>), dim3(grid), dim3(block), 0, s, a);
  else if (mode == dev::MODE_ENUM)
    hipLaunchKernelGGL((dev::k_dnf_scan<dev::MODE_ENUM>), dim3(grid), dim3(block), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_batch(int log2w, int var, const BatchArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (var) {
    case 0: return launch_batch_w<0>(log2w, a, grid, block, lds, s);
    case 1: return launch_batch_w<1>(log2w, a, grid, block, lds, s);
    case 2: return launch_batch_w<2>(log2w, a, grid, block, lds, s);
    case 3: return launch_batch_w<3>(log2w, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *block_sums, uint64_t *total,
                       hipStream_t s) {
  const uint64_t nb = (n + dev::SCAN_BLOCK - 1) / dev::SCAN_BLOCK;
  if (nb == 0) {
    hipLaunchKernelGGL(dev::k_set_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(dev::k_scan_reduce, dim3((unsigned)nb), dim3(dev::SCAN_THREADS), 0, s, in, n, block_sums);
  hipLaunchKernelGGL(dev::k_scan_sums, dim3(1), dim3(dev::SCAN_THREADS), 0, s, block_sums, nb, total);
  hipLaunchKernelGGL(dev::k_scan_apply, dim3((unsigned)nb), dim3(dev::SCAN_THREADS), 0, s, in, n, block_sums, out);
  return hipGetLastError();
}

uint64_t scan_block_count(uint64_t n) { return (n + dev::SCAN_BLOCK - 1) / dev::SCAN_BLOCK; }

hipError_t launch_zero(uint64_t *p, uint64_t n, uint32_t *head, hipStream_t s) {
  const uint64_t threads = n > 0 ? n : 1;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  hipLaunchKernelGGL(dev::k_zero_u64, dim3(grid), dim3(256), 0, s, p, n, head);
  return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(dev::k_set_u64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace fbg
