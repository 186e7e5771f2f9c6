// fbg_device.h -- gfx950 kernels for evaluating Boolean terms on the free
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
//   k_batch<LOG2W, VAR, MODE>  many programs, persistent waves popping work
//                         items (program, tiles t0 + k step) from eight
//                         device queues, one per XCD, with stealing; counts,
//                         and with MODE_DNF the DNF vectors too
//   k_scan_*              exclusive scan of per-tile counts
//   k_zero_*, k_set_u64   fills (used instead of memset so that a caller may
//                         capture the launches into a graph)
//
// The kernel templates live here; each eval_*.hip / batch.hip / misc.hip
// translation unit instantiates and launches its share of them, so that the
// library builds in parallel.
#ifndef FBG_DEVICE_H
#define FBG_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbg_asm16.h"
#include "fbg_isa.h"
#include "fbg_kernels.h"

namespace fbg {
namespace dev {

enum { MODE_COUNT = 0, MODE_DNF = 1, MODE_TILECNT = 2, MODE_ENUM = 3 };

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }


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

// ---- the general part of a program (after the clause prefix)
//
// Every operation on cur is one v_bitop3 per word whose truth table the
// encoder chose (w0 bits 8..15): inputs cur (0xF0), T or the register (0xCC)
// and the word pattern P(i) (0xAA).  The cases below are every table the
// encoder emits; a switch on a wave-uniform value costs a few scalar
// instructions, after which each word is a single VALU instruction.
#define FBG_LIT_TABLES(X) \
  X(0xEE) X(0x11) X(0x66) X(0x99) X(0xE0) X(0x10) X(0x60) X(0xFE) X(0xF1) X(0xF6) \
  X(0x1E) X(0xE1) X(0x96) X(0x1F) X(0xEF) X(0x9F) X(0x01) X(0x0E) X(0x09) X(0x69)
#define FBG_REG_TABLES(X) \
  X(0xC0) X(0x30) X(0xFC) X(0xF3) X(0x3C) X(0xC3) X(0x3F) X(0xCF) X(0x03) X(0x0C) X(0xCC) X(0x33)

// Any truth table, bit by bit (never reached with the encoder's tables).
__device__ __forceinline__ uint32_t bitop3_any(uint32_t a, uint32_t b, uint32_t c, uint32_t tt) {
  uint32_t r = 0;
#pragma unroll
  for (uint32_t m = 0; m < 8; m++) {
    if (!((tt >> m) & 1u)) continue;
    r |= ((m & 4u) ? a : ~a) & ((m & 2u) ? b : ~b) & ((m & 1u) ? c : ~c);
  }
  return r;
}

// cur = bitop3(cur, b, c) in place: the tied operand keeps cur in the same
// registers in every case of the dispatch, so the cases merge without copies.
#define FBG_BITOP3_INPLACE(d, b, c, tt) \
  asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:" #tt : "+v"(d) : "v"(b), "s"(c))
#define FBG_BITOP3_INPLACE_2(d, b, tt) asm("v_bitop3_b32 %0, %0, %1, 0 bitop3:" #tt : "+v"(d) : "v"(b))

template <int W>
__device__ __forceinline__ void lit_op(uint32_t tt, uint32_t (&cur)[W], uint32_t T, const uint32_t (&P)[W]) {
  switch (tt) {
#define FBG_CASE(x)                                                                    \
  case x:                                                                              \
    _Pragma("unroll") for (int i = 0; i < W; i++) FBG_BITOP3_INPLACE(cur[i], T, P[i], x); \
    break;
    FBG_LIT_TABLES(FBG_CASE)
#undef FBG_CASE
    default:
#pragma unroll
      for (int i = 0; i < W; i++) cur[i] = bitop3_any(cur[i], T, P[i], tt);
  }
}

// The same for a literal set without word-index literals (P = 0 on every
// word): no pattern words are loaded.
template <int W>
__device__ __forceinline__ void lit_op0(uint32_t tt, uint32_t (&cur)[W], uint32_t T) {
  switch (tt) {
#define FBG_CASE(x)                                                                    \
  case x:                                                                              \
    _Pragma("unroll") for (int i = 0; i < W; i++) FBG_BITOP3_INPLACE_2(cur[i], T, x); \
    break;
    FBG_LIT_TABLES(FBG_CASE)
#undef FBG_CASE
    default:
#pragma unroll
      for (int i = 0; i < W; i++) cur[i] = bitop3_any(cur[i], T, 0u, tt);
  }
}

template <int W>
__device__ __forceinline__ void reg_op(uint32_t tt, uint32_t (&cur)[W], const uint32_t (&R)[W]) {
  switch (tt) {
#define FBG_CASE(x)                                                                    \
  case x:                                                                              \
    _Pragma("unroll") for (int i = 0; i < W; i++) FBG_BITOP3_INPLACE_2(cur[i], R[i], x); \
    break;
    FBG_REG_TABLES(FBG_CASE)
#undef FBG_CASE
    default:
#pragma unroll
      for (int i = 0; i < W; i++) cur[i] = bitop3_any(cur[i], R[i], 0u, tt);
  }
}

// Registers 0..kVgprRegs-1 live in VGPRs (selected by a wave-uniform switch);
// higher ones in LDS, W*64 words each (the launch sizes LDS for those only).
static_assert(kVgprRegs == 4, "the register switches below name registers 0..3");

// The VGPR state of the general part: cur and the first kVgprRegs
// registers.  A kernel keeps one per wave across all its tiles and clears it
// once: every program writes cur and a register before reading them, so a
// tile needs no reset.
template <int W>
struct GenState {
  uint32_t cur[W];
  uint32_t rv[kVgprRegs][W];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < W; i++) cur[i] = 0u;
#pragma unroll
    for (uint32_t r = 0; r < kVgprRegs; r++)
#pragma unroll
      for (int i = 0; i < W; i++) rv[r][i] = 0u;
  }
};

template <int LOG2W>
__device__ __forceinline__ void run_general(code_ptr w, const code_ptr table, uint32_t nins, uint64_t U0,
                                            uint32_t lane, uint32_t (&acc)[1 << LOG2W],
                                            GenState<1 << LOG2W> &st, uint32_t *__restrict__ regs) {
  constexpr int W = 1 << LOG2W;
  uint32_t (&cur)[W] = st.cur;
  uint32_t tmp[W];
  for (uint32_t pc = 0; pc < nins; ++pc, w += FBG_INS_WORDS) {
    const u32x8 ins = *(const __attribute__((address_space(4))) u32x8 *)w;
    const uint32_t w0 = ins[0];
    const uint32_t op = w0 & 15u;
    const uint32_t tt = (w0 >> FBG_F_SHIFT) & 0xFFu;
    if (op <= FBG_OP_OPL) {  // LDL / OPL (the encoder keeps CL in the clause block)
      const uint64_t lm = (uint64_t)ins[2] | ((uint64_t)ins[3] << 32);
      const uint64_t sel = (uint64_t)ins[4] | ((uint64_t)ins[5] << 32);
      uint32_t T;
      if (!(w0 & FBG_XORSET)) {
        const uint64_t neg = (uint64_t)ins[6] | ((uint64_t)ins[7] << 32);
        const uint64_t lmq = lm | (((U0 & sel) != neg) ? ~0ull : 0ull);
        T = __builtin_amdgcn_inverse_ballot_w64(lmq) ? ~0u : ins[1];
      } else {
        const uint32_t S = ins[1] ^ ((__popcll(U0 & sel) & 1) ? ~0u : 0u);
        T = lane_part(lm) ^ S;
      }
      if (w0 & FBG_HASPAT) {
        const code_ptr Pp = table + (w0 >> FBG_ARG_SHIFT);
        uint32_t P[W];
#pragma unroll
        for (int i = 0; i < W; i++) P[i] = Pp[i];
        lit_op<W>(tt, cur, T, P);
      } else {
        lit_op0<W>(tt, cur, T);
      }
      continue;
    }
    const uint32_t r = w0 >> FBG_ARG_SHIFT;
    switch (op) {
      case FBG_OP_ST:
        switch (r) {
#define FBG_ST(k) \
  case k:         \
    _Pragma("unroll") for (int i = 0; i < W; i++) st.rv[k][i] = cur[i]; \
    break;
          FBG_ST(0) FBG_ST(1) FBG_ST(2) FBG_ST(3)
#undef FBG_ST
          default: {
            uint32_t *R = regs + (size_t)(r - kVgprRegs) * (W * 64) + lane;
#pragma unroll
            for (int i = 0; i < W; i++) R[i * 64] = cur[i];
          }
        }
        if (w0 & FBG_INVOUT) {
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = ~cur[i];
        }
        break;
      case FBG_OP_OPR:
      case FBG_OP_LDR:
        switch (r) {
          case 0: reg_op<W>(tt, cur, st.rv[0]); break;
          case 1: reg_op<W>(tt, cur, st.rv[1]); break;
          case 2: reg_op<W>(tt, cur, st.rv[2]); break;
          case 3: reg_op<W>(tt, cur, st.rv[3]); break;
          default: {
            const uint32_t *R = regs + (size_t)(r - kVgprRegs) * (W * 64) + lane;
#pragma unroll
            for (int i = 0; i < W; i++) tmp[i] = R[i * 64];
            reg_op<W>(tt, cur, tmp);
          }
        }
        break;
      case FBG_OP_ACC:
        if (w0 & FBG_INV) {
#pragma unroll
          for (int i = 0; i < W; i++) acc[i] &= ~cur[i];
        } else {
#pragma unroll
          for (int i = 0; i < W; i++) acc[i] &= cur[i];
        }
        if (w0 & FBG_INVOUT) {
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = ~cur[i];
        }
        break;
      default:  // FBG_OP_NOT; an INVOUT on it (a folded second NOT) cancels it
        if (!(w0 & FBG_INVOUT)) {
#pragma unroll
          for (int i = 0; i < W; i++) cur[i] = ~cur[i];
        }
        break;
    }
  }
}

// One chunk of the clause block: the tile tests of its clauses (lane l takes
// clause l mod 32; one compare across the wave) and U, the clauses of the
// chunk that neither a lane nor a tile literal satisfies on this lane.
__device__ __forceinline__ uint32_t chunk_tile_bits(const uint32_t *__restrict__ ch, uint32_t nc, uint64_t U0,
                                                    uint32_t lane) {
  const uint32_t c = min(lane & (FBG_CB_CHUNK - 1u), nc - 1u);
  const uint4 td = *(const uint4 *)(ch + FBG_CB_CHUNK_HDR + 64 + 4 * c);
  const uint64_t sel = (uint64_t)td.x | ((uint64_t)td.y << 32);
  const uint64_t neg = (uint64_t)td.z | ((uint64_t)td.w << 32);
  return (uint32_t)__ballot((U0 & sel) != neg);
}

// Top bits of the runs (keys) of a chunk that meet U (fbg_isa.h).
__device__ __forceinline__ uint32_t runs_false(uint32_t U, uint32_t T, uint32_t F) {
  return (((U & ~T) + F) | U) & T;
}

// G & (m | ~x): v_bitop3 over (G = 0xF0, m = 0xCC, x = 0xAA).
constexpr uint32_t kTT_KEY = 0xF0u & (0xCCu | (~0xAAu & 0xFFu));
// m | ~x over (m = 0xF0, x = 0xCC).
constexpr uint32_t kTT_ORNOT = (0xF0u | (~0xCCu & 0xFFu)) & 0xFFu;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) char *code_byte_ptr;

// The clause block (fbg_isa.h): the per-lane products G_g of the static
// groups chunk by chunk, acc from them by a product tree that also applies
// the keys of the first multi chunk at their levels, then any later multi
// chunk on the W words.
template <int LOG2W>
__device__ __forceinline__ void run_clauses(const uint32_t *__restrict__ cb_g, const code_ptr table, uint64_t U0,
                                            uint32_t lane, uint32_t (&acc)[1 << LOG2W]) {
  constexpr int W = 1 << LOG2W;
  constexpr int NG = 1 + 2 * LOG2W;
  const code_ptr cb = (code_ptr)cb_g;
  const uint32_t nstat = cb[1], nmulti = cb[2];
  uint32_t G[NG];
#pragma unroll
  for (int g = 0; g < NG; g++) G[g] = ~0u;
  const uint32_t *ch = cb_g + FBG_CB_HDR;
  for (uint32_t k = 0; k < nstat; ++k) {
    const code_ptr h = (code_ptr)ch;
    const u32x16 hd = *(const __attribute__((address_space(4))) u32x16 *)h;
    const uint32_t nc = hd[0];
    const uint32_t lb = ch[FBG_CB_CHUNK_HDR + lane];
    const uint32_t S = chunk_tile_bits(ch, nc, U0, lane);
    const uint32_t A = runs_false(~(lb | S), hd[2], hd[3]);
    // keys by group; hd[5 + g] is where group g's keys end (bytes)
    const code_byte_ptr hb = (code_byte_ptr)h;
    uint32_t off = (FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4;
#pragma unroll
    for (int g = 0; g < NG; g++) {
      for (; off < hd[5 + g]; off += 8) {
        const u32x2 km = *(const __attribute__((address_space(4))) u32x2 *)(hb + off);
        const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int)A, km[0], 1u);
        G[g] = __builtin_amdgcn_bitop3_b32(G[g], km[1], x, kTT_KEY);
      }
    }
    ch += hd[1];
  }
  // the first multi chunk: its false runs now, its keys inside the tree
  u32x16 mh = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t Am = 0, moff = 0;
  const code_byte_ptr mb = (code_byte_ptr)ch;
  if (nmulti) {
    mh = *(const __attribute__((address_space(4))) u32x16 *)ch;
    const uint32_t lb = ch[FBG_CB_CHUNK_HDR + lane];
    Am = runs_false(~(lb | chunk_tile_bits(ch, mh[0], U0, lane)), mh[2], mh[3]);
    moff = (FBG_CB_CHUNK_HDR + 64 + 4 * mh[0]) * 4;
  }
  // level j + 1 of the tree: the 2^(j+1) products of the words' low j + 1
  // bits; a multi key of level j + 1 acts on the nodes of its half
  acc[0] = G[0];
#pragma unroll
  for (int j = 0; j < LOG2W; j++) {
#pragma unroll
    for (int v = 0; v < (1 << j); v++) {
      acc[v | (1 << j)] = acc[v] & G[2 + 2 * j];
      acc[v] = acc[v] & G[1 + 2 * j];
    }
    if (j >= 1) {
#pragma unroll
      for (int half = 0; half < 2; half++) {
        for (; moff < mh[5 + 2 * (j - 1) + half]; moff += 16) {
          const u32x4 kq = *(const __attribute__((address_space(4))) u32x4 *)(mb + moff);
          const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int)Am, kq[0], 1u);
          const uint32_t T = __builtin_amdgcn_bitop3_b32(kq[1], x, 0u, kTT_ORNOT);
          const code_ptr P = table + kq[2];
#pragma unroll
          for (int v = 0; v < (1 << j); v++)
            acc[(half << j) | v] = __builtin_amdgcn_bitop3_b32(T, acc[(half << j) | v], P[v], kTT_AND_OR);
        }
      }
    }
  }
  // later multi chunks (more than 32 multi clauses): on the W words
  if (nmulti > 1) {
    ch += mh[1];
    for (uint32_t k = 1; k < nmulti; ++k) {
      const code_ptr h = (code_ptr)ch;
      const u32x16 hd = *(const __attribute__((address_space(4))) u32x16 *)h;
      const uint32_t nc = hd[0];
      const uint32_t lb = ch[FBG_CB_CHUNK_HDR + lane];
      const uint32_t A = runs_false(~(lb | chunk_tile_bits(ch, nc, U0, lane)), hd[2], hd[3]);
      const code_byte_ptr hb = (code_byte_ptr)h;
      for (uint32_t off = (FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4; off < hd[5]; off += 16) {
        const u32x4 kq = *(const __attribute__((address_space(4))) u32x4 *)(hb + off);
        const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int)A, kq[0], 1u);
        const uint32_t T = __builtin_amdgcn_bitop3_b32(kq[1], x, 0u, kTT_ORNOT);
        const code_ptr P = table + kq[2];
#pragma unroll
        for (int i = 0; i < W; i++) acc[i] = __builtin_amdgcn_bitop3_b32(T, acc[i], P[i], kTT_AND_OR);
      }
      ch += hd[1];
    }
  }
}

// The uniform-cofactor test of one tile (lane-parallel: each lane may ask
// about another tile): 0 when a clause made only of tile literals is false on
// the whole tile, which makes the program false there (acc only loses bits
// after the clause block), else 1.  The encoder lists the tile selectors of
// every such clause in a table at the end of the clause block, its length in
// the first static chunk's h[4]; they are read as scalars.  Every lane runs
// it (no divergent branch around it), and the result is a 0/1 word, not a
// lane-mask boolean.
template <int LOG2W>
__device__ __forceinline__ uint32_t tile_alive(const uint32_t *__restrict__ cb_g, uint64_t t) {
  const code_ptr cb = (code_ptr)cb_g;
  if (cb[1] == 0) return 1u;
  const uint32_t k = cb[FBG_CB_HDR + 4];
  const code_ptr td = cb + cb[0] - 4 * k;
  const uint64_t U0 = t << LOG2W;
  uint32_t dead = 0u;
  for (uint32_t c = 0; c < k; ++c) {
    const u32x4 e = *(const __attribute__((address_space(4))) u32x4 *)(td + 4 * c);
    const uint64_t sel = (uint64_t)e[0] | ((uint64_t)e[1] << 32);
    const uint64_t neg = (uint64_t)e[2] | ((uint64_t)e[3] << 32);
    dead |= (uint32_t)((U0 & sel) == neg);
  }
  return dead ^ 1u;
}

// A bijection of [0, n): cycle-walking over a bijection of the bits-bit
// integers (2^bits >= n > 2^(bits - 1), mask = 2^bits - 1), two rounds of an
// xor-shift (invertible for a shift >= 1) and a multiplication by an odd
// constant (invertible modulo 2^bits).  The walk from x < n ends: following
// the permutation's cycle through x returns to x.
__device__ __forceinline__ uint64_t tile_hash(uint64_t x, uint64_t n, uint32_t bits, uint64_t mask) {
  const uint32_t h = bits > 1 ? bits >> 1 : 1u;
  do {
    x = ((x ^ (x >> h)) * 0x9E3779B97F4A7C15ull) & mask;
    x = ((x ^ (x >> h)) * 0xD6E8FEB86659FD93ull) & mask;
    x ^= x >> h;
  } while (x >= n);
  return x;
}

// Visit the tiles first, first + stride, ... below end.  body(t, alive):
// alive = false means the tile is known to be all zeros (uniform cofactor)
// and need not be evaluated.  With COF the wave tests the next 64 tiles at
// once, one per lane, and visits only the live ones, or (ALL) every tile,
// the dead ones with alive = false.  Lanes past the end test some tile
// beyond it; the valid mask removes them.  With HASH (COF only: a launch in
// which wave w of nw visits w, w + nw, ... of the tiles [0, end)) the k-th
// tile a wave visits is tile_hash of that index instead: the tiles that
// survive the test often share their low index bits, and a power-of-two
// stride would give them all to a few waves.
template <int LOG2W, bool COF, bool ALL, bool HASH = false, typename Body>
__device__ __forceinline__ void for_tiles(const uint32_t *__restrict__ code, uint64_t first, uint64_t stride,
                                          uint64_t end, uint32_t lane, Body &&body) {
  if (!COF) {
    for (uint64_t t = first; t < end; t += stride) body(t, true);
    return;
  }
  uint32_t bits = 0;
  if (HASH)
    while ((1ull << bits) < end) bits++;
  const uint64_t mask = bits >= 64 ? ~0ull : (1ull << bits) - 1;
  for (uint64_t q0 = 0; first + q0 * stride < end; q0 += 64) {
    const uint64_t il = first + (q0 + lane) * stride;
    const uint64_t valid = __ballot(il < end);
    const uint64_t tl = HASH && il < end ? tile_hash(il, end, bits, mask) : il;
    const uint64_t alive = __ballot(tile_alive<LOG2W>(code, tl) != 0u) & valid;
    uint64_t todo = ALL ? valid : alive;
    while (todo) {
      const uint32_t l = (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      // lane l's tile, read as a scalar (l is wave-uniform)
      const uint64_t t = HASH ? (uint64_t)__builtin_amdgcn_readlane((uint32_t)tl, l) |
                                    (uint64_t)__builtin_amdgcn_readlane((uint32_t)(tl >> 32), l) << 32
                              : first + (q0 + l) * stride;
      body(t, ((alive >> l) & 1ull) != 0);
    }
  }
}

// Interpret one program over the W words of this lane in tile group U0: the
// clause block, then (GEN) the instructions after it.
// regs: this wave's LDS registers; at 16 words per lane the registers from
// lds_bytes on (byte offsets in the jump-table form) live in global memory at
// gregs instead (a block per wave).
template <int LOG2W, bool GEN>
__device__ __forceinline__ void run_program(const uint32_t *__restrict__ code_g, uint32_t nins, uint64_t U0,
                                            uint32_t lane, uint32_t (&acc)[1 << LOG2W],
                                            GenState<1 << LOG2W> &st, uint32_t *__restrict__ regs,
                                            uint32_t lds_bytes = 0, uint32_t *gregs = nullptr,
                                            uint32_t j16_any = 0) {
  const code_ptr cb = (code_ptr)code_g;
  const code_ptr ins = cb + cb[0];
  const code_ptr table = ins + FBG_TABLE_OFFSET(nins, LOG2W);
  if constexpr (GEN && LOG2W == FBG_J16_LOG2W) {
    // programs without clauses (most general programs) skip the block and
    // its product tree: acc starts all-ones (wave-uniform test); only here,
    // where the register map is fixed anyway, so the other kernels keep
    // their register allocation
    if (cb[1] + cb[2] == 0) {
#pragma unroll
      for (int i = 0; i < (1 << LOG2W); i++) acc[i] = ~0u;
    } else {
      run_clauses<LOG2W>(code_g, table, U0, lane, acc);
    }
  } else {
    run_clauses<LOG2W>(code_g, table, U0, lane, acc);
  }
  if (!GEN) return;
  if constexpr (LOG2W == FBG_J16_LOG2W) {
    // the jump-table form; LDS registers at this wave's block, 64 bytes a lane
    const uint32_t lds_lane =
        (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint32_t *)regs) + lane * 64u;
    run_general_j16((const uint32_t *)(uintptr_t)ins, (const uint32_t *)(uintptr_t)table, U0, lds_lane, lds_bytes,
                    gregs, lane, acc, j16_any);
  } else {
    run_general<LOG2W>(ins, table, nins, U0, lane, acc, st, regs);
  }
}

// Store a tile of the XCD-local layout (fbg_kernels.h): the program's
// renamed variables put the lane's words 4g .. 4g+3 side by side, so each
// group is one 16-byte store to 1 KiB unit g & 3 of the tile's piece g >> 2
// (the second piece 8 pieces, 32 KiB, after the first).  dst = the first
// piece + 4 lane words, 16-byte aligned.  (Instantiated for every W; called
// at W = 32 only.)
template <int W>
__device__ __forceinline__ void store_xcd_tile(const uint32_t (&acc)[W], uint32_t *dst) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int g = 0; g < W / 4; g++) {
    const u32x4 v = {acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
    __builtin_nontemporal_store(v, (u32x4 *)(dst + (g >> 2) * 8192 + (g & 3) * 256));
  }
}

// Zero the words of this lane that lie beyond the valuation space.
template <int LOG2W>
__device__ __forceinline__ void mask_tail(uint32_t (&acc)[1 << LOG2W], uint64_t U0, uint32_t lane,
                                          uint64_t nslices, int n) {
  constexpr int W = 1 << LOG2W;
  if ((U0 + W) * 64 > nslices) {  // wave-uniform
    // valid words of the tile, at most 64 W: 32-bit compares per word
    const uint64_t base = U0 * 64;
    const uint32_t rem = (uint32_t)min(nslices > base ? nslices - base : 0ull, (unsigned long long)W * 64);
    // word i of this lane is valid when 64 i + lane < rem, i.e. when
    // d = rem - lane exceeds 64 i: one VGPR and an immediate per word, no
    // per-word lane constants kept across the tile loop
    const int d = (int)rem - (int)lane;
#pragma unroll
    for (int i = 0; i < W; i++) acc[i] = d > 64 * i ? acc[i] : 0u;
    if (n < FBG_SLICE_BITS) acc[0] &= (uint32_t)((1ull << (1u << n)) - 1u);
  }
}

// Wave sums.  ds_swizzle exchanges within each half of the wave with the
// lane pattern in the instruction (no address registers to keep live across
// the tile loop); the two halves meet through v_readlane.  The result is
// wave-uniform.
template <int XOR>
__device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (XOR << 10));
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  v += swz_xor<16>(v);
  v += swz_xor<8>(v);
  v += swz_xor<4>(v);
  v += swz_xor<2>(v);
  v += swz_xor<1>(v);
  return (uint32_t)__builtin_amdgcn_readlane(v, 0) + (uint32_t)__builtin_amdgcn_readlane(v, 32);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#define FBG_SUM_STEP(x)                                                   \
  {                                                                       \
    const uint64_t t = ((uint64_t)hi << 32 | lo) +                        \
                       ((uint64_t)swz_xor<x>(hi) << 32 | swz_xor<x>(lo)); \
    lo = (uint32_t)t;                                                     \
    hi = (uint32_t)(t >> 32);                                             \
  }
  FBG_SUM_STEP(16) FBG_SUM_STEP(8) FBG_SUM_STEP(4) FBG_SUM_STEP(2) FBG_SUM_STEP(1)
#undef FBG_SUM_STEP
  // readlane returns int: widen through uint32_t, never by sign extension
  const uint64_t a = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 0) << 32 |
                     (uint32_t)__builtin_amdgcn_readlane(lo, 0);
  const uint64_t b = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 32) << 32 |
                     (uint32_t)__builtin_amdgcn_readlane(lo, 32);
  return a + b;
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
    if (__ballot(x != 0u) == 0ull) continue;  // wave-uniform: no model in this word of any lane
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

// DNF write-out and count of one tile: the words past the valuation space
// are cleared (only the single tile of a program smaller than one tile has
// any), the words inside the output stored, and the models of this lane
// counted.  A whole tile's stores are issued unconditionally (streaming: the
// vector is not read back by this kernel).
template <int LOG2W>
__device__ __forceinline__ uint32_t store_count_tile(const uint32_t (&acc)[1 << LOG2W], uint64_t U0, uint32_t lane,
                                                     uint64_t nslices, int n, uint32_t *out32, uint64_t out_slices) {
  constexpr int W = 1 << LOG2W;
  uint32_t *dst = out32 + U0 * 64 + lane;
  uint32_t c = 0;
  if ((U0 + W) * 64 <= nslices) {  // wave-uniform; out_slices >= nslices
#pragma unroll
    for (int i = 0; i < W; i++) {
      __builtin_nontemporal_store(acc[i], dst + i * 64);
      c += __popc(acc[i]);
    }
  } else {
    const uint64_t base = U0 * 64;
    const uint32_t rem = (uint32_t)min(nslices > base ? nslices - base : 0ull, (unsigned long long)W * 64);
    const uint32_t rem_out = (uint32_t)min(out_slices > base ? out_slices - base : 0ull, (unsigned long long)W * 64);
    const uint32_t m0 = n < FBG_SLICE_BITS ? (uint32_t)((1ull << (1u << n)) - 1u) : ~0u;
#pragma unroll
    for (int i = 0; i < W; i++) {
      // word (i, lane) of the tile is valid when lane < rem - 64 i (a
      // wave-uniform bound: no per-word lane constants)
      uint32_t v = (int)lane < (int)rem - 64 * i ? acc[i] : 0u;
      if (i == 0) v &= m0;
      if ((int)lane < (int)rem_out - 64 * i) dst[i * 64] = v;
      c += __popc(v);
    }
  }
  return c;
}

// Store the W words of this lane; the stores of a whole tile are issued
// unconditionally (streaming: the vector is not read back by this kernel).
template <int LOG2W>
__device__ __forceinline__ void store_tile(const uint32_t (&acc)[1 << LOG2W], uint64_t U0, uint32_t lane,
                                           uint32_t *out32, uint64_t out_slices) {
  constexpr int W = 1 << LOG2W;
  uint32_t *dst = out32 + U0 * 64 + lane;
  if ((U0 + W) * 64 <= out_slices) {  // wave-uniform
#pragma unroll
    for (int i = 0; i < W; i++) __builtin_nontemporal_store(acc[i], dst + i * 64);
  } else {
#pragma unroll
    for (int i = 0; i < W; i++)
      if ((U0 + i) * 64 + lane < out_slices) dst[i * 64] = acc[i];
  }
}

// Waves per SIMD each evaluator instance is compiled for (its VGPR budget),
// as many as fit without spilling: programs made of clauses alone fit 8
// (<= 64 VGPRs), the uniform-cofactor variant 7 at W = 32; the general
// interpreter 6 at W <= 8, 4 at W = 16 (124 VGPRs: cur, acc and four
// registers per word) and is left unconstrained above.
constexpr int min_waves(int log2w, int var) {
  return (var & 1) ? (log2w <= 3 ? 6 : (log2w == 4 ? 4 : 1)) : ((var & 2) && log2w == 5 ? 7 : 8);
}

template <int LOG2W, int MODE, int VAR>
__global__ __launch_bounds__(256, min_waves(LOG2W, VAR)) void k_eval(EvalArgs a) {
  constexpr int W = 1 << LOG2W;
  extern __shared__ uint32_t lds[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  uint32_t *regs = lds + (size_t)wib * a.nregs * (W * 64);
  const uint64_t wave = (uint64_t)blockIdx.x * wpb + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
  uint64_t total = 0;
  GenState<W> st;
  if (VAR & 1) st.clear();
  // dead tiles (uniform cofactor) still write their zeros in DNF mode;
  // counting and compaction skip them, and so does the tile-count pass,
  // whose counts the host clears beforehand
  constexpr bool ALL = MODE == MODE_DNF;
  for_tiles<LOG2W, (VAR & 2) != 0, ALL, true>(a.code, wave, nwaves, a.ntiles, lane, [&](uint64_t t, bool alive) {
    const uint64_t U0 = t << LOG2W;
    if (MODE == MODE_ENUM) {
      if (a.tile_counts[t] == 0u) return;  // no model in this tile
    }
    uint32_t acc[W];
    if (LOG2W == 5 && VAR == 0 && MODE == MODE_DNF && a.xcd_code) {
      // XCD-local layout (fbg_kernels.h): full tiles only (n >= 21), output
      // 16-byte aligned
      run_program<LOG2W, false>(a.xcd_code, a.nins, U0, lane, acc, st, regs);
      store_xcd_tile(acc, a.out32 + (((t >> 2) & 7) + 16 * (t & 3) + 64 * (t >> 5)) * 1024 + lane * 4);
      return;
    }
    if (alive) {
      run_program<LOG2W, (VAR & 1) != 0>(a.code, a.nins, U0, lane, acc, st, regs, a.nregs * (W * 256u), nullptr,
                                         a.j16_any);
      mask_tail<LOG2W>(acc, U0, lane, a.nslices, a.n);
    } else {
#pragma unroll
      for (int i = 0; i < W; i++) acc[i] = 0u;
    }
    if (MODE == MODE_COUNT) {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < W; i++) c += __popc(acc[i]);
      total += c;
    } else if (MODE == MODE_DNF) {
      store_tile<LOG2W>(acc, U0, lane, a.out32, a.out_slices);
    } else if (MODE == MODE_TILECNT) {
      tile_count_out<LOG2W>(acc, lane, a.tile_counts + t);
    } else {
      tile_compact<LOG2W>(acc, U0, lane, a.tile_offsets[t], a.out_idx, a.capacity);
    }
  });
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
    const uint32_t *src = a.out32 + U0 * 64 + lane;
    if ((U0 + W) * 64 <= a.nslices) {  // wave-uniform: a whole tile, every load issued at once
#pragma unroll
      for (int i = 0; i < W; i++) acc[i] = __builtin_nontemporal_load(src + i * 64);
    } else {
#pragma unroll
      for (int i = 0; i < W; i++) {
        const uint64_t s = (U0 + i) * 64 + lane;
        acc[i] = s < a.nslices ? src[i * 64] : 0u;
      }
    }
    if (MODE == MODE_TILECNT)
      tile_count_out<LOG2W>(acc, lane, a.tile_counts + t);
    else
      tile_compact<LOG2W>(acc, U0, lane, a.tile_offsets[t], a.out_idx, a.capacity);
  }
}

// ---------------------------------------------------------------- batches

// MODE_COUNT adds each program's model count into its slot; MODE_DNF also
// writes the program's DNF vector (BatchProg.out32).  The item and program
// tables are read-only during the launch: scalar loads, so tile indices and
// code pointers stay wave-uniform.
template <int LOG2W, int VAR, int MODE>
__global__ __launch_bounds__(256, min_waves(LOG2W, VAR)) void k_batch(BatchArgs a) {
  constexpr int W = 1 << LOG2W;
  extern __shared__ uint32_t lds[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  uint32_t *regs = lds + (size_t)wib * a.max_regs * (W * 64);
  // registers beyond the LDS block: this wave's block of global scratch
  uint32_t *gregs = a.gscratch ? a.gscratch + ((size_t)blockIdx.x * (blockDim.x >> 6) + wib) * a.gstride : nullptr;
  typedef const __attribute__((address_space(4))) BatchItem *item_ptr;
  typedef const __attribute__((address_space(4))) BatchProg *prog_ptr;
  // A wave adds its count to a program's slot once per run of items of
  // that program, not once per item: same-address device atomics serialize.
  uint64_t total = 0;
  uint32_t cur_slot = ~0u;
  GenState<W> st;
  if (VAR & 1) st.clear();
  auto process = [&](uint32_t item) {
    const item_ptr it = (item_ptr)a.items + item;
    const uint64_t t0 = it->t0, t1 = it->t1, step = it->step;
    const uint32_t slot = it->slot;
    const prog_ptr p = (prog_ptr)a.progs + it->prog;
    if (slot != cur_slot) {  // wave-uniform
      const uint64_t s = wave_sum_u64(total);
      if (lane == 0 && s) atomicAdd((unsigned long long *)(a.counts + cur_slot), (unsigned long long)s);
      total = 0;
      cur_slot = slot;
    }
    for_tiles<LOG2W, (VAR & 2) != 0, MODE == MODE_DNF>(p->code, t0, step, t1, lane, [&](uint64_t t, bool alive) {
      const uint64_t U0 = t << LOG2W;
      uint32_t acc[W];
      if (alive) {
        run_program<LOG2W, (VAR & 1) != 0>(p->code, p->nins, U0, lane, acc, st, regs, a.max_regs * (W * 256u), gregs,
                                           a.j16_any);
      } else {
#pragma unroll
        for (int i = 0; i < W; i++) acc[i] = 0u;
      }
      uint32_t c = 0;
      if (MODE == MODE_DNF) {
        c = store_count_tile<LOG2W>(acc, U0, lane, p->nslices, p->n, p->out32, p->out_slices);
      } else {
        mask_tail<LOG2W>(acc, U0, lane, p->nslices, p->n);
#pragma unroll
        for (int i = 0; i < W; i++) c += __popc(acc[i]);
      }
      total += c;
      if (MODE == MODE_DNF && p->tile_counts) {  // for a later batched enumeration
        const uint32_t tc = wave_sum_u32(c);
        if (lane == 0) p->tile_counts[t] = tc;
      }
    });
  };
  // Items come sorted by cost, largest first, dealt over kQueues queues:
  // queue q holds items q, q + kQueues, ...  A wave pops from the queue of
  // its XCD (workgroups go to the XCDs round-robin), then from the others
  // until all are drained; a drained queue is seen by a plain read before
  // any atomic is spent on it.
  const uint32_t q0 = blockIdx.x % kQueues;
  for (uint32_t k = 0; k < kQueues; ++k) {
    const uint32_t q = (q0 + k) % kQueues;
    uint32_t *head = a.head + q * kQueueStride;
    if (k > 0 && q + kQueues * __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)head) >= a.nitems) continue;
    for (;;) {
      uint32_t r = 0;
      if (lane == 0) r = atomicAdd(head, 1u);
      const uint32_t item = q + kQueues * __builtin_amdgcn_readfirstlane(r);  // lane 0 took the item
      if (item >= a.nitems) break;  // this queue is drained
      process(item);
    }
  }
  const uint64_t s = wave_sum_u64(total);
  if (lane == 0 && s) atomicAdd((unsigned long long *)(a.counts + cur_slot), (unsigned long long)s);
}

// Batched DNF write-out of a plan of clause-only programs without the uniform
// cofactor, on a grid of fresh blocks whose waves take a.run consecutive
// tiles each: the blocks start in order, so the waves write the vectors in
// order together, and no wave spends a queue pop or a count atomic.  a.items
// holds the plan's programs, one entry each, with [t0, t1) its tiles in the
// plan's tile order (ascending, contiguous, a.nitems >= 1); wave w takes plan
// tiles [w run, (w + 1) run), each tile finding its own program (a run may
// cross from one program into the next).  Every program has a
// tile-count array: the tile's model count goes there, and the program's count
// is the later sum over them (k_sum_tile_counts).
template <int LOG2W>
__global__ __launch_bounds__(256, min_waves(LOG2W, 0)) void k_batch_direct(BatchArgs a) {
  constexpr int W = 1 << LOG2W;
  typedef const __attribute__((address_space(4))) BatchItem *item_ptr;
  typedef const __attribute__((address_space(4))) BatchProg *prog_ptr;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  const uint64_t g0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wib) * a.run;
  const item_ptr items = (item_ptr)a.items;
  const uint64_t end = items[a.nitems - 1].t1;
  if (g0 >= end) return;
  uint32_t lo = 0, hi = a.nitems;  // the entry with t0 <= g0 < t1, found once
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (items[mid].t0 <= g0)
      lo = mid;
    else
      hi = mid;
  }
  for (uint64_t g = g0; g < g0 + a.run && g < end; ++g) {  // wave-uniform
    while (g >= items[lo].t1) lo++;  // the run crossed into the next program
    const item_ptr it = items + lo;
    if (g < it->t0) continue;  // padding in front of a program of the XCD-local layout
    const prog_ptr p = (prog_ptr)a.progs + it->prog;
    const uint64_t t = g - it->t0;
    const uint64_t U0 = t << LOG2W;
    uint32_t acc[W];
    GenState<W> st;  // unused: clause-only programs
    if (LOG2W == 5 && p->xcd_code && p->chunk_counts) {
      // XCD-local layout (fbg_kernels.h): the renamed program's tile t is
      // the pieces x + 8 h + 16 (t & 3) + 64 (t >> 5) of the vector, h = 0, 1
      // (words 0..15 and 16..31 of each lane), x = bits 2..4 of t; full tiles
      // only (n >= 21), output 16-byte aligned
      run_program<LOG2W, false>(p->xcd_code, p->nins, U0, lane, acc, st, nullptr);
      const uint64_t piece = ((t >> 2) & 7) + 16 * (t & 3) + 64 * (t >> 5);
      store_xcd_tile(acc, p->out32 + piece * 1024 + lane * 4);
      uint32_t c0 = 0, c1 = 0;
#pragma unroll
      for (int i = 0; i < W; i++) {
        if (i < 16)
          c0 += __popc(acc[i]);
        else
          c1 += __popc(acc[i]);
      }
      c0 = wave_sum_u32(c0);
      c1 = wave_sum_u32(c1);
      // the two piece counts side by side, in tile order: the four waves of a
      // block fill 32 contiguous bytes
      if (lane == 0) *(uint2 *)(p->chunk_counts + 2 * t) = make_uint2(c0, c1);
    } else {
      run_program<LOG2W, false>(p->code, p->nins, U0, lane, acc, st, nullptr);
      const uint32_t c = store_count_tile<LOG2W>(acc, U0, lane, p->nslices, p->n, p->out32, p->out_slices);
      const uint32_t tc = wave_sum_u32(c);
      if (lane == 0) p->tile_counts[t] = tc;
    }
  }
}

#ifdef FBG_DEVICE_BATCH_KERNELS  // defined once, in batch.hip
// Counts after k_batch_direct: block (m, y) adds its share of the tile counts
// of entry m's program into that program's count slot (zeroed before).  For a
// program of the XCD-local layout it first forms each tile count from the
// counts of the tile's two 4 KiB pieces.
__global__ __launch_bounds__(256) void k_sum_tile_counts(BatchArgs a) {
  __shared__ uint64_t part[4];
  const BatchItem &it = a.items[blockIdx.x];
  const BatchProg &p = a.progs[it.prog];
  uint64_t s = 0;
  const bool xcd = p.xcd_code && p.chunk_counts;
  for (uint64_t t = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; t < p.ntiles; t += (uint64_t)gridDim.y * blockDim.x) {
    if (xcd) {
      // tile t of the vector is pieces 2t and 2t + 1; piece c came from
      // tile (c & 7) << 2 | (c >> 4 & 3) | (c >> 6) << 5 of the renamed
      // program, its half c >> 3 & 1
      uint32_t v = 0;
      for (uint64_t c = 2 * t; c < 2 * t + 2; c++) {
        const uint64_t k = ((c & 7) << 2) | ((c >> 4) & 3) | ((c >> 6) << 5);
        v += p.chunk_counts[2 * k + ((c >> 3) & 1)];
      }
      p.tile_counts[t] = v;
      s += v;
    } else {
      s += p.tile_counts[t];
    }
  }
  s = wave_sum_u64(s);
  if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (uint32_t w = 0; w < (blockDim.x >> 6); w++) tot += part[w];
    if (tot) atomicAdd((unsigned long long *)(a.counts + it.slot), (unsigned long long)tot);
  }
}

#endif

// Batched enumeration from the stored DNF vectors: every wave strides over
// the global tile list of all programs (tile counts and their exclusive scan
// concatenated in program order), skips programs of the other plan and tiles
// without models, and compacts the models of a tile into its program's list.
template <int LOG2W>
__global__ __launch_bounds__(256) void k_batch_compact(BatchEnumArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = uni(threadIdx.x) >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wib;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  typedef const __attribute__((address_space(4))) EnumProg *enum_ptr;
  // one tile with models per wave and step, from the list k_list_tiles built
  const uint32_t nlist = *a.nlist;
  for (uint64_t k = wave; k < nlist; k += nwaves) {
    const uint64_t g = a.list[k];
    // the program owning global tile g: tile0 ascends with the program index
    uint32_t lo = 0, hi = a.np;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (((enum_ptr)a.progs)[mid].tile0 <= g) lo = mid; else hi = mid;
    }
    const enum_ptr p = (enum_ptr)a.progs + lo;
    if (p->log2w != (uint32_t)LOG2W || p->capacity == 0) continue;
    const uint64_t t = g - p->tile0;
    const uint64_t U0 = t << LOG2W;
    constexpr int W = 1 << LOG2W;
    uint32_t acc[W];
    const uint32_t *src = p->dnf + U0 * 64 + lane;
#pragma unroll
    for (int i = 0; i < W; i++) {
      const uint64_t sidx = (U0 + i) * 64 + lane;
      acc[i] = sidx < p->nslices ? src[i * 64] : 0u;
    }
    const uint64_t first = a.offsets[g] - a.offsets[p->tile0];
    tile_compact<LOG2W>(acc, U0, lane, first, p->out, p->capacity);
  }
}

#ifdef FBG_DEVICE_BATCH_KERNELS
// The global indices of the tiles that hold models, in any order (every
// tile's output position comes from the scan, not from the list order).
__global__ __launch_bounds__(256) void k_list_tiles(BatchEnumArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.total_tiles; g += stride)
    if (a.tile_counts[g] != 0u) a.list[atomicAdd(a.nlist, 1u)] = (uint32_t)g;
}

#endif

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

#ifdef FBG_DEVICE_MISC_KERNELS  // defined once, in misc.hip
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

// p[0..n) = 0 and head[0..nhead) = 0 (queue heads and list counters).
__global__ void k_zero_u64(uint64_t *p, uint64_t n, uint32_t *head, uint32_t nhead) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i < nhead) head[i] = 0;
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

#endif

}  // namespace dev
}  // namespace fbg

#endif
