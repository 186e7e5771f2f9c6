/*
 * fbg_isa.h -- the device program format interpreted by the evaluator.
 *
 * Index layout.  The 2^n valuations are cut into 32-bit words ("slices"):
 * slice s holds valuations 32s .. 32s+31 (Section 2.3 blocks with k = 5).  A
 * wave of 64 lanes evaluates one tile of 64*W slices; lane l and word i of
 * tile t hold slice s = (t*W + i)*64 + l.  The bits of a valuation index mu
 * therefore fall into four classes:
 *   bits 0..4                 position inside the 32-bit word: generator k
 *                             is the constant mask MASK_k (0xAAAAAAAA, ...)
 *   bits 5..10                the lane l: generator k is all-ones or zero
 *                             per lane (bit k-5 of l)
 *   bits 11..11+log2(W)-1     the word index i inside the lane
 *   bits 11+log2(W) ..        the tile t, the same for the whole wave
 * so every generator word is synthesised from (l, i, t) and no generator
 * vector is ever read from memory (Section 2.2 defines b_k bit mu = bit k of
 * mu).
 *
 * Literal sets.  An OR (or XOR) of literals factors over those classes:
 *   L = mconst  OP  V(l)  OP  P(i)  OP  Q(t),       OP in {|, ^}
 * with mconst the OP of the in-word literals, V(l) = -(bit l of lanemask),
 * P(i) = -(bit i of pat), and Q(t) = -( ((U0 ^ neg) & sel) != 0 ) for OR,
 * -( parity(U0 & sel) ) for XOR, where U0 = t*W is the slice group index of
 * word 0 (the word-index bits are zero in U0; sel/neg only use bits >= log2 W).
 * A literal set may be inverted (INV), which makes AND-sets of literals.
 *
 * Registers per slice: acc (the running conjunction, starts all-ones), cur
 * (the value being built) and R[0..nregs) in LDS.
 *
 * Instruction: 8 x uint32.
 *   w0 bits 0..3   opcode
 *      bit 4       XORSET  literal set combines with XOR (else OR)
 *      bit 5       HASLANE lanemask != 0
 *      bit 6       INV     second operand inverted (literal set / register)
 *      bit 7       INVOUT  invert cur after the operation
 *      bits 8..9   f       binary function for OPL/OPR: 0 AND, 1 OR, 2 XOR
 *      bits 8..15  (CL only) index of the pattern entry of pat, see below
 *      bits 16..31 pat (literal-set ops) or register index (register ops)
 *   w1           mconst
 *   w2, w3       lanemask (lo, hi)
 *   w4, w5       sel (lo, hi)
 *   w6, w7       neg (lo, hi)
 * Opcodes:
 *   CL   acc &= L            LDL  cur = L            OPL  cur = f(cur, L)
 *   ST   R[r] = cur          OPR  cur = f(cur, R[r]^inv)
 *   ACC  acc &= cur ^ inv    LDR  cur = R[r] ^ inv   NOT  cur = ~cur
 * CL carries plain OR-sets only (no XORSET, no INV).
 *
 * Pattern table.  After the nins instructions comes a table of W-word
 * entries; entry e holds P(0..W-1) = -(bit i of pat) for one pattern, entry 0
 * is all zeros.  A clause reads its W values with one scalar load instead of
 * extracting W bits.  Per-word patterns are ORs of literals over the log2 W
 * word-index bits, so there are at most 3^(log2 W) <= 81 of them.
 */
#ifndef FBG_ISA_H
#define FBG_ISA_H

#include <stdint.h>

#define FBG_OP_CL 1u
#define FBG_OP_LDL 2u
#define FBG_OP_OPL 3u
#define FBG_OP_ST 4u
#define FBG_OP_OPR 5u
#define FBG_OP_ACC 6u
#define FBG_OP_LDR 7u
#define FBG_OP_NOT 8u

#define FBG_XORSET (1u << 4)
#define FBG_HASLANE (1u << 5)
#define FBG_INV (1u << 6)
#define FBG_INVOUT (1u << 7)
#define FBG_F_SHIFT 8
#define FBG_F_AND 0u
#define FBG_F_OR 1u
#define FBG_F_XOR 2u
#define FBG_ARG_SHIFT 16

#define FBG_INS_WORDS 8
#define FBG_LANE_BITS 6  /* 64 lanes per wave */
#define FBG_SLICE_BITS 5 /* 32 valuations per word */
#define FBG_TILE_BASE_BIT (FBG_SLICE_BITS + FBG_LANE_BITS) /* 11 */

/* In-word generator masks: bit j of MASK_k is bit k of j (Section 2.2). */
static inline uint32_t fbg_inword_mask(int k) {
  static const uint32_t m[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
  return m[k];
}

#endif
