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
 * Registers per slice: acc (the running conjunction), cur (the value being
 * built) and R[0..nregs) (the first few in VGPRs, the rest in LDS).
 *
 * Clause block.  The leading clauses of a program (its top-level conjunction
 * of OR-sets) are not instructions: they form a block that comes first in
 * the encoded program and sets acc.  Write a clause as T_c(l, t) | P_c(i),
 * with T_c = mconst | V(l) | Q(t) and P_c the OR of its word-index literals.
 * P_c is the only part that depends on the word, so clauses are grouped by
 * it; by distributivity AND_c (T_c | P) = (AND_c T_c) | P, and a group costs
 * one per-lane product whatever its size.  Groups:
 *   0          no word literal: applies to every word
 *   1 + 2j + v one word literal, on word-index bit j, false on the words
 *              whose bit j is v
 *   multi      two or more word literals: P(i) from the pattern table
 * With G_g the per-lane product of group g, the static groups give
 *   acc[i] = G_0 & AND_j G_{1 + 2j + (bit j of i)},
 * which the kernels build as a product tree, level by level (2W - 2 ANDs per
 * tile): level j + 1 holds the 2^(j+1) products of the words' low j + 1
 * bits.  A multi key whose highest word literal is on bit j (false where bit
 * j is v) touches only the level-(j + 1) nodes of the half v, and within it
 * the nodes its lower word literals leave false: it is applied there, 2^j
 * operations instead of W, and the tree carries it to the words.  The keys of
 * the first multi chunk act this way; later multi chunks (more than 32 such
 * clauses) act on the W words after the tree.
 *
 * Chunks.  Clauses are packed FBG_CB_CHUNK to a chunk, static and multi
 * clauses in separate chunks.  A chunk stores per lane the bits Lb[l] (bit c:
 * lane l satisfies clause c through a lane literal; bits >= nc are set) and
 * per clause the tile selectors (sel_c, neg_c).  One compare across lanes
 * (lane l takes clause l mod 32) gives S (bit c: a tile literal of clause c
 * holds, (U0 & sel_c) != neg_c), and U(l) = ~(Lb[l] | S) marks the clauses
 * left false on lane l by everything but their in-word and word literals.  A
 * key gathers a run of consecutive clauses of one group with the same
 * in-word part m: G_g &= (some clause of the run is in U) ? m : all-ones.
 * With T the top bits of the runs and F the other bits of runs longer than
 * one, the carries of ((U & ~T) + F) stop at the top of each run, so
 *   A = (((U & ~T) + F) | U) & T
 * has the top bit of a run set exactly when the run meets U: one add for all
 * the keys of a chunk, then one bit extract and one v_bitop3 per key.
 *
 * Block layout (uint32 words):
 *   cb[0] size of the block in words (the instructions start there)
 *   cb[1] static chunks   cb[2] multi chunks   cb[3] clauses
 *   then the chunks (static ones first), each:
 *     h[0] clauses nc (1 .. FBG_CB_CHUNK)   h[1] chunk size in words
 *     h[2] T   h[3] F
 *     h[4] first static chunk only: the length of the uniform-cofactor
 *          table
 *     h[5 ..] end of each slot's keys, in bytes from the chunk start; slots
 *          are the groups 0 .. 2 log2 W (static), the (level j, half v)
 *          pairs 2 (j - 1) + v (first multi chunk), or one (later ones)
 *     Lb[64]; (sel lo, sel hi, neg lo, neg hi) x nc
 *     keys: static (top bit, m); multi (top bit, m, pattern offset, 0), the
 *     pattern of the first multi chunk's keys over the 2^j nodes of their
 *     half
 *     zero padding to a multiple of 4 words
 *   then the uniform-cofactor table, the last 4 h[4] words of the block:
 *   (sel lo, sel hi, neg lo, neg hi) of every clause made only of tile
 *   literals (such a clause is constant on a tile; where it is false the
 *   whole tile is)
 *
 * Instruction: 8 x uint32.
 *   w0 bits 0..3   opcode
 *      bit 4       XORSET  literal set combines with XOR (else OR)
 *      bit 5       HASPAT  the literal set has word-index literals: the
 *                          kernel loads its W pattern words (else P = 0)
 *      bit 6       INV     second operand inverted (literal set / register)
 *      bit 7       INVOUT  invert cur after the operation
 *      bits 8..15  tt      LDL/OPL/LDR/OPR: the 8-bit truth table of the
 *                          v_bitop3_b32 the kernel applies per word, over
 *                          (cur = 0xF0, lane value T or register = 0xCC,
 *                          word pattern P(i) = 0xAA), with the operation,
 *                          the set's inversion and the output inversion
 *                          folded in (INV / INVOUT are then clear)
 *      bits 16..31 pattern offset (literal-set ops) or register index
 *                  (register ops)
 *   w1           mconst
 *   w2, w3       lanemask (lo, hi)
 *   w4, w5       sel (lo, hi)
 *   w6, w7       neg (lo, hi)
 * Opcodes (the instructions after the clause block; acc starts as the
 * block's value, cur as zero):
 *   CL   acc &= L            LDL  cur = L            OPL  cur = f(cur, L)
 *   ST   R[r] = cur          OPR  cur = f(cur, R[r]^inv)
 *   ACC  acc &= cur ^ inv    LDR  cur = R[r] ^ inv   NOT  cur = ~cur
 * CL carries plain OR-sets only (no XORSET, no INV).
 *
 * Pattern table.  After the nins instructions comes a table of W-word
 * entries; entry e holds P(0..W-1) = -(bit i of pat) for one pattern, entry 0
 * is all zeros.  An operation reads its W values with scalar loads instead of
 * extracting W bits.  Per-word patterns are ORs of literals over the log2 W
 * word-index bits, so there are at most 3^(log2 W) <= 243 of them.
 *
 * Jump-table form (16 words per lane only).  At 16 words per lane the
 * instructions after the clause block use another encoding, run by an
 * interpreter that jumps straight to the code of each instruction instead of
 * deciding among the cases with a chain of compares (kernels: fbg_asm16.h).
 * Literal-set instructions take 8 x uint32, all others 2:
 *   w0 bits 0..15   byte offset of the instruction's case in the jump table
 *                   (case number x FBG_J16_SLOT)
 *      bits 16..31  literal sets with word-index literals: byte offset of
 *                   their 16 pattern words in the pattern table
 *   w1           literal sets: mconst; register ops: the register's place,
 *                r x 16 for VGPR registers (r < 3: a VGPR index offset),
 *                (r - 3) x 4096 for LDS registers (a byte offset); unused
 *                by ACC and NOT
 *   w2..w7       literal sets only: lanemask, sel, neg as above
 * The case fixes the operation, its truth table and the instruction's length
 * (the case fetches the next instruction that far on); the cases are listed
 * below (FBG_J16_*).  A case END, padded to 8 words, follows the last
 * instruction, and the pattern table starts after it; the number of
 * instructions given for this form counts its length in units of 2 words,
 * END included.  The short forms halve the program bytes the scalar cache
 * streams through per tile.  LDS registers hold a lane's 16 words
 * contiguously (64 bytes per lane, 4096 per register and wave).
 *
 * Chains.  Two or more literal-set operations in a row, none with word
 * literals, act on cur through per-lane values only: bit by bit the chain
 * maps cur to (cur & X) | (~cur & Y), where X is what the chain makes of an
 * all-ones cur and Y what it makes of zero.  The jump-table form runs such a
 * run as XYF (X = f(~0, T), Y = f(0, T) for its first operation), XYM (X =
 * f(X, T), Y = f(Y, T) for each further one but the last) and XYL (the last:
 * X and Y updated, then per word one v_bitop3 over (cur, X, Y)): per lane two
 * operations per set instead of one per word, and one pass over the words
 * for the whole run.  X and Y live only inside a chain (an XYF always starts
 * one, an XYL always ends it).  In the plain form's terms (the disassembly
 * and the emulator) they are the opcodes XYF, XYM and XYL, which the plain
 * encoding never contains.
 *
 * Merged stores.  A store of cur into a VGPR register after which cur is dead
 * (the next instruction loads cur without reading it, or the program ends)
 * merges into the instruction before it when that one can write the register
 * itself: the last set of a chain (XYS: the chain's result goes to R[r], r x
 * 16 in bits 16..31 of w0), a literal set without word literals (LIS, r x 16
 * in the same place) or an operation on that same register (ORS: R[r] =
 * f(cur, R[r])).  cur keeps its old value; nothing reads it.  In the plain
 * form's terms they are the opcodes XYS, LIS and ORS.
 *
 * Merged ACC.  Likewise an ACC (acc &= cur, or acc &= ~cur) after which cur
 * is dead merges into the operation before it when that is an operation on
 * a VGPR register (ORA) or a literal set without word literals (LIA): one
 * v_bitop3 per word over (acc, cur, R[r] or T) computes acc AND the
 * operation's result.  In the plain form's terms: the opcode ACM.
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
/* chain operations: only as the decoded jump-table form (see Chains) */
#define FBG_OP_XYF 9u
#define FBG_OP_XYM 10u
#define FBG_OP_XYL 11u
/* a store merged into the instruction before it (see Merged stores): only
   as the decoded jump-table form */
#define FBG_OP_XYS 12u
#define FBG_OP_ORS 13u
#define FBG_OP_LIS 14u
/* an ACC merged into the operation before it (see Merged ACC): only as the
   decoded jump-table form; FBG_HASPAT marks the register form */
#define FBG_OP_ACM 15u

#define FBG_XORSET (1u << 4)
#define FBG_HASPAT (1u << 5)
#define FBG_INV (1u << 6)
#define FBG_INVOUT (1u << 7)
#define FBG_F_SHIFT 8
#define FBG_F_AND 0u
#define FBG_F_OR 1u
#define FBG_F_XOR 2u
#define FBG_ARG_SHIFT 16

#define FBG_INS_WORDS 8
/* Words per lane of the jump-table form, and where the pattern table starts
   (in words after the first instruction): after the nins instructions, or
   in the jump-table form after nins units of FBG_J16_UNIT words (END
   included). */
#define FBG_J16_LOG2W 4
#define FBG_J16_VGPR_REGS 3   /* registers 0..2 in VGPRs, the rest in LDS */
#define FBG_TABLE_OFFSET(nins, log2w) ((log2w) == FBG_J16_LOG2W ? (nins) * FBG_J16_UNIT : (nins) * FBG_INS_WORDS)
#define FBG_J16_UNIT 2u       /* words per length unit of the jump-table form */
#define FBG_J16_SHORT_WORDS 2u /* register, ACC and NOT instructions */
#define FBG_CB_HDR 4        /* words of the clause-block header */
#define FBG_CB_CHUNK 32     /* clauses per chunk */
#define FBG_CB_CHUNK_HDR 16 /* words of a chunk header */
#define FBG_LANE_BITS 6  /* 64 lanes per wave */
#define FBG_SLICE_BITS 5 /* 32 valuations per word */
#define FBG_TILE_BASE_BIT (FBG_SLICE_BITS + FBG_LANE_BITS) /* 11 */

/* Jump-table form: case numbers; each case's code fills one slot of
   FBG_J16_SLOT bytes. */
#define FBG_J16_SLOT 256u
#define FBG_J16_END 0u          /* leave the interpreter */
#define FBG_J16_NOT 1u          /* cur = ~cur */
#define FBG_J16_ACC 2u          /* + (INV ? 1 : 0) + (INVOUT ? 2 : 0): acc &= cur (^ ~0) */
#define FBG_J16_ST_V 6u         /* + (INVOUT ? 1 : 0): R[r] = cur, r < 4 */
#define FBG_J16_ST_L 8u         /* + (INVOUT ? 1 : 0): R[r] = cur, r >= 4 */
#define FBG_J16_REG_V 10u       /* + table index (FBG_J16_REG_TABLES): cur = tt(cur, R[r]) */
#define FBG_J16_REG_L 22u
#define FBG_J16_LIT_OR 34u      /* OR-set, no word literal: + index in FBG_J16_NP_TABLES */
#define FBG_J16_LIT_XOR 46u     /* XOR-set, no word literal: + index in FBG_J16_NP_TABLES */
#define FBG_J16_LIT_OR_P 58u    /* OR-set with word literals: + index in FBG_J16_OR_TABLES */
#define FBG_J16_LIT_XOR_P 70u   /* XOR-set with word literals: + index in FBG_J16_XOR_TABLES */
#define FBG_J16_XYF_OR 78u      /* first set of a chain, OR-set: + index in FBG_J16_NP_TABLES */
#define FBG_J16_XYF_XOR 90u     /* first set of a chain, XOR-set */
#define FBG_J16_XYM_OR 102u     /* further set of a chain, OR-set */
#define FBG_J16_XYM_XOR 114u    /* further set of a chain, XOR-set */
#define FBG_J16_XYL_OR 126u     /* last set of a chain, then cur = (cur & X) | (~cur & Y) */
#define FBG_J16_XYL_XOR 138u
#define FBG_J16_ORS 150u        /* + table index: R[r] = tt(cur, R[r]), cur left as it was (VGPR registers) */
#define FBG_J16_XYS_OR 162u     /* last set of a chain, the result into R[r] instead of cur: + table index */
#define FBG_J16_XYS_XOR 174u
#define FBG_J16_LIS_OR 186u     /* literal set without word literals, the result into R[r]: + table index */
#define FBG_J16_LIS_XOR 198u
#define FBG_J16_ORA 210u        /* + table index: acc = tt(acc, cur, R[r]), cur left (an operation and ACC) */
#define FBG_J16_LIA_OR 222u     /* + table index: acc = tt(acc, cur, T), cur left (a literal set and ACC) */
#define FBG_J16_LIA_XOR 234u
#define FBG_J16_NCASES 246u
/* Truth tables of the cases, over (cur = 0xF0, T or R = 0xCC, P = 0xAA).
   Without word literals P is 0, so only the bits of 0x55 matter. */
#define FBG_J16_REG_TABLES(X) X(0xC0) X(0x30) X(0xFC) X(0xF3) X(0x3C) X(0xC3) X(0x3F) X(0xCF) X(0x03) X(0x0C) X(0xCC) X(0x33)
#define FBG_J16_NP_TABLES(X) X(0x44) X(0x11) X(0x40) X(0x10) X(0x15) X(0x45) X(0x54) X(0x51) X(0x01) X(0x04) X(0x14) X(0x41)
#define FBG_J16_OR_TABLES(X) X(0xEE) X(0x11) X(0xE0) X(0x10) X(0x1F) X(0xEF) X(0xFE) X(0xF1) X(0x01) X(0x0E) X(0x1E) X(0xE1)
#define FBG_J16_XOR_TABLES(X) X(0x66) X(0x99) X(0x60) X(0x9F) X(0xF6) X(0x09) X(0x96) X(0x69)
/* Merged ACC, over (acc = 0xF0, cur = 0xCC, R or T = 0xAA): acc AND the
   operation of the register table (or the literal table) of the same index */
#define FBG_J16_ORA_TABLES(X) X(0x80) X(0x40) X(0xE0) X(0xD0) X(0x60) X(0x90) X(0x70) X(0xB0) X(0x10) X(0x20) X(0xA0) X(0x50)
#define FBG_J16_LIA_TABLES(X) X(0xA0) X(0x50) X(0x80) X(0x40) X(0x70) X(0xB0) X(0xE0) X(0xD0) X(0x10) X(0x20) X(0x60) X(0x90)

/* In-word generator masks: bit j of MASK_k is bit k of j (Section 2.2). */
static inline uint32_t fbg_inword_mask(int k) {
  static const uint32_t m[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
  return m[k];
}

#endif
