// fbg_asm16.h -- the general part of a program at 16 words per lane, run as
// a jump table (the instruction format is the jump-table form of fbg_isa.h).
//
// The interpreter of fbg_device.h decides among its cases with a chain of
// scalar compares and branches, about 25 scalar instructions for the 16 VALU
// instructions of one program instruction; the scalar unit, which issues no
// faster than the VALU, then bounds the loop.  Here every instruction carries
// the byte offset of its case, and one s_setpc_b64 enters the case's code
// directly (2 scalar instructions on the table's 64 KiB boundary, 4
// elsewhere).  Each case fetches the next instruction before its VALU work,
// so the fetch is waited for only at the next dispatch.
//
// Register map (fixed; the C++ side sees acc as a pinned in/out operand and
// every other register below as clobbered):
//   v14         T, the lane value of a literal set (of a set without word
//               literals: its lane part, the rest in s73)
//   v15         LDS address
//   v[16:31]    cur, word i in v[16+i]
//   v[32:79]    registers 0..2 in VGPRs, register r word i in v[32+16r+i]
//               (read and written through VGPR index mode, M0 = 16 r)
//   v[80:95]    a register read back from LDS; inside a chain of literal
//               sets (fbg_isa.h) v80 = X and v81 = Y instead
//   v[96:111]   acc
// leaving v[0:13] and v[112:127] to the compiler for what lives across (four
// waves share a SIMD; two VGPR registers and five waves measured slower).
//   s[48:55]    the current instruction, s[56:71] its pattern words,
//   s[72:75]    scratch (s73: the rest of a lane value, above),
//   s[76:77]    the table's address (copy B) or bits 16..31 of it in s77
//               (copy A), s[78:79] the jump target (s79 its bits 32..63 in
//               copy A), s80 the instruction offset, s81 the pattern offset,
//   s83         M0 saved (index mode changes M0; restored on exit),
//   s[84:85]    where the interpreter returns to
// All 64 lanes are active (the kernels call it on full waves).
#ifndef FBG_ASM16_H
#define FBG_ASM16_H

#include <stdint.h>

#include "fbg_isa.h"

namespace fbg {
namespace dev {

typedef uint32_t j16_u32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t j16_u32x2 __attribute__((ext_vector_type(2)));

#define FBG_J16_STR2(x) #x
#define FBG_J16_STR(x) FBG_J16_STR2(x)
#define FBG_J16_W16(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

// Fetch the next instruction into s[48:55]: 32 bytes further after a
// literal-set instruction (NEXT_L), 8 after the others (NEXT_S).  The load
// reads 32 bytes either way; the END that closes the program is 32 bytes
// long, so it never reads past the program.
#define FBG_J16_NEXT_L "s_add_u32 s80, s80, 32\n" "s_load_dwordx8 s[48:55], %[code], s80\n"
#define FBG_J16_NEXT_S "s_add_u32 s80, s80, 8\n" "s_load_dwordx8 s[48:55], %[code], s80\n"
// Wait for it and jump to its case: an assembler macro (fbgdisp), defined
// once per copy of the table (FBG_J16_PROGRAM).  The offset is bits 0..15 of
// the instruction's first word, so no instruction word can send the jump
// outside the table's 256 slots (those past the last case exit).
#define FBG_J16_DISPATCH "fbgdisp%=\n"
// The table on a 64 KiB boundary: s77 holds bits 16..31 of its address and
// s79 bits 32..63, so the jump target is the offset packed under s77.
#define FBG_J16_DISPATCH_ALIGNED "s_waitcnt lgkmcnt(0)\n" "s_pack_ll_b32_b16 s78, s48, s77\n" "s_setpc_b64 s[78:79]\n"
// Anywhere: s[76:77] holds its address; the offset, cut to a whole slot, is
// added to it.
#define FBG_J16_DISPATCH_ANY                                                                           \
  "s_waitcnt lgkmcnt(0)\n" "s_and_b32 s78, s48, 0xff00\n" "s_add_u32 s78, s76, s78\n" "s_addc_u32 s79, s77, 0\n" \
  "s_setpc_b64 s[78:79]\n"
// Start of case k: its slot of the table (an .org that moves backwards, i.e.
// a case longer than its slot, is an assembly error).
#define FBG_J16_CASE(k) ".org Lc%=\\s+(" FBG_J16_STR(k) ")*256\n"

// per-word bodies
#define FBG_J16_NOTCUR(i) "v_not_b32 v[16+" #i "], v[16+" #i "]\n"
#define FBG_J16_ACCAND(i) "v_and_b32 v[96+" #i "], v[96+" #i "], v[16+" #i "]\n"
#define FBG_J16_ACCANDN(i) "v_bitop3_b32 v[96+" #i "], v[96+" #i "], v[16+" #i "], 0 bitop3:0x30\n"
#define FBG_J16_STV(i) "v_mov_b32 v[32+" #i "], v[16+" #i "]\n"

// The lane value T (v14) of the current literal set, from its lane mask,
// in-word constant and tile selectors (fbg_isa.h): OR-sets all-ones where a
// lane or tile literal holds, else mconst; XOR-sets the lane part XOR mconst
// XOR the parity of the tile literals.
#define FBG_J16_T_OR                           \
  "s_and_b64 s[72:73], %[u0], s[52:53]\n"      \
  "s_cmp_lg_u64 s[72:73], s[54:55]\n"          \
  "s_cselect_b64 s[74:75], -1, s[50:51]\n"     \
  "v_mov_b32 v14, s49\n"                       \
  "v_cndmask_b32_e64 v14, v14, -1, s[74:75]\n"
#define FBG_J16_T_XOR                          \
  "s_and_b64 s[72:73], %[u0], s[52:53]\n"      \
  "s_bcnt1_i32_b64 s72, s[72:73]\n"            \
  "s_bfe_i32 s72, s72, 0x10000\n"              \
  "s_xor_b32 s72, s72, s49\n"                  \
  "v_cndmask_b32_e64 v14, 0, -1, s[50:51]\n"   \
  "v_xor_b32 v14, s72, v14\n"
// A set without word literals needs no VGPR for T: v14 holds its lane part
// (all-ones or zero per lane) and s73 the rest, so that T = v14 | s73
// (OR-sets: s73 = all-ones when a tile literal holds, else mconst) or
// T = v14 ^ s73 (XOR-sets: s73 = mconst XOR the parity of the tile
// literals).  The cases' tables fold that OR or XOR in, and every word still
// takes one v_bitop3_b32 over (cur, v14, s73): one VALU instruction less per
// set than forming T, and no scalar one more.
#define FBG_J16_M_OR                           \
  "s_and_b64 s[72:73], %[u0], s[52:53]\n"      \
  "s_cmp_lg_u64 s[72:73], s[54:55]\n"          \
  "s_cselect_b32 s73, -1, s49\n"               \
  "v_cndmask_b32_e64 v14, 0, -1, s[50:51]\n"
#define FBG_J16_M_XOR                          \
  "s_and_b64 s[72:73], %[u0], s[52:53]\n"      \
  "s_bcnt1_i32_b64 s73, s[72:73]\n"            \
  "s_bfe_i32 s73, s73, 0x10000\n"              \
  "s_xor_b32 s73, s73, s49\n"                  \
  "v_cndmask_b32_e64 v14, 0, -1, s[50:51]\n"
// Load the set's 16 pattern words (issued before T is formed).
#define FBG_J16_PLOAD "s_lshr_b32 s81, s48, 16\n" "s_load_dwordx16 s[56:71], %[tab], s81\n"

// Case bodies parameterised by a truth table TT.
#define FBG_J16_LITM_W(i, TT) "v_bitop3_b32 v[16+" #i "], v[16+" #i "], v14, s73 bitop3:" TT "\n"
#define FBG_J16_LITP_W(i, TT) "v_bitop3_b32 v[16+" #i "], v[16+" #i "], v14, s[56+" #i "] bitop3:" TT "\n"
#define FBG_J16_REGV_W(i, TT) "v_bitop3_b32 v[16+" #i "], v[16+" #i "], v[32+" #i "], 0 bitop3:" TT "\n"
#define FBG_J16_REGL_W(i, TT) "v_bitop3_b32 v[16+" #i "], v[16+" #i "], v[80+" #i "], 0 bitop3:" TT "\n"
#define FBG_J16_EACH(M, TT)                                                                             \
  M(0, TT) M(1, TT) M(2, TT) M(3, TT) M(4, TT) M(5, TT) M(6, TT) M(7, TT) M(8, TT) M(9, TT) M(10, TT) \
  M(11, TT) M(12, TT) M(13, TT) M(14, TT) M(15, TT)

// literal set without word literals: lane part, fetch, 16 x v_bitop3(cur,
// v14, s73)
#define FBG_J16_C_LITOR(TT) FBG_J16_M_OR FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LITM_W, #TT) FBG_J16_DISPATCH
#define FBG_J16_C_LITXOR(TT) FBG_J16_M_XOR FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LITM_W, #TT) FBG_J16_DISPATCH
// with word literals: the pattern words come in with the next instruction
#define FBG_J16_C_LITORP(TT) \
  FBG_J16_PLOAD FBG_J16_T_OR "s_waitcnt lgkmcnt(0)\n" FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LITP_W, #TT) FBG_J16_DISPATCH
#define FBG_J16_C_LITXORP(TT) \
  FBG_J16_PLOAD FBG_J16_T_XOR "s_waitcnt lgkmcnt(0)\n" FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LITP_W, #TT) FBG_J16_DISPATCH
// register in VGPRs: index mode offsets the register operand by 16 r
#define FBG_J16_C_REGV(TT)                                                                          \
  "s_set_gpr_idx_on s49, gpr_idx(SRC1)\n" FBG_J16_NEXT_S "s_nop 1\n" FBG_J16_EACH(FBG_J16_REGV_W, #TT) \
  "s_set_gpr_idx_off\n" FBG_J16_DISPATCH
// register beyond the VGPRs: in LDS when its offset is inside this wave's
// LDS block (%[ldsb] bytes), else in the wave's global-memory block (the
// code of FBG_J16_G_REGL, before the table); four 16-byte reads per lane,
// then the operation
#define FBG_J16_C_REGL(TT)                                                                \
  "s_cmp_lt_u32 s49, %[ldsb]\n"                                                          \
  "s_cbranch_scc0 LG" #TT "%=\\s\n"                                                          \
  "v_add_u32 v15, s49, %[lb]\n"                                                           \
  "ds_read_b128 v[80:83], v15\n"                                                         \
  "ds_read_b128 v[84:87], v15 offset:16\n"                                               \
  "ds_read_b128 v[88:91], v15 offset:32\n"                                               \
  "ds_read_b128 v[92:95], v15 offset:48\n" FBG_J16_NEXT_S "s_waitcnt lgkmcnt(0)\n"         \
  FBG_J16_EACH(FBG_J16_REGL_W, #TT) FBG_J16_DISPATCH

// the global-memory half: the same register read from the wave's block at
// %[gb], lane l at 64 l (%[l64]); earlier stores of this wave are waited for
#define FBG_J16_G_REGL(TT)                                                                \
  "LG" #TT "%=\\s:\n"                                                                        \
  "s_sub_u32 s72, s49, %[ldsb]\n"                                                         \
  "v_add_u32 v15, s72, %[l64]\n"                                                          \
  "s_waitcnt vmcnt(0)\n"                                                                  \
  "global_load_dwordx4 v[80:83], v15, %[gb]\n"                                            \
  "global_load_dwordx4 v[84:87], v15, %[gb] offset:16\n"                                  \
  "global_load_dwordx4 v[88:91], v15, %[gb] offset:32\n"                                  \
  "global_load_dwordx4 v[92:95], v15, %[gb] offset:48\n" FBG_J16_NEXT_S                   \
  "s_waitcnt vmcnt(0) lgkmcnt(0)\n" FBG_J16_EACH(FBG_J16_REGL_W, #TT) FBG_J16_DISPATCH

// chains (fbg_isa.h): the first set sets X and Y from cur = all-ones and cur
// = zero, each further set updates them, and the last one then applies them
// to the words: cur = (cur & X) | (~cur & Y)
#define FBG_J16_XYF(TT) \
  "v_bitop3_b32 v80, -1, v14, s73 bitop3:" TT "\n" "v_bitop3_b32 v81, 0, v14, s73 bitop3:" TT "\n"
#define FBG_J16_XYM(TT) \
  "v_bitop3_b32 v80, v80, v14, s73 bitop3:" TT "\n" "v_bitop3_b32 v81, v81, v14, s73 bitop3:" TT "\n"
#define FBG_J16_C_XYF_OR(TT) FBG_J16_M_OR FBG_J16_NEXT_L FBG_J16_XYF(#TT) FBG_J16_DISPATCH
#define FBG_J16_C_XYF_XOR(TT) FBG_J16_M_XOR FBG_J16_NEXT_L FBG_J16_XYF(#TT) FBG_J16_DISPATCH
#define FBG_J16_C_XYM_OR(TT) FBG_J16_M_OR FBG_J16_NEXT_L FBG_J16_XYM(#TT) FBG_J16_DISPATCH
#define FBG_J16_C_XYM_XOR(TT) FBG_J16_M_XOR FBG_J16_NEXT_L FBG_J16_XYM(#TT) FBG_J16_DISPATCH
#define FBG_J16_XYAPPLY(i) "v_bitop3_b32 v[16+" #i "], v[16+" #i "], v80, v81 bitop3:0xca\n"
#define FBG_J16_C_XYL_OR(TT) \
  FBG_J16_M_OR FBG_J16_NEXT_L FBG_J16_XYM(#TT) FBG_J16_W16(FBG_J16_XYAPPLY) FBG_J16_DISPATCH
#define FBG_J16_C_XYL_XOR(TT) \
  FBG_J16_M_XOR FBG_J16_NEXT_L FBG_J16_XYM(#TT) FBG_J16_W16(FBG_J16_XYAPPLY) FBG_J16_DISPATCH

// merged stores (fbg_isa.h): ORS writes the operation's result into the
// register it reads (index mode on the second source and the destination);
// XYS updates X and Y, then writes the chain's result into R[r] (index mode on
// the destination only, switched on after the X and Y updates)
#define FBG_J16_ORS_W(i, TT) "v_bitop3_b32 v[32+" #i "], v[16+" #i "], v[32+" #i "], 0 bitop3:" TT "\n"
#define FBG_J16_C_ORS(TT)                                                                                \
  "s_set_gpr_idx_on s49, gpr_idx(SRC1,DST)\n" FBG_J16_NEXT_S "s_nop 1\n" FBG_J16_EACH(FBG_J16_ORS_W, #TT) \
  "s_set_gpr_idx_off\n" FBG_J16_DISPATCH
#define FBG_J16_XYSTORE(i) "v_bitop3_b32 v[32+" #i "], v[16+" #i "], v80, v81 bitop3:0xca\n"
#define FBG_J16_XYS_TAIL(TT)                                                                            \
  FBG_J16_XYM(TT) "s_lshr_b32 s72, s48, 16\n" "s_set_gpr_idx_on s72, gpr_idx(DST)\n" FBG_J16_NEXT_L \
  "s_nop 1\n" FBG_J16_W16(FBG_J16_XYSTORE) "s_set_gpr_idx_off\n" FBG_J16_DISPATCH
#define FBG_J16_C_XYS_OR(TT) FBG_J16_M_OR FBG_J16_XYS_TAIL(#TT)
#define FBG_J16_C_XYS_XOR(TT) FBG_J16_M_XOR FBG_J16_XYS_TAIL(#TT)
// LIS: a literal set's operation, its result into R[r] (index mode on the
// destination)
#define FBG_J16_LIS_W(i, TT) "v_bitop3_b32 v[32+" #i "], v[16+" #i "], v14, s73 bitop3:" TT "\n"
#define FBG_J16_LIS_TAIL(TT)                                                                          \
  "s_lshr_b32 s72, s48, 16\n" "s_set_gpr_idx_on s72, gpr_idx(DST)\n" FBG_J16_NEXT_L "s_nop 1\n" \
  FBG_J16_EACH(FBG_J16_LIS_W, TT) "s_set_gpr_idx_off\n" FBG_J16_DISPATCH
#define FBG_J16_C_LIS_OR(TT) FBG_J16_M_OR FBG_J16_LIS_TAIL(#TT)
#define FBG_J16_C_LIS_XOR(TT) FBG_J16_M_XOR FBG_J16_LIS_TAIL(#TT)
// merged ACC (fbg_isa.h): acc = tt(acc, cur, R[r]) with index mode on the
// third source, or acc = tt(acc, cur, T)
#define FBG_J16_ORA_W(i, TT) "v_bitop3_b32 v[96+" #i "], v[96+" #i "], v[16+" #i "], v[32+" #i "] bitop3:" TT "\n"
#define FBG_J16_C_ORA(TT)                                                                             \
  "s_set_gpr_idx_on s49, gpr_idx(SRC2)\n" FBG_J16_NEXT_S "s_nop 1\n" FBG_J16_EACH(FBG_J16_ORA_W, #TT) \
  "s_set_gpr_idx_off\n" FBG_J16_DISPATCH
#define FBG_J16_LIA_W(i, TT) "v_bitop3_b32 v[96+" #i "], v[96+" #i "], v[16+" #i "], v14 bitop3:" TT "\n"
#define FBG_J16_C_LIA_OR(TT) FBG_J16_T_OR FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LIA_W, #TT) FBG_J16_DISPATCH
#define FBG_J16_C_LIA_XOR(TT) FBG_J16_T_XOR FBG_J16_NEXT_L FBG_J16_EACH(FBG_J16_LIA_W, #TT) FBG_J16_DISPATCH

#define FBG_J16_C_ST_V(INVOUT)                                                                  \
  "s_set_gpr_idx_on s49, gpr_idx(DST)\n" FBG_J16_NEXT_S "s_nop 1\n" FBG_J16_W16(FBG_J16_STV)     \
  "s_set_gpr_idx_off\n" INVOUT FBG_J16_DISPATCH
#define FBG_J16_C_ST_L(INVOUT, G)                                             \
  "s_cmp_lt_u32 s49, %[ldsb]\n"                                              \
  "s_cbranch_scc0 LGST" #G "%=\\s\n"                                             \
  "v_add_u32 v15, s49, %[lb]\n"                                               \
  "ds_write_b128 v15, v[16:19]\n"                                             \
  "ds_write_b128 v15, v[20:23] offset:16\n"                                   \
  "ds_write_b128 v15, v[24:27] offset:32\n"                                   \
  "ds_write_b128 v15, v[28:31] offset:48\n" FBG_J16_NEXT_S INVOUT FBG_J16_DISPATCH
#define FBG_J16_G_ST_L(INVOUT, G)                                             \
  "LGST" #G "%=\\s:\n"                                                           \
  "s_sub_u32 s72, s49, %[ldsb]\n"                                            \
  "v_add_u32 v15, s72, %[l64]\n"                                             \
  "global_store_dwordx4 v15, v[16:19], %[gb]\n"                              \
  "global_store_dwordx4 v15, v[20:23], %[gb] offset:16\n"                    \
  "global_store_dwordx4 v15, v[24:27], %[gb] offset:32\n"                    \
  "global_store_dwordx4 v15, v[28:31], %[gb] offset:48\n" FBG_J16_NEXT_S INVOUT FBG_J16_DISPATCH
// cur inverted after a store: the store has read cur first
#define FBG_J16_INVOUT_CUR FBG_J16_W16(FBG_J16_NOTCUR)
#define FBG_J16_INVOUT_AFTER_DS "s_waitcnt lgkmcnt(0)\n" FBG_J16_W16(FBG_J16_NOTCUR)
#define FBG_J16_INVOUT_AFTER_VM "s_waitcnt vmcnt(0)\n" FBG_J16_W16(FBG_J16_NOTCUR)

// The cases in table order (case k at Lc + 256 k).
#define FBG_J16_CASES_REG(MAC, BASE)                                                                         \
  FBG_J16_CASE(BASE + 0) MAC(0xC0) FBG_J16_CASE(BASE + 1) MAC(0x30) FBG_J16_CASE(BASE + 2) MAC(0xFC)        \
  FBG_J16_CASE(BASE + 3) MAC(0xF3) FBG_J16_CASE(BASE + 4) MAC(0x3C) FBG_J16_CASE(BASE + 5) MAC(0xC3)        \
  FBG_J16_CASE(BASE + 6) MAC(0x3F) FBG_J16_CASE(BASE + 7) MAC(0xCF) FBG_J16_CASE(BASE + 8) MAC(0x03)        \
  FBG_J16_CASE(BASE + 9) MAC(0x0C) FBG_J16_CASE(BASE + 10) MAC(0xCC) FBG_J16_CASE(BASE + 11) MAC(0x33)
// Twelve cases from a list of twelve tables (FBG_J16_APPLY splits the list
// into arguments).
#define FBG_J16_APPLY(M, ARGS) M ARGS
#define FBG_J16_CASES12(MAC, B, t0, t1, t2, t3, t4, t5, t6, t7, t8, t9, t10, t11)                          \
  FBG_J16_CASE(B + 0) MAC(t0) FBG_J16_CASE(B + 1) MAC(t1) FBG_J16_CASE(B + 2) MAC(t2)                       \
  FBG_J16_CASE(B + 3) MAC(t3) FBG_J16_CASE(B + 4) MAC(t4) FBG_J16_CASE(B + 5) MAC(t5)                       \
  FBG_J16_CASE(B + 6) MAC(t6) FBG_J16_CASE(B + 7) MAC(t7) FBG_J16_CASE(B + 8) MAC(t8)                       \
  FBG_J16_CASE(B + 9) MAC(t9) FBG_J16_CASE(B + 10) MAC(t10) FBG_J16_CASE(B + 11) MAC(t11)
// The tables of the sets without word literals (FBG_J16_NP_TABLES, over
// cur and T) with T = v14 | s73 (ORT) or T = v14 ^ s73 (XORT) folded in, in
// the same order; the ORT tables are also those of the OR-sets with word
// literals (their P is OR-ed into T).  Checked below.
#define FBG_J16_ORT_LIST 0xEE, 0x11, 0xE0, 0x10, 0x1F, 0xEF, 0xFE, 0xF1, 0x01, 0x0E, 0x1E, 0xE1
#define FBG_J16_XORT_LIST 0x66, 0x99, 0x60, 0x90, 0x9F, 0x6F, 0xF6, 0xF9, 0x09, 0x06, 0x96, 0x69
#define FBG_J16_CASES_ORT(MAC, BASE) FBG_J16_APPLY(FBG_J16_CASES12, (MAC, BASE, FBG_J16_ORT_LIST))
#define FBG_J16_CASES_XORT(MAC, BASE) FBG_J16_APPLY(FBG_J16_CASES12, (MAC, BASE, FBG_J16_XORT_LIST))

#define FBG_J16_LISTED(t) t,
constexpr uint32_t kJ16NpTables[] = {FBG_J16_NP_TABLES(FBG_J16_LISTED)};
constexpr uint32_t kJ16OrtTables[] = {FBG_J16_ORT_LIST};
constexpr uint32_t kJ16XortTables[] = {FBG_J16_XORT_LIST};
// tt over (a, b, c) = (0xF0, 0xCC, 0xAA) as tt0(a, b OP c, 0)
constexpr uint32_t j16_fold(uint32_t tt0, bool is_xor) {
  uint32_t r = 0;
  for (uint32_t x = 0; x < 8; x++) {
    const uint32_t a = x >> 2, b = (x >> 1) & 1u, c = x & 1u;
    const uint32_t t = is_xor ? (b ^ c) : (b | c);
    r |= ((tt0 >> ((a << 2) | (t << 1))) & 1u) << x;
  }
  return r;
}
constexpr bool j16_folded_tables_agree() {
  for (int k = 0; k < 12; k++)
    if (j16_fold(kJ16NpTables[k], false) != kJ16OrtTables[k] || j16_fold(kJ16NpTables[k], true) != kJ16XortTables[k])
      return false;
  return true;
}
static_assert(sizeof kJ16NpTables / sizeof kJ16NpTables[0] == 12 && j16_folded_tables_agree(),
              "ORT / XORT tables are the NP tables with the lane part and s73 folded in");

#define FBG_J16_CASES_ORA(MAC, BASE)                                                                         \
  FBG_J16_CASE(BASE + 0) MAC(0x80) FBG_J16_CASE(BASE + 1) MAC(0x40) FBG_J16_CASE(BASE + 2) MAC(0xE0)        \
  FBG_J16_CASE(BASE + 3) MAC(0xD0) FBG_J16_CASE(BASE + 4) MAC(0x60) FBG_J16_CASE(BASE + 5) MAC(0x90)        \
  FBG_J16_CASE(BASE + 6) MAC(0x70) FBG_J16_CASE(BASE + 7) MAC(0xB0) FBG_J16_CASE(BASE + 8) MAC(0x10)        \
  FBG_J16_CASE(BASE + 9) MAC(0x20) FBG_J16_CASE(BASE + 10) MAC(0xA0) FBG_J16_CASE(BASE + 11) MAC(0x50)
#define FBG_J16_CASES_LIA(MAC, BASE)                                                                         \
  FBG_J16_CASE(BASE + 0) MAC(0xA0) FBG_J16_CASE(BASE + 1) MAC(0x50) FBG_J16_CASE(BASE + 2) MAC(0x80)        \
  FBG_J16_CASE(BASE + 3) MAC(0x40) FBG_J16_CASE(BASE + 4) MAC(0x70) FBG_J16_CASE(BASE + 5) MAC(0xB0)        \
  FBG_J16_CASE(BASE + 6) MAC(0xE0) FBG_J16_CASE(BASE + 7) MAC(0xD0) FBG_J16_CASE(BASE + 8) MAC(0x10)        \
  FBG_J16_CASE(BASE + 9) MAC(0x20) FBG_J16_CASE(BASE + 10) MAC(0x60) FBG_J16_CASE(BASE + 11) MAC(0x90)
#define FBG_J16_CASES_XORP(MAC, BASE)                                                                        \
  FBG_J16_CASE(BASE + 0) MAC(0x66) FBG_J16_CASE(BASE + 1) MAC(0x99) FBG_J16_CASE(BASE + 2) MAC(0x60)        \
  FBG_J16_CASE(BASE + 3) MAC(0x9F) FBG_J16_CASE(BASE + 4) MAC(0xF6) FBG_J16_CASE(BASE + 5) MAC(0x09)        \
  FBG_J16_CASE(BASE + 6) MAC(0x96) FBG_J16_CASE(BASE + 7) MAC(0x69)

// clang-format off
// The table of cases, an assembler macro emitted twice: fbgtab <label
// suffix>, <alignment as a power of two>.  Its exit returns to the address
// in s[84:85].
#define FBG_J16_TABLE                                                                                        \
  ".macro fbgtab%= s, a\n"                                                                                   \
  ".p2align \\a\n"                                                                                           \
  "Lc%=\\s:\n"                                                                                                \
  FBG_J16_CASE(0)  "s_branch Ld%=\\s\n"                                                                         \
  FBG_J16_CASE(1)  FBG_J16_NEXT_S FBG_J16_W16(FBG_J16_NOTCUR) FBG_J16_DISPATCH                                \
  FBG_J16_CASE(2)  FBG_J16_NEXT_S FBG_J16_W16(FBG_J16_ACCAND) FBG_J16_DISPATCH                                \
  FBG_J16_CASE(3)  FBG_J16_NEXT_S FBG_J16_W16(FBG_J16_ACCANDN) FBG_J16_DISPATCH                               \
  FBG_J16_CASE(4)  FBG_J16_NEXT_S FBG_J16_W16(FBG_J16_ACCAND) FBG_J16_INVOUT_CUR FBG_J16_DISPATCH             \
  FBG_J16_CASE(5)  FBG_J16_NEXT_S FBG_J16_W16(FBG_J16_ACCANDN) FBG_J16_INVOUT_CUR FBG_J16_DISPATCH            \
  FBG_J16_CASE(6)  FBG_J16_C_ST_V("")                                                                        \
  FBG_J16_CASE(7)  FBG_J16_C_ST_V(FBG_J16_INVOUT_CUR)                                                        \
  FBG_J16_CASE(8)  FBG_J16_C_ST_L("", 0)                                                                     \
  FBG_J16_CASE(9)  FBG_J16_C_ST_L(FBG_J16_INVOUT_AFTER_DS, 1)                                                \
  FBG_J16_CASES_REG(FBG_J16_C_REGV, 10)                                                                      \
  FBG_J16_CASES_REG(FBG_J16_C_REGL, 22)                                                                      \
  FBG_J16_CASES_ORT(FBG_J16_C_LITOR, 34)                                                                      \
  FBG_J16_CASES_XORT(FBG_J16_C_LITXOR, 46)                                                                     \
  FBG_J16_CASES_ORT(FBG_J16_C_LITORP, 58)                                                                    \
  FBG_J16_CASES_XORP(FBG_J16_C_LITXORP, 70)                                                                  \
  FBG_J16_CASES_ORT(FBG_J16_C_XYF_OR, 78)                                                                     \
  FBG_J16_CASES_XORT(FBG_J16_C_XYF_XOR, 90)                                                                    \
  FBG_J16_CASES_ORT(FBG_J16_C_XYM_OR, 102)                                                                    \
  FBG_J16_CASES_XORT(FBG_J16_C_XYM_XOR, 114)                                                                   \
  FBG_J16_CASES_ORT(FBG_J16_C_XYL_OR, 126)                                                                    \
  FBG_J16_CASES_XORT(FBG_J16_C_XYL_XOR, 138)                                                                   \
  FBG_J16_CASES_REG(FBG_J16_C_ORS, 150)                                                                      \
  FBG_J16_CASES_ORT(FBG_J16_C_XYS_OR, 162)                                                                    \
  FBG_J16_CASES_XORT(FBG_J16_C_XYS_XOR, 174)                                                                   \
  FBG_J16_CASES_ORT(FBG_J16_C_LIS_OR, 186)                                                                    \
  FBG_J16_CASES_XORT(FBG_J16_C_LIS_XOR, 198)                                                                   \
  FBG_J16_CASES_ORA(FBG_J16_C_ORA, 210)                                                                      \
  FBG_J16_CASES_LIA(FBG_J16_C_LIA_OR, 222)                                                                   \
  FBG_J16_CASES_LIA(FBG_J16_C_LIA_XOR, 234)                                                                  \
  FBG_J16_CASE(246) "s_branch Ld%=\\s\n" FBG_J16_CASE(247) "s_branch Ld%=\\s\n" FBG_J16_CASE(248) "s_branch Ld%=\\s\n"   \
  FBG_J16_CASE(249) "s_branch Ld%=\\s\n" FBG_J16_CASE(250) "s_branch Ld%=\\s\n" FBG_J16_CASE(251) "s_branch Ld%=\\s\n"   \
  FBG_J16_CASE(252) "s_branch Ld%=\\s\n" FBG_J16_CASE(253) "s_branch Ld%=\\s\n" FBG_J16_CASE(254) "s_branch Ld%=\\s\n"   \
  FBG_J16_CASE(255)                                                                                          \
  "Ld%=\\s:\n"                                                                                                \
  "s_setpc_b64 s[84:85]\n"                                                                                   \
  FBG_J16_G_REGL(0xC0) FBG_J16_G_REGL(0x30) FBG_J16_G_REGL(0xFC) FBG_J16_G_REGL(0xF3) FBG_J16_G_REGL(0x3C)   \
  FBG_J16_G_REGL(0xC3) FBG_J16_G_REGL(0x3F) FBG_J16_G_REGL(0xCF) FBG_J16_G_REGL(0x03) FBG_J16_G_REGL(0x0C)   \
  FBG_J16_G_REGL(0xCC) FBG_J16_G_REGL(0x33)                                                                  \
  FBG_J16_G_ST_L("", 0) FBG_J16_G_ST_L(FBG_J16_INVOUT_AFTER_VM, 1)                                          \
  ".endm\n"

// The interpreter: return address into s[84:85]; the first instruction's
// fetch; then into the table on its 64 KiB boundary (copy A) or, should the
// code object not have been loaded on such a boundary or %[any] ask for it,
// into copy B with the longer dispatch.  Both copies sit in a section of their own, so that the
// compiler's branches around this statement do not span them.
#define FBG_J16_PROGRAM                                                                                      \
  "s_mov_b32 s83, m0\n"                                                                                      \
  "s_getpc_b64 s[84:85]\n"                                                                                   \
  "Lr%=:\n"                                                                                                  \
  "s_add_u32 s84, s84, Lret%=-Lr%=\n"                                                                        \
  "s_addc_u32 s85, s85, 0\n"                                                                                 \
  "s_mov_b32 s80, 0\n"                                                                                       \
  "s_load_dwordx8 s[48:55], %[code], s80\n"                                                                  \
  "s_cmp_lg_u32 %[any], 0\n"                                                                                \
  "s_cbranch_scc1 Lany%=\n"                                                                                  \
  "s_getpc_b64 s[76:77]\n"                                                                                   \
  "s_add_u32 s76, s76, Lc%=A@rel32@lo+4\n"                                                                   \
  "s_addc_u32 s77, s77, Lc%=A@rel32@hi+12\n"                                                                 \
  "s_and_b32 s72, s76, 0xffff\n"                                                                             \
  "s_cmp_lg_u32 s72, 0\n"                                                                                    \
  "s_cbranch_scc1 Lany%=\n"                                                                                  \
  "s_mov_b32 s79, s77\n"                                                                                     \
  "s_lshr_b32 s77, s76, 16\n"                                                                                \
  FBG_J16_DISPATCH_ALIGNED                                                                                   \
  "Lany%=:\n"                                                                                                \
  "s_getpc_b64 s[76:77]\n"                                                                                   \
  "s_add_u32 s76, s76, Lc%=B@rel32@lo+4\n"                                                                   \
  "s_addc_u32 s77, s77, Lc%=B@rel32@hi+12\n"                                                                 \
  FBG_J16_DISPATCH_ANY                                                                                       \
  ".pushsection .text.fbg_j16, \"ax\", @progbits\n"                                                          \
  FBG_J16_TABLE                                                                                              \
  ".macro fbgdisp%=\n" FBG_J16_DISPATCH_ALIGNED ".endm\n"                                                    \
  "fbgtab%= A, 16\n"                                                                                         \
  ".purgem fbgdisp%=\n"                                                                                      \
  ".macro fbgdisp%=\n" FBG_J16_DISPATCH_ANY ".endm\n"                                                        \
  "fbgtab%= B, 8\n"                                                                                          \
  ".purgem fbgdisp%=\n"                                                                                      \
  ".purgem fbgtab%=\n"                                                                                       \
  ".popsection\n"                                                                                            \
  "Lret%=:\n"                                                                                                \
  "s_mov_b32 m0, s83\n"
// clang-format on

static_assert(FBG_J16_NCASES == 246 && FBG_J16_SLOT == 256 && FBG_J16_XYF_OR == 78 && FBG_J16_XYF_XOR == 90 &&
                  FBG_J16_XYM_OR == 102 && FBG_J16_XYM_XOR == 114 && FBG_J16_XYL_OR == 126 &&
                  FBG_J16_XYL_XOR == 138 && FBG_J16_ORS == 150 && FBG_J16_XYS_OR == 162 && FBG_J16_XYS_XOR == 174 &&
                  FBG_J16_LIS_OR == 186 && FBG_J16_LIS_XOR == 198 && FBG_J16_ORA == 210 && FBG_J16_LIA_OR == 222 &&
                  FBG_J16_LIA_XOR == 234,
              "the case list of FBG_J16_PROGRAM: 246 cases, then exits up to slot 255 (FBG_J16_DISPATCH)");

// Run the general part of a program (jump-table form at `code`, its pattern
// table at `table`) on the 16 words of this lane of tile group U0.  acc comes
// in as the clause block's value and leaves as the program's.  Registers from
// 3 on sit at byte offset 4096 (r - 3): below `lds_bytes` in LDS, at
// `lds_lane` (this wave's LDS block + 64 lane); from `lds_bytes` on in global
// memory, at `gbase` (this wave's block) + offset - lds_bytes + 64 lane.
// `any` non-zero runs copy B of the table (both copies compute the same).
__device__ __forceinline__ void run_general_j16(const uint32_t *code, const uint32_t *table, uint64_t U0,
                                                uint32_t lds_lane, uint32_t lds_bytes, uint32_t *gbase,
                                                uint32_t lane, uint32_t (&acc)[16], uint32_t any) {
  j16_u32x16 a;
#pragma unroll
  for (int i = 0; i < 16; i++) a[i] = acc[i];
  j16_u32x16 d0, d1, d2, d3, d4;
  j16_u32x2 d6;
  const uint64_t c = (uint64_t)code, t = (uint64_t)table, g = (uint64_t)gbase;
  const uint32_t l64 = lane * 64u;
  asm volatile(FBG_J16_PROGRAM
               : "+{v[96:111]}"(a), "=&{v[16:31]}"(d0), "=&{v[32:47]}"(d1), "=&{v[48:63]}"(d2),
                 "=&{v[64:79]}"(d3), "=&{v[80:95]}"(d4), "=&{v[14:15]}"(d6)
               : [code] "s"(c), [tab] "s"(t), [u0] "s"(U0), [lb] "v"(lds_lane), [ldsb] "s"(lds_bytes),
                 [gb] "s"(g), [l64] "v"(l64), [any] "s"(any)
               : "s48", "s49", "s50", "s51", "s52", "s53", "s54", "s55", "s56", "s57", "s58", "s59", "s60", "s61",
                 "s62", "s63", "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75",
                 "s76", "s77", "s78", "s79", "s80", "s81", "s83", "s84", "s85", "scc", "memory");
#pragma unroll
  for (int i = 0; i < 16; i++) acc[i] = a[i];
}

}  // namespace dev
}  // namespace fbg

#endif
