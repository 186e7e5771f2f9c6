// fbg_internal.h -- host-side structures shared by the compiler, the runtime
// and the C ABI.  Not installed; the public interface is include/fbg.h.
#ifndef FBG_INTERNAL_H
#define FBG_INTERNAL_H

#include <stdint.h>

#include <string>
#include <vector>

#include "fbg_isa.h"

namespace fbg {

// A literal: variable k, complemented or not.
struct Lit {
  int k;
  bool neg;
};

// OR (or XOR) of literals, optionally inverted.
struct LitSet {
  bool is_xor = false;
  bool inv = false;
  std::vector<Lit> lits;
};

// Host form of one device instruction, before the words-per-lane dependent
// encoding.  Registers are virtual until allocation, physical after.
struct HIns {
  uint32_t op = 0;
  LitSet ls;          // CL, LDL, OPL
  uint32_t f = 0;     // OPL, OPR
  int reg = -1;       // ST, OPR, LDR
  bool inv = false;   // OPR, ACC, LDR (the register / cur operand inverted)
  bool invout = false;
};

struct Compiled {
  int n = 0;
  int const_value = -1;   // -1, or 0/1 when the formula folded to a constant
  uint64_t l2in = 0;      // AND/XOR nodes reachable from the root
  int nregs = 0;
  int n_clause_instr = 0;
  std::vector<HIns> code;
};

// Parse and compile.  Returns 0, or an fbg_status with msg / offset set.
// subst (n entries or null): -1 / -2 replace the variable by 0 / 1, j >= 0 by
// the program's variable j < n_free; out.n is n_free (n without subst).
int compile_formula(const char *src, int n, Compiled &out, std::string &msg, int64_t &offset,
                    const int32_t *subst = nullptr, int n_free = 0);

// Encode for words-per-lane 2^log2w (W <= 32).  Appends the clause block,
// FBG_INS_WORDS words per instruction after it (the jump-table form at
// 16 words per lane, closed by END), then the pattern table (a multiple of 4
// words in all); returns the instruction count.  *err (if given) is set when
// the program cannot be encoded.
uint32_t encode_program(const Compiled &c, int log2w, std::vector<uint32_t> &words, std::string *err = nullptr);

// Number of leading clause (CL) instructions; no CL follows them.
uint32_t leading_clauses(const Compiled &c);

// The same program with its variables renamed: variable k becomes to[k]
// (to a permutation of 0 .. n-1).  Evaluated at index j it gives the
// original's value at the index whose bit k is bit to[k] of j.
Compiled permute_variables(const Compiled &c, const std::vector<int> &to);

// The renaming behind the XCD-local DNF write-out at 32 words per lane
// (fbg_kernels.h), for n >= kXcdMinVars: with it, word i of lane l of tile t
// of the renamed program is the DNF word at index
//   piece(t, i >> 4) * 1024 + ((i >> 2) & 3) * 256 + 4 l + (i & 3),
//   piece(t, h) = ((t >> 2) & 7) + 16 (t & 3) + 64 (t >> 5) + 8 h,
// so that each lane writes its words 4g .. 4g+3 with one 16-byte store.
std::vector<int> xcd_write_out_permutation(int n);

// VALU instructions per 32-bit slice the evaluator issues for an encoded
// program (a static count per tile, divided by the words per lane; the
// popcount and store epilogue excluded).
double valu_per_slice(const std::vector<uint32_t> &words, uint32_t nins, int log2w, uint32_t nregs);
// Estimated cost per tile of the general part of a program in the
// jump-table form (16 words per lane), in the steps of tile_cost: its VALU
// instructions per word, and half a step per instruction for the dispatch.
double j16_general_cost(const std::vector<uint32_t> &words, uint32_t nins);

// Listing of an encoded program.
std::string disasm_program(const std::vector<uint32_t> &words, uint32_t nins, int log2w);

// Host interpretation of an encoded program, slice by slice (debug aid).
// Writes 2^max(n-5,0) 32-bit slices into out32 (zeroed tail for n < 5).
// cof: read the program the way the uniform-cofactor kernels do.
void emulate_program(const std::vector<uint32_t> &words, uint32_t nins, int nregs, int n, int log2w, bool cof,
                     uint32_t *out32);

}  // namespace fbg

#endif
