// Host-only driver of the compiler and encoder for the sanitizer build
// (tests/test_host_sanitizers.py builds it with -fsanitize=address,undefined
// from this file and compiler.cpp alone; no HIP).
//
// Input on stdin, repeated: a line "n nbytes", then nbytes of formula text.
// For each case it prints "ERR <status>" when the text does not compile,
// else one line per words-per-lane setting and evaluation variant:
//   "<log2w> <cof> <hex words of the emulated DNF vector>"
// and walks the listing and the VALU count of every encoding.  For n >= 21
// it also prints "X <hex words>": the 32-words-per-lane encoding of the
// program with the variables renamed for the XCD-local DNF write-out,
// emulated, and each emulated word (tile t, word i, lane l) put at the index
// the write-out kernel stores it to.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <string>
#include <vector>

#include "fbg_internal.h"

int main() {
  int n;
  long len;
  while (scanf("%d %ld", &n, &len) == 2) {
    if (getchar() != '\n' || len < 0 || len > (1l << 24)) return 2;
    std::string text((size_t)len, '\0');
    if (len && fread(&text[0], 1, (size_t)len, stdin) != (size_t)len) return 2;
    fbg::Compiled c;
    std::string msg;
    int64_t off = -1;
    const int st = fbg::compile_formula(text.c_str(), n, c, msg, off);
    if (st != 0) {
      printf("ERR %d\n", st);
      continue;
    }
    const uint64_t slices = c.n >= 5 ? (1ull << (c.n - 5)) : 1ull;
    const uint64_t words64 = c.n >= 6 ? (1ull << (c.n - 6)) : 1ull;
    for (int l = 0; l <= 5; l++) {
      std::vector<uint32_t> words;
      std::string err;
      const uint32_t nins = fbg::encode_program(c, l, words, &err);
      if (!err.empty()) {
        printf("ERR encode %s\n", err.c_str());
        continue;
      }
      (void)fbg::disasm_program(words, nins, l);
      (void)fbg::valu_per_slice(words, nins, l, (uint32_t)c.nregs);
      for (int cof = 0; cof < 2; cof++) {
        std::vector<uint32_t> out32((size_t)(slices < 2 ? 2 : slices), 0u);
        fbg::emulate_program(words, nins, c.nregs, c.n, l, cof != 0, out32.data());
        printf("%d %d", l, cof);
        for (uint64_t w = 0; w < words64; w++)
          printf(" %llx", (unsigned long long)((uint64_t)out32[2 * w] | ((uint64_t)out32[2 * w + 1] << 32)));
        printf("\n");
      }
    }
    if (c.n >= 21) {
      const fbg::Compiled x = fbg::permute_variables(c, fbg::xcd_write_out_permutation(c.n));
      std::vector<uint32_t> words;
      std::string err;
      const uint32_t nins = fbg::encode_program(x, 5, words, &err);
      std::vector<uint32_t> em((size_t)slices, 0u), out32((size_t)slices, 0u);
      fbg::emulate_program(words, nins, x.nregs, x.n, 5, false, em.data());
      for (uint64_t s = 0; s < slices; s++) {
        const uint64_t l = s & 63, i = (s >> 6) & 31, t = s >> 11;
        const uint64_t piece = ((t >> 2) & 7) + 16 * (t & 3) + 64 * (t >> 5) + 8 * (i >> 4);
        out32[(size_t)(piece * 1024 + ((i >> 2) & 3) * 256 + 4 * l + (i & 3))] = em[(size_t)s];
      }
      printf("X");
      for (uint64_t w = 0; w < words64; w++)
        printf(" %llx", (unsigned long long)((uint64_t)out32[2 * w] | ((uint64_t)out32[2 * w + 1] << 32)));
      printf("\n");
    }
  }
  return 0;
}
