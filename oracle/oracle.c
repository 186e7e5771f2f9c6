/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the free-Boolean-
 * generator path.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does, and this
 * file shares no code with it (own parser, own evaluator).
 *
 * What it computes (Section 2.3, Proposition "prop22"; Section 3.2 for the
 * count and the models): for a Boolean term t(x0..x{n-1}) the vector
 * d = t(b_0..b_{n-1}) of length 2^n whose bit mu is t evaluated at the
 * valuation mu, i.e. the full DNF of t.  The number of models is the number
 * of 1-bits of d; the models are the positions of those bits.
 *
 * Readings of the paper fixed here (the paper leaves them open):
 *  - variable xk is bit k of the valuation index mu (LSB first); with this
 *    order the index bits line up with the columns of the matrix M of
 *    Section 2.2 (column i = binary expansion of i);
 *  - DNF word w holds valuations 64w .. 64w+63, valuation mu at bit mu&63;
 *    bits at or above 2^n are zero;
 *  - the formula is the conjunction of all assertions of the text (a system
 *    of equations phi_i = 1, Section 5.1);
 *  - operators ~ & ^ | with Python precedence (Section 4.2), ^ being the
 *    symmetric difference the paper writes as +; constants 0 and 1.
 *
 * Two evaluators:
 *  orc_*        per valuation, recursive over the syntax tree, one memo slot
 *               per named temporary (the definition written out);
 *  orc_bitpar_* the blocked evaluation of Section 2.3 with 64-bit blocks:
 *               generator blocks b_kj are formed from the definition of M
 *               and the term is applied to whole blocks (a cross-check of the
 *               per-valuation evaluator, and the paper's own CPU variant).
 *
 * Parallelism: both split the index range into contiguous chunks, one per
 * thread, and concatenate results in chunk order.  No other reordering.
 */
#define _GNU_SOURCE
#include <ctype.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

enum { K_C0, K_C1, K_VAR, K_TMP, K_NOT, K_AND, K_OR, K_XOR };

typedef struct {
  int kind;
  int a, b; /* VAR: a = k; TMP: a = temp index; NOT: a; binary: a, b */
} onode;

typedef struct {
  onode *nodes;
  int nn, ncap;
  char **tmp_name;
  int *tmp_root;
  int ntmp, tcap;
  int *asserts;
  int na, acap;
  int max_var; /* largest variable index used, -1 if none */
} oformula;

static __thread char g_err[512];

const char *orc_error(void) { return g_err; }

/* ------------------------------------------------------------------ parse */

typedef struct {
  const char *s;
  size_t pos;
  oformula *f;
  int failed;
} oparser;

static void perr(oparser *p, const char *msg) {
  if (!p->failed)
    snprintf(g_err, sizeof g_err, "parse error at offset %zu: %s", p->pos, msg);
  p->failed = 1;
}

static int add_node(oformula *f, int kind, int a, int b) {
  if (f->nn == f->ncap) {
    f->ncap = f->ncap ? 2 * f->ncap : 256;
    f->nodes = (onode *)realloc(f->nodes, sizeof(onode) * (size_t)f->ncap);
  }
  f->nodes[f->nn].kind = kind;
  f->nodes[f->nn].a = a;
  f->nodes[f->nn].b = b;
  return f->nn++;
}

/* skip blanks and comments, not statement separators */
static void skip_ws(oparser *p) {
  for (;;) {
    char c = p->s[p->pos];
    if (c == ' ' || c == '\t' || c == '\r') {
      p->pos++;
    } else if (c == '#') {
      while (p->s[p->pos] && p->s[p->pos] != '\n') p->pos++;
    } else {
      return;
    }
  }
}

static int is_ident_start(char c) { return isalpha((unsigned char)c) || c == '_'; }
static int is_ident_char(char c) { return isalnum((unsigned char)c) || c == '_'; }

/* is s[0..len) of the form x<digits>? returns the index or -1 */
static long var_index(const char *s, size_t len) {
  if (len < 2 || s[0] != 'x') return -1;
  long v = 0;
  for (size_t i = 1; i < len; i++) {
    if (!isdigit((unsigned char)s[i])) return -1;
    v = v * 10 + (s[i] - '0');
    if (v > 1000000) return -2;
  }
  return v;
}

static int find_tmp(oformula *f, const char *s, size_t len) {
  for (int t = f->ntmp - 1; t >= 0; t--)
    if (strlen(f->tmp_name[t]) == len && memcmp(f->tmp_name[t], s, len) == 0) return t;
  return -1;
}

static int parse_or(oparser *p);

static int parse_atom(oparser *p) {
  skip_ws(p);
  char c = p->s[p->pos];
  if (c == '~') {
    p->pos++;
    int a = parse_atom(p);
    if (p->failed) return -1;
    return add_node(p->f, K_NOT, a, -1);
  }
  if (c == '(') {
    p->pos++;
    int a = parse_or(p);
    if (p->failed) return -1;
    skip_ws(p);
    if (p->s[p->pos] != ')') {
      perr(p, "expected ')'");
      return -1;
    }
    p->pos++;
    return a;
  }
  if (isdigit((unsigned char)c)) {
    size_t st = p->pos;
    while (isdigit((unsigned char)p->s[p->pos])) p->pos++;
    if (p->pos - st == 1 && c == '0') return add_node(p->f, K_C0, -1, -1);
    if (p->pos - st == 1 && c == '1') return add_node(p->f, K_C1, -1, -1);
    p->pos = st;
    perr(p, "only the constants 0 and 1 are allowed");
    return -1;
  }
  if (is_ident_start(c)) {
    size_t st = p->pos;
    while (is_ident_char(p->s[p->pos])) p->pos++;
    size_t len = p->pos - st;
    long v = var_index(p->s + st, len);
    if (v >= 0) {
      if (v > p->f->max_var) p->f->max_var = (int)v;
      return add_node(p->f, K_VAR, (int)v, -1);
    }
    if (v == -2) {
      p->pos = st;
      perr(p, "variable index too large");
      return -1;
    }
    int t = find_tmp(p->f, p->s + st, len);
    if (t < 0) {
      p->pos = st;
      perr(p, "undefined name");
      return -1;
    }
    return add_node(p->f, K_TMP, t, -1);
  }
  perr(p, "expected an operand");
  return -1;
}

static int parse_and(oparser *p) {
  int a = parse_atom(p);
  for (;;) {
    if (p->failed) return -1;
    skip_ws(p);
    if (p->s[p->pos] != '&') return a;
    p->pos++;
    int b = parse_atom(p);
    if (p->failed) return -1;
    a = add_node(p->f, K_AND, a, b);
  }
}

static int parse_xor(oparser *p) {
  int a = parse_and(p);
  for (;;) {
    if (p->failed) return -1;
    skip_ws(p);
    if (p->s[p->pos] != '^') return a;
    p->pos++;
    int b = parse_and(p);
    if (p->failed) return -1;
    a = add_node(p->f, K_XOR, a, b);
  }
}

static int parse_or(oparser *p) {
  int a = parse_xor(p);
  for (;;) {
    if (p->failed) return -1;
    skip_ws(p);
    if (p->s[p->pos] != '|') return a;
    p->pos++;
    int b = parse_xor(p);
    if (p->failed) return -1;
    a = add_node(p->f, K_OR, a, b);
  }
}

static void free_formula(oformula *f) {
  for (int t = 0; t < f->ntmp; t++) free(f->tmp_name[t]);
  free(f->tmp_name);
  free(f->tmp_root);
  free(f->nodes);
  free(f->asserts);
  memset(f, 0, sizeof *f);
}

static int parse_formula(const char *src, oformula *f) {
  memset(f, 0, sizeof *f);
  f->max_var = -1;
  oparser p = {src, 0, f, 0};
  g_err[0] = 0;
  for (;;) {
    skip_ws(&p);
    char c = src[p.pos];
    if (c == 0) break;
    if (c == '\n' || c == ';') {
      p.pos++;
      continue;
    }
    /* definition?  IDENT ws '=' */
    int is_def = 0;
    size_t st = p.pos, len = 0;
    if (is_ident_start(c)) {
      size_t q = p.pos;
      while (is_ident_char(src[q])) q++;
      len = q - st;
      size_t r = q;
      while (src[r] == ' ' || src[r] == '\t') r++;
      if (src[r] == '=') {
        if (var_index(src + st, len) != -1) {
          perr(&p, "cannot assign to a variable");
          free_formula(f);
          return -1;
        }
        if (find_tmp(f, src + st, len) >= 0) {
          perr(&p, "name defined twice");
          free_formula(f);
          return -1;
        }
        is_def = 1;
        p.pos = r + 1;
      }
    }
    int root = parse_or(&p);
    if (p.failed) {
      free_formula(f);
      return -1;
    }
    skip_ws(&p);
    c = src[p.pos];
    if (c != 0 && c != '\n' && c != ';') {
      perr(&p, "unexpected character");
      free_formula(f);
      return -1;
    }
    if (is_def) {
      if (f->ntmp == f->tcap) {
        f->tcap = f->tcap ? 2 * f->tcap : 64;
        f->tmp_name = (char **)realloc(f->tmp_name, sizeof(char *) * (size_t)f->tcap);
        f->tmp_root = (int *)realloc(f->tmp_root, sizeof(int) * (size_t)f->tcap);
      }
      char *nm = (char *)malloc(len + 1);
      memcpy(nm, src + st, len);
      nm[len] = 0;
      f->tmp_name[f->ntmp] = nm;
      f->tmp_root[f->ntmp] = root;
      f->ntmp++;
    } else {
      if (f->na == f->acap) {
        f->acap = f->acap ? 2 * f->acap : 64;
        f->asserts = (int *)realloc(f->asserts, sizeof(int) * (size_t)f->acap);
      }
      f->asserts[f->na++] = root;
    }
  }
  if (f->na == 0) {
    snprintf(g_err, sizeof g_err, "no assertion in the formula");
    free_formula(f);
    return -1;
  }
  return 0;
}

static int check_n(const oformula *f, int n, int nmax) {
  if (n < 0 || n > nmax) {
    snprintf(g_err, sizeof g_err, "n=%d out of range [0,%d]", n, nmax);
    return -1;
  }
  if (f->max_var >= n) {
    snprintf(g_err, sizeof g_err, "variable x%d used but n=%d", f->max_var, n);
    return -1;
  }
  return 0;
}

/* ---------------------------------------------- per-valuation evaluation */

typedef struct {
  const oformula *f;
  uint64_t mu;
  uint64_t gen;       /* memo generation = valuation being evaluated + 1 */
  uint64_t *memo_gen; /* per temporary */
  uint8_t *memo_val;
} vctx;

static int ev(vctx *c, int id) {
  const onode *nd = &c->f->nodes[id];
  switch (nd->kind) {
    case K_C0: return 0;
    case K_C1: return 1;
    case K_VAR: return (int)((c->mu >> nd->a) & 1u);
    case K_TMP: {
      int t = nd->a;
      if (c->memo_gen[t] != c->gen) {
        c->memo_val[t] = (uint8_t)ev(c, c->f->tmp_root[t]);
        c->memo_gen[t] = c->gen;
      }
      return c->memo_val[t];
    }
    case K_NOT: return !ev(c, nd->a);
    case K_AND: return ev(c, nd->a) ? ev(c, nd->b) : 0;
    case K_OR: return ev(c, nd->a) ? 1 : ev(c, nd->b);
    case K_XOR: return ev(c, nd->a) ^ ev(c, nd->b);
  }
  return 0;
}

/* t(mu): the conjunction of all assertions at valuation mu */
static int eval_valuation(vctx *c, uint64_t mu) {
  c->mu = mu;
  c->gen = mu + 1;
  for (int i = 0; i < c->f->na; i++)
    if (!ev(c, c->f->asserts[i])) return 0;
  return 1;
}

static void vctx_init(vctx *c, const oformula *f) {
  c->f = f;
  c->memo_gen = (uint64_t *)calloc((size_t)(f->ntmp + 1), sizeof(uint64_t));
  c->memo_val = (uint8_t *)calloc((size_t)(f->ntmp + 1), 1);
}

static void vctx_free(vctx *c) {
  free(c->memo_gen);
  free(c->memo_val);
}

typedef struct {
  const oformula *f;
  uint64_t lo, hi; /* valuation range [lo, hi) */
  uint64_t count;
  uint64_t *dnf;   /* optional: whole-vector words */
  uint64_t *models;
  uint64_t nmodels, mcap;
  uint64_t keep; /* keep at most this many models (the first ones in range) */
  int want_models;
} vjob;

static void *vjob_run(void *arg) {
  vjob *j = (vjob *)arg;
  vctx c;
  vctx_init(&c, j->f);
  for (uint64_t mu = j->lo; mu < j->hi; mu++) {
    if (eval_valuation(&c, mu)) {
      j->count++;
      if (j->dnf) j->dnf[mu >> 6] |= (uint64_t)1 << (mu & 63);
      if (j->want_models && j->nmodels < j->keep) {
        if (j->nmodels == j->mcap) {
          j->mcap = j->mcap ? 2 * j->mcap : 1024;
          j->models = (uint64_t *)realloc(j->models, sizeof(uint64_t) * j->mcap);
        }
        j->models[j->nmodels++] = mu;
      }
    }
  }
  vctx_free(&c);
  return NULL;
}

static int default_threads(int threads) {
  if (threads > 0) return threads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

/* Split [lo, hi) into contiguous chunks aligned to 64 valuations. */
static int run_range(const oformula *f, uint64_t lo, uint64_t hi, int threads, uint64_t *dnf, int want_models,
                     uint64_t *count, uint64_t *models, uint64_t cap, uint64_t *total);

static int run_valuations(const oformula *f, int n, int threads, uint64_t *dnf, int want_models,
                          uint64_t *count, uint64_t *models, uint64_t cap, uint64_t *total) {
  return run_range(f, 0, (uint64_t)1 << n, threads, dnf, want_models, count, models, cap, total);
}

static int run_range(const oformula *f, uint64_t lo, uint64_t hi, int threads, uint64_t *dnf, int want_models,
                     uint64_t *count, uint64_t *models, uint64_t cap, uint64_t *total) {
  uint64_t total_v = hi;
  int T = default_threads(threads);
  uint64_t w0 = lo / 64;
  uint64_t words = (total_v + 63) / 64 - w0;
  if ((uint64_t)T > words) T = (int)words;
  if (T < 1) T = 1;
  vjob *jobs = (vjob *)calloc((size_t)T, sizeof(vjob));
  pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
  for (int t = 0; t < T; t++) {
    uint64_t wlo = w0 + words * (uint64_t)t / (uint64_t)T, whi = w0 + words * (uint64_t)(t + 1) / (uint64_t)T;
    jobs[t].f = f;
    jobs[t].lo = wlo * 64 > lo ? wlo * 64 : lo;
    jobs[t].hi = whi * 64 < total_v ? whi * 64 : total_v;
    jobs[t].dnf = dnf;
    jobs[t].want_models = want_models;
    jobs[t].keep = cap;
  }
  for (int t = 1; t < T; t++) pthread_create(&th[t], NULL, vjob_run, &jobs[t]);
  vjob_run(&jobs[0]);
  for (int t = 1; t < T; t++) pthread_join(th[t], NULL);
  uint64_t cnt = 0, written = 0;
  for (int t = 0; t < T; t++) {
    cnt += jobs[t].count;
    if (want_models) {
      for (uint64_t i = 0; i < jobs[t].nmodels && written < cap; i++) models[written++] = jobs[t].models[i];
      free(jobs[t].models);
    }
  }
  if (count) *count = cnt;
  if (total) *total = cnt;
  free(jobs);
  free(th);
  return 0;
}

#define ORC_NMAX 48

int orc_count(const char *src, int n, int threads, uint64_t *out_count) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, ORC_NMAX)) {
    free_formula(&f);
    return -1;
  }
  run_valuations(&f, n, threads, NULL, 0, out_count, NULL, 0, NULL);
  free_formula(&f);
  return 0;
}

/* out must hold max(1, 2^(n-6)) words; it is cleared first. */
int orc_dnf(const char *src, int n, int threads, uint64_t *out, uint64_t out_words) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, 40)) {
    free_formula(&f);
    return -1;
  }
  uint64_t need = n >= 6 ? ((uint64_t)1 << (n - 6)) : 1;
  if (out_words < need) {
    snprintf(g_err, sizeof g_err, "out_words %llu < %llu", (unsigned long long)out_words,
             (unsigned long long)need);
    free_formula(&f);
    return -1;
  }
  memset(out, 0, sizeof(uint64_t) * need);
  run_valuations(&f, n, threads, out, 0, NULL, NULL, 0, NULL);
  free_formula(&f);
  return 0;
}

/* Ascending model indices, at most cap of them; *total = number of models. */
int orc_models(const char *src, int n, int threads, uint64_t *out, uint64_t cap, uint64_t *total) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, ORC_NMAX)) {
    free_formula(&f);
    return -1;
  }
  run_valuations(&f, n, threads, NULL, 1, NULL, out, cap, total);
  free_formula(&f);
  return 0;
}

/* Models among the valuations lo <= mu < hi (a bounded sample of the count). */
int orc_count_range(const char *src, int n, uint64_t lo, uint64_t hi, int threads, uint64_t *out_count) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, ORC_NMAX)) {
    free_formula(&f);
    return -1;
  }
  uint64_t top = (uint64_t)1 << n;
  if (hi > top) hi = top;
  if (lo >= hi) {
    *out_count = 0;
    free_formula(&f);
    return 0;
  }
  run_range(&f, lo, hi, threads, NULL, 0, out_count, NULL, 0, NULL);
  free_formula(&f);
  return 0;
}

/* t(mu) for each listed valuation; out[i] = 0/1. */
int orc_eval_at(const char *src, int n, const uint64_t *idx, uint64_t m, uint8_t *out) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, 63)) {
    free_formula(&f);
    return -1;
  }
  vctx c;
  vctx_init(&c, &f);
  for (uint64_t i = 0; i < m; i++) {
    if (n < 64 && (idx[i] >> n) != 0) {
      snprintf(g_err, sizeof g_err, "valuation %llu out of range", (unsigned long long)idx[i]);
      vctx_free(&c);
      free_formula(&f);
      return -1;
    }
    out[i] = (uint8_t)eval_valuation(&c, idx[i]);
  }
  vctx_free(&c);
  free_formula(&f);
  return 0;
}

/* Number of letters the text mentions: 1 + largest variable index (0 if none),
   and the number of assertions and temporaries, for test introspection. */
int orc_describe(const char *src, int *nvars, int *nasserts, int *ntemps) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  *nvars = f.max_var + 1;
  *nasserts = f.na;
  *ntemps = f.ntmp;
  free_formula(&f);
  return 0;
}

/* ---------------------------------------------- blocked (bit-parallel) */

/*
 * Section 2.3: every generator b_k is cut into blocks of 2^6 = 64 bits and the
 * term is applied to the blocks b_kj bitwise.  Block j of b_k holds bit k of
 * the indices 64j .. 64j+63 (row k of M restricted to those columns):
 *   k < 6 : bit k of the offset 0..63, the same pattern for every block;
 *   k >= 6: bit k-6 of j, i.e. the block is all ones or all zeros.
 */
typedef struct {
  const oformula *f;
  uint64_t j;
  uint64_t low[6];
  uint64_t *memo_gen;
  uint64_t *memo_val;
  uint64_t gen;
} bctx;

static uint64_t generator_block(const bctx *c, int k) {
  if (k < 6) return c->low[k];
  return ((c->j >> (k - 6)) & 1u) ? ~(uint64_t)0 : 0;
}

static uint64_t evb(bctx *c, int id) {
  const onode *nd = &c->f->nodes[id];
  switch (nd->kind) {
    case K_C0: return 0;
    case K_C1: return ~(uint64_t)0;
    case K_VAR: return generator_block(c, nd->a);
    case K_TMP: {
      int t = nd->a;
      if (c->memo_gen[t] != c->gen) {
        c->memo_val[t] = evb(c, c->f->tmp_root[t]);
        c->memo_gen[t] = c->gen;
      }
      return c->memo_val[t];
    }
    case K_NOT: return ~evb(c, nd->a);
    case K_AND: return evb(c, nd->a) & evb(c, nd->b);
    case K_OR: return evb(c, nd->a) | evb(c, nd->b);
    case K_XOR: return evb(c, nd->a) ^ evb(c, nd->b);
  }
  return 0;
}

typedef struct {
  const oformula *f;
  int n;
  uint64_t wlo, whi;
  uint64_t count;
  uint64_t *dnf;
} bjob;

static void *bjob_run(void *arg) {
  bjob *b = (bjob *)arg;
  bctx c;
  c.f = b->f;
  for (int k = 0; k < 6; k++) {
    uint64_t w = 0;
    for (int bit = 0; bit < 64; bit++)
      if ((bit >> k) & 1) w |= (uint64_t)1 << bit;
    c.low[k] = w;
  }
  c.memo_gen = (uint64_t *)calloc((size_t)(b->f->ntmp + 1), sizeof(uint64_t));
  c.memo_val = (uint64_t *)calloc((size_t)(b->f->ntmp + 1), sizeof(uint64_t));
  uint64_t tail = b->n >= 6 ? ~(uint64_t)0 : (((uint64_t)1 << ((uint64_t)1 << b->n)) - 1);
  for (uint64_t j = b->wlo; j < b->whi; j++) {
    c.j = j;
    c.gen = j + 1;
    uint64_t d = ~(uint64_t)0;
    for (int i = 0; i < b->f->na && d; i++) d &= evb(&c, b->f->asserts[i]);
    d &= tail;
    b->count += (uint64_t)__builtin_popcountll(d);
    if (b->dnf) b->dnf[j] = d;
  }
  free(c.memo_gen);
  free(c.memo_val);
  return NULL;
}

static int run_blocks(const oformula *f, int n, int threads, uint64_t *dnf, uint64_t *count) {
  uint64_t words = n >= 6 ? ((uint64_t)1 << (n - 6)) : 1;
  int T = default_threads(threads);
  if ((uint64_t)T > words) T = (int)words;
  bjob *jobs = (bjob *)calloc((size_t)T, sizeof(bjob));
  pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
  for (int t = 0; t < T; t++) {
    jobs[t].f = f;
    jobs[t].n = n;
    jobs[t].wlo = words * (uint64_t)t / (uint64_t)T;
    jobs[t].whi = words * (uint64_t)(t + 1) / (uint64_t)T;
    jobs[t].dnf = dnf;
  }
  for (int t = 1; t < T; t++) pthread_create(&th[t], NULL, bjob_run, &jobs[t]);
  bjob_run(&jobs[0]);
  for (int t = 1; t < T; t++) pthread_join(th[t], NULL);
  uint64_t cnt = 0;
  for (int t = 0; t < T; t++) cnt += jobs[t].count;
  if (count) *count = cnt;
  free(jobs);
  free(th);
  return 0;
}

int orc_bitpar_count(const char *src, int n, int threads, uint64_t *out_count) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, ORC_NMAX)) {
    free_formula(&f);
    return -1;
  }
  run_blocks(&f, n, threads, NULL, out_count);
  free_formula(&f);
  return 0;
}

int orc_bitpar_dnf(const char *src, int n, int threads, uint64_t *out, uint64_t out_words) {
  oformula f;
  if (parse_formula(src, &f)) return -1;
  if (check_n(&f, n, 40)) {
    free_formula(&f);
    return -1;
  }
  uint64_t need = n >= 6 ? ((uint64_t)1 << (n - 6)) : 1;
  if (out_words < need) {
    snprintf(g_err, sizeof g_err, "out_words too small");
    free_formula(&f);
    return -1;
  }
  run_blocks(&f, n, threads, out, NULL);
  free_formula(&f);
  return 0;
}

/* ------------------------------------------------------------------------
 * Unlabeled models (Section 3.2: kappa_{T,n} is the number of non-isomorphic
 * models of size n).  Two labeled models are isomorphic when a permutation of
 * the domain maps one onto the other; a permutation acts on valuations by
 * moving the value of each letter to the letter it maps that letter to.
 * perms holds the action of every permutation of the group on the n letters
 * (perms[p*n + k] = image of letter k); the orbits are counted as the number
 * of distinct smallest images, computed model by model.
 * ---------------------------------------------------------------------- */

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y);
}

int orc_orbits(const char *src, int n, const int32_t *perms, int nperm, int threads, uint64_t *out_orbits,
               uint64_t *out_models) {
  uint64_t total = 0;
  if (n < 0 || n > 40 || nperm <= 0) {
    snprintf(g_err, sizeof g_err, "orbits: n=%d nperm=%d out of range", n, nperm);
    return -1;
  }
  for (int p = 0; p < nperm; p++)
    for (int k = 0; k < n; k++)
      if (perms[(size_t)p * n + k] < 0 || perms[(size_t)p * n + k] >= n) {
        snprintf(g_err, sizeof g_err, "orbits: perms[%d][%d] out of range", p, k);
        return -1;
      }
  if (orc_count(src, n, threads, &total)) return -1;
  uint64_t *m = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
  if (!m) {
    snprintf(g_err, sizeof g_err, "orbits: out of memory");
    return -1;
  }
  uint64_t got = 0;
  if (orc_models(src, n, threads, m, total, &got)) {
    free(m);
    return -1;
  }
  for (uint64_t i = 0; i < total; i++) {
    uint64_t best = UINT64_MAX;
    for (int p = 0; p < nperm; p++) {
      const int32_t *pi = perms + (size_t)p * n;
      uint64_t img = 0;
      for (int k = 0; k < n; k++)
        if ((m[i] >> k) & 1u) img |= 1ull << pi[k];
      if (img < best) best = img;
    }
    m[i] = best;
  }
  qsort(m, total, sizeof(uint64_t), cmp_u64);
  uint64_t orbits = 0;
  for (uint64_t i = 0; i < total; i++)
    if (i == 0 || m[i] != m[i - 1]) orbits++;
  free(m);
  *out_orbits = orbits;
  if (out_models) *out_models = total;
  return 0;
}
