// compiler.cpp -- formula text to straight-line bitwise program.
//
// Section 4.1 of the paper: the engine builds a computing tree for the formula
// and the Reduction submodule removes the constants 0 and 1.  Here the text is
// parsed into a hash-consed graph of 2-input AND / XOR nodes with complemented
// edges (OR is AND with complemented inputs and output), which gives constant
// folding, common-subexpression elimination and dead-code removal by
// construction.  Code generation then:
//   * splits the root into top-level conjuncts (the equations of a system,
//     Section 5.1, and the clauses of a CNF);
//   * turns every sub-term that is an OR, AND or XOR of literals into one
//     literal-set operand (fbg_isa.h), whatever its width;
//   * evaluates the remaining structure in post order through a current value
//     and LDS registers, registers being allocated by a linear scan over the
//     emitted code.
#include <pthread.h>
#include <string.h>
#include <sys/mman.h>
#include <ucontext.h>

#include <algorithm>
#include <array>
#include <set>
#include <cctype>
#include <new>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/fbg.h"
#include "fbg_internal.h"

namespace fbg {
namespace {

// ------------------------------------------------------------------ graph

enum : uint8_t { NK_CONST = 0, NK_VAR = 1, NK_AND = 2, NK_XOR = 3 };

struct GNode {
  uint8_t kind;
  uint32_t a, b;  // VAR: a = variable; AND/XOR: child edges
};

// Edge = node << 1 | complement.  Node 0 is the constant false.
typedef uint32_t Edge;
constexpr Edge kFalse = 0, kTrue = 1;

struct Graph {
  std::vector<GNode> nodes;
  std::unordered_map<uint64_t, uint32_t> table;
  std::vector<uint32_t> vars;  // node of variable k, 0 if none yet

  Graph() { nodes.push_back({NK_CONST, 0, 0}); }

  // room for about m nodes without rehashing
  void reserve(size_t m) {
    nodes.reserve(m + 1);
    table.reserve(m);
  }

  uint32_t node_of(uint8_t kind, uint32_t a, uint32_t b) {
    uint64_t key = ((uint64_t)kind << 62) ^ ((uint64_t)a << 31) ^ (uint64_t)b;
    auto it = table.find(key);
    if (it != table.end()) {
      const GNode &g = nodes[it->second];
      if (g.kind == kind && g.a == a && g.b == b) return it->second;
      // key collision (only for gigantic graphs): fall back to a linear probe
      for (uint32_t i = 1; i < nodes.size(); i++)
        if (nodes[i].kind == kind && nodes[i].a == a && nodes[i].b == b) return i;
    }
    uint32_t id = (uint32_t)nodes.size();
    nodes.push_back({kind, a, b});
    table.emplace(key, id);
    return id;
  }

  Edge var(int k) {
    if ((size_t)k >= vars.size()) vars.resize((size_t)k + 1, 0u);
    if (vars[(size_t)k]) return vars[(size_t)k] << 1;
    const uint32_t id = node_of(NK_VAR, (uint32_t)k, 0);
    vars[(size_t)k] = id;
    return id << 1;
  }

  Edge And(Edge a, Edge b) {
    if (a > b) std::swap(a, b);
    if (a == kFalse) return kFalse;
    if (a == kTrue) return b;
    if (a == b) return a;
    if ((a ^ 1u) == b) return kFalse;
    return node_of(NK_AND, a, b) << 1;
  }

  Edge Xor(Edge a, Edge b) {
    uint32_t c = (a ^ b) & 1u;
    a &= ~1u;
    b &= ~1u;
    if (a > b) std::swap(a, b);
    if (a == kFalse) return b ^ c;
    if (a == b) return kFalse ^ c;
    return (node_of(NK_XOR, a, b) << 1) ^ c;
  }

  Edge Or(Edge a, Edge b) { return And(a ^ 1u, b ^ 1u) ^ 1u; }
};

// ----------------------------------------------------------------- parser

struct Tok {
  enum Kind { END, SEP, LP, RP, NOT, AND, XOR, OR, EQ, CONST, VAR, NAME } kind;
  int64_t pos;
  int64_t val;  // CONST value, VAR index
  std::string name;
};

struct Parser {
  const char *src;
  int n;
  Graph &g;
  std::vector<Tok> toks;
  size_t p = 0;
  std::unordered_map<std::string, Edge> names;
  std::string msg;
  int64_t off = -1;
  int status = FBG_OK;

  // Substitution (Section 3.3, killing variables): subst[k] = -1 or -2
  // replaces xk by the constant 0 or 1, which the graph folds away (the
  // Reduction of Section 4.1); subst[k] = j >= 0 makes xk the program's
  // variable j (several letters may share one).  Null: every xk is itself.
  const int32_t *subst = nullptr;

  Parser(const char *s, int nv, Graph &gr) : src(s), n(nv), g(gr) {}

  bool fail(int st, int64_t at, const std::string &m) {
    if (status == FBG_OK) {
      status = st;
      off = at;
      msg = m;
    }
    return false;
  }

  bool lex() {
    toks.reserve(strlen(src) / 2 + 2);
    int64_t i = 0;
    for (;;) {
      char c = src[i];
      if (c == 0) {
        toks.push_back({Tok::END, i, 0, {}});
        return true;
      }
      if (c == ' ' || c == '\t' || c == '\r') {
        i++;
        continue;
      }
      if (c == '#') {
        while (src[i] && src[i] != '\n') i++;
        continue;
      }
      Tok t{Tok::END, i, 0, {}};
      switch (c) {
        case '\n':
        case ';': t.kind = Tok::SEP; i++; break;
        case '(': t.kind = Tok::LP; i++; break;
        case ')': t.kind = Tok::RP; i++; break;
        case '~': t.kind = Tok::NOT; i++; break;
        case '&': t.kind = Tok::AND; i++; break;
        case '^': t.kind = Tok::XOR; i++; break;
        case '|': t.kind = Tok::OR; i++; break;
        case '=': t.kind = Tok::EQ; i++; break;
        default:
          if (isdigit((unsigned char)c)) {
            int64_t st = i;
            while (isdigit((unsigned char)src[i])) i++;
            if (i - st != 1 || (c != '0' && c != '1'))
              return fail(FBG_E_PARSE, st, "only the constants 0 and 1 are allowed");
            t.kind = Tok::CONST;
            t.val = c - '0';
          } else if (isalpha((unsigned char)c) || c == '_') {
            int64_t st = i;
            while (isalnum((unsigned char)src[i]) || src[i] == '_') i++;
            const int64_t len = i - st;
            bool isvar = len >= 2 && c == 'x';
            for (int64_t q = st + 1; isvar && q < i; q++) isvar = isdigit((unsigned char)src[q]) != 0;
            if (isvar) {
              if (len > 9) return fail(FBG_E_RANGE, st, "variable index too large");
              t.kind = Tok::VAR;
              t.val = 0;
              for (int64_t q = st + 1; q < i; q++) t.val = 10 * t.val + (src[q] - '0');
            } else {
              t.kind = Tok::NAME;
              t.name.assign(src + st, (size_t)len);
            }
          } else {
            return fail(FBG_E_PARSE, i, std::string("unexpected character '") + c + "'");
          }
      }
      toks.push_back(t);
    }
  }

  const Tok &peek() const { return toks[p]; }

  // precedence climbing over | (1), ^ (2), & (3); ~ is a prefix operator
  bool primary(Edge &e) {
    const Tok &t = toks[p];
    switch (t.kind) {
      case Tok::NOT: {
        p++;
        Edge a;
        if (!primary(a)) return false;
        e = a ^ 1u;
        return true;
      }
      case Tok::LP: {
        p++;
        if (!expr(e, 1)) return false;
        if (toks[p].kind != Tok::RP) return fail(FBG_E_PARSE, toks[p].pos, "expected ')'");
        p++;
        return true;
      }
      case Tok::CONST: p++; e = t.val ? kTrue : kFalse; return true;
      case Tok::VAR:
        if (t.val >= n) return fail(FBG_E_RANGE, t.pos, "variable x" + std::to_string(t.val) + " >= n");
        p++;
        if (!subst)
          e = g.var((int)t.val);
        else if (subst[t.val] < 0)
          e = subst[t.val] == -2 ? kTrue : kFalse;
        else
          e = g.var(subst[t.val]);
        return true;
      case Tok::NAME: {
        auto it = names.find(t.name);
        if (it == names.end()) return fail(FBG_E_PARSE, t.pos, "undefined name '" + t.name + "'");
        p++;
        e = it->second;
        return true;
      }
      default: return fail(FBG_E_PARSE, t.pos, "expected an operand");
    }
  }

  static int prec(Tok::Kind k) { return k == Tok::OR ? 1 : k == Tok::XOR ? 2 : k == Tok::AND ? 3 : 0; }

  bool expr(Edge &e, int minp) {
    if (!primary(e)) return false;
    for (;;) {
      Tok::Kind k = toks[p].kind;
      int pr = prec(k);
      if (pr == 0 || pr < minp) return true;
      p++;
      Edge r;
      if (!expr(r, pr + 1)) return false;  // left associative
      e = (k == Tok::OR) ? g.Or(e, r) : (k == Tok::XOR) ? g.Xor(e, r) : g.And(e, r);
    }
  }

  bool program(Edge &root) {
    if (!lex()) return false;
    g.reserve(toks.size());
    root = kTrue;
    int nassert = 0;
    for (;;) {
      while (peek().kind == Tok::SEP) p++;
      if (peek().kind == Tok::END) break;
      bool def = peek().kind == Tok::NAME && toks[p + 1].kind == Tok::EQ;
      if (peek().kind == Tok::VAR && toks[p + 1].kind == Tok::EQ)
        return fail(FBG_E_PARSE, peek().pos, "cannot assign to a variable");
      std::string name;
      if (def) {
        name = peek().name;
        if (names.count(name)) return fail(FBG_E_PARSE, peek().pos, "name '" + name + "' defined twice");
        p += 2;
      }
      Edge e;
      if (!expr(e, 1)) return false;
      if (peek().kind != Tok::SEP && peek().kind != Tok::END)
        return fail(FBG_E_PARSE, peek().pos, "unexpected token");
      if (def) {
        names[name] = e;
      } else {
        root = g.And(root, e);
        nassert++;
      }
    }
    if (nassert == 0) return fail(FBG_E_PARSE, 0, "no assertion in the formula");
    return true;
  }
};

// ---------------------------------------------------------------- codegen

struct Codegen {
  Graph &g;
  std::vector<uint32_t> fanout;      // per node, parents among reachable nodes
  std::vector<HIns> code;
  std::unordered_map<uint32_t, int> stored;  // node -> virtual register
  int nvregs = 0;

  explicit Codegen(Graph &gr) : g(gr) {}

  bool is_var(Edge e) const { return g.nodes[e >> 1].kind == NK_VAR; }
  Lit lit_of(Edge e) const { return Lit{(int)g.nodes[e >> 1].a, (e & 1u) != 0}; }

  // Reachable AND/XOR nodes and their fan-out (iterative DFS).
  uint64_t analyse(Edge root) {
    fanout.assign(g.nodes.size(), 0);
    std::vector<uint8_t> seen(g.nodes.size(), 0);
    std::vector<uint32_t> stack{root >> 1};
    uint64_t gates = 0;
    seen[root >> 1] = 1;
    while (!stack.empty()) {
      uint32_t v = stack.back();
      stack.pop_back();
      const GNode &nd = g.nodes[v];
      if (nd.kind != NK_AND && nd.kind != NK_XOR) continue;
      gates++;
      for (uint32_t c : {nd.a >> 1, nd.b >> 1}) {
        fanout[c]++;
        if (!seen[c]) {
          seen[c] = 1;
          stack.push_back(c);
        }
      }
    }
    return gates;
  }

  // If edge e is an OR / AND / XOR of literals only, describe it as a
  // literal set.  Flattening passes through shared nodes too: a literal set
  // costs one instruction wherever it is used.
  bool literal_set(Edge e, LitSet &ls) {
    const GNode &top = g.nodes[e >> 1];
    ls = LitSet();
    if (top.kind == NK_VAR) {
      ls.lits.push_back(lit_of(e));
      return true;
    }
    if (top.kind == NK_AND) {
      // e = AND(leaves) (possibly complemented); leaves through plain AND edges
      std::vector<Edge> stack{top.a, top.b};
      std::vector<Lit> leaves;
      while (!stack.empty()) {
        Edge c = stack.back();
        stack.pop_back();
        const GNode &nd = g.nodes[c >> 1];
        if (nd.kind == NK_AND && !(c & 1u)) {
          stack.push_back(nd.a);
          stack.push_back(nd.b);
        } else if (nd.kind == NK_VAR) {
          leaves.push_back(lit_of(c));
        } else {
          return false;
        }
      }
      // AND(l) = ~OR(~l); ~AND(l) = OR(~l)
      for (Lit &l : leaves) l.neg = !l.neg;
      ls.lits = std::move(leaves);
      ls.inv = !(e & 1u);
      return true;
    }
    if (top.kind == NK_XOR) {
      std::vector<Edge> stack{top.a, top.b};
      bool parity = (e & 1u) != 0;
      std::vector<Lit> leaves;
      while (!stack.empty()) {
        Edge c = stack.back();
        stack.pop_back();
        const GNode &nd = g.nodes[c >> 1];
        if (nd.kind == NK_XOR) {
          parity ^= (c & 1u) != 0;
          stack.push_back(nd.a);
          stack.push_back(nd.b);
        } else if (nd.kind == NK_VAR) {
          leaves.push_back(Lit{(int)nd.a, false});
          parity ^= (c & 1u) != 0;
        } else {
          return false;
        }
      }
      ls.is_xor = true;
      ls.lits = std::move(leaves);
      ls.inv = parity;
      return true;
    }
    return false;
  }

  void emit(const HIns &h) { code.push_back(h); }
  void emit(HIns &&h) { code.push_back(std::move(h)); }

  // Invert cur: fold into the previous cur-writing instruction when possible.
  void emit_not() {
    if (!code.empty()) {
      HIns &last = code.back();
      if (last.op != FBG_OP_ST && last.op != FBG_OP_CL && last.op != FBG_OP_ACC) {
        last.invout = !last.invout;
        return;
      }
    }
    HIns h;
    h.op = FBG_OP_NOT;
    emit(h);
  }

  // value of edge e into cur
  void gen_edge(Edge e) {
    LitSet ls;
    if (literal_set(e, ls)) {
      HIns h;
      h.op = FBG_OP_LDL;
      h.ls = ls;
      emit(h);
      return;
    }
    gen_node(e >> 1);
    if (e & 1u) emit_not();
  }

  // Operand list of a node: flatten through single-use children of the same
  // kind that are not already stored.
  void operands(uint32_t v, std::vector<Edge> &ops, bool &parity) {
    const GNode &top = g.nodes[v];
    uint8_t kind = top.kind;
    parity = false;
    std::vector<Edge> stack{top.a, top.b};
    while (!stack.empty()) {
      Edge c = stack.back();
      stack.pop_back();
      uint32_t cn = c >> 1;
      const GNode &nd = g.nodes[cn];
      bool through = nd.kind == kind && fanout[cn] == 1 && !stored.count(cn);
      if (kind == NK_AND) through = through && !(c & 1u);
      if (through) {
        if (kind == NK_XOR) parity ^= (c & 1u) != 0;
        stack.push_back(nd.a);
        stack.push_back(nd.b);
      } else {
        ops.push_back(c);
      }
    }
    // duplicates: AND keeps one; XOR cancels pairs (x ^ x = 0, x ^ ~x = 1)
    std::sort(ops.begin(), ops.end());
    std::vector<Edge> out;
    for (size_t i = 0; i < ops.size();) {
      size_t j = i;
      if (kind == NK_XOR) {
        // group by node, ignoring complement
        while (j < ops.size() && (ops[j] >> 1) == (ops[i] >> 1)) j++;
        bool odd = ((j - i) & 1u) != 0;
        bool par = false;
        for (size_t q = i; q < j; q++) par ^= (ops[q] & 1u) != 0;
        parity ^= par;
        if (odd) out.push_back(ops[i] & ~1u);
      } else {
        while (j < ops.size() && ops[j] == ops[i]) j++;
        out.push_back(ops[i]);
      }
      i = j;
    }
    ops.swap(out);
  }

  void gen_node(uint32_t v) {
    auto it = stored.find(v);
    if (it != stored.end()) {
      HIns h;
      h.op = FBG_OP_LDR;
      h.reg = it->second;
      emit(h);
      return;
    }
    const GNode &nd = g.nodes[v];
    bool is_and = nd.kind == NK_AND;
    uint32_t f = is_and ? FBG_F_AND : FBG_F_XOR;
    std::vector<Edge> ops;
    bool parity = false;
    operands(v, ops, parity);

    // AND with x and ~x among the operands is false; the hashed graph folds
    // direct pairs, flattening can still bring them together.
    if (is_and) {
      std::unordered_set<Edge> have(ops.begin(), ops.end());
      for (Edge e : ops)
        if (have.count(e ^ 1u)) {
          HIns h;
          h.op = FBG_OP_LDL;  // empty OR-set = 0
          emit(h);
          store_if_shared(v);
          return;
        }
    }

    std::vector<Lit> plain;
    std::vector<LitSet> sets;
    std::vector<Edge> general;
    for (Edge e : ops) {
      LitSet ls;
      if (is_var(e)) {
        plain.push_back(lit_of(e));
      } else if (literal_set(e, ls)) {
        sets.push_back(ls);
      } else {
        general.push_back(e);
      }
    }
    if (!plain.empty()) {
      LitSet ls;
      if (is_and) {  // AND(l) = ~OR(~l)
        for (Lit l : plain) ls.lits.push_back(Lit{l.k, !l.neg});
        ls.inv = true;
      } else {
        ls.is_xor = true;
        ls.lits = plain;
      }
      sets.insert(sets.begin(), ls);
    }
    // an XOR's parity goes into one of its XOR literal sets if it has one
    if (!is_and && parity) {
      for (LitSet &ls : sets)
        if (ls.is_xor) {
          ls.inv = !ls.inv;
          parity = false;
          break;
        }
    }
    // Stored operands first (cheap register reads), then the others by
    // decreasing register need, so that the operand needing most registers
    // is evaluated while no partial result is held (Sethi-Ullman order).
    std::stable_sort(general.begin(), general.end(), [&](Edge a, Edge b) {
      const bool sa = stored.count(a >> 1) != 0, sb = stored.count(b >> 1) != 0;
      if (sa != sb) return sa;
      return !sa && need(a >> 1) > need(b >> 1);
    });

    bool have_cur = false;
    if (!general.empty()) {
      // start from a general operand that is not stored if there is one, so
      // that stored ones combine through OPR without a reload
      size_t first = 0;
      for (size_t i = 0; i < general.size(); i++)
        if (!stored.count(general[i] >> 1)) {
          first = i;
          break;
        }
      gen_edge(general[first]);
      general.erase(general.begin() + (long)first);
      have_cur = true;
      for (Edge e : general) {
        auto s = stored.find(e >> 1);
        if (s != stored.end()) {
          HIns h;
          h.op = FBG_OP_OPR;
          h.f = f;
          h.reg = s->second;
          h.inv = (e & 1u) != 0;
          emit(h);
        } else {
          int t = nvregs++;
          HIns st;
          st.op = FBG_OP_ST;
          st.reg = t;
          emit(st);
          gen_edge(e);
          HIns h;
          h.op = FBG_OP_OPR;
          h.f = f;
          h.reg = t;
          emit(h);
        }
      }
    }
    for (const LitSet &ls : sets) {
      HIns h;
      h.ls = ls;
      if (!have_cur) {
        h.op = FBG_OP_LDL;
        have_cur = true;
      } else {
        h.op = FBG_OP_OPL;
        h.f = f;
      }
      emit(h);
    }
    if (!have_cur) {  // cannot happen for a hashed AND/XOR node
      HIns h;
      h.op = FBG_OP_LDL;
      h.ls.inv = is_and;  // neutral element
      emit(h);
    }
    if (parity) emit_not();
    store_if_shared(v);
  }

  // Registers the evaluation of node v needs, estimated on the tree view of
  // the graph (shared nodes counted as computed in place): an operand that is
  // a literal set needs none; the first general operand is evaluated with no
  // partial result held, every later one while the partial result of the
  // node sits in a register, so it needs its own need plus one.
  std::unordered_map<uint32_t, uint32_t> need_memo;
  uint32_t need(uint32_t v) {
    auto it = need_memo.find(v);
    if (it != need_memo.end()) return it->second;
    need_memo[v] = 0;  // cycles cannot occur; this guards a revisit during the walk
    std::vector<Edge> ops;
    bool parity;
    operands(v, ops, parity);
    std::vector<uint32_t> ns;
    for (Edge e : ops) {
      LitSet ls;
      if (is_var(e) || literal_set(e, ls)) continue;
      ns.push_back(need(e >> 1));
    }
    std::sort(ns.begin(), ns.end(), std::greater<uint32_t>());
    uint32_t r = 0;
    for (size_t j = 0; j < ns.size(); j++) r = std::max<uint32_t>(r, ns[j] + (j > 0 ? 1u : 0u));
    need_memo[v] = r;
    return r;
  }

  void store_if_shared(uint32_t v) {
    if (fanout[v] > 1) {
      int r = nvregs++;
      HIns st;
      st.op = FBG_OP_ST;
      st.reg = r;
      emit(st);
      stored[v] = r;
    }
  }

  void top(Edge root, int &n_clause) {
    // conjuncts: flatten plain AND edges from the root through single-use nodes
    std::vector<Edge> conj;
    std::vector<Edge> stack{root};
    while (!stack.empty()) {
      Edge e = stack.back();
      stack.pop_back();
      const GNode &nd = g.nodes[e >> 1];
      if (nd.kind == NK_AND && !(e & 1u) && (e == root || fanout[e >> 1] == 1)) {
        stack.push_back(nd.b);
        stack.push_back(nd.a);
      } else {
        conj.push_back(e);
      }
    }
    std::unordered_set<Edge> seen;
    std::vector<Edge> uniq;
    for (Edge e : conj)
      if (seen.insert(e).second) uniq.push_back(e);
    for (Edge e : uniq)
      if (seen.count(e ^ 1u)) {  // x & ~x
        code.clear();
        HIns h;
        h.op = FBG_OP_CL;  // acc &= 0
        emit(h);
        n_clause = 1;
        return;
      }
    // Clauses first, as one prefix of CL instructions (the kernels run that
    // prefix in a loop of its own); then XOR / AND sets of literals through
    // cur; then the general conjuncts.
    n_clause = 0;
    code.reserve(uniq.size() + 16);
    std::vector<Edge> general;
    std::vector<LitSet> other_sets;
    for (Edge e : uniq) {
      LitSet ls;
      if (literal_set(e, ls)) {
        if (!ls.is_xor && !ls.inv) {
          HIns h;
          h.op = FBG_OP_CL;
          h.ls = std::move(ls);
          emit(std::move(h));
          n_clause++;
        } else {
          other_sets.push_back(std::move(ls));
        }
      } else {
        general.push_back(e);
      }
    }
    for (const LitSet &ls : other_sets) {
      HIns h;
      h.op = FBG_OP_LDL;
      h.ls = ls;
      emit(h);
      HIns a;
      a.op = FBG_OP_ACC;
      emit(a);
    }
    for (Edge e : general) {
      gen_node(e >> 1);
      HIns h;
      h.op = FBG_OP_ACC;
      h.inv = (e & 1u) != 0;
      emit(h);
    }
  }
};

// Linear-scan allocation of virtual registers to the fewest physical ones.
int allocate_registers(std::vector<HIns> &code, int nv) {
  if (nv == 0) return 0;
  std::vector<long> last(nv, -1);
  for (long i = 0; i < (long)code.size(); i++) {
    const HIns &h = code[i];
    if ((h.op == FBG_OP_OPR || h.op == FBG_OP_LDR) && h.reg >= 0) last[h.reg] = i;
  }
  // drop stores that are never read
  std::vector<HIns> kept;
  std::vector<long> remap(code.size(), -1);
  for (long i = 0; i < (long)code.size(); i++) {
    if (code[i].op == FBG_OP_ST && last[code[i].reg] < 0) continue;
    remap[i] = (long)kept.size();
    kept.push_back(code[i]);
  }
  for (int r = 0; r < nv; r++)
    if (last[r] >= 0) last[r] = remap[last[r]];
  code.swap(kept);
  std::vector<int> phys(nv, -1);
  std::vector<int> free_list;
  int used = 0;
  for (long i = 0; i < (long)code.size(); i++) {
    HIns &h = code[i];
    if (h.op == FBG_OP_ST) {
      int p;
      if (!free_list.empty()) {
        std::sort(free_list.begin(), free_list.end(), std::greater<int>());
        p = free_list.back();
        free_list.pop_back();
      } else {
        p = used++;
      }
      phys[h.reg] = p;
      h.reg = p;
    } else if (h.op == FBG_OP_OPR || h.op == FBG_OP_LDR) {
      int v = h.reg;
      h.reg = phys[v];
      if (last[v] == i) free_list.push_back(phys[v]);
    }
  }
  return used;
}

struct CompileJob {
  const char *src;
  int n;        // variables of the text
  int n_free;   // variables of the program
  const int32_t *subst = nullptr;
  Compiled *out;
  std::string msg;
  int64_t off = -1;
  int status = FBG_OK;
};

void compile_job(CompileJob *job);

// Entry of the compile on its own stack: nothing may propagate out of it
// (an allocation failure becomes FBG_E_NOMEM).
void *compile_thread(void *arg) {
  CompileJob *job = (CompileJob *)arg;
  try {
    compile_job(job);
  } catch (const std::bad_alloc &) {
    job->status = FBG_E_NOMEM;
    job->msg = "out of host memory while compiling";
  } catch (...) {
    job->status = FBG_E_INVAL;
    job->msg = "internal error while compiling";
  }
  return nullptr;
}

void compile_job(CompileJob *job) {
  Graph g;
  Parser ps(job->src, job->n, g);
  ps.subst = job->subst;
  Edge root;
  if (!ps.program(root)) {
    job->status = ps.status;
    job->msg = ps.msg;
    job->off = ps.off;
    return;
  }
  Compiled &c = *job->out;
  c = Compiled();
  c.n = job->n_free;
  if (root == kFalse || root == kTrue) {
    c.const_value = root == kTrue ? 1 : 0;
    if (root == kFalse) {
      HIns h;
      h.op = FBG_OP_CL;  // acc &= (empty OR-set) = 0
      c.code.push_back(h);
      c.n_clause_instr = 1;
    }
    return;
  }
  Codegen cg(g);
  c.l2in = cg.analyse(root);
  cg.top(root, c.n_clause_instr);
  c.code.swap(cg.code);
  c.nregs = allocate_registers(c.code, cg.nvregs);
}

// Deeply nested text recurses in the parser and the code generator, so the
// work runs on a large stack of its own: 512 MiB of address space per
// calling thread, reserved on its first compile (pages are committed only as
// the recursion touches them) behind a guard page, entered with swapcontext
// in the caller's own thread.  A thread created per compile (the first
// design) cost about 0.1 ms and a long-lived worker thread about 0.03 ms per
// hand-over, most of a small compile.  Under AddressSanitizer, which does not
// follow stack switches, and if the reservation fails, a thread with such a
// stack runs the job instead.
constexpr size_t kCompileStack = (size_t)512 << 20;

struct CompileStack {
  void *base = nullptr;
  bool failed = false;
  ~CompileStack() {
    if (base) munmap(base, kCompileStack);
  }
};
thread_local CompileStack t_stack;
thread_local CompileJob *t_job = nullptr;

void compile_on_switched_stack() { compile_thread(t_job); }

bool run_on_big_stack(CompileJob *job) {
#if defined(__SANITIZE_ADDRESS__)
  (void)job;
  return false;
#else
  CompileStack &st = t_stack;
  if (!st.base && !st.failed) {
    void *p = mmap(nullptr, kCompileStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1,
                   0);
    if (p == MAP_FAILED || mprotect(p, 4096, PROT_NONE) != 0) {  // guard page at the low end
      if (p != MAP_FAILED) munmap(p, kCompileStack);
      st.failed = true;
    } else {
      st.base = p;
    }
  }
  if (!st.base) return false;
  ucontext_t caller, callee;
  if (getcontext(&callee) != 0) return false;
  callee.uc_stack.ss_sp = st.base;
  callee.uc_stack.ss_size = kCompileStack;
  callee.uc_link = &caller;
  makecontext(&callee, compile_on_switched_stack, 0);
  t_job = job;
  const bool ok = swapcontext(&caller, &callee) == 0;
  t_job = nullptr;
  return ok;
#endif
}

}  // namespace

int compile_formula(const char *src, int n, Compiled &out, std::string &msg, int64_t &offset,
                    const int32_t *subst, int n_free) {
  CompileJob job;
  job.src = src;
  job.n = n;
  job.n_free = subst ? n_free : n;
  job.out = &out;
  job.subst = subst;
  if (!run_on_big_stack(&job)) {
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, kCompileStack);
    pthread_t th;
    if (pthread_create(&th, &attr, compile_thread, &job) != 0) {
      compile_thread(&job);
    } else {
      pthread_join(th, nullptr);
    }
    pthread_attr_destroy(&attr);
  }
  msg = job.msg;
  offset = job.off;
  return job.status;
}

// ---------------------------------------------------------------- encoding

namespace {

struct SetWords {
  uint32_t flags = 0, pat = 0, mconst = 0;
  uint64_t lanemask = 0, sel = 0, neg = 0;
};

// bit i of kIndexBitMask64[j] = bit j of i
constexpr uint64_t kIndexBitMask64[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                                         0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

SetWords encode_set(const LitSet &ls, int log2w) {
  SetWords s;
  const int W = 1 << log2w;
  const int tile_bit = FBG_TILE_BASE_BIT + log2w;
  bool taut = false;
  for (const Lit &l : ls.lits) {
    uint32_t negmask = l.neg ? ~0u : 0u;
    if (l.k < FBG_SLICE_BITS) {
      uint32_t m = fbg_inword_mask(l.k) ^ negmask;
      if (ls.is_xor) s.mconst ^= m; else s.mconst |= m;
    } else if (l.k < FBG_TILE_BASE_BIT) {
      // the lanes whose index has bit k - 5 set (clear, for a negated literal)
      const uint64_t m = kIndexBitMask64[l.k - FBG_SLICE_BITS] ^ (l.neg ? ~0ull : 0ull);
      if (ls.is_xor) s.lanemask ^= m; else s.lanemask |= m;
    } else if (l.k < tile_bit) {
      // likewise the words of a lane, of W
      const uint32_t wmask = W == 32 ? ~0u : (1u << W) - 1u;
      const uint32_t m = ((uint32_t)kIndexBitMask64[l.k - FBG_TILE_BASE_BIT] ^ (l.neg ? ~0u : 0u)) & wmask;
      if (ls.is_xor) s.pat ^= m; else s.pat |= m;
    } else {
      uint64_t b = 1ull << (l.k - FBG_TILE_BASE_BIT);
      if (ls.is_xor) {
        s.sel ^= b;
        if (l.neg) s.mconst ^= ~0u;
      } else if (s.sel & b) {
        if (((s.neg & b) != 0) != l.neg) taut = true;
      } else {
        s.sel |= b;
        if (l.neg) s.neg |= b;
      }
    }
  }
  if (taut) s.mconst = ~0u;
  if (ls.is_xor) {
    s.flags |= FBG_XORSET;
    if (ls.inv) s.mconst ^= ~0u;
  } else if (ls.inv) {
    s.flags |= FBG_INV;
  }
  return s;
}

}  // namespace

namespace {
uint32_t table_f(uint32_t f, uint32_t a, uint32_t b) {
  return (f == FBG_F_AND ? (a & b) : f == FBG_F_OR ? (a | b) : (a ^ b)) & 0xFFu;
}
}  // namespace

namespace {

// Group of a clause at tiling log2w, from the words on which its word-index
// literals hold (pat): 0 (no word literal), 1 + 2j + v (one literal on word
// bit j, false on the words whose bit j is v), kMulti, or kAlwaysTrue.
constexpr int kMulti = -1, kAlwaysTrue = -2;

int group_of(uint32_t pat, int log2w) {
  const int W = 1 << log2w;
  const uint32_t full = W == 32 ? ~0u : ((1u << W) - 1u);
  pat &= full;
  if (pat == 0) return 0;
  if (pat == full) return kAlwaysTrue;
  for (int j = 0; j < log2w; j++) {
    const uint32_t ones = (uint32_t)kIndexBitMask64[j] & full;  // the words whose bit j is 1
    if (pat == ones) return 1 + 2 * j;             // x: false where bit j = 0
    if (pat == (full & ~ones)) return 1 + 2 * j + 1;  // ~x: false where bit j = 1
  }
  return kMulti;
}

struct BlockClause {
  SetWords s;
  int group;
  bool tile_only;  // only tile literals (or none at all)
  int top = 0;     // multi: highest word bit j of its word literals
  int top_v = 0;   // multi: the value of bit j on which that literal is false
};

int pattern_entry(std::vector<uint32_t> &pats, uint32_t pat) {
  size_t e = 0;
  while (e < pats.size() && pats[e] != pat) e++;
  if (e == pats.size()) pats.push_back(pat);
  return (int)e;
}

// One chunk of at most FBG_CB_CHUNK clauses; see fbg_isa.h for the layout.
// The clauses arrive sorted so that each key is a run of consecutive
// clauses: one group and in-word part (static), one level, half, pattern and
// in-word part (multi).  kind: 0 static, 1 the first multi chunk (its keys
// act inside the product tree), 2 a later multi chunk (after the tree).
void emit_chunk(const std::vector<BlockClause> &cl, size_t lo, size_t hi, int kind, int log2w,
                std::vector<uint32_t> &pats, std::vector<uint32_t> &out) {
  const uint32_t nc = (uint32_t)(hi - lo);
  const int W = 1 << log2w;
  const size_t base = out.size();
  out.resize(base + FBG_CB_CHUNK_HDR, 0u);
  out[base + 0] = nc;
  // lane bits: clause c holds on lane l through a lane literal; padding set
  const size_t lanes = out.size();
  out.resize(lanes + 64, nc == FBG_CB_CHUNK ? 0u : ~0u << nc);
  for (uint32_t c = 0; c < nc; c++)
    for (uint64_t m = cl[lo + c].s.lanemask; m; m &= m - 1) out[lanes + (size_t)__builtin_ctzll(m)] |= 1u << c;
  for (uint32_t c = 0; c < nc; c++) {
    const SetWords &s = cl[lo + c].s;
    out.push_back((uint32_t)s.sel);
    out.push_back((uint32_t)(s.sel >> 32));
    out.push_back((uint32_t)s.neg);
    out.push_back((uint32_t)(s.neg >> 32));
  }
  // runs of equal keys; a run [a, b) has its top bit b - 1 in T and the bits
  // below it in F
  auto same = [&](uint32_t a, uint32_t b) {
    const BlockClause &x = cl[lo + a], &y = cl[lo + b];
    if (x.s.mconst != y.s.mconst || x.tile_only != y.tile_only) return false;
    if (kind == 0) return x.group == y.group;
    return x.s.pat == y.s.pat && x.top == y.top && x.top_v == y.top_v;
  };
  // slot of a key: its group (static), its (level, half) (tree), or 0 (late)
  auto slot = [&](const BlockClause &x) {
    return kind == 0 ? x.group : kind == 1 ? 2 * (x.top - 1) + x.top_v : 0;
  };
  const int nslots = kind == 0 ? 1 + 2 * log2w : kind == 1 ? 2 * (log2w - 1) : 1;
  const uint32_t kw = kind == 0 ? 2u : 4u;  // words per key
  uint32_t T = 0, F = 0;
  std::vector<uint32_t> keys;
  std::vector<uint32_t> counts((size_t)std::max(nslots, 1), 0u);
  for (uint32_t a = 0; a < nc;) {
    uint32_t b = a + 1;
    while (b < nc && same(a, b)) b++;
    T |= 1u << (b - 1);
    for (uint32_t c = a; c + 1 < b; c++) F |= 1u << c;
    const BlockClause &x = cl[lo + a];
    keys.push_back(b - 1);
    keys.push_back(x.s.mconst);
    if (kind != 0) {
      uint32_t pat = x.s.pat;
      if (kind == 1) {
        // the node pattern of level top + 1 in the half top_v: node v < 2^top
        // stands for the words whose low top + 1 bits are v | top_v << top
        const uint32_t half = 1u << x.top;
        pat = ~0u;
        for (uint32_t v = 0; v < half; v++)
          if (!((x.s.pat >> (v | ((uint32_t)x.top_v << x.top))) & 1u)) pat &= ~(1u << v);
      }
      keys.push_back((uint32_t)(pattern_entry(pats, pat) * W));
      keys.push_back(0u);
    }
    counts[(size_t)slot(x)]++;
    a = b;
  }
  out.insert(out.end(), keys.begin(), keys.end());
  out[base + 2] = T;
  out[base + 3] = F;
  // end of each slot's keys, in bytes from the chunk start
  uint32_t end = (uint32_t)(FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4u;
  for (int sl = 0; sl < nslots; sl++) {
    end += counts[(size_t)sl] * kw * 4u;
    out[base + 5 + sl] = end;
  }
  while ((out.size() - base) % 4) out.push_back(0u);
  out[base + 1] = (uint32_t)(out.size() - base);
}

}  // namespace

namespace {

// registers below this one live in VGPRs in the jump-table form
constexpr uint32_t kJ16V = FBG_J16_VGPR_REGS;

#define FBG_LIST(x) x,
const uint32_t kJ16Reg[] = {FBG_J16_REG_TABLES(FBG_LIST)};
const uint32_t kJ16Np[] = {FBG_J16_NP_TABLES(FBG_LIST)};
const uint32_t kJ16Or[] = {FBG_J16_OR_TABLES(FBG_LIST)};
const uint32_t kJ16Xor[] = {FBG_J16_XOR_TABLES(FBG_LIST)};
const uint32_t kJ16Ora[] = {FBG_J16_ORA_TABLES(FBG_LIST)};
const uint32_t kJ16Lia[] = {FBG_J16_LIA_TABLES(FBG_LIST)};
#undef FBG_LIST

template <size_t N>
int table_index(const uint32_t (&list)[N], uint32_t tt) {
  for (size_t k = 0; k < N; k++)
    if (list[k] == tt) return (int)k;
  return -1;
}

// Words of a jump-table instruction of case cs: literal sets (chains
// included) take 8, register, ACC and NOT instructions 2.
uint32_t j16_words(uint32_t cs) {
  const bool lit = (cs >= FBG_J16_LIT_OR && cs < FBG_J16_ORS) || (cs >= FBG_J16_XYS_OR && cs < FBG_J16_ORA) ||
                   cs >= FBG_J16_LIA_OR;
  return lit ? FBG_INS_WORDS : FBG_J16_SHORT_WORDS;
}

// Rewrite the nins instructions at words[at..] into the jump-table form
// (fbg_isa.h) and close them with END; returns the length of that form in
// units of FBG_J16_UNIT words, END included (a NOT with INVOUT, which changes
// nothing, is dropped; runs of literal sets become chains).  *err is set
// when an instruction has no case (the code generator emits none such).
uint32_t to_jump_table(std::vector<uint32_t> &words, size_t at, uint32_t nins, std::string *err) {
  std::vector<std::array<uint32_t, FBG_INS_WORDS>> out;
  std::vector<uint32_t> pop;  // the plain opcode of each entry of out
  out.reserve(nins);
  pop.reserve(nins);
  auto missing = [&](const char *what, uint32_t tt) {
    if (err && err->empty()) *err = std::string("internal: no jump-table case for ") + what + " table " +
                                    std::to_string(tt);
  };
  for (uint32_t k = 0; k < nins; k++) {
    const uint32_t *g = &words[at + (size_t)k * FBG_INS_WORDS];
    std::array<uint32_t, FBG_INS_WORDS> w{};
    const uint32_t op = g[0] & 15u, tt = (g[0] >> FBG_F_SHIFT) & 0xFFu, arg = g[0] >> FBG_ARG_SHIFT;
    const uint32_t invout = (g[0] & FBG_INVOUT) ? 1u : 0u;
    uint32_t cs = 0;
    if (op == FBG_OP_LDL || op == FBG_OP_OPL) {
      const bool x = (g[0] & FBG_XORSET) != 0;
      int idx;
      if (!(g[0] & FBG_HASPAT)) {
        idx = table_index(kJ16Np, tt & 0x55u);
        cs = (x ? FBG_J16_LIT_XOR : FBG_J16_LIT_OR) + (uint32_t)idx;
      } else {
        idx = x ? table_index(kJ16Xor, tt) : table_index(kJ16Or, tt);
        cs = (x ? FBG_J16_LIT_XOR_P : FBG_J16_LIT_OR_P) + (uint32_t)idx;
        w[0] = (arg * 4u) << 16;  // the pattern words' byte offset
      }
      if (idx < 0) missing("literal", tt);
      for (int j = 1; j < FBG_INS_WORDS; j++) w[j] = g[j];
    } else if (op == FBG_OP_ST) {
      cs = (arg < kJ16V ? FBG_J16_ST_V : FBG_J16_ST_L) + invout;
      w[1] = arg < kJ16V ? arg * 16u : (arg - kJ16V) * 4096u;
    } else if (op == FBG_OP_OPR || op == FBG_OP_LDR) {
      const int idx = table_index(kJ16Reg, tt);
      if (idx < 0) missing("register", tt);
      cs = (arg < kJ16V ? FBG_J16_REG_V : FBG_J16_REG_L) + (uint32_t)idx;
      w[1] = arg < kJ16V ? arg * 16u : (arg - kJ16V) * 4096u;
    } else if (op == FBG_OP_ACC) {
      cs = FBG_J16_ACC + ((g[0] & FBG_INV) ? 1u : 0u) + 2u * invout;
    } else if (op == FBG_OP_NOT) {
      if (invout) continue;  // NOT then NOT
      cs = FBG_J16_NOT;
    } else {
      missing("opcode", op);
    }
    w[0] |= cs * FBG_J16_SLOT;
    out.push_back(w);
    pop.push_back(op);
  }
  // Runs of kMinChain or more literal sets without word literals become
  // chains: XYF, XYM ..., XYM, XYL (fbg_isa.h, Chains).
  constexpr size_t kMinChain = 2;
  auto case_of = [&](size_t k) { return (out[k][0] & 0xFFFFu) / FBG_J16_SLOT; };
  auto chainable = [&](size_t k) { return case_of(k) >= FBG_J16_LIT_OR && case_of(k) < FBG_J16_LIT_OR_P; };
  for (size_t k = 0; k < out.size();) {
    size_t e = k;
    while (e < out.size() && chainable(e)) e++;
    if (e - k >= kMinChain) {
      for (size_t j = k; j < e; j++) {
        const uint32_t cs = case_of(j);
        const bool x = cs >= FBG_J16_LIT_XOR;
        const uint32_t idx = cs - (x ? FBG_J16_LIT_XOR : FBG_J16_LIT_OR);
        const uint32_t first = x ? FBG_J16_XYF_XOR : FBG_J16_XYF_OR, further = x ? FBG_J16_XYM_XOR : FBG_J16_XYM_OR,
                       last = x ? FBG_J16_XYL_XOR : FBG_J16_XYL_OR;
        const uint32_t ncs = (j == k ? first : j + 1 == e ? last : further) + idx;
        out[j][0] = (out[j][0] & ~0xFFFFu) | ncs * FBG_J16_SLOT;
      }
    }
    k = e > k ? e : k + 1;
  }
  // A store into a VGPR register after which cur is dead (the next
  // instruction loads cur without reading it, or the program ends) merges
  // into the instruction before it when that one can write the register
  // itself: the last set of a chain (XYS), a literal set without word
  // literals (LIS) or an operation with that same register (ORS, both
  // operands then addressed with the register's index).
  auto st_v = [&](size_t k) {
    const uint32_t cs = case_of(k);
    return cs == FBG_J16_ST_V || cs == FBG_J16_ST_V + 1;
  };
  auto dead_after = [&](size_t k) {
    return k + 1 >= out.size() || pop[k + 1] == FBG_OP_LDL || pop[k + 1] == FBG_OP_LDR;
  };
  {
    std::vector<std::array<uint32_t, FBG_INS_WORDS>> merged;
    std::vector<uint32_t> mpop;
    merged.reserve(out.size());
    for (size_t k = 0; k < out.size(); k++) {
      const uint32_t cs = case_of(k);
      if (k + 1 < out.size() && st_v(k + 1) && dead_after(k + 1)) {
        if (cs >= FBG_J16_XYL_OR && cs < FBG_J16_XYL_OR + 24) {
          std::array<uint32_t, FBG_INS_WORDS> w = out[k];
          w[0] = ((out[k + 1][1] & 0xFFFFu) << 16) | (FBG_J16_XYS_OR + (cs - FBG_J16_XYL_OR)) * FBG_J16_SLOT;
          merged.push_back(w);
          mpop.push_back(FBG_OP_ST);
          k++;
          continue;
        }
        if (cs >= FBG_J16_LIT_OR && cs < FBG_J16_LIT_OR_P) {
          std::array<uint32_t, FBG_INS_WORDS> w = out[k];
          w[0] = ((out[k + 1][1] & 0xFFFFu) << 16) | (FBG_J16_LIS_OR + (cs - FBG_J16_LIT_OR)) * FBG_J16_SLOT;
          merged.push_back(w);
          mpop.push_back(FBG_OP_ST);
          k++;
          continue;
        }
        if (cs >= FBG_J16_REG_V && cs < FBG_J16_REG_L && out[k][1] == out[k + 1][1]) {
          std::array<uint32_t, FBG_INS_WORDS> w = out[k];
          w[0] = (FBG_J16_ORS + (cs - FBG_J16_REG_V)) * FBG_J16_SLOT;
          merged.push_back(w);
          mpop.push_back(FBG_OP_ST);
          k++;
          continue;
        }
      }
      merged.push_back(out[k]);
      mpop.push_back(pop[k]);
    }
    out.swap(merged);
    pop.swap(mpop);
  }
  // An ACC after which cur is dead merges into the operation before it: an
  // operation on a VGPR register (ORA) or a literal set without word literals
  // (LIA) then ANDs its result into acc directly (ACC's inversion folded into
  // the operation's table).
  {
    std::vector<std::array<uint32_t, FBG_INS_WORDS>> merged;
    std::vector<uint32_t> mpop;
    merged.reserve(out.size());
    for (size_t k = 0; k < out.size(); k++) {
      const uint32_t cs = case_of(k);
      if (k + 1 < out.size() && case_of(k + 1) >= FBG_J16_ACC && case_of(k + 1) < FBG_J16_ACC + 4 &&
          dead_after(k + 1)) {
        const bool inv = ((case_of(k + 1) - FBG_J16_ACC) & 1u) != 0;  // acc &= ~cur
        if (cs >= FBG_J16_REG_V && cs < FBG_J16_REG_L) {
          const uint32_t t = kJ16Reg[cs - FBG_J16_REG_V];
          const int idx = table_index(kJ16Reg, inv ? ~t & 0xFFu : t);
          std::array<uint32_t, FBG_INS_WORDS> w = out[k];
          w[0] = (FBG_J16_ORA + (uint32_t)idx) * FBG_J16_SLOT;
          merged.push_back(w);
          mpop.push_back(FBG_OP_ACC);
          k++;
          continue;
        }
        if (cs >= FBG_J16_LIT_OR && cs < FBG_J16_LIT_OR_P) {
          const bool x = cs >= FBG_J16_LIT_XOR;
          const uint32_t t = kJ16Np[cs - (x ? FBG_J16_LIT_XOR : FBG_J16_LIT_OR)];
          const int idx = table_index(kJ16Np, inv ? ~t & 0x55u : t);
          std::array<uint32_t, FBG_INS_WORDS> w = out[k];
          w[0] = ((x ? FBG_J16_LIA_XOR : FBG_J16_LIA_OR) + (uint32_t)idx) * FBG_J16_SLOT;
          merged.push_back(w);
          mpop.push_back(FBG_OP_ACC);
          k++;
          continue;
        }
      }
      merged.push_back(out[k]);
      mpop.push_back(pop[k]);
    }
    out.swap(merged);
    pop.swap(mpop);
  }
  // lay out: literal sets (and chain members) in full, the others short
  std::vector<uint32_t> flat;
  flat.reserve(out.size() * FBG_INS_WORDS + FBG_INS_WORDS);
  for (const auto &w : out) {
    const uint32_t len = j16_words((w[0] & 0xFFFFu) / FBG_J16_SLOT);
    flat.insert(flat.end(), w.begin(), w.begin() + len);
  }
  flat.resize(flat.size() + FBG_INS_WORDS, 0u);  // END, full length
  words.resize(at);
  words.insert(words.end(), flat.begin(), flat.end());
  return (uint32_t)(flat.size() / FBG_J16_UNIT);
}

}  // namespace

// One jump-table instruction back in the plain form (the same semantics: an
// LDL is an OPL whose table ignores cur; chain members keep their chain
// opcodes).  Returns the instruction's length in words, 0 for END.
static uint32_t from_jump_table(const uint32_t *w, uint32_t g[FBG_INS_WORDS]) {
  for (int j = 0; j < FBG_INS_WORDS; j++) g[j] = 0;
  const uint32_t cs = (w[0] & 0xFFFFu) / FBG_J16_SLOT;
  if (cs == FBG_J16_END || cs >= FBG_J16_NCASES) return 0;
  if (cs >= FBG_J16_ORA) {  // acc = tt(acc, cur, R[r] or T)
    if (cs < FBG_J16_LIA_OR) {
      g[0] = FBG_OP_ACM | FBG_HASPAT | (kJ16Ora[cs - FBG_J16_ORA] << FBG_F_SHIFT) | ((w[1] / 16u) << FBG_ARG_SHIFT);
      return FBG_J16_SHORT_WORDS;
    }
    const uint32_t k = cs - FBG_J16_LIA_OR;
    g[0] = FBG_OP_ACM | (k >= 12 ? FBG_XORSET : 0u) | (kJ16Lia[k % 12] << FBG_F_SHIFT);
    for (int j = 1; j < FBG_INS_WORDS; j++) g[j] = w[j];
    return FBG_INS_WORDS;
  }
  if (cs >= FBG_J16_XYS_OR) {  // a chain's last set, or a literal set, into R[r]
    const uint32_t k = (cs - FBG_J16_XYS_OR) % 24, op = cs >= FBG_J16_LIS_OR ? FBG_OP_LIS : FBG_OP_XYS;
    const uint32_t r = (w[0] >> 16) / 16u;
    g[0] = op | (k >= 12 ? FBG_XORSET : 0u) | (kJ16Np[k % 12] << FBG_F_SHIFT) | (r << FBG_ARG_SHIFT);
    for (int j = 1; j < FBG_INS_WORDS; j++) g[j] = w[j];
    return FBG_INS_WORDS;
  }
  if (cs >= FBG_J16_ORS) {  // R[r] = tt(cur, R[r])
    g[0] = FBG_OP_ORS | (kJ16Reg[cs - FBG_J16_ORS] << FBG_F_SHIFT) | ((w[1] / 16u) << FBG_ARG_SHIFT);
    return FBG_J16_SHORT_WORDS;
  }
  if (cs >= FBG_J16_XYF_OR) {
    const uint32_t k = cs - FBG_J16_XYF_OR;  // 12 cases per (first / further / last, OR / XOR)
    const uint32_t ops[3] = {FBG_OP_XYF, FBG_OP_XYM, FBG_OP_XYL};
    g[0] = ops[k / 24] | ((k / 12) % 2 ? FBG_XORSET : 0u) | (kJ16Np[k % 12] << FBG_F_SHIFT);
    for (int j = 1; j < FBG_INS_WORDS; j++) g[j] = w[j];
    return FBG_INS_WORDS;
  }
  if (cs >= FBG_J16_LIT_OR) {
    uint32_t tt, flags = 0, arg = 0;
    if (cs >= FBG_J16_LIT_XOR_P) {
      tt = kJ16Xor[cs - FBG_J16_LIT_XOR_P], flags = FBG_XORSET | FBG_HASPAT;
    } else if (cs >= FBG_J16_LIT_OR_P) {
      tt = kJ16Or[cs - FBG_J16_LIT_OR_P], flags = FBG_HASPAT;
    } else if (cs >= FBG_J16_LIT_XOR) {
      tt = kJ16Np[cs - FBG_J16_LIT_XOR], flags = FBG_XORSET;
    } else {
      tt = kJ16Np[cs - FBG_J16_LIT_OR];
    }
    if (flags & FBG_HASPAT) arg = (w[0] >> 16) / 4u;
    g[0] = FBG_OP_OPL | flags | (tt << FBG_F_SHIFT) | (arg << FBG_ARG_SHIFT);
    for (int j = 1; j < FBG_INS_WORDS; j++) g[j] = w[j];
    return FBG_INS_WORDS;
  }
  if (cs >= FBG_J16_REG_V) {
    const bool lds = cs >= FBG_J16_REG_L;
    const uint32_t tt = kJ16Reg[cs - (lds ? FBG_J16_REG_L : FBG_J16_REG_V)];
    const uint32_t r = lds ? kJ16V + w[1] / 4096u : w[1] / 16u;
    g[0] = FBG_OP_OPR | (tt << FBG_F_SHIFT) | (r << FBG_ARG_SHIFT);
  } else if (cs >= FBG_J16_ST_V) {
    const bool lds = cs >= FBG_J16_ST_L;
    const uint32_t r = lds ? kJ16V + w[1] / 4096u : w[1] / 16u;
    g[0] = FBG_OP_ST | (r << FBG_ARG_SHIFT) | ((cs - (lds ? FBG_J16_ST_L : FBG_J16_ST_V)) ? FBG_INVOUT : 0u);
  } else if (cs >= FBG_J16_ACC) {
    const uint32_t v = cs - FBG_J16_ACC;
    g[0] = FBG_OP_ACC | ((v & 1u) ? FBG_INV : 0u) | ((v & 2u) ? FBG_INVOUT : 0u);
  } else {
    g[0] = FBG_OP_NOT;
  }
  return FBG_J16_SHORT_WORDS;
}

uint32_t encode_program(const Compiled &c, int log2w, std::vector<uint32_t> &words, std::string *err) {
  const size_t base = words.size();
  const int W = 1 << log2w;
  const int tile_bit = FBG_TILE_BASE_BIT + log2w;
  std::vector<uint32_t> pats{0u};  // pattern table, entry 0 = no per-word literal
  size_t ncl = 0;
  while (ncl < c.code.size() && c.code[ncl].op == FBG_OP_CL) ncl++;

  // ---- the clause block
  std::vector<BlockClause> stat, multi;
  std::set<std::array<uint64_t, 4>> seen;
  for (size_t k = 0; k < ncl; k++) {
    BlockClause b;
    b.s = encode_set(c.code[k].ls, log2w);
    if (b.s.mconst == ~0u) continue;  // a tautology
    b.group = group_of(b.s.pat, log2w);
    if (b.group == kAlwaysTrue) continue;
    // the same clause twice (the same literals in another order) once
    const std::array<uint64_t, 4> id{(uint64_t)b.s.mconst << 32 | b.s.pat, b.s.lanemask, b.s.sel, b.s.neg};
    if (!seen.insert(id).second) continue;
    b.tile_only = true;
    b.top = -1;
    for (const Lit &l : c.code[k].ls.lits) {
      b.tile_only = b.tile_only && l.k >= tile_bit;
      const int j = l.k - FBG_TILE_BASE_BIT;
      if (j >= 0 && j < log2w && j > b.top) {
        b.top = j;
        b.top_v = l.neg ? 1 : 0;  // x is false where the bit is 0, ~x where it is 1
      }
    }
    (b.group == kMulti ? multi : stat).push_back(b);
  }
  // clauses made only of tile literals first (their keys stay apart from the
  // others'; the uniform-cofactor table at the end of the block lists them
  // again), then by group and in-word part so that equal keys share a chunk
  std::stable_sort(stat.begin(), stat.end(), [](const BlockClause &a, const BlockClause &b) {
    if (a.tile_only != b.tile_only) return a.tile_only;
    if (a.group != b.group) return a.group < b.group;
    return a.s.mconst < b.s.mconst;
  });
  // multi clauses by (level, half) so that the first chunk's keys come in
  // the order the product tree meets them, then by pattern and in-word part
  std::stable_sort(multi.begin(), multi.end(), [](const BlockClause &a, const BlockClause &b) {
    if (a.top != b.top) return a.top < b.top;
    if (a.top_v != b.top_v) return a.top_v < b.top_v;
    if (a.s.pat != b.s.pat) return a.s.pat < b.s.pat;
    return a.s.mconst < b.s.mconst;
  });
  std::vector<uint32_t> block(FBG_CB_HDR, 0u);
  uint32_t nstat = 0, nmulti = 0;
  for (size_t lo = 0; lo < stat.size(); lo += FBG_CB_CHUNK, nstat++)
    emit_chunk(stat, lo, std::min(stat.size(), lo + FBG_CB_CHUNK), 0, log2w, pats, block);
  for (size_t lo = 0; lo < multi.size(); lo += FBG_CB_CHUNK, nmulti++)
    emit_chunk(multi, lo, std::min(multi.size(), lo + FBG_CB_CHUNK), lo == 0 ? 1 : 2, log2w, pats, block);
  // the uniform-cofactor table: the tile selectors of every clause made only
  // of tile literals, at the end of the block; its length in the first
  // static chunk's h[4] (such clauses are static, so that chunk exists)
  uint32_t ncof = 0;
  for (const BlockClause &b : stat) {
    if (!b.tile_only) continue;
    block.push_back((uint32_t)b.s.sel);
    block.push_back((uint32_t)(b.s.sel >> 32));
    block.push_back((uint32_t)b.s.neg);
    block.push_back((uint32_t)(b.s.neg >> 32));
    ncof++;
  }
  if (nstat > 0) block[FBG_CB_HDR + 4] = ncof;
  block[0] = (uint32_t)block.size();
  block[1] = nstat;
  block[2] = nmulti;
  block[3] = (uint32_t)(stat.size() + multi.size());
  words.insert(words.end(), block.begin(), block.end());

  // ---- the instructions after the clauses (the kernels run no CL there: a
  // clause after other instructions becomes LDL + ACC; the code generator
  // emits none)
  std::vector<HIns> gen;
  for (size_t idx = ncl; idx < c.code.size(); idx++) {
    if (c.code[idx].op == FBG_OP_CL) {
      HIns l = c.code[idx];
      l.op = FBG_OP_LDL;
      gen.push_back(l);
      HIns a;
      a.op = FBG_OP_ACC;
      gen.push_back(a);
    } else {
      gen.push_back(c.code[idx]);
    }
  }
  const size_t ins_base = words.size();
  for (const HIns &h : gen) {
    uint32_t w[FBG_INS_WORDS] = {0, 0, 0, 0, 0, 0, 0, 0};
    w[0] = h.op;
    if (h.op == FBG_OP_CL || h.op == FBG_OP_LDL || h.op == FBG_OP_OPL) {
      SetWords s = encode_set(h.ls, log2w);
      if (h.op == FBG_OP_CL) s.flags &= ~(uint32_t)(FBG_XORSET | FBG_INV);
      // at most 3^5 = 243 entries of at most 32 words: the offset fits 16 bits
      const int e = pattern_entry(pats, s.pat);
      w[0] |= s.flags | ((uint32_t)(e * W) << FBG_ARG_SHIFT) | (e != 0 ? FBG_HASPAT : 0u);
      w[1] = s.mconst;
      w[2] = (uint32_t)s.lanemask;
      w[3] = (uint32_t)(s.lanemask >> 32);
      w[4] = (uint32_t)s.sel;
      w[5] = (uint32_t)(s.sel >> 32);
      w[6] = (uint32_t)s.neg;
      w[7] = (uint32_t)(s.neg >> 32);
    } else {
      if (h.inv) w[0] |= FBG_INV;
      if (h.reg >= 0) w[0] |= (uint32_t)h.reg << FBG_ARG_SHIFT;
    }
    // Operations on cur: the v_bitop3 truth table over (cur = 0xF0, T or the
    // register = 0xCC, P(i) = 0xAA) with the inversions folded in.
    if (h.op == FBG_OP_LDL || h.op == FBG_OP_OPL) {
      uint32_t L = (w[0] & FBG_XORSET) ? (0xCCu ^ 0xAAu) : (0xCCu | 0xAAu);  // XOR-set inversion is in mconst
      if (w[0] & FBG_INV) L = ~L & 0xFFu;
      w[0] &= ~(uint32_t)FBG_INV;
      uint32_t t = h.op == FBG_OP_LDL ? L : table_f(h.f, 0xF0u, L);
      if (h.invout) t = ~t & 0xFFu;
      w[0] |= t << FBG_F_SHIFT;
    } else if (h.op == FBG_OP_OPR || h.op == FBG_OP_LDR) {
      const uint32_t R = h.inv ? 0x33u : 0xCCu;
      uint32_t t = h.op == FBG_OP_LDR ? R : table_f(h.f, 0xF0u, R);
      if (h.invout) t = ~t & 0xFFu;
      w[0] = (w[0] & ~(uint32_t)FBG_INV) | (t << FBG_F_SHIFT);
    } else if (h.invout) {
      w[0] |= FBG_INVOUT;  // ST, ACC, NOT: cur inverted afterwards
    }
    words.insert(words.end(), w, w + FBG_INS_WORDS);
  }
  uint32_t nins = (uint32_t)((words.size() - ins_base) / FBG_INS_WORDS);
  if (log2w == FBG_J16_LOG2W) nins = to_jump_table(words, ins_base, nins, err);
  for (uint32_t pat : pats)
    for (int i = 0; i < W; i++) words.push_back(((pat >> i) & 1u) ? ~0u : 0u);
  while ((words.size() - base) % 4) words.push_back(0u);
  return nins;
}

// VALU instructions per tile of the general part in the jump-table form, and
// its instructions (dispatches), W words per lane.
static void j16_general_work(const uint32_t *ins, uint32_t nins, uint32_t W, double &valu, uint32_t &dispatches) {
  double per_tile = 0;
  uint32_t n = 0;
  const size_t end = (size_t)nins * FBG_J16_UNIT;
  for (size_t at = 0; at < end;) {
    const uint32_t cs = (ins[at] & 0xFFFFu) / FBG_J16_SLOT;
    if (cs == FBG_J16_END || cs >= FBG_J16_NCASES) break;
    at += j16_words(cs);
    n++;
    if (cs >= FBG_J16_LIA_OR) {
      per_tile += 2 + W;  // the lane value, one v_bitop3 per word into acc
    } else if (cs >= FBG_J16_ORA) {
      per_tile += W;  // one v_bitop3 per word into acc
    } else if (cs >= FBG_J16_LIS_OR) {
      per_tile += 1 + W;  // the lane part, one v_bitop3 per word into the register
    } else if (cs >= FBG_J16_XYS_OR) {
      per_tile += 3 + W;  // the lane part, X and Y, then one v_bitop3 per word
    } else if (cs >= FBG_J16_ORS) {
      per_tile += W;  // one v_bitop3 per word into the register
    } else if (cs >= FBG_J16_XYL_OR) {
      per_tile += 3 + W;  // the lane part, X and Y, then one v_bitop3 per word
    } else if (cs >= FBG_J16_XYF_OR) {
      per_tile += 3;  // the lane part, then X and Y
    } else if (cs >= FBG_J16_LIT_OR_P) {
      per_tile += 2 + W;  // the lane value, one v_bitop3 per word
    } else if (cs >= FBG_J16_LIT_OR) {
      per_tile += 1 + W;  // the lane part, one v_bitop3 per word
    } else if (cs >= FBG_J16_REG_V) {
      per_tile += W + (cs >= FBG_J16_REG_L ? 1 : 0);
    } else if (cs >= FBG_J16_ST_V) {
      const bool lds = cs >= FBG_J16_ST_L;
      per_tile += (lds ? 1 : W) + ((cs - (lds ? FBG_J16_ST_L : FBG_J16_ST_V)) ? W : 0);
    } else if (cs >= FBG_J16_ACC) {
      per_tile += W + ((cs - FBG_J16_ACC) >= 2 ? W : 0);
    } else if (cs == FBG_J16_NOT) {
      per_tile += W;
    }
  }
  valu = per_tile;
  dispatches = n;
}

double valu_per_slice(const std::vector<uint32_t> &words, uint32_t nins, int log2w, uint32_t nregs) {
  // The per-tile VALU instructions of the kernels, instruction by
  // instruction of the encoding (run_clauses and run_general in
  // fbg_device.h, the cases of fbg_asm16.h).
  const uint32_t W = 1u << log2w;
  if (words.empty()) return 0.0;
  const uint32_t *cb = words.data();
  double per_tile = 0;
  const uint32_t *ch = cb + FBG_CB_HDR;
  const uint32_t nchunks = cb[1] + cb[2];
  // a chunk: the tile compare of its clauses (64-bit and, compare), U and the
  // segmented add of its runs (about 6), then per key a bit extract and a
  // v_bitop3; first multi chunk keys act on 2^j tree nodes, later ones on W
  for (uint32_t k = 0; k < nchunks; k++) {
    const int kind = k < cb[1] ? 0 : k == cb[1] ? 1 : 2;
    const uint32_t nc = ch[0];
    per_tile += 8;
    uint32_t off = (uint32_t)(FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4u;
    const int nslots = kind == 0 ? 1 + 2 * log2w : kind == 1 ? 2 * (log2w - 1) : 1;
    for (int sl = 0; sl < nslots; sl++)
      for (; off < ch[5 + sl]; off += kind == 0 ? 8u : 16u) {
        per_tile += 2;
        if (kind == 1) per_tile += (double)(1u << (1 + sl / 2));
        if (kind == 2) per_tile += W;
      }
    ch += ch[1];
  }
  if (nchunks) per_tile += 2.0 * W - 2.0;  // the product tree
  const uint32_t *ins = cb + cb[0];
  if (log2w == FBG_J16_LOG2W) {
    // jump-table form: per instruction its case's VALU work
    double valu;
    uint32_t dispatches;
    j16_general_work(ins, nins, W, valu, dispatches);
    per_tile += valu;
    (void)nregs;
    return per_tile / W;
  }
  for (uint32_t pc = 0; pc < nins; pc++) {
    const uint32_t w0 = ins[(size_t)pc * FBG_INS_WORDS];
    const uint32_t op = w0 & 15u;
    const uint32_t r = w0 >> FBG_ARG_SHIFT;
    if (op == FBG_OP_CL || op == FBG_OP_LDL || op == FBG_OP_OPL) {
      per_tile += 1 + W;  // the lane value of the set, one v_bitop3 per word
    } else if (op == FBG_OP_ST) {
      per_tile += r < 4 ? W : 0;  // a VGPR copy; LDS registers are ds_write
    } else {
      per_tile += W;  // OPR / LDR / ACC / NOT
    }
    if ((op == FBG_OP_ST || op == FBG_OP_ACC || op == FBG_OP_NOT) && (w0 & FBG_INVOUT)) per_tile += W;
  }
  (void)nregs;
  return per_tile / W;
}

double j16_general_cost(const std::vector<uint32_t> &words, uint32_t nins) {
  if (words.empty()) return 0.0;
  double valu;
  uint32_t dispatches;
  j16_general_work(words.data() + words[0], nins, 1u << FBG_J16_LOG2W, valu, dispatches);
  return valu / (1u << FBG_J16_LOG2W) + 0.5 * dispatches;
}

Compiled permute_variables(const Compiled &c, const std::vector<int> &to) {
  Compiled r = c;
  for (HIns &h : r.code)
    for (Lit &l : h.ls.lits) l.k = to[(size_t)l.k];
  return r;
}

std::vector<int> xcd_write_out_permutation(int n) {
  // Word-index bits of the kernel's (tile t, word i, lane l), as
  // (t << 11) | (i << 6) | l, and the bits of the DNF word they address:
  //   l0..l5 -> 2..7    i0, i1 -> 0, 1    i2, i3 -> 8, 9    i4 -> 13
  //   t0, t1 -> 14, 15  t2..t4 -> 10..12  t5.. -> 16..
  // Variable 5 + b of the formula (DNF word bit b) becomes variable 5 + k
  // of the program, k the kernel bit that lands on b.
  static const int kernel_bit_of[16] = {6, 7, 0, 1, 2, 3, 4, 5, 8, 9, 13, 14, 15, 10, 11, 12};
  std::vector<int> to((size_t)n);
  for (int k = 0; k < n; k++) to[(size_t)k] = k;
  for (int b = 0; b < 16 && 5 + b < n; b++) to[(size_t)(5 + b)] = 5 + kernel_bit_of[b];
  return to;
}

uint32_t leading_clauses(const Compiled &c) {
  // the code generator emits every clause before any other instruction
  uint32_t k = 0;
  while (k < c.code.size() && c.code[k].op == FBG_OP_CL) k++;
  return k;
}

std::string disasm_program(const std::vector<uint32_t> &words, uint32_t nins, int log2w) {
  static const char *ops[] = {"?",   "CL",  "LDL", "OPL", "ST",  "OPR", "ACC", "LDR",
                              "NOT", "XYF", "XYM", "XYL", "XYS", "ORS", "LIS", "ACM"};
  const int W = 1 << log2w;
  const uint32_t *cb = words.data();
  const uint32_t *ins = cb + cb[0];
  const uint32_t *table = ins + FBG_TABLE_OFFSET(nins, log2w);
  char buf[256];
  std::string out = "; words per lane " + std::to_string(W) + "\n";
  snprintf(buf, sizeof buf, "; clause block: %u clauses, %u static chunks, %u multi chunks\n", cb[3], cb[1], cb[2]);
  out += buf;
  const uint32_t *ch = cb + FBG_CB_HDR;
  for (uint32_t k = 0; k < cb[1] + cb[2]; k++) {
    const int kind = k < cb[1] ? 0 : k == cb[1] ? 1 : 2;
    static const char *kinds[] = {"static", "multi-tree", "multi"};
    const uint32_t nc = ch[0];
    snprintf(buf, sizeof buf, "chunk %u %s clauses=%u cofactor=%u tops=%08x fill=%08x\n", k, kinds[kind], nc,
             k == 0 && kind == 0 ? ch[4] : 0u, ch[2], ch[3]);
    out += buf;
    const uint32_t *td = ch + FBG_CB_CHUNK_HDR + 64;
    for (uint32_t c = 0; c < nc; c++) {
      uint64_t lm = 0;
      for (int lane = 0; lane < 64; lane++)
        if ((ch[FBG_CB_CHUNK_HDR + lane] >> c) & 1u) lm |= 1ull << lane;
      snprintf(buf, sizeof buf, "  clause %u lane=%016llx sel=%08x%08x neg=%08x%08x\n", c, (unsigned long long)lm,
               td[4 * c + 1], td[4 * c], td[4 * c + 3], td[4 * c + 2]);
      out += buf;
    }
    uint32_t off = (uint32_t)(FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4u;
    const int nslots = kind == 0 ? 1 + 2 * log2w : kind == 1 ? 2 * (log2w - 1) : 1;
    for (int sl = 0; sl < nslots; sl++) {
      for (; off < ch[5 + sl]; off += kind == 0 ? 8u : 16u) {
        const uint32_t *key = ch + off / 4;
        if (kind == 0) {
          snprintf(buf, sizeof buf, "  key group=%d top=%u mconst=%08x\n", sl, key[0], key[1]);
        } else {
          const int j = kind == 1 ? 1 + sl / 2 : log2w;
          const int n = kind == 1 ? 1 << j : W;
          uint32_t pat = 0;
          for (int v = 0; v < n; v++)
            if (table[key[2] + v]) pat |= 1u << v;
          if (kind == 1)
            snprintf(buf, sizeof buf, "  key multi level=%d half=%d top=%u mconst=%08x nodes=%08x\n", j, sl % 2,
                     key[0], key[1], pat);
          else
            snprintf(buf, sizeof buf, "  key multi top=%u mconst=%08x pat=%08x\n", key[0], key[1], pat);
        }
        out += buf;
      }
    }
    ch += ch[1];
  }
  if (log2w == FBG_J16_LOG2W) out += "; jump-table form (listed in the plain form's terms)\n";
  const bool j16 = log2w == FBG_J16_LOG2W;
  const size_t end = (size_t)nins * (j16 ? FBG_J16_UNIT : FBG_INS_WORDS);
  size_t pc = 0;
  for (size_t at = 0; at < end; pc++) {
    uint32_t gw[FBG_INS_WORDS];
    const uint32_t *w = &ins[at];
    if (j16) {
      const uint32_t len = from_jump_table(w, gw);
      if (!len) break;
      at += len;
      w = gw;
    } else {
      at += FBG_INS_WORDS;
    }
    uint32_t op = w[0] & 15u;
    uint32_t arg = w[0] >> FBG_ARG_SHIFT;
    const char *name = ops[op];
    if (op == FBG_OP_ACM && (w[0] & FBG_HASPAT)) {
      snprintf(buf, sizeof buf, "%4zu %-3s tt=%02x r%u\n", pc, name, (w[0] >> FBG_F_SHIFT) & 0xFFu, arg);
    } else if (op == FBG_OP_ACM) {
      snprintf(buf, sizeof buf, "%4zu %-3s tt=%02x set=%s mconst=%08x lane=%08x%08x sel=%08x%08x neg=%08x%08x\n", pc,
               name, (w[0] >> FBG_F_SHIFT) & 0xFFu, (w[0] & FBG_XORSET) ? "xor" : "or", w[1], w[3], w[2], w[5], w[4],
               w[7], w[6]);
    } else if (op == FBG_OP_XYS || op == FBG_OP_LIS) {
      snprintf(buf, sizeof buf,
               "%4zu %-3s tt=%02x set=%s mconst=%08x lane=%08x%08x sel=%08x%08x neg=%08x%08x into r%u\n", pc, name,
               (w[0] >> FBG_F_SHIFT) & 0xFFu, (w[0] & FBG_XORSET) ? "xor" : "or", w[1], w[3], w[2], w[5], w[4], w[7],
               w[6], arg);
    } else if (op == FBG_OP_CL || op == FBG_OP_LDL || op == FBG_OP_OPL || op == FBG_OP_XYF || op == FBG_OP_XYM ||
        op == FBG_OP_XYL) {
      uint32_t pat = 0;
      for (int i = 0; i < W; i++)
        if (table[arg + i]) pat |= 1u << i;
      char tt[16] = "";
      if (op != FBG_OP_CL) snprintf(tt, sizeof tt, "tt=%02x ", (w[0] >> FBG_F_SHIFT) & 0xFFu);
      snprintf(buf, sizeof buf,
               "%4zu %-3s %sset=%s mconst=%08x lane=%08x%08x pat=%08x sel=%08x%08x neg=%08x%08x\n",
               pc, name, tt, (w[0] & FBG_XORSET) ? "xor" : "or", w[1], w[3], w[2], pat, w[5],
               w[4], w[7], w[6]);
    } else if (op == FBG_OP_OPR || op == FBG_OP_LDR || op == FBG_OP_ORS) {
      snprintf(buf, sizeof buf, "%4zu %-3s tt=%02x r%u\n", pc, name, (w[0] >> FBG_F_SHIFT) & 0xFFu, arg);
    } else {
      snprintf(buf, sizeof buf, "%4zu %-3s r%u%s%s\n", pc, name, arg, (w[0] & FBG_INV) ? " inv" : "",
               (w[0] & FBG_INVOUT) ? " invout" : "");
    }
    out += buf;
  }
  return out;
}

// ---------------------------------------------------------------- emulator

namespace {

// The lane value T of a literal set at (lane, tile group U0), formed the way
// the kernels form it: every literal but the per-word ones.
inline uint32_t set_lane_value(const uint32_t *w, uint32_t lane, uint64_t U0) {
  uint64_t lanemask = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
  uint64_t sel = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
  uint64_t neg = (uint64_t)w[6] | ((uint64_t)w[7] << 32);
  uint32_t V = ((lanemask >> lane) & 1u) ? ~0u : 0u;
  if (w[0] & FBG_XORSET) return V ^ w[1] ^ ((__builtin_popcountll(U0 & sel) & 1) ? ~0u : 0u);
  return (V || ((U0 ^ neg) & sel)) ? ~0u : w[1];
}

// v_bitop3: bit m of tt is the result for inputs (a, b, c) = bits of m.
inline uint32_t bitop3(uint32_t tt, uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r = 0;
  for (uint32_t m = 0; m < 8; m++)
    if ((tt >> m) & 1u) r |= ((m & 4u) ? a : ~a) & ((m & 2u) ? b : ~b) & ((m & 1u) ? c : ~c);
  return r;
}

// The clause block at (lane, word i, tile group U0), read the way the kernels
// read it; the product tree is written here as its closed form.  With cof,
// a false clause made only of tile literals ends the tile, as in the
// uniform-cofactor kernels.
uint32_t clause_block_value(const uint32_t *cb, const uint32_t *table, int log2w, uint32_t lane, uint32_t i,
                            uint64_t U0, bool cof) {
  uint32_t G[1 + 2 * 5];
  for (uint32_t &g : G) g = ~0u;
  const uint32_t *ch = cb + FBG_CB_HDR;
  if (cof && cb[1] > 0) {  // the uniform-cofactor table at the end of the block
    const uint32_t ncof = ch[4];
    const uint32_t *td = cb + cb[0] - 4 * ncof;
    for (uint32_t c = 0; c < ncof; c++) {
      const uint64_t sel = (uint64_t)td[4 * c] | ((uint64_t)td[4 * c + 1] << 32);
      const uint64_t neg = (uint64_t)td[4 * c + 2] | ((uint64_t)td[4 * c + 3] << 32);
      if ((U0 & sel) == neg) return 0u;
    }
  }
  uint32_t extra = ~0u;  // the multi keys' factors of word i
  for (uint32_t k = 0; k < cb[1] + cb[2]; k++) {
    const int kind = k < cb[1] ? 0 : k == cb[1] ? 1 : 2;
    const uint32_t nc = ch[0];
    const uint32_t *td = ch + FBG_CB_CHUNK_HDR + 64;
    uint32_t S = 0;
    for (uint32_t c = 0; c < nc; c++) {
      const uint64_t sel = (uint64_t)td[4 * c] | ((uint64_t)td[4 * c + 1] << 32);
      const uint64_t neg = (uint64_t)td[4 * c + 2] | ((uint64_t)td[4 * c + 3] << 32);
      if ((U0 & sel) != neg) S |= 1u << c;
    }
    const uint32_t U = ~(ch[FBG_CB_CHUNK_HDR + lane] | S);
    // the clauses of a key are the run of bits ending at its top bit, after
    // the previous key's top bit
    auto run_false = [&](uint32_t top) {
      uint32_t lo = top;
      while (lo > 0 && !((ch[2] >> (lo - 1)) & 1u)) lo--;
      const uint32_t run = (uint32_t)(((2ull << top) - 1) & ~((1ull << lo) - 1));
      return (U & run) != 0;
    };
    uint32_t off = (uint32_t)(FBG_CB_CHUNK_HDR + 64 + 4 * nc) * 4u;  // bytes
    const int nslots = kind == 0 ? 1 + 2 * log2w : kind == 1 ? 2 * (log2w - 1) : 1;
    for (int sl = 0; sl < nslots; sl++) {
      for (; off < ch[5 + sl]; off += kind == 0 ? 8u : 16u) {
        const uint32_t *key = ch + off / 4;
        if (!run_false(key[0])) continue;
        if (kind == 0) {
          G[sl] &= key[1];
        } else if (kind == 1) {
          const int j = 1 + sl / 2;  // level j + 1, half bit j = sl % 2
          if (((i >> j) & 1u) == (uint32_t)(sl % 2)) extra &= key[1] | table[key[2] + (i & ((1u << j) - 1u))];
        } else {
          extra &= key[1] | table[key[2] + i];
        }
      }
    }
    ch += ch[1];
  }
  uint32_t acc = G[0] & extra;
  for (int j = 0; j < log2w; j++) acc &= G[1 + 2 * j + ((i >> j) & 1u)];
  return acc;
}

}  // namespace

void emulate_program(const std::vector<uint32_t> &words, uint32_t nins, int nregs, int n, int log2w, bool cof,
                     uint32_t *out32) {
  const uint64_t slices = n >= FBG_SLICE_BITS ? (1ull << (n - FBG_SLICE_BITS)) : 1ull;
  const uint64_t W = 1ull << log2w;
  std::vector<uint32_t> R((size_t)nregs + 1, 0);
  const uint32_t *cb = words.data();
  const uint32_t *ins = cb + cb[0];
  const uint32_t *table = ins + FBG_TABLE_OFFSET(nins, log2w);
  // the jump-table form, read back into the plain form once
  std::vector<uint32_t> plain;
  if (log2w == FBG_J16_LOG2W) {
    uint32_t g[FBG_INS_WORDS];
    const size_t end = (size_t)nins * FBG_J16_UNIT;
    for (size_t at = 0; at < end;) {
      const uint32_t len = from_jump_table(&ins[at], g);
      if (!len) break;
      at += len;
      plain.insert(plain.end(), g, g + FBG_INS_WORDS);
    }
    ins = plain.data();
    nins = (uint32_t)(plain.size() / FBG_INS_WORDS);
  }
  for (uint64_t s = 0; s < slices; s++) {
    uint32_t lane = (uint32_t)(s & 63u);
    uint64_t U = s >> FBG_LANE_BITS;
    uint32_t i = (uint32_t)(U & (W - 1));
    uint64_t U0 = U - i;
    uint32_t acc = clause_block_value(cb, table, log2w, lane, i, U0, cof), cur = 0, X = 0, Y = 0;
    for (size_t pc = 0; pc < nins; pc++) {
      const uint32_t *w = &ins[pc * FBG_INS_WORDS];
      uint32_t op = w[0] & 15u;
      uint32_t tt = (w[0] >> FBG_F_SHIFT) & 0xFFu;
      uint32_t arg = w[0] >> FBG_ARG_SHIFT;
      uint32_t inv = (w[0] & FBG_INV) ? ~0u : 0u;
      switch (op) {
        case FBG_OP_CL: acc &= set_lane_value(w, lane, U0) | table[arg + i]; break;
        case FBG_OP_LDL:
        case FBG_OP_OPL: cur = bitop3(tt, cur, set_lane_value(w, lane, U0), table[arg + i]); break;
        case FBG_OP_ST: R[arg] = cur; break;
        case FBG_OP_OPR:
        case FBG_OP_LDR: cur = bitop3(tt, cur, R[arg], 0u); break;
        case FBG_OP_ACC: acc &= cur ^ inv; break;
        case FBG_OP_NOT: cur = ~cur; break;
        case FBG_OP_XYF:
          X = bitop3(tt, ~0u, set_lane_value(w, lane, U0), 0u);
          Y = bitop3(tt, 0u, set_lane_value(w, lane, U0), 0u);
          break;
        case FBG_OP_XYM:
          X = bitop3(tt, X, set_lane_value(w, lane, U0), 0u);
          Y = bitop3(tt, Y, set_lane_value(w, lane, U0), 0u);
          break;
        case FBG_OP_XYL:
          X = bitop3(tt, X, set_lane_value(w, lane, U0), 0u);
          Y = bitop3(tt, Y, set_lane_value(w, lane, U0), 0u);
          cur = (cur & X) | (~cur & Y);
          break;
        case FBG_OP_XYS:  // cur keeps its value
          X = bitop3(tt, X, set_lane_value(w, lane, U0), 0u);
          Y = bitop3(tt, Y, set_lane_value(w, lane, U0), 0u);
          R[arg] = (cur & X) | (~cur & Y);
          break;
        case FBG_OP_ORS: R[arg] = bitop3(tt, cur, R[arg], 0u); break;  // cur keeps its value
        case FBG_OP_LIS: R[arg] = bitop3(tt, cur, set_lane_value(w, lane, U0), 0u); break;  // cur too
        case FBG_OP_ACM:  // cur keeps its value
          acc = bitop3(tt, acc, cur, (w[0] & FBG_HASPAT) ? R[arg] : set_lane_value(w, lane, U0));
          break;
      }
      if (w[0] & FBG_INVOUT) cur = ~cur;
    }
    if (n < FBG_SLICE_BITS) acc &= (uint32_t)((1ull << (1u << n)) - 1u);
    out32[s] = acc;
  }
  if (n < 6) {
    // the DNF has one 64-bit word: clear the upper slice if it is not valid
    if (slices < 2) out32[1] = 0;
  }
}

}  // namespace fbg
