// oracle.cc -- reference implementation of certified-split lexing.
//
// TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, serial, deliberately
// unoptimised code whose every step can be checked against the paper by eye.
// It shares nothing with the HIP library: its own regex parser, its own NFA
// construction and simulation, its own automaton construction and its own
// certificate checker.
//
// Paper map
//   Section 3 (Preliminaries)      -> longest_match(), lex_serial()
//   Section 4, Definitions 1-2     -> analyse(): reentrant, exact map
//   Section 4, Corollary 2         -> analyse(): useful = certified AND q0-live
//   Section 4.1 (trim to Q+)       -> trim_and_minimise()
//   Section 4.1 (minimisation that keeps a missing transition apart from a
//                dead one)         -> trim_and_minimise(), Moore refinement
//   Section 5, Definition 3        -> analyse(): discard map via T(q) subset I
//   Section 6.1 (reverse closure
//                seeded by kept accepting states) -> analyse()
//   Theorem 2 (witness w = u b v)  -> orc_witness()
//   Theorems 1, 3, Corollary 1     -> lex_chunked()
//   Section 6.1 (exhaustive sweep) -> orc_bruteforce()
//   Section 7.1 (reserved byte)    -> orc_compile_framed()
//
// Parity status: every function here is pinned by the CPU test-suite
// (printed examples, closed forms, brute force, a library regex engine);
// the pins are listed in the tests that exercise them.

#include "oracle.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

namespace {

// ---------------------------------------------------------------- byte sets
struct ByteSet {
  uint64_t w[4] = {0, 0, 0, 0};
  void add(int b) { w[b >> 6] |= (uint64_t)1 << (b & 63); }
  bool has(int b) const { return (w[b >> 6] >> (b & 63)) & 1; }
  void add_range(int lo, int hi) {
    for (int b = lo; b <= hi; ++b) add(b);
  }
  void invert() {
    for (auto &x : w) x = ~x;
  }
  bool empty() const { return !(w[0] | w[1] | w[2] | w[3]); }
};

// ---------------------------------------------------------------- regex AST
// Byte-regex dialect: literals, '.', classes [..] and [^..] with ranges,
// groups, '|', postfix * + ? {m} {m,} {m,n}, escapes \n \t \r \f \v \0 \xHH
// and a backslash before any non-alphanumeric byte.  The language is over
// bytes; an empty class is rejected (the dialect has no empty-language atom).
enum NodeKind { N_EPS, N_SET, N_CAT, N_ALT, N_STAR, N_PLUS, N_OPT, N_REP };

struct Node {
  NodeKind kind;
  ByteSet set;
  std::vector<int> kids;
  int lo = 0, hi = 0;  // N_REP bounds; hi < 0 means unbounded
};

struct RegexParser {
  const uint8_t *p;
  size_t n;
  size_t i = 0;
  std::vector<Node> &nodes;
  std::string err;

  RegexParser(const uint8_t *p_, size_t n_, std::vector<Node> &nodes_) : p(p_), n(n_), nodes(nodes_) {}

  int add(Node nd) {
    nodes.push_back(std::move(nd));
    return (int)nodes.size() - 1;
  }
  bool fail(const char *msg) {
    if (err.empty()) {
      char buf[160];
      snprintf(buf, sizeof buf, "%s at offset %zu", msg, i);
      err = buf;
    }
    return false;
  }
  static int hexval(uint8_t c) {
    if (c >= '0' && c <= '9') return c - '0';
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    if (c >= 'A' && c <= 'F') return c - 'A' + 10;
    return -1;
  }
  // Reads the escape after a backslash at p[i-1]; returns the byte or -1.
  int escape() {
    if (i >= n) {
      fail("dangling backslash");
      return -1;
    }
    uint8_t c = p[i++];
    switch (c) {
      case 'n': return '\n';
      case 't': return '\t';
      case 'r': return '\r';
      case 'f': return '\f';
      case 'v': return '\v';
      case 'b': return '\b';
      case '0': return 0;
      case 'x': {
        if (i + 2 > n || hexval(p[i]) < 0 || hexval(p[i + 1]) < 0) {
          fail("bad \\x escape");
          return -1;
        }
        int v = hexval(p[i]) * 16 + hexval(p[i + 1]);
        i += 2;
        return v;
      }
      default:
        if ((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9')) {
          fail("unknown escape");
          return -1;
        }
        return c;
    }
  }
  int parse_class() {  // p[i-1] == '['
    ByteSet s;
    bool neg = false;
    if (i < n && p[i] == '^') {
      neg = true;
      ++i;
    }
    bool first = true;
    for (;;) {
      if (i >= n) {
        fail("unterminated class");
        return -1;
      }
      uint8_t c = p[i];
      if (c == ']' && !first) {
        ++i;
        break;
      }
      first = false;
      ++i;
      int lo = c;
      if (c == '\\') {
        lo = escape();
        if (lo < 0) return -1;
      }
      if (i + 1 < n && p[i] == '-' && p[i + 1] != ']') {
        ++i;
        uint8_t d = p[i++];
        int hi = d;
        if (d == '\\') {
          hi = escape();
          if (hi < 0) return -1;
        }
        if (hi < lo) {
          fail("reversed range");
          return -1;
        }
        s.add_range(lo, hi);
      } else {
        s.add(lo);
      }
    }
    if (neg) s.invert();
    if (s.empty()) {
      fail("empty class");
      return -1;
    }
    Node nd;
    nd.kind = N_SET;
    nd.set = s;
    return add(nd);
  }
  int parse_atom() {
    uint8_t c = p[i++];
    Node nd;
    if (c == '(') {
      int r = parse_alt();
      if (r < 0) return -1;
      if (i >= n || p[i] != ')') {
        fail("missing )");
        return -1;
      }
      ++i;
      return r;
    }
    if (c == '[') return parse_class();
    nd.kind = N_SET;
    if (c == '.') {
      nd.set.add_range(0, 255);
    } else if (c == '\\') {
      int b = escape();
      if (b < 0) return -1;
      nd.set.add(b);
    } else if (c == '*' || c == '+' || c == '?' || c == '{' || c == ')' || c == '|') {
      --i;
      fail("misplaced operator");
      return -1;
    } else {
      nd.set.add(c);
    }
    return add(nd);
  }
  bool read_int(int &v) {
    size_t s = i;
    v = 0;
    while (i < n && p[i] >= '0' && p[i] <= '9') {
      v = v * 10 + (p[i] - '0');
      if (v > 1000) return fail("repeat bound too large");
      ++i;
    }
    return i > s;
  }
  int parse_repeat() {
    int a = parse_atom();
    if (a < 0) return -1;
    while (i < n) {
      uint8_t c = p[i];
      Node nd;
      if (c == '*') nd.kind = N_STAR;
      else if (c == '+') nd.kind = N_PLUS;
      else if (c == '?') nd.kind = N_OPT;
      else if (c == '{') {
        ++i;
        int lo, hi;
        if (!read_int(lo)) {
          fail("bad repeat");
          return -1;
        }
        hi = lo;
        if (i < n && p[i] == ',') {
          ++i;
          if (i < n && p[i] == '}') hi = -1;
          else if (!read_int(hi) || hi < lo) {
            fail("bad repeat");
            return -1;
          }
        }
        if (i >= n || p[i] != '}') {
          fail("bad repeat");
          return -1;
        }
        nd.kind = N_REP;
        nd.lo = lo;
        nd.hi = hi;
      } else {
        break;
      }
      ++i;
      nd.kids.push_back(a);
      a = add(nd);
    }
    return a;
  }
  int parse_concat() {
    Node nd;
    nd.kind = N_CAT;
    while (i < n && p[i] != '|' && p[i] != ')') {
      int r = parse_repeat();
      if (r < 0) return -1;
      nd.kids.push_back(r);
    }
    if (nd.kids.empty()) nd.kind = N_EPS;
    if (nd.kids.size() == 1) return nd.kids[0];
    return add(nd);
  }
  int parse_alt() {
    Node nd;
    nd.kind = N_ALT;
    for (;;) {
      int r = parse_concat();
      if (r < 0) return -1;
      nd.kids.push_back(r);
      if (i < n && p[i] == '|') {
        ++i;
        continue;
      }
      break;
    }
    if (nd.kids.size() == 1) return nd.kids[0];
    return add(nd);
  }
  int parse() {
    int r = parse_alt();
    if (r < 0) return -1;
    if (i != n) {
      fail("unbalanced )");
      return -1;
    }
    return r;
  }
};

// -------------------------------------------------------- Thompson NFA
// Each state has at most one byte edge (set -> to) and any number of
// epsilon edges.  One start and one final state per token kind.
struct NState {
  ByteSet on;
  int to = -1;
  std::vector<int> eps;
};

struct Nfa {
  std::vector<NState> st;
  int fresh() {
    st.emplace_back();
    return (int)st.size() - 1;
  }
  struct Frag {
    int start, end;
  };
  // Builds a fresh fragment for AST node `id` (called once per copy for
  // bounded repeats, so copies never share states).
  Frag build(const std::vector<Node> &ast, int id) {
    const Node &nd = ast[id];
    Frag f{-1, -1};
    switch (nd.kind) {
      case N_EPS: {
        f.start = fresh();
        f.end = fresh();
        st[f.start].eps.push_back(f.end);
        return f;
      }
      case N_SET: {
        f.start = fresh();
        f.end = fresh();
        st[f.start].on = nd.set;
        st[f.start].to = f.end;
        return f;
      }
      case N_CAT: {
        Frag a = build(ast, nd.kids[0]);
        f.start = a.start;
        int end = a.end;
        for (size_t k = 1; k < nd.kids.size(); ++k) {
          Frag b = build(ast, nd.kids[k]);
          st[end].eps.push_back(b.start);
          end = b.end;
        }
        f.end = end;
        return f;
      }
      case N_ALT: {
        f.start = fresh();
        f.end = fresh();
        for (int k : nd.kids) {
          Frag b = build(ast, k);
          st[f.start].eps.push_back(b.start);
          st[b.end].eps.push_back(f.end);
        }
        return f;
      }
      case N_STAR: {  // e*: zero or more
        f.start = fresh();
        f.end = fresh();
        Frag b = build(ast, nd.kids[0]);
        st[f.start].eps.push_back(b.start);
        st[f.start].eps.push_back(f.end);
        st[b.end].eps.push_back(b.start);
        st[b.end].eps.push_back(f.end);
        return f;
      }
      case N_PLUS: {  // e+: one or more
        f.start = fresh();
        f.end = fresh();
        Frag b = build(ast, nd.kids[0]);
        st[f.start].eps.push_back(b.start);
        st[b.end].eps.push_back(b.start);
        st[b.end].eps.push_back(f.end);
        return f;
      }
      case N_OPT: {  // e?: zero or one
        f.start = fresh();
        f.end = fresh();
        Frag b = build(ast, nd.kids[0]);
        st[f.start].eps.push_back(b.start);
        st[f.start].eps.push_back(f.end);
        st[b.end].eps.push_back(f.end);
        return f;
      }
      case N_REP: {  // e{lo,hi}: lo mandatory copies, then optional ones
        f.start = fresh();
        int end = f.start;
        for (int k = 0; k < nd.lo; ++k) {
          Frag b = build(ast, nd.kids[0]);
          st[end].eps.push_back(b.start);
          end = b.end;
        }
        if (nd.hi < 0) {
          Frag b = build(ast, nd.kids[0]);  // then e*
          int out = fresh();
          st[end].eps.push_back(b.start);
          st[end].eps.push_back(out);
          st[b.end].eps.push_back(b.start);
          st[b.end].eps.push_back(out);
          end = out;
        } else {
          int out = fresh();
          for (int k = nd.lo; k < nd.hi; ++k) {
            Frag b = build(ast, nd.kids[0]);
            st[end].eps.push_back(b.start);
            st[end].eps.push_back(out);
            end = b.end;
          }
          st[end].eps.push_back(out);
          end = out;
        }
        f.end = end;
        return f;
      }
    }
    return f;
  }
};

}  // namespace

struct orc_set {
  Nfa nfa;
  std::vector<int> start, final_;  // per kind
  std::vector<int32_t> prio;
  std::vector<uint8_t> discard;
  // scratch for the NFA simulation (a set is used by one thread at a time)
  mutable std::vector<uint64_t> mark;
  mutable uint64_t gen = 0;
  mutable std::vector<int> stack, cur, nxt;
};

namespace {

// Adds the epsilon-closure of s to `out`, stamping visited states with gen.
void closure_add(const orc_set *S, int s, std::vector<int> &out) {
  std::vector<int> &stack = S->stack;
  stack.clear();
  stack.push_back(s);
  while (!stack.empty()) {
    int x = stack.back();
    stack.pop_back();
    if (S->mark[x] == S->gen) continue;
    S->mark[x] = S->gen;
    out.push_back(x);
    for (int y : S->nfa.st[x].eps) stack.push_back(y);
  }
}

// Length of the longest non-empty prefix of w[i, n) in L(kind), or 0 if there
// is none (Section 3: tokens have positive length, so the empty match of a
// nullable pattern never counts).
uint64_t longest_match(const orc_set *S, int kind, const uint8_t *w, uint64_t i, uint64_t n) {
  std::vector<int> &cur = S->cur, &nxt = S->nxt;
  cur.clear();
  ++S->gen;
  closure_add(S, S->start[kind], cur);
  const int fin = S->final_[kind];
  uint64_t best = 0;
  for (uint64_t j = i; j < n && !cur.empty(); ++j) {
    ++S->gen;
    nxt.clear();
    for (int x : cur) {
      const NState &ns = S->nfa.st[x];
      if (ns.to >= 0 && ns.on.has(w[j])) closure_add(S, ns.to, nxt);
    }
    std::swap(cur, nxt);
    for (int x : cur)
      if (x == fin) {
        best = j + 1 - i;
        break;
      }
  }
  return best;
}

struct Tok {
  uint8_t kind;
  uint32_t len;
  uint64_t off;
};

// The serial longest-match scan of Section 3: at each offset take the longest
// positive-length match over all kinds, break a same-length tie by the lower
// priority number and then the lower kind index, emit it and restart; halt
// when no kind matches.  Returns con(w).
uint64_t lex_serial(const orc_set *S, const uint8_t *w, uint64_t n, std::vector<Tok> &out) {
  const int K = (int)S->start.size();
  uint64_t i = 0;
  while (i < n) {
    uint64_t best_len = 0;
    int best = -1;
    for (int k = 0; k < K; ++k) {
      uint64_t l = longest_match(S, k, w, i, n);
      if (l == 0) continue;
      if (l > best_len || (l == best_len && (S->prio[k] < S->prio[best] ||
                                             (S->prio[k] == S->prio[best] && k < best)))) {
        best_len = l;
        best = k;
      }
    }
    if (best < 0) break;  // no positive-length accepting prefix: halt at i
    out.push_back(Tok{(uint8_t)best, (uint32_t)best_len, i});
    i += best_len;
  }
  return i;
}

// pi_I of Section 5: delete every pair whose kind is discarded.
std::vector<Tok> project(const orc_set *S, const std::vector<Tok> &t) {
  std::vector<Tok> r;
  for (const Tok &x : t)
    if (!S->discard[x.kind]) r.push_back(x);
  return r;
}

// Chunked scan: every slice is a whole input; concatenate in order; stop
// after the first slice that halts before its end (Corollary 1, and the
// same rule in discard mode).  Returns the error offset (n if none).
uint64_t lex_chunked(const orc_set *S, const uint8_t *w, uint64_t n, const std::vector<uint64_t> &cuts,
                     std::vector<Tok> &out) {
  uint64_t lo = 0;
  for (size_t j = 0; j <= cuts.size(); ++j) {
    uint64_t hi = j < cuts.size() ? cuts[j] : n;
    std::vector<Tok> part;
    uint64_t con = lex_serial(S, w + lo, hi - lo, part);
    for (Tok &t : part) {
      t.off += lo;
      out.push_back(t);
    }
    if (con < hi - lo) return lo + con;
    lo = hi;
  }
  return n;
}

// ------------------------------------------------ automaton construction
struct Dfa {
  int n = 0;
  int q0 = 0;
  std::vector<int> next;  // n * 256, -1 = undefined
  std::vector<int> acc;   // n, -1 = not accepting
};

// Subset construction over the union of the per-kind NFAs.  tau(S) is the
// kind with the lowest (priority, index) among those whose final state is in
// S: the compile-time resolution of same-length ties described in Section 3.
Dfa subset_construct(const orc_set *S) {
  Dfa d;
  std::map<std::vector<int>, int> id;
  std::vector<std::vector<int>> sets;
  auto intern = [&](std::vector<int> v) {
    std::sort(v.begin(), v.end());
    auto it = id.find(v);
    if (it != id.end()) return it->second;
    int k = (int)sets.size();
    id.emplace(v, k);
    sets.push_back(v);
    return k;
  };
  std::vector<int> init;
  ++S->gen;
  for (int s : S->start) closure_add(S, s, init);
  intern(init);
  for (size_t q = 0; q < sets.size(); ++q) {
    d.next.resize((q + 1) * 256, -1);
    for (int b = 0; b < 256; ++b) {
      std::vector<int> t;
      ++S->gen;
      for (int x : sets[q]) {
        const NState &ns = S->nfa.st[x];
        if (ns.to >= 0 && ns.on.has(b)) closure_add(S, ns.to, t);
      }
      if (!t.empty()) d.next[q * 256 + b] = intern(t);
    }
  }
  d.n = (int)sets.size();
  d.q0 = 0;
  d.acc.assign(d.n, -1);
  const int K = (int)S->start.size();
  for (int q = 0; q < d.n; ++q) {
    for (int x : sets[q])
      for (int k = 0; k < K; ++k)
        if (x == S->final_[k]) {
          int &a = d.acc[q];
          if (a < 0 || S->prio[k] < S->prio[a] || (S->prio[k] == S->prio[a] && k < a)) a = k;
        }
  }
  return d;
}

// Section 4.1: restrict to Q+ (reachable and co-accessible), keep only the
// transitions between live states (delta+), then merge states with the same
// accepting label and, byte by byte, the same target class -- a missing
// transition counting as its own target, never as a dead state.  The result
// has every state live.  Returns false if q0 is not live.
bool trim_and_minimise(const Dfa &in, Dfa &out) {
  const int n = in.n;
  std::vector<char> reach(n, 0), coacc(n, 0);
  std::deque<int> work{in.q0};
  reach[in.q0] = 1;
  while (!work.empty()) {
    int q = work.front();
    work.pop_front();
    for (int b = 0; b < 256; ++b) {
      int t = in.next[q * 256 + b];
      if (t >= 0 && !reach[t]) {
        reach[t] = 1;
        work.push_back(t);
      }
    }
  }
  std::vector<std::vector<int>> pred(n);
  for (int q = 0; q < n; ++q)
    for (int b = 0; b < 256; ++b) {
      int t = in.next[q * 256 + b];
      if (t >= 0) pred[t].push_back(q);
    }
  for (int q = 0; q < n; ++q)
    if (in.acc[q] >= 0) {
      coacc[q] = 1;
      work.push_back(q);
    }
  while (!work.empty()) {
    int q = work.front();
    work.pop_front();
    for (int p : pred[q])
      if (!coacc[p]) {
        coacc[p] = 1;
        work.push_back(p);
      }
  }
  std::vector<char> live(n);
  for (int q = 0; q < n; ++q) live[q] = reach[q] && coacc[q];
  if (!live[in.q0]) return false;
  auto dplus = [&](int q, int b) {
    int t = in.next[q * 256 + b];
    return (t >= 0 && live[t]) ? t : -1;
  };
  // Moore refinement over the live states.
  std::vector<int> cls(n, -1);
  {
    std::map<int, int> lab;
    for (int q = 0; q < n; ++q)
      if (live[q]) {
        auto it = lab.find(in.acc[q]);
        if (it == lab.end()) it = lab.emplace(in.acc[q], (int)lab.size()).first;
        cls[q] = it->second;
      }
  }
  int ncls = 0;
  for (int q = 0; q < n; ++q) ncls = std::max(ncls, cls[q] + 1);
  for (;;) {
    std::map<std::vector<int>, int> sig;
    std::vector<int> ncl(n, -1);
    for (int q = 0; q < n; ++q) {
      if (!live[q]) continue;
      std::vector<int> key;
      key.reserve(257);
      key.push_back(cls[q]);
      for (int b = 0; b < 256; ++b) {
        int t = dplus(q, b);
        key.push_back(t < 0 ? -1 : cls[t]);
      }
      auto it = sig.find(key);
      if (it == sig.end()) it = sig.emplace(key, (int)sig.size()).first;
      ncl[q] = it->second;
    }
    int m = (int)sig.size();
    cls.swap(ncl);
    if (m == ncls) break;
    ncls = m;
  }
  // Quotient automaton, numbered so that q0's class comes first.
  std::vector<int> ren(ncls, -1), rep;
  int k = 0;
  ren[cls[in.q0]] = k++;
  rep.push_back(in.q0);
  for (int q = 0; q < n; ++q)
    if (live[q] && ren[cls[q]] < 0) {
      ren[cls[q]] = k++;
      rep.push_back(q);
    }
  out.n = k;
  out.q0 = 0;
  out.next.assign((size_t)k * 256, -1);
  out.acc.assign(k, -1);
  for (int c = 0; c < k; ++c) {
    int q = rep[c];
    out.acc[c] = in.acc[q];
    for (int b = 0; b < 256; ++b) {
      int t = dplus(q, b);
      if (t >= 0) out.next[c * 256 + b] = ren[cls[t]];
    }
  }
  return true;
}

void setbit(uint8_t *m, int b) { m[b >> 3] |= (uint8_t)(1u << (b & 7)); }
bool getbit(const uint8_t *m, int b) { return (m[b >> 3] >> (b & 7)) & 1; }

// Definitions 1-3 and the useful sets of Corollary 2 / Proposition 2, on an
// automaton whose states are all live (so delta = delta+).
void analyse(const Dfa &d, const std::vector<uint8_t> &discard, orc_cert_info *out) {
  const int n = d.n, q0 = d.q0;
  auto dp = [&](int q, int b) { return d.next[q * 256 + b]; };
  // Definition 1, tested as "some live transition enters q0".
  bool reent = false;
  for (int q = 0; q < n; ++q)
    for (int b = 0; b < 256; ++b)
      if (dp(q, b) == q0) reent = true;
  // T(q) subset I  <=>  q cannot reach an accepting state whose token is kept.
  std::vector<std::vector<int>> pred(n);
  for (int q = 0; q < n; ++q)
    for (int b = 0; b < 256; ++b)
      if (dp(q, b) >= 0) pred[dp(q, b)].push_back(q);
  std::vector<char> reaches_kept(n, 0);
  std::deque<int> work;
  for (int q = 0; q < n; ++q)
    if (d.acc[q] >= 0 && !discard[d.acc[q]]) {
      reaches_kept[q] = 1;
      work.push_back(q);
    }
  while (!work.empty()) {
    int q = work.front();
    work.pop_front();
    for (int p : pred[q])
      if (!reaches_kept[p]) {
        reaches_kept[p] = 1;
        work.push_back(p);
      }
  }
  for (int b = 0; b < 256; ++b) {
    const int t0 = dp(q0, b);
    bool exact = true, modi = true, consumed = false;
    for (int q = 0; q < n; ++q) {
      int t = dp(q, b);
      if (t < 0) continue;
      consumed = true;
      // Definition 2: only q0 may consume b, and then q0 must not be re-entrant.
      bool A = (q == q0) && !reent;
      if (!A) exact = false;
      // Definition 3, clause C: tau(q) defined, delta+(q0,b) = delta+(q,b),
      // and T(q) within I.
      bool C = d.acc[q] >= 0 && t0 >= 0 && t0 == t && !reaches_kept[q];
      if (!(A || C)) modi = false;
    }
    if (consumed) setbit(out->consumed, b);
    if (t0 >= 0) setbit(out->q0_live, b);
    if (exact) setbit(out->exact_raw, b);
    if (modi) setbit(out->discard_raw, b);
    if (exact && t0 >= 0) setbit(out->exact_useful, b);
    if (modi && t0 >= 0) setbit(out->discard_useful, b);
  }
  out->nstates = n;
  out->q0_live_state = 1;
  out->reentrant = reent ? 1 : 0;
}

// Cert of an arbitrary automaton: trim, minimise, analyse.
int cert_of_dfa(const Dfa &d, const std::vector<uint8_t> &discard, orc_cert_info *out, Dfa *minimised) {
  memset(out, 0, sizeof *out);
  Dfa m;
  if (!trim_and_minimise(d, m)) {
    // q0 not live: the token set accepts nothing; Definition 2 quantifies
    // over an empty Q+, so every byte is certified and none is useful.
    for (int b = 0; b < 256; ++b) {
      setbit(out->exact_raw, b);
      setbit(out->discard_raw, b);
    }
    out->q0_live_state = 0;
    if (minimised) *minimised = Dfa{};
    return ORC_OK;
  }
  analyse(m, discard, out);
  if (minimised) *minimised = m;
  return ORC_OK;
}

// Shortest byte path in d from `from` to any state satisfying goal(), using
// only bytes allowed by `allow`; the path may be empty unless nonempty is set.
// Returns false when none exists.
template <class Goal>
bool shortest_path(const Dfa &d, int from, Goal goal, bool nonempty, const ByteSet &allow,
                   std::vector<uint8_t> &path) {
  path.clear();
  if (!nonempty && goal(from)) return true;
  std::vector<int> par(d.n, -2), pb(d.n, -1);
  std::deque<int> work;
  // Level 1 from `from`; the goal may be `from` itself via a nonempty cycle.
  std::vector<std::pair<int, int>> first;
  for (int b = 0; b < 256; ++b) {
    if (!allow.has(b)) continue;
    int t = d.next[from * 256 + b];
    if (t >= 0 && par[t] == -2) {
      par[t] = -1;
      pb[t] = b;
      work.push_back(t);
    }
  }
  while (!work.empty()) {
    int q = work.front();
    work.pop_front();
    if (goal(q)) {
      std::vector<uint8_t> rev;
      for (int x = q; x >= 0 && par[x] != -2; x = par[x]) {
        rev.push_back((uint8_t)pb[x]);
        if (par[x] == -1) break;
      }
      path.assign(rev.rbegin(), rev.rend());
      return true;
    }
    for (int b = 0; b < 256; ++b) {
      if (!allow.has(b)) continue;
      int t = d.next[q * 256 + b];
      if (t >= 0 && par[t] == -2) {
        par[t] = q;
        pb[t] = b;
        work.push_back(t);
      }
    }
  }
  return false;
}

// Theorem 2's witness for an uncertified, live-consumed byte b on the
// minimised automaton m: pick a consuming q != q0 if one exists (u = a path
// q0 -> q, nonempty), else q = q0 re-entrant (u = a nonempty cycle q0 -> q0);
// v = a path from delta+(q, b) to acceptance.  Returns false if no witness
// exists over the allowed bytes.
bool make_witness(const Dfa &m, int b, const ByteSet &allow, std::vector<uint8_t> &w, uint64_t &boff) {
  int q = -1;
  for (int x = 0; x < m.n; ++x)
    if (x != m.q0 && m.next[x * 256 + b] >= 0) {
      std::vector<uint8_t> tmp;
      if (shortest_path(m, m.q0, [&](int y) { return y == x; }, true, allow, tmp)) {
        q = x;
        break;
      }
    }
  std::vector<uint8_t> u, v;
  if (q >= 0) {
    shortest_path(m, m.q0, [&](int y) { return y == q; }, true, allow, u);
  } else {
    if (m.next[m.q0 * 256 + b] < 0) return false;
    if (!shortest_path(m, m.q0, [&](int y) { return y == m.q0; }, true, allow, u)) return false;
    q = m.q0;
  }
  int t = m.next[q * 256 + b];
  if (!shortest_path(m, t, [&](int y) { return m.acc[y] >= 0; }, false, allow, v)) return false;
  w = u;
  w.push_back((uint8_t)b);
  w.insert(w.end(), v.begin(), v.end());
  boff = u.size();
  return true;
}

bool same(const std::vector<Tok> &a, const std::vector<Tok> &b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].kind != b[i].kind || a[i].len != b[i].len) return false;
  return true;
}

}  // namespace

// ================================================================ C API
extern "C" {

orc_set *orc_compile_framed(const orc_def *defs, uint32_t ndefs, uint32_t r, int r_discard, char *err,
                            size_t errlen) {
  // r < 256 reserves byte r; r == 256 (orc_compile) reserves nothing.
  auto seterr = [&](const std::string &m) {
    if (err && errlen) {
      snprintf(err, errlen, "%s", m.c_str());
    }
  };
  uint32_t limit = r < 256 ? 254 : 255;
  if (!defs || ndefs == 0 || ndefs > limit || r > 256) {
    seterr("need 1.." + std::to_string(limit) + " token definitions and a byte below 256");
    return nullptr;
  }
  orc_set *S = new orc_set;
  for (uint32_t k = 0; k < ndefs; ++k) {
    if (!defs[k].pattern) {
      seterr("null pattern");
      delete S;
      return nullptr;
    }
    std::vector<Node> ast;
    RegexParser P((const uint8_t *)defs[k].pattern, strlen(defs[k].pattern), ast);
    int root = P.parse();
    if (root < 0) {
      seterr("kind " + std::to_string(k) + ": " + P.err);
      delete S;
      return nullptr;
    }
    if (r < 256) {
      // the reserved byte leaves every class: no word of this kind contains it
      for (Node &nd : ast)
        if (nd.kind == N_SET) nd.set.w[r >> 6] &= ~((uint64_t)1 << (r & 63));
    }
    Nfa::Frag f = S->nfa.build(ast, root);
    S->start.push_back(f.start);
    S->final_.push_back(f.end);
    S->prio.push_back(defs[k].priority);
    S->discard.push_back(defs[k].discard ? 1 : 0);
  }
  if (r < 256) {
    // the reserved byte's own kind: the one-byte word r
    std::vector<Node> ast(1);
    ast[0].kind = N_SET;
    ast[0].set.add((int)r);
    Nfa::Frag f = S->nfa.build(ast, 0);
    S->start.push_back(f.start);
    S->final_.push_back(f.end);
    S->prio.push_back(0);
    S->discard.push_back(r_discard ? 1 : 0);
  }
  S->mark.assign(S->nfa.st.size(), 0);
  return S;
}

orc_set *orc_compile(const orc_def *defs, uint32_t ndefs, char *err, size_t errlen) {
  return orc_compile_framed(defs, ndefs, 256, 0, err, errlen);
}

void orc_free(orc_set *s) { delete s; }

uint32_t orc_nkinds(const orc_set *s) { return s ? (uint32_t)s->start.size() : 0; }

int orc_lex(const orc_set *s, const uint8_t *w, uint64_t n, int discard_filter, uint8_t *kinds,
            uint32_t *lens, uint64_t *offs, uint64_t cap, uint64_t *ntok, uint64_t *con) {
  if (!s || (!w && n) || !ntok || !con) return ORC_EINVAL;
  std::vector<Tok> t;
  *con = lex_serial(s, w, n, t);
  if (discard_filter) t = project(s, t);
  *ntok = t.size();
  if (t.size() > cap) return ORC_ECAP;
  for (size_t i = 0; i < t.size(); ++i) {
    if (kinds) kinds[i] = t[i].kind;
    if (lens) lens[i] = t[i].len;
    if (offs) offs[i] = t[i].off;
  }
  return ORC_OK;
}

int orc_cert(const orc_set *s, orc_cert_info *out) {
  if (!s || !out) return ORC_EINVAL;
  Dfa d = subset_construct(s);
  return cert_of_dfa(d, s->discard, out, nullptr);
}

int orc_cert_table(int32_t nstates, int32_t q0, const int32_t *next, const int32_t *accept,
                   const uint8_t *discard, int32_t ntok, orc_cert_info *out) {
  if (nstates <= 0 || q0 < 0 || q0 >= nstates || !next || !accept || !out || ntok < 0)
    return ORC_EINVAL;
  Dfa d;
  d.n = nstates;
  d.q0 = q0;
  d.next.assign(next, next + (size_t)nstates * 256);
  d.acc.assign(accept, accept + nstates);
  for (int v : d.next)
    if (v < -1 || v >= nstates) return ORC_EINVAL;
  for (int v : d.acc)
    if (v < -1 || v >= ntok) return ORC_EINVAL;
  std::vector<uint8_t> disc(std::max(ntok, 1), 0);
  for (int t = 0; t < ntok; ++t) disc[t] = discard ? (discard[t] ? 1 : 0) : 0;
  return cert_of_dfa(d, disc, out, nullptr);
}

int64_t orc_witness(const orc_set *s, int b, uint8_t *out, uint64_t cap, uint64_t *b_offset) {
  if (!s || b < 0 || b > 255 || !b_offset) return ORC_EINVAL;
  Dfa d = subset_construct(s), m;
  orc_cert_info info;
  cert_of_dfa(d, s->discard, &info, &m);
  if (!info.q0_live_state || getbit(info.exact_raw, b) || !getbit(info.consumed, b)) return 0;
  ByteSet all;
  all.add_range(0, 255);
  std::vector<uint8_t> w;
  uint64_t boff = 0;
  if (!make_witness(m, b, all, w, boff)) return ORC_EINVAL;  // cannot happen (Theorem 2)
  if (w.size() > cap) return ORC_ECAP;
  if (out) memcpy(out, w.data(), w.size());
  *b_offset = boff;
  return (int64_t)w.size();
}

int orc_lex_chunked(const orc_set *s, const uint8_t *w, uint64_t n, const uint64_t *cuts, uint64_t ncuts,
                    int discard_filter, uint8_t *kinds, uint32_t *lens, uint64_t cap, uint64_t *ntok,
                    uint64_t *err_off) {
  if (!s || (!w && n) || !ntok || !err_off || (ncuts && !cuts)) return ORC_EINVAL;
  std::vector<uint64_t> c(cuts, cuts + ncuts);
  for (size_t j = 0; j < c.size(); ++j)
    if (c[j] == 0 || c[j] >= n || (j && c[j] <= c[j - 1])) return ORC_EINVAL;
  std::vector<Tok> t;
  *err_off = lex_chunked(s, w, n, c, t);
  if (discard_filter) t = project(s, t);
  *ntok = t.size();
  if (t.size() > cap) return ORC_ECAP;
  for (size_t i = 0; i < t.size(); ++i) {
    if (kinds) kinds[i] = t[i].kind;
    if (lens) lens[i] = t[i].len;
  }
  return ORC_OK;
}

int orc_bruteforce(const orc_set *s, const uint8_t *alphabet, uint32_t nalpha, uint32_t maxlen,
                   uint64_t *stats) {
  if (!s || !alphabet || !nalpha || !stats || maxlen > 16) return ORC_EINVAL;
  for (int i = 0; i < ORC_BF_NSTATS; ++i) stats[i] = 0;
  Dfa d = subset_construct(s), m;
  orc_cert_info ci;
  cert_of_dfa(d, s->discard, &ci, &m);
  ByteSet alpha;
  for (uint32_t a = 0; a < nalpha; ++a) alpha.add(alphabet[a]);

  bool inside_seen[256] = {false};  // byte seen strictly inside a token
  bool unsafe_i[256] = {false};     // splitting at every occurrence broke pi_I

  std::vector<uint8_t> w;
  std::vector<uint32_t> digit;
  for (uint32_t len = 1; len <= maxlen; ++len) {
    digit.assign(len, 0);
    w.assign(len, alphabet[0]);
    for (;;) {
      ++stats[ORC_BF_STRINGS];
      std::vector<Tok> ser;
      const uint64_t con = lex_serial(s, w.data(), len, ser);
      const bool full = con == len;
      if (full) ++stats[ORC_BF_TOKENIZABLE];
      std::vector<char> bnd(len + 1, 0);
      bnd[0] = 1;
      for (const Tok &t : ser) bnd[t.off + t.len] = 1;
      const std::vector<Tok> ser_i = project(s, ser);

      // Lemma 1 (and Lemma 3 for offsets before con(w)): a certified byte
      // below con(w) sits on a boundary.
      for (uint64_t i = 1; i < len; ++i) {
        if (i < con && getbit(ci.exact_raw, w[i]) && !bnd[i]) ++stats[ORC_BF_LEMMA1_VIOL];
        if (full && !bnd[i]) inside_seen[w[i]] = true;
      }
      // Splits at useful certified occurrences: all at once, then each alone.
      for (int mode = 0; mode < 2; ++mode) {
        const uint8_t *map = mode == 0 ? ci.exact_useful : ci.discard_useful;
        std::vector<uint64_t> all;
        for (uint64_t i = 1; i < len; ++i)
          if (getbit(map, w[i])) all.push_back(i);
        if (all.empty()) continue;
        std::vector<std::vector<uint64_t>> plans{all};
        if (all.size() > 1)
          for (uint64_t c : all) plans.push_back({c});
        for (const auto &plan : plans) {
          ++stats[ORC_BF_MODE_SPLITS];
          std::vector<Tok> ch;
          uint64_t err = lex_chunked(s, w.data(), len, plan, ch);
          bool ok;
          if (mode == 0) ok = same(ch, ser) && err == con;
          else ok = same(project(s, ch), ser_i) && err == con;
          if (!ok) {
            if (mode == 0) ++stats[full ? ORC_BF_THM1_VIOL : ORC_BF_COR1_VIOL];
            else ++stats[full ? ORC_BF_THM3_VIOL : ORC_BF_MALFORMED_I_VIOL];
          }
        }
      }
      // The paper's sweep: split at every noninitial occurrence of each
      // alphabet byte and compare the pi_I images (tokenizable strings only).
      if (full) {
        for (uint32_t a = 0; a < nalpha; ++a) {
          const uint8_t b = alphabet[a];
          if (unsafe_i[b]) continue;
          std::vector<uint64_t> plan;
          for (uint64_t i = 1; i < len; ++i)
            if (w[i] == b) plan.push_back(i);
          if (plan.empty()) continue;
          std::vector<Tok> ch;
          uint64_t err = lex_chunked(s, w.data(), len, plan, ch);
          if (!(same(project(s, ch), ser_i) && err == con)) unsafe_i[b] = true;
        }
      }
      // next string (odometer)
      uint32_t p = 0;
      while (p < len) {
        if (++digit[p] < nalpha) {
          w[p] = alphabet[digit[p]];
          break;
        }
        digit[p] = 0;
        w[p] = alphabet[0];
        ++p;
      }
      if (p == len) break;
    }
  }
  // Proposition 3: exact certificates are certified modulo any I.
  for (int b = 0; b < 256; ++b)
    if (getbit(ci.exact_raw, b) && !getbit(ci.discard_raw, b)) ++stats[ORC_BF_PROP3_VIOL];
  // Theorem 2 and the sweep's pair counts, over the alphabet.
  for (uint32_t a = 0; a < nalpha; ++a) {
    const int b = alphabet[a];
    if (!ci.q0_live_state || !getbit(ci.consumed, b)) continue;
    ++stats[ORC_BF_PAIRS_CONSUMED];
    if (getbit(ci.discard_raw, b)) ++stats[ORC_BF_PAIRS_ADMITTED_I];
    else if (!unsafe_i[b]) ++stats[ORC_BF_PAIRS_REFUSED_SAFE];
    if (getbit(ci.exact_raw, b)) continue;
    if (inside_seen[b]) ++stats[ORC_BF_NECESSITY_FOUND];
    ByteSet all;
    all.add_range(0, 255);
    std::vector<uint8_t> wit;
    uint64_t boff = 0;
    if (!make_witness(m, b, all, wit, boff)) {
      ++stats[ORC_BF_WITNESS_VIOL];
      continue;
    }
    std::vector<Tok> t;
    uint64_t con = lex_serial(s, wit.data(), wit.size(), t);
    if (!(con == wit.size() && t.size() == 1 && boff >= 1 && boff < wit.size()))
      ++stats[ORC_BF_WITNESS_VIOL];
    // If a witness fits within the alphabet and the bound, the enumeration
    // must have seen b strictly inside a token.
    std::vector<uint8_t> wa;
    if (make_witness(m, b, alpha, wa, boff) && wa.size() <= maxlen && !inside_seen[b])
      ++stats[ORC_BF_NECESSITY_VIOL];
  }
  return ORC_OK;
}

}  // extern "C"
