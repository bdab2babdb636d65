// compile.cc -- token-set compiler: byte regex -> Glushkov position automaton ->
// class-compressed subset DFA -> trimmed, Hopcroft-minimised automaton -> certificate
// maps -> packed GPU tables.
//
// Paper map
//   Section 3     tau resolves same-length ties by (priority, index) at compile time
//   Section 4.1   Q+ = reachable AND co-accessible; delta+ keeps edges inside Q+;
//                 the minimiser keeps a missing transition apart from a dead one
//   Definition 1  re-entrant q0: some live edge enters q0
//   Definition 2  exact map; Corollary 2 useful = certified AND delta+(q0,b) defined
//   Definition 3  modulo-I map; Section 6.1 decides T(q) within I with one reverse
//                 closure seeded by accepting states of kept tokens
//   Section 6     every sweep visits each (state, class) entry a constant number of times
#include "compile.h"

#include <algorithm>
#include <cctype>
#include <cstring>
#include <map>
#include <numeric>

namespace lexc {
namespace {

// ------------------------------------------------------------------ byte sets
struct Set256 {
  uint32_t w[8] = {0};
  void on(unsigned b) { w[b >> 5] |= 1u << (b & 31); }
  void off(unsigned b) { w[b >> 5] &= ~(1u << (b & 31)); }
  bool in(unsigned b) const { return (w[b >> 5] >> (b & 31)) & 1u; }
  void span(unsigned a, unsigned z) {
    for (unsigned b = a; b <= z; ++b) on(b);
  }
  void flip() {
    for (uint32_t &x : w) x = ~x;
  }
  bool none() const {
    for (uint32_t x : w)
      if (x) return false;
    return true;
  }
  bool operator==(const Set256 &o) const { return memcmp(w, o.w, sizeof w) == 0; }
  bool operator<(const Set256 &o) const { return memcmp(w, o.w, sizeof w) < 0; }
};

// ------------------------------------------------------------- regex parser
// Binary syntax tree; bounded repeats are expanded during the position build.
struct Re {
  enum Op { kEps, kSet, kCat, kAlt, kStar, kPlus, kOpt, kRep } op = kEps;
  Set256 set;
  int l = -1, r = -1;
  int lo = 0, hi = 0;  // kRep; hi == -1: unbounded
};

class ReParser {
 public:
  ReParser(const std::string &src, std::vector<Re> &tree) : s_(src), t_(tree) {}
  int run() {
    int root = alt();
    if (root >= 0 && at_ < s_.size()) return bad("unexpected ')'");
    return root;
  }
  const std::string &error() const { return err_; }

 private:
  const std::string &s_;
  std::vector<Re> &t_;
  size_t at_ = 0;
  std::string err_;

  bool more() const { return at_ < s_.size(); }
  unsigned char peek() const { return (unsigned char)s_[at_]; }
  unsigned char take() { return (unsigned char)s_[at_++]; }
  int bad(const char *what) {
    if (err_.empty()) err_ = std::string(what) + " at offset " + std::to_string(at_);
    return -1;
  }
  int node(Re r) {
    t_.push_back(r);
    return (int)t_.size() - 1;
  }
  int bin(Re::Op op, int l, int r) {
    Re x;
    x.op = op;
    x.l = l;
    x.r = r;
    return node(x);
  }
  static int hexdig(unsigned char c) {
    if (c >= '0' && c <= '9') return c - '0';
    c |= 0x20;
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    return -1;
  }
  // Byte denoted by the escape whose backslash was just consumed, or -1.
  int escaped() {
    if (!more()) return bad("trailing backslash");
    unsigned char c = take();
    static const char kFrom[] = "ntrfvb0";
    static const unsigned char kTo[] = {'\n', '\t', '\r', '\f', '\v', '\b', 0};
    if (const char *hit = strchr(kFrom, c); hit && c) return kTo[hit - kFrom];
    if (c == 'x') {
      if (at_ + 2 > s_.size()) return bad("short \\x escape");
      int h = hexdig(take()), l = hexdig(take());
      if (h < 0 || l < 0) return bad("bad \\x escape");
      return h * 16 + l;
    }
    if (isalnum(c)) return bad("unsupported escape");
    return c;
  }
  int alt() {
    int lhs = seq();
    while (lhs >= 0 && more() && peek() == '|') {
      take();
      int rhs = seq();
      if (rhs < 0) return -1;
      lhs = bin(Re::kAlt, lhs, rhs);
    }
    return lhs;
  }
  int seq() {
    int acc = -1;
    while (more() && peek() != '|' && peek() != ')') {
      int f = post();
      if (f < 0) return -1;
      acc = acc < 0 ? f : bin(Re::kCat, acc, f);
    }
    if (acc < 0) acc = node(Re{});  // empty sequence = epsilon
    return acc;
  }
  bool number(int &v) {
    if (!more() || !isdigit(peek())) return false;
    v = 0;
    while (more() && isdigit(peek())) {
      v = v * 10 + (take() - '0');
      if (v > 1000) return false;
    }
    return true;
  }
  int post() {
    int x = prim();
    while (x >= 0 && more()) {
      unsigned char c = peek();
      if (c == '*' || c == '+' || c == '?') {
        take();
        x = bin(c == '*' ? Re::kStar : c == '+' ? Re::kPlus : Re::kOpt, x, -1);
      } else if (c == '{') {
        take();
        Re r;
        r.op = Re::kRep;
        r.l = x;
        if (!number(r.lo)) return bad("bad {m,n}");
        r.hi = r.lo;
        if (more() && peek() == ',') {
          take();
          if (more() && peek() == '}') r.hi = -1;
          else if (!number(r.hi) || r.hi < r.lo) return bad("bad {m,n}");
        }
        if (!more() || take() != '}') return bad("bad {m,n}");
        x = node(r);
      } else {
        break;
      }
    }
    return x;
  }
  int klass() {
    Set256 set;
    bool negate = more() && peek() == '^';
    if (negate) take();
    bool first = true;
    for (;;) {
      if (!more()) return bad("unterminated [");
      unsigned char c = take();
      if (c == ']' && !first) break;
      first = false;
      int lo = c == '\\' ? escaped() : c;
      if (lo < 0) return -1;
      int hi = lo;
      if (at_ + 1 < s_.size() && peek() == '-' && s_[at_ + 1] != ']') {
        take();
        unsigned char d = take();
        hi = d == '\\' ? escaped() : d;
        if (hi < 0) return -1;
        if (hi < lo) return bad("empty range");
      }
      set.span((unsigned)lo, (unsigned)hi);
    }
    if (negate) set.flip();
    if (set.none()) return bad("class matches no byte");
    Re r;
    r.op = Re::kSet;
    r.set = set;
    return node(r);
  }
  int prim() {
    unsigned char c = take();
    switch (c) {
      case '(': {
        int inner = alt();
        if (inner < 0) return -1;
        if (!more() || take() != ')') return bad("missing ')'");
        return inner;
      }
      case '[':
        return klass();
      case '*': case '+': case '?': case '{': case '|': case ')':
        --at_;
        return bad("operator without operand");
      default: {
        Re r;
        r.op = Re::kSet;
        if (c == '.') r.set.span(0, 255);
        else if (c == '\\') {
          int b = escaped();
          if (b < 0) return -1;
          r.set.on((unsigned)b);
        } else {
          r.set.on(c);
        }
        return node(r);
      }
    }
  }
};

// ---------------------------------------------------- Glushkov positions
struct Positions {
  std::vector<Set256> set;      // byte set of each position
  std::vector<int> kind;        // token kind of each position
  std::vector<std::vector<int>> follow;
  std::vector<char> last;       // position ends a word of its kind
};
struct Summary {
  bool nullable = false;
  std::vector<int> first, last;
};

constexpr size_t kMaxPositions = 1u << 16;

bool glushkov(const std::vector<Re> &t, int id, int kind, Positions &P, Summary &out) {
  const Re &r = t[id];
  out = Summary{};
  switch (r.op) {
    case Re::kEps:
      out.nullable = true;
      return true;
    case Re::kSet: {
      if (P.set.size() >= kMaxPositions) return false;
      int p = (int)P.set.size();
      P.set.push_back(r.set);
      P.kind.push_back(kind);
      P.follow.emplace_back();
      P.last.push_back(0);
      out.first = {p};
      out.last = {p};
      return true;
    }
    case Re::kCat: {
      Summary a, b;
      if (!glushkov(t, r.l, kind, P, a) || !glushkov(t, r.r, kind, P, b)) return false;
      for (int x : a.last) P.follow[x].insert(P.follow[x].end(), b.first.begin(), b.first.end());
      out.nullable = a.nullable && b.nullable;
      out.first = a.first;
      if (a.nullable) out.first.insert(out.first.end(), b.first.begin(), b.first.end());
      out.last = b.last;
      if (b.nullable) out.last.insert(out.last.end(), a.last.begin(), a.last.end());
      return true;
    }
    case Re::kAlt: {
      Summary a, b;
      if (!glushkov(t, r.l, kind, P, a) || !glushkov(t, r.r, kind, P, b)) return false;
      out.nullable = a.nullable || b.nullable;
      out.first = a.first;
      out.first.insert(out.first.end(), b.first.begin(), b.first.end());
      out.last = a.last;
      out.last.insert(out.last.end(), b.last.begin(), b.last.end());
      return true;
    }
    case Re::kStar:
    case Re::kPlus:
    case Re::kOpt: {
      Summary a;
      if (!glushkov(t, r.l, kind, P, a)) return false;
      if (r.op != Re::kOpt)
        for (int x : a.last) P.follow[x].insert(P.follow[x].end(), a.first.begin(), a.first.end());
      out = a;
      if (r.op != Re::kPlus) out.nullable = true;
      return true;
    }
    case Re::kRep: {
      // e{lo,hi} = e^lo (e?)^(hi-lo), or e^lo e* when unbounded; each copy gets
      // fresh positions.
      Summary acc;
      acc.nullable = true;
      auto append = [&](const Summary &b) {
        for (int x : acc.last) P.follow[x].insert(P.follow[x].end(), b.first.begin(), b.first.end());
        std::vector<int> first = acc.first;
        if (acc.nullable) first.insert(first.end(), b.first.begin(), b.first.end());
        std::vector<int> last = b.last;
        if (b.nullable) last.insert(last.end(), acc.last.begin(), acc.last.end());
        acc.first = first;
        acc.last = last;
        acc.nullable = acc.nullable && b.nullable;
      };
      for (int k = 0; k < r.lo; ++k) {
        Summary b;
        if (!glushkov(t, r.l, kind, P, b)) return false;
        append(b);
      }
      if (r.hi < 0) {
        Summary b;
        if (!glushkov(t, r.l, kind, P, b)) return false;
        for (int x : b.last) P.follow[x].insert(P.follow[x].end(), b.first.begin(), b.first.end());
        b.nullable = true;
        append(b);
      } else {
        for (int k = r.lo; k < r.hi; ++k) {
          Summary b;
          if (!glushkov(t, r.l, kind, P, b)) return false;
          b.nullable = true;
          append(b);
        }
      }
      out = acc;
      return true;
    }
  }
  return false;
}

void sort_unique(std::vector<int> &v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

// Partition of the 256 bytes into classes that no position set separates.
int byte_classes(const std::vector<Set256> &sets, uint8_t cls[256]) {
  std::vector<int> id(256, 0);
  int n = 1;
  std::vector<Set256> distinct(sets);
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  for (const Set256 &s : distinct) {
    std::map<std::pair<int, bool>, int> remap;
    for (int b = 0; b < 256; ++b) {
      auto key = std::make_pair(id[b], s.in((unsigned)b));
      auto it = remap.find(key);
      if (it == remap.end()) it = remap.emplace(key, (int)remap.size()).first;
      id[b] = it->second;
    }
    n = (int)remap.size();
  }
  for (int b = 0; b < 256; ++b) cls[b] = (uint8_t)id[b];
  return n;
}

constexpr int kMaxStates = 4000;

// Subset construction over position sets.  State 0 is the initial state (the
// pseudo-position "before any byte"), whose successors are the first positions
// of every kind and which accepts the nullable kinds.
bool subset_dfa(const Positions &P, const std::vector<Summary> &kinds, const std::vector<TokDef> &defs,
                Dfa &d, std::string &err) {
  d.nclasses = byte_classes(P.set, d.cls);
  std::vector<int> rep(d.nclasses, -1);
  for (int b = 255; b >= 0; --b) rep[d.cls[b]] = b;
  std::vector<int> init_follow;
  for (const Summary &k : kinds) init_follow.insert(init_follow.end(), k.first.begin(), k.first.end());
  sort_unique(init_follow);

  std::map<std::vector<int>, int> index;
  std::vector<std::vector<int>> states;
  states.push_back({-1});
  index[{-1}] = 0;
  d.next.clear();
  for (size_t q = 0; q < states.size(); ++q) {
    if ((int)states.size() > kMaxStates) {
      err = "automaton exceeds " + std::to_string(kMaxStates) + " states";
      return false;
    }
    d.next.resize((q + 1) * d.nclasses, -1);
    for (int c = 0; c < d.nclasses; ++c) {
      const unsigned b = (unsigned)rep[c];
      std::vector<int> to;
      for (int p : states[q]) {
        const std::vector<int> &succ = p < 0 ? init_follow : P.follow[p];
        for (int x : succ)
          if (P.set[x].in(b)) to.push_back(x);
      }
      if (to.empty()) continue;
      sort_unique(to);
      auto it = index.find(to);
      if (it == index.end()) {
        it = index.emplace(to, (int)states.size()).first;
        states.push_back(to);
      }
      d.next[q * d.nclasses + c] = it->second;
    }
  }
  d.nstates = (int)states.size();
  d.acc.assign(d.nstates, -1);
  auto better = [&](int k, int cur) {
    return cur < 0 || defs[k].priority < defs[cur].priority ||
           (defs[k].priority == defs[cur].priority && k < cur);
  };
  for (int q = 0; q < d.nstates; ++q) {
    int &a = d.acc[q];
    if (q == 0) {
      for (size_t k = 0; k < kinds.size(); ++k)
        if (kinds[k].nullable && better((int)k, a)) a = (int)k;
    } else {
      for (int p : states[q])
        if (P.last[p] && better(P.kind[p], a)) a = P.kind[p];
    }
  }
  return true;
}

// Section 4.1: keep Q+ (forward sweep from q0, reverse sweep from accepting
// states), drop edges leaving it, then minimise.  Minimisation is Hopcroft's
// partition refinement over a completed automaton in which every missing (or
// dead) transition goes to an explicit SINK carrying a label of its own, so a
// missing transition is never identified with any live state.  Returns false
// when q0 is not live.
bool trim_minimise(const Dfa &in, Dfa &out) {
  const int n = in.nstates, C = in.nclasses;
  std::vector<char> fwd(n, 0), bwd(n, 0);
  std::vector<int> stack{0};
  fwd[0] = 1;
  while (!stack.empty()) {
    int q = stack.back();
    stack.pop_back();
    for (int c = 0; c < C; ++c) {
      int t = in.next[q * C + c];
      if (t >= 0 && !fwd[t]) {
        fwd[t] = 1;
        stack.push_back(t);
      }
    }
  }
  // reverse index, built once per class row (Section 6)
  std::vector<std::vector<int>> into(n);
  for (int q = 0; q < n; ++q)
    for (int c = 0; c < C; ++c)
      if (in.next[q * C + c] >= 0) into[in.next[q * C + c]].push_back(q);
  for (int q = 0; q < n; ++q)
    if (in.acc[q] >= 0) {
      bwd[q] = 1;
      stack.push_back(q);
    }
  while (!stack.empty()) {
    int q = stack.back();
    stack.pop_back();
    for (int p : into[q])
      if (!bwd[p]) {
        bwd[p] = 1;
        stack.push_back(p);
      }
  }
  if (!(fwd[0] && bwd[0])) return false;
  std::vector<int> live_id(n, -1);
  std::vector<int> live;
  for (int q = 0; q < n; ++q)
    if (fwd[q] && bwd[q]) {
      live_id[q] = (int)live.size();
      live.push_back(q);
    }
  const int L = (int)live.size();
  const int SINK = L, N = L + 1;
  std::vector<int> f((size_t)N * C);
  for (int i = 0; i < L; ++i)
    for (int c = 0; c < C; ++c) {
      int t = in.next[live[i] * C + c];
      f[(size_t)i * C + c] = (t >= 0 && live_id[t] >= 0) ? live_id[t] : SINK;
    }
  for (int c = 0; c < C; ++c) f[(size_t)SINK * C + c] = SINK;

  // inverse transitions per class
  std::vector<std::vector<std::vector<int>>> inv(C, std::vector<std::vector<int>>(N));
  for (int q = 0; q < N; ++q)
    for (int c = 0; c < C; ++c) inv[c][f[(size_t)q * C + c]].push_back(q);

  // initial partition: by accepting label; SINK alone
  std::vector<int> block(N);
  std::vector<std::vector<int>> members;
  {
    std::map<int, int> bylabel;
    for (int i = 0; i < L; ++i) {
      int lab = in.acc[live[i]];
      auto it = bylabel.find(lab);
      if (it == bylabel.end()) {
        it = bylabel.emplace(lab, (int)members.size()).first;
        members.emplace_back();
      }
      block[i] = it->second;
      members[it->second].push_back(i);
    }
    block[SINK] = (int)members.size();
    members.push_back({SINK});
  }
  std::vector<std::vector<char>> queued;
  std::vector<std::pair<int, int>> work;
  for (int B = 0; B < (int)members.size(); ++B) {
    queued.emplace_back(C, 1);
    for (int c = 0; c < C; ++c) work.emplace_back(B, c);
  }
  std::vector<int> hits(N, 0);
  std::vector<char> marked(N, 0);
  while (!work.empty()) {
    auto [A, c] = work.back();
    work.pop_back();
    queued[A][c] = 0;
    std::vector<int> X;
    for (int t : members[A])
      for (int q : inv[c][t]) X.push_back(q);
    std::vector<int> touched;
    for (int q : X) {
      if (marked[q]) continue;
      marked[q] = 1;
      if (hits[block[q]]++ == 0) touched.push_back(block[q]);
    }
    for (int Y : touched) {
      if (hits[Y] < (int)members[Y].size()) {
        std::vector<int> in_x, out_x;
        for (int q : members[Y]) (marked[q] ? in_x : out_x).push_back(q);
        const int Z = (int)members.size();
        // Y keeps the larger part, Z takes the smaller one
        if (in_x.size() > out_x.size()) std::swap(in_x, out_x);
        members[Y] = out_x;
        members.push_back(in_x);
        for (int q : in_x) block[q] = Z;
        // Hopcroft's rule: if (Y, d) is pending it now stands for the larger
        // half and (Z, d) is added; otherwise the smaller half Z suffices.
        // Either way (Z, d) is enqueued.
        queued.emplace_back(C, 1);
        for (int d = 0; d < C; ++d) work.emplace_back(Z, d);
      }
    }
    for (int q : X) marked[q] = 0;
    for (int Y : touched) hits[Y] = 0;
  }
  // quotient: q0's block first, SINK's block dropped
  const int nb = (int)members.size();
  std::vector<int> newid(nb, -1);
  int k = 0;
  newid[block[live_id[0]]] = k++;
  for (int i = 0; i < L; ++i)
    if (newid[block[i]] < 0) newid[block[i]] = k++;
  out.nstates = k;
  out.nclasses = C;
  memcpy(out.cls, in.cls, sizeof out.cls);
  out.next.assign((size_t)k * C, -1);
  out.acc.assign(k, -1);
  for (int i = 0; i < L; ++i) {
    const int s = newid[block[i]];
    out.acc[s] = in.acc[live[i]];
    for (int c = 0; c < C; ++c) {
      int t = f[(size_t)i * C + c];
      if (t != SINK) out.next[(size_t)s * C + c] = newid[block[t]];
    }
  }
  return true;
}

void bit_on(uint8_t *m, int b) { m[b >> 3] |= (uint8_t)(1u << (b & 7)); }

// Definitions 1-3 on the minimised live automaton, one decision per byte class.
void certify(Compiled &R) {
  const Dfa &d = R.dfa;
  const int n = d.nstates, C = d.nclasses;
  auto step = [&](int q, int c) { return d.next[(size_t)q * C + c]; };
  R.reentrant = false;
  for (int q = 0; q < n && !R.reentrant; ++q)
    for (int c = 0; c < C; ++c)
      if (step(q, c) == 0) {
        R.reentrant = true;
        break;
      }
  // kept_reach[q]: some accepting state of a kept kind is reachable from q, i.e.
  // T(q) is not within I.  One backward closure from the kept accepting states.
  std::vector<std::vector<int>> into(n);
  for (int q = 0; q < n; ++q)
    for (int c = 0; c < C; ++c)
      if (step(q, c) >= 0) into[step(q, c)].push_back(q);
  std::vector<char> kept_reach(n, 0);
  std::vector<int> stack;
  for (int q = 0; q < n; ++q)
    if (d.acc[q] >= 0 && !R.discard[d.acc[q]]) {
      kept_reach[q] = 1;
      stack.push_back(q);
    }
  while (!stack.empty()) {
    int q = stack.back();
    stack.pop_back();
    for (int p : into[q])
      if (!kept_reach[p]) {
        kept_reach[p] = 1;
        stack.push_back(p);
      }
  }
  std::vector<char> ex(C, 1), mo(C, 1), live0(C, 0);
  for (int c = 0; c < C; ++c) {
    const int t0 = step(0, c);
    live0[c] = t0 >= 0;
    for (int q = 0; q < n; ++q) {
      const int t = step(q, c);
      if (t < 0) continue;
      const bool clause_a = q == 0 && !R.reentrant;
      const bool clause_c = d.acc[q] >= 0 && t0 >= 0 && t == t0 && !kept_reach[q];
      if (!clause_a) ex[c] = 0;
      if (!clause_a && !clause_c) mo[c] = 0;
    }
  }
  memset(R.exact_raw, 0, 32);
  memset(R.discard_raw, 0, 32);
  memset(R.exact_useful, 0, 32);
  memset(R.discard_useful, 0, 32);
  memset(R.q0_live_bytes, 0, 32);
  for (int b = 0; b < 256; ++b) {
    const int c = d.cls[b];
    if (ex[c]) bit_on(R.exact_raw, b);
    if (mo[c]) bit_on(R.discard_raw, b);
    if (live0[c]) bit_on(R.q0_live_bytes, b);
    if (ex[c] && live0[c]) bit_on(R.exact_useful, b);
    if (mo[c] && live0[c]) bit_on(R.discard_useful, b);
  }
  R.monotone = true;
  for (int q = 0; q < n; ++q) {
    if (d.acc[q] < 0) continue;
    for (int c = 0; c < C; ++c) {
      int t = step(q, c);
      if (t >= 0 && d.acc[t] < 0) R.monotone = false;
    }
  }
}

// Packs the walker tables (layout in compile.h).  The start row is q0's row
// without q0's own accepting label: a token never has length zero (Section 3).
void pack(Compiled &R) {
  const Dfa &d = R.dfa;
  const int S = R.q0_live ? d.nstates : 0;
  R.row_sink = 1 + S;
  R.row_fail = R.monotone ? -1 : 2 + S;
  R.nrows = R.monotone ? 2 + S : 3 + S;
  const uint32_t sink = row_state(R.row_sink);
  const uint32_t fail = R.monotone ? sink : row_state(R.row_fail);
  auto row_of = [](int q) { return row_state(1 + q); };
  R.rowkind.assign(R.nrows, 0xFF);
  for (int q = 0; q < S; ++q)
    if (d.acc[q] >= 0) R.rowkind[1 + q] = (uint8_t)d.acc[q];
  for (int mode = 0; mode < 2; ++mode) {
    auto counted = [&](int kind) { return mode == 0 || !R.discard[kind]; };
    std::vector<uint32_t> &T = R.table[mode];
    T.assign((size_t)R.nrows * 256, 0);
    auto enter = [&](int t) { return row_of(t) | (d.acc[t] >= 0 ? kAcc : 0u); };
    auto at = [&](int row, int b) -> uint32_t & { return T[(size_t)row * 256 + (b ^ row_swizzle(row))]; };
    for (int b = 0; b < 256; ++b) {
      const int c = d.cls[b];
      const int t0 = S ? d.next[c] : -1;
      at(0, b) = t0 >= 0 ? enter(t0) : sink;
      for (int q = 0; q < S; ++q) {
        const int t = d.next[(size_t)q * d.nclasses + c];
        uint32_t e;
        if (t >= 0) {
          e = enter(t);
        } else if (d.acc[q] >= 0) {
          e = kEmit | ((uint32_t)d.acc[q] << kKindShift) | (counted(d.acc[q]) ? kCount : 0u) |
              (t0 >= 0 ? enter(t0) : sink);
        } else {
          e = fail;
        }
        at(1 + q, b) = e;
      }
      at(R.row_sink, b) = sink;
      if (!R.monotone) at(R.row_fail, b) = fail;
    }
    std::vector<uint8_t> &I = R.rowinfo[mode];
    I.assign(R.nrows, 0);
    for (int q = 0; q < S; ++q)
      if (d.acc[q] >= 0) I[1 + q] = kInfoAcc | (counted(d.acc[q]) ? kInfoCount : 0);
  }
}

bool finish(Compiled &R, const Dfa &raw, std::string &err) {
  Dfa m;
  R.q0_live = trim_minimise(raw, m);
  if (!R.q0_live) {
    // the token set accepts nothing: every byte is certified, none usefully
    memset(R.exact_raw, 0xFF, 32);
    memset(R.discard_raw, 0xFF, 32);
    R.dfa = Dfa{};
    R.monotone = true;
    R.reentrant = false;
  } else {
    R.dfa = m;
    certify(R);
  }
  pack(R);
  if (R.nrows > kMaxRows) {
    err = "too many states for the packed table";
    return false;
  }
  return true;
}

}  // namespace

bool compile_defs(const std::vector<TokDef> &defs, Compiled &R, std::string &err) {
  if (defs.empty() || defs.size() > 255) {
    err = "need 1..255 token definitions";
    return false;
  }
  Positions P;
  std::vector<Summary> kinds(defs.size());
  R = Compiled{};
  R.nkinds = (int)defs.size();
  for (size_t k = 0; k < defs.size(); ++k) {
    std::vector<Re> tree;
    ReParser parser(defs[k].pattern, tree);
    int root = parser.run();
    if (root < 0) {
      err = "definition " + std::to_string(k) + ": " + parser.error();
      return false;
    }
    if (defs[k].exclude >= 0)
      for (Re &x : tree)
        if (x.op == Re::kSet) x.set.off((unsigned)defs[k].exclude);
    if (!glushkov(tree, root, (int)k, P, kinds[k])) {
      err = "definition " + std::to_string(k) + ": pattern too large";
      return false;
    }
    for (int x : kinds[k].last) P.last[x] = 1;
    R.discard.push_back(defs[k].discard ? 1 : 0);
  }
  for (auto &f : P.follow) sort_unique(f);
  Dfa raw;
  if (!subset_dfa(P, kinds, defs, raw, err)) return false;
  return finish(R, raw, err);
}

bool compile_table(int nstates, int q0, const int32_t *next, const int32_t *accept,
                   const std::vector<uint8_t> &discard, Compiled &R, std::string &err) {
  R = Compiled{};
  if (nstates <= 0 || nstates > kMaxStates || q0 < 0 || q0 >= nstates) {
    err = "bad state count or initial state";
    return false;
  }
  R.nkinds = (int)discard.size();
  R.discard = discard;
  // Renumber so that q0 is state 0; classes = identical byte columns.
  std::vector<int> ren(nstates);
  std::iota(ren.begin(), ren.end(), 0);
  std::swap(ren[0], ren[q0]);  // ren[old] = new
  Dfa raw;
  raw.nstates = nstates;
  std::map<std::vector<int32_t>, int> colid;
  for (int b = 0; b < 256; ++b) {
    std::vector<int32_t> col(nstates);
    for (int q = 0; q < nstates; ++q) {
      int32_t t = next[(size_t)q * 256 + b];
      if (t < -1 || t >= nstates) {
        err = "transition target out of range";
        return false;
      }
      col[ren[q]] = t < 0 ? -1 : ren[t];
    }
    auto it = colid.find(col);
    if (it == colid.end()) it = colid.emplace(col, (int)colid.size()).first;
    raw.cls[b] = (uint8_t)it->second;
  }
  raw.nclasses = (int)colid.size();
  raw.next.assign((size_t)nstates * raw.nclasses, -1);
  for (auto &kv : colid)
    for (int q = 0; q < nstates; ++q) raw.next[(size_t)q * raw.nclasses + kv.second] = kv.first[q];
  raw.acc.assign(nstates, -1);
  for (int q = 0; q < nstates; ++q) {
    int a = accept[q];
    if (a < -1 || a >= R.nkinds || a > 254) {
      err = "accepting token out of range";
      return false;
    }
    raw.acc[ren[q]] = a;
  }
  return finish(R, raw, err);
}

}  // namespace lexc
