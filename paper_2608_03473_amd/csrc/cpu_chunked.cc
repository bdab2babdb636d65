// cpu_chunked.cc -- the multithreaded chunked lexer on the host CPU cores: a baseline to
// time the GPU path against, never called by any GPU entry point (lex_run and the batch
// entry points have no CPU fallback).
//
// It is the paper's executor (Section 6): an equal-division plan cuts the buffer before
// the first useful certified byte at or after each multiple of the chunk length L
// (Definition 2 with Corollary 2 in exact mode, Definition 3 with Proposition 2 modulo I);
// worker threads take chunks from an atomic counter and scan each one from the start
// state with the longest-match loop of Section 3, treating the chunk's end as the end of
// input; the per-chunk (kind, length) streams are then concatenated in chunk order, up to
// and including the first chunk that halts (Corollary 1), whose halt offset is con(w).
// By Theorem 1 and Theorem 3 the result is the serial scan's.
//
// The scan walks the library's packed table of the mode (compile.h): one u32 per (row,
// byte) holding the next row, the COUNT / EMIT / ACC flags and the emitted kind, so a
// byte costs one dependent load from a table of nrows KiB that stays in L1.  A monotone
// automaton (no live edge from an accepting to a non-accepting state) never falls back,
// and its loop writes every step's candidate token and advances the output count by the
// COUNT bit, with no branch per byte.  A non-monotone automaton keeps the last accepting
// position and re-scans from it when the walk reaches the FAIL row (plain backtracking:
// the baseline does not bound failed lookahead).
//
// Outputs: each chunk writes its tokens into the caller's arrays at the chunk's own byte
// offset (a chunk of m bytes has at most m tokens), then the chunks are compacted to their
// final offsets.  Every destination lies at or before its source, so a chunk is moved once
// every earlier chunk whose source its destination overlaps has been moved.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/lex.h"
#include "compile.h"

namespace lexcpu {

struct Walker {
  const uint8_t *table;  // packed table as bytes: entry of (state, b) at state ^ (b << 2)
  const uint8_t *rowinfo;
  const uint8_t *rowkind;
  uint32_t sink, fail;   // row states (entry & kStateMask form)
  bool mono;
};

inline uint32_t entry(const Walker &w, uint32_t st, uint8_t b) {
  uint32_t x;
  memcpy(&x, w.table + (st ^ ((uint32_t)b << 2)), 4);
  return x;
}

inline uint32_t row_of(uint32_t st) { return st >> lexc::kRowShift; }

struct Slice {
  uint64_t ntok = 0;
  uint64_t halt = UINT64_MAX;  // absolute halt offset, or none
};

// Scans w[s, e) from the start state with e as end of input; writes tokens at kinds[s..],
// lens[s..] (at most e - s of them).
Slice scan_slice(const Walker &W, const uint8_t *in, uint64_t s, uint64_t e, uint8_t *kinds, uint32_t *lens) {
  Slice out;
  uint8_t *ko = kinds + s;
  uint32_t *lo = lens + s;
  uint64_t cnt = 0, tok = s;
  uint32_t st = 0;  // row 0: token start
  if (W.mono) {
    for (uint64_t p = s; p < e; ++p) {
      const uint32_t x = entry(W, st, in[p]);
      const uint32_t emit = (x >> 1) & 1;
      // a candidate token (kind, p - tok) at slot cnt; kept iff COUNT (which implies EMIT)
      ko[cnt] = (uint8_t)(x >> lexc::kKindShift);
      lo[cnt] = (uint32_t)(p - tok);
      cnt += x & 1;
      tok = emit ? p : tok;
      st = x & lexc::kStateMask;
      if (__builtin_expect(st == W.sink, 0)) break;
    }
  } else {
    uint64_t lacc = s;  // position after the last accepting step of the current token
    uint32_t lrow = 0;  // the accepting row reached there
    uint64_t p = s;
    for (;;) {
      bool fall = false;
      if (p == e) {  // end of input inside a token that is not accepting: fall back
        if (st == 0 || st == W.sink || (W.rowinfo[row_of(st)] & lexc::kInfoAcc)) break;
        fall = true;
      } else {
        const uint32_t x = entry(W, st, in[p]);
        if (x & lexc::kEmit) {
          if (x & lexc::kCount) {
            ko[cnt] = (uint8_t)(x >> lexc::kKindShift);
            lo[cnt] = (uint32_t)(p - tok);
            ++cnt;
          }
          tok = p;
        }
        st = x & lexc::kStateMask;
        ++p;
        if (x & lexc::kAcc) lacc = p, lrow = st;
        if (st == W.sink) break;
        fall = st == W.fail;  // no longer a token: fall back to the last accepting position
      }
      if (fall) {
        if (lacc <= tok) {  // no accepting prefix since the token started: halt there
          st = W.sink;
          break;
        }
        const uint32_t r = row_of(lrow);
        if (W.rowinfo[r] & lexc::kInfoCount) {
          ko[cnt] = W.rowkind[r];
          lo[cnt] = (uint32_t)(lacc - tok);
          ++cnt;
        }
        tok = p = lacc;
        st = 0;
      }
    }
  }
  if (st == W.sink) {
    out.halt = tok;
  } else if (st != 0) {
    const uint32_t r = row_of(st);
    if (W.rowinfo[r] & lexc::kInfoAcc) {
      if (W.rowinfo[r] & lexc::kInfoCount) {
        ko[cnt] = W.rowkind[r];
        lo[cnt] = (uint32_t)(e - tok);
        ++cnt;
      }
    } else {
      out.halt = tok;  // monotone: no accepting prefix of the pending token
    }
  }
  out.ntok = cnt;
  return out;
}

}  // namespace lexcpu

// Internal access to a compiled lexer's host tables (defined in runtime.hip).
const lexc::Compiled &lex_compiled(const lex_dfa *d);

extern "C" int lex_cpu_chunked(const lex_dfa *d, const uint8_t *bytes, uint64_t n, int mode, uint8_t *kinds,
                               uint32_t *lens, uint64_t cap, uint64_t chunk_bytes, uint32_t nthreads,
                               lex_result *result) {
  if (!d || !result || (!bytes && n) || mode < 0 || mode > 2) return LEX_EINVAL;
  if (n && (!kinds || !lens || cap < n)) return LEX_EINVAL;
  if (n > 0xFFFFFFF0ull) return LEX_ELIMIT;
  const lexc::Compiled &c = lex_compiled(d);
  const int m = mode & 1;
  lexcpu::Walker W;
  W.table = reinterpret_cast<const uint8_t *>(c.table[m].data());
  W.rowinfo = c.rowinfo[m].data();
  W.rowkind = c.rowkind.data();
  W.sink = lexc::row_state(c.row_sink);
  W.fail = c.row_fail >= 0 ? lexc::row_state(c.row_fail) : W.sink;
  W.mono = c.monotone;
  const uint8_t *map = m ? c.discard_useful : c.exact_useful;
  bool cert[256], any = false;
  for (int b = 0; b < 256; ++b) any |= (cert[b] = (map[b >> 3] >> (b & 7)) & 1);
  if (mode == LEX_MODE_SERIAL) any = false;
  const uint64_t L = chunk_bytes ? chunk_bytes : 64 << 10;
  unsigned T = nthreads ? nthreads : std::max(1u, std::thread::hardware_concurrency());

  // Equal-division plan: the first useful certified byte at or after each k * L.
  std::vector<uint64_t> cuts{0};
  if (any && n > L) {
    for (uint64_t t = L; t < n; t += L) {
      uint64_t x = std::max(t, cuts.back());
      while (x < n && !cert[bytes[x]]) ++x;
      if (x >= n) break;
      if (x > cuts.back()) cuts.push_back(x);
    }
  }
  cuts.push_back(n);
  const size_t K = cuts.size() - 1;
  std::vector<lexcpu::Slice> sl(K);
  T = (unsigned)std::min<size_t>(T, std::max<size_t>(K, 1));

  // Scan: workers take chunks in order from a counter.
  std::atomic<size_t> next{0};
  auto scan_worker = [&]() {
    for (size_t j; (j = next.fetch_add(1, std::memory_order_relaxed)) < K;)
      sl[j] = lexcpu::scan_slice(W, bytes, cuts[j], cuts[j + 1], kinds, lens);
  };
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < T; ++i) pool.emplace_back(scan_worker);
  scan_worker();
  for (auto &t : pool) t.join();
  pool.clear();

  // Concatenation up to the first halting chunk (Corollary 1).
  size_t keep = K;
  uint64_t con = n;
  for (size_t j = 0; j < K; ++j)
    if (sl[j].halt != UINT64_MAX) {
      keep = j + 1;
      con = sl[j].halt;
      break;
    }
  std::vector<uint64_t> dst(keep + 1, 0);
  for (size_t j = 0; j < keep; ++j) dst[j + 1] = dst[j] + sl[j].ntok;
  std::vector<std::atomic<uint8_t>> moved(keep);
  for (auto &f : moved) f.store(0, std::memory_order_relaxed);
  next.store(0);
  auto move_worker = [&]() {
    for (size_t j; (j = next.fetch_add(1, std::memory_order_relaxed)) < keep;) {
      const uint64_t src = cuts[j], to = dst[j], cnt = sl[j].ntok;
      // earlier chunks whose tokens still sit where this chunk's go must have moved
      for (size_t i = 0; i < j && cuts[i] < to + cnt; ++i)
        while (!moved[i].load(std::memory_order_acquire)) std::this_thread::yield();
      if (cnt && src != to) {
        memmove(kinds + to, kinds + src, cnt);
        memmove(lens + to, lens + src, cnt * 4);
      }
      moved[j].store(1, std::memory_order_release);
    }
  };
  for (unsigned i = 1; i < T; ++i) pool.emplace_back(move_worker);
  move_worker();
  for (auto &t : pool) t.join();

  result->ntokens = dst[keep];
  result->error_offset = con;
  result->status = LEX_OK;
  result->nslices = (uint32_t)K;
  return LEX_OK;
}
