/*
 * gen.c -- seeded synthetic inputs shaped like the paper's workloads.
 *
 * Input generation only: nothing here lexes, classifies or certifies.  Both the
 * library's tests/benchmarks and the oracle's tests draw their inputs from here.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014).  Distributions are
 * written out below rather than taken from a standard library, so a corpus is
 * the same byte for byte on every platform:
 *   uniform [0,1)      u = (x >> 11) * 2^-53
 *   geometric, mean m  on {1,2,..}: ceil(ln u / ln(1 - 1/m))   (u in (0,1))
 *   geometric0, mean m on {0,1,..}: geometric(m + 1) - 1
 *   Poisson(l)         Knuth's product-of-uniforms method
 *   normal             Box-Muller
 *   log-normal         exp(ln(median) + sigma * z)
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
  uint64_t s;
} rng_t;

static uint64_t next64(rng_t *r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double unif(rng_t *r) { return (double)(next64(r) >> 11) * (1.0 / 9007199254740992.0); }
static double unif_pos(rng_t *r) { /* (0, 1) */
  double u;
  do u = unif(r);
  while (u <= 0.0);
  return u;
}
static uint64_t below(rng_t *r, uint64_t n) { return (uint64_t)(unif(r) * (double)n); }
static uint64_t geometric(rng_t *r, double mean) {
  if (mean <= 1.0) return 1;
  double g = ceil(log(unif_pos(r)) / log(1.0 - 1.0 / mean));
  if (g < 1.0) g = 1.0;
  if (g > 1e9) g = 1e9;
  return (uint64_t)g;
}
static uint64_t geometric0(rng_t *r, double mean) { return geometric(r, mean + 1.0) - 1; }
static uint64_t poisson(rng_t *r, double lambda) {
  double L = exp(-lambda), p = 1.0;
  uint64_t k = 0;
  do {
    ++k;
    p *= unif(r);
  } while (p > L);
  return k - 1;
}
static double normal(rng_t *r) {
  double u1 = unif_pos(r), u2 = unif(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ------------------------------------------------------------ output buffer */
typedef struct {
  uint8_t *p;
  uint64_t n, cap;
} out_t;
static int put(out_t *o, uint8_t c) {
  if (o->n >= o->cap) return 0;
  o->p[o->n++] = c;
  return 1;
}
static int puts_(out_t *o, const char *s) {
  while (*s)
    if (!put(o, (uint8_t)*s++)) return 0;
  return 1;
}

static const char *const OPS[24] = {"+", "-", "*", "/", "%", "=", "==", "!=", "<", "<=", ">", ">=",
                                    "&&", "||", "!", "(", ")", "{", "}", "[", "]", ";", ",", "."};
static const char ALPHA[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz_";
static const char ALNUM[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789_";

static uint8_t printable(rng_t *r) { return (uint8_t)(0x20 + below(r, 0x7F - 0x20)); }

/* One C-like line into o (without its newline).  Returns 0 if it did not fit.
 * Kinds: IDENT .35, INT .15, OP .25, STR .05, LCOMMENT .05 (+ BCOMMENT .05 when
 * block comments are enabled), normalised; a line comment ends the line.  When *rs is
 * set and the line has a token, the record separator 0x1E goes right before its first
 * token (a token boundary: the byte before is the previous line's newline) and *rs is
 * cleared. */
static int clike_line(rng_t *r, out_t *o, int bcomment, int *rs) {
  uint64_t k = poisson(r, 8.0);
  const double w[6] = {0.35, 0.15, 0.25, 0.05, 0.05, 0.05};
  const int nk = bcomment ? 6 : 5;
  double tot = 0;
  for (int i = 0; i < nk; ++i) tot += w[i];
  for (uint64_t t = 0; t < k; ++t) {
    if (!t && *rs) {
      if (!put(o, 0x1E)) return 0;
      *rs = 0;
    }
    if (t) {
      uint64_t sp = 1 + below(r, 4);
      for (uint64_t s = 0; s < sp; ++s)
        if (!put(o, unif(r) < 0.9 ? ' ' : '\t')) return 0;
    }
    double u = unif(r) * tot;
    int kind = 0;
    while (kind < nk - 1 && u >= w[kind]) u -= w[kind++];
    switch (kind) {
      case 0: { /* IDENT */
        uint64_t len = geometric(r, 6.0);
        if (!put(o, (uint8_t)ALPHA[below(r, sizeof ALPHA - 1)])) return 0;
        for (uint64_t i = 1; i < len; ++i)
          if (!put(o, (uint8_t)ALNUM[below(r, sizeof ALNUM - 1)])) return 0;
        break;
      }
      case 1: { /* INT */
        uint64_t len = geometric(r, 3.0);
        for (uint64_t i = 0; i < len; ++i)
          if (!put(o, (uint8_t)('0' + below(r, 10)))) return 0;
        break;
      }
      case 2: /* OP */
        if (!puts_(o, OPS[below(r, 24)])) return 0;
        break;
      case 3: { /* STR */
        static const char esc[] = "ntr0\"\\";
        uint64_t items = geometric0(r, 8.0);
        if (!put(o, '"')) return 0;
        for (uint64_t i = 0; i < items; ++i) {
          if (unif(r) < 0.9) {
            uint8_t c;
            do c = printable(r);
            while (c == '"' || c == '\\');
            if (!put(o, c)) return 0;
          } else {
            if (!put(o, '\\') || !put(o, (uint8_t)esc[below(r, 6)])) return 0;
          }
        }
        if (!put(o, '"')) return 0;
        break;
      }
      case 4: { /* LCOMMENT, ends the line */
        uint64_t len = geometric0(r, 20.0);
        if (!puts_(o, "//")) return 0;
        for (uint64_t i = 0; i < len; ++i)
          if (!put(o, printable(r))) return 0;
        return 1;
      }
      case 5: { /* BCOMMENT: printable bytes plus newline, never forming the closer */
        uint64_t len = geometric0(r, 40.0);
        uint8_t prev = '*'; /* the opener's star: the body may not start with '/' */
        if (!puts_(o, "/*")) return 0;
        for (uint64_t i = 0; i < len; ++i) {
          uint8_t c;
          do c = unif(r) < 0.05 ? '\n' : printable(r);
          while (prev == '*' && c == '/');
          if (!put(o, c)) return 0;
          prev = c;
        }
        if (!puts_(o, "*/")) return 0;
        break;
      }
    }
  }
  return 1;
}

/* C-like corpus of exactly n bytes: lines of Poisson(8) tokens separated by
 * runs of 1-4 spaces/tabs, each line ended by a newline; the tail that cannot
 * hold another whole line is padded with newlines.  frame > 0: a framed
 * document, records of frame lines each opened by 0x1E before their first token
 * (deferred to the next line that has one); no other byte of the corpus is 0x1E. */
void wl_clike(uint8_t *buf, uint64_t n, uint64_t seed, int bcomment, uint64_t frame) {
  rng_t r = {seed};
  out_t o = {buf, 0, n};
  int rs = 0;
  for (uint64_t line = 0;; ++line) {
    uint64_t mark = o.n;
    if (frame && line % frame == 0) rs = 1;
    if (!clike_line(&r, &o, bcomment, &rs) || !put(&o, '\n')) {
      o.n = mark;
      break;
    }
  }
  memset(buf + o.n, '\n', n - o.n);
}

/* ------------------------------------------------------------------- JSON */
static int indent(out_t *o, int k) {
  for (int i = 0; i < k; ++i)
    if (!put(o, ' ')) return 0;
  return 1;
}
static int json_value(rng_t *r, out_t *o, int depth);

static int json_container(rng_t *r, out_t *o, int depth, int is_obj) {
  uint64_t m = 1 + below(r, 8);
  if (!puts_(o, is_obj ? "{\n" : "[\n")) return 0;
  for (uint64_t i = 0; i < m; ++i) {
    if (i && !puts_(o, ",\n")) return 0;
    if (!indent(o, 2 * (depth + 1))) return 0;
    if (is_obj) {
      uint64_t kl = 3 + below(r, 10);
      if (!put(o, '"')) return 0;
      for (uint64_t j = 0; j < kl; ++j)
        if (!put(o, (uint8_t)ALPHA[below(r, 52)])) return 0;
      if (!puts_(o, "\": ")) return 0;
    }
    if (!json_value(r, o, depth + 1)) return 0;
  }
  if (!put(o, '\n') || !indent(o, 2 * depth) || !put(o, is_obj ? '}' : ']')) return 0;
  return 1;
}

/* A value at nesting depth `depth`: top-level containers have depth 0 and a
 * container may open at depths 0..5, so containers nest at most 6 deep; a
 * nested value drawn at depth 6 is re-drawn among the leaves. */
static int json_value(rng_t *r, out_t *o, int depth) {
  double u = unif(r);
  if (u >= 0.8 && depth >= 6) u = unif(r) * 0.8; /* re-draw among the leaves */
  if (u < 0.40) {                                 /* string */
    static const char *const esc[] = {"\\\"", "\\\\", "\\/", "\\b", "\\f", "\\n", "\\r", "\\t"};
    static const char HEX[] = "0123456789abcdefABCDEF";
    uint64_t items = geometric0(r, 12.0);
    if (!put(o, '"')) return 0;
    for (uint64_t i = 0; i < items; ++i) {
      if (unif(r) < 0.95) {
        uint8_t c;
        do c = printable(r);
        while (c == '"' || c == '\\');
        if (!put(o, c)) return 0;
      } else {
        uint64_t e = below(r, 9);
        if (e < 8) {
          if (!puts_(o, esc[e])) return 0;
        } else {
          if (!puts_(o, "\\u")) return 0;
          for (int h = 0; h < 4; ++h)
            if (!put(o, (uint8_t)HEX[below(r, 22)])) return 0;
        }
      }
    }
    return put(o, '"');
  }
  if (u < 0.70) { /* number */
    if (unif(r) < 0.3 && !put(o, '-')) return 0;
    if (unif(r) < 0.1) {
      if (!put(o, '0')) return 0;
    } else {
      uint64_t d = below(r, 6);
      if (!put(o, (uint8_t)('1' + below(r, 9)))) return 0;
      for (uint64_t i = 0; i < d; ++i)
        if (!put(o, (uint8_t)('0' + below(r, 10)))) return 0;
    }
    if (unif(r) < 0.4) {
      uint64_t d = 1 + below(r, 6);
      if (!put(o, '.')) return 0;
      for (uint64_t i = 0; i < d; ++i)
        if (!put(o, (uint8_t)('0' + below(r, 10)))) return 0;
    }
    if (unif(r) < 0.1) {
      uint64_t d = 1 + below(r, 3);
      if (!put(o, unif(r) < 0.5 ? 'e' : 'E')) return 0;
      double s = unif(r);
      if (s < 1.0 / 3 && !put(o, '+')) return 0;
      if (s >= 1.0 / 3 && s < 2.0 / 3 && !put(o, '-')) return 0;
      for (uint64_t i = 0; i < d; ++i)
        if (!put(o, (uint8_t)('0' + below(r, 10)))) return 0;
    }
    return 1;
  }
  if (u < 0.80) { /* keyword */
    static const char *const kw[] = {"true", "false", "null"};
    return puts_(o, kw[below(r, 3)]);
  }
  return json_container(r, o, depth, unif(r) < 0.5);
}

/* Pretty-printed JSON of exactly n bytes: top-level objects/arrays separated by
 * newlines (2-space indent); the tail is padded with newlines. */
void wl_json(uint8_t *buf, uint64_t n, uint64_t seed) {
  rng_t r = {seed};
  out_t o = {buf, 0, n};
  for (;;) {
    uint64_t mark = o.n;
    if (!json_container(&r, &o, 0, unif(&r) < 0.5) || !put(&o, '\n')) {
      o.n = mark;
      break;
    }
  }
  memset(buf + o.n, '\n', n - o.n);
}

/* --------------------------------------------------------- scalar draws */
void wl_lognormal_sizes(uint64_t *out, uint64_t count, double median, double sigma, uint64_t lo,
                        uint64_t hi, uint64_t seed) {
  rng_t r = {seed};
  for (uint64_t i = 0; i < count; ++i) {
    double v = exp(log(median) + sigma * normal(&r));
    if (v < (double)lo) v = (double)lo;
    if (v > (double)hi) v = (double)hi;
    out[i] = (uint64_t)llround(v);
  }
}
void wl_uniform(double *out, uint64_t count, uint64_t seed) {
  rng_t r = {seed};
  for (uint64_t i = 0; i < count; ++i) out[i] = unif(&r);
}
void wl_exponential(double *out, uint64_t count, double rate, uint64_t seed) {
  rng_t r = {seed};
  for (uint64_t i = 0; i < count; ++i) out[i] = -log(unif_pos(&r)) / rate;
}
/* Seed of the i-th sub-stream of `seed` (one SplitMix64 output). */
uint64_t wl_substream(uint64_t seed, uint64_t i) {
  rng_t r = {seed ^ (0xD1B54A32D192ED03ull * (i + 1))};
  return next64(&r);
}
