/*
 * oracle.h -- reference (test-only) implementation of certified-split lexing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing under oracle/ is part of the product:
 * only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * Everything here is plain, serial and slow on purpose:
 *   - the lexer matches every token definition directly by simulating one
 *     Thompson NFA per kind (Section 3, the longest-match scanner with the
 *     priority tie-break), never a DFA;
 *   - the certificate checker builds its own automaton (union NFA ->
 *     subset construction -> trim to the live subautomaton -> Moore
 *     refinement) and evaluates Definitions 1-3 literally;
 *   - the chunked checker lexes each slice as a whole input and applies
 *     the truncation rule of Corollary 1.
 *
 * Conventions
 *   kinds are u8 (at most 255 definitions), lengths are u32;
 *   a return value < 0 is an error (see ORC_E*), errors carry a message in
 *   the caller's buffer.
 */
#ifndef PAPER_ORACLE_H
#define PAPER_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,   /* bad argument */
  ORC_ESYNTAX = -2,  /* pattern does not parse */
  ORC_ECAP = -3,     /* output capacity too small */
  ORC_ELIMIT = -4    /* too many kinds / states */
};

/* One token definition: a byte regex, its tie-break priority (lower wins a
 * same-length tie, then the lower index), and whether the kind is in the
 * discarded set I (Section 5). */
typedef struct {
  const char *pattern;
  int32_t priority;
  uint8_t discard;
} orc_def;

typedef struct orc_set orc_set;

/* Parse every pattern and build its Thompson NFA.  NULL on error (message in
 * err).  The set is immutable afterwards. */
orc_set *orc_compile(const orc_def *defs, uint32_t ndefs, char *err, size_t errlen);
/* Framing at the producer (Section 7.1): the byte r is reserved -- removed from every
 * byte class of every pattern, so no token contains it -- and given a kind of its own,
 * kind ndefs, whose only word is r (priority 0, discarded iff r_discard). */
orc_set *orc_compile_framed(const orc_def *defs, uint32_t ndefs, uint32_t r, int r_discard, char *err,
                            size_t errlen);
void orc_free(orc_set *s);
uint32_t orc_nkinds(const orc_set *s);

/* Serial maximal-munch scan of w[0, n) (Section 3).  Writes up to cap tokens;
 * *ntok receives the number of tokens emitted (before any discard filter
 * when discard_filter == 0; kept tokens only when it is 1, i.e. the image
 * pi_I of Section 5), *con the final committed offset con(w).  If offs is
 * non-NULL the start offset of each written token is stored there.
 * Returns ORC_OK, or ORC_ECAP when more than cap tokens would be written
 * (*ntok still holds the full count). */
int orc_lex(const orc_set *s, const uint8_t *w, uint64_t n, int discard_filter,
            uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
            uint64_t *ntok, uint64_t *con);

/* Certificate summary. Bit b of a 32-byte map is (map[b >> 3] >> (b & 7)) & 1. */
typedef struct {
  uint8_t exact_raw[32];      /* Definition 2, vacuous symbols included      */
  uint8_t discard_raw[32];    /* Definition 3, vacuous symbols included      */
  uint8_t exact_useful[32];   /* Corollary 2: exact_raw  AND q0-live bytes   */
  uint8_t discard_useful[32]; /* Proposition 2: discard_raw AND q0-live      */
  uint8_t q0_live[32];        /* bytes b with delta+(q0, b) defined          */
  uint8_t consumed[32];       /* bytes some live state consumes live         */
  int32_t nstates;            /* states of the trimmed, minimised automaton  */
  int32_t q0_live_state;      /* 1 if q0 is in Q+                            */
  int32_t reentrant;          /* Definition 1                                */
  int32_t reserved;
} orc_cert_info;

/* Certificates of a compiled token set (Sections 4 and 6). */
int orc_cert(const orc_set *s, orc_cert_info *out);

/* Certificates of a hand-built automaton, as in the examples of Section 4.1:
 * next[q * 256 + b] is the target state or -1, accept[q] the token of an
 * accepting state or -1, discard[t] marks t in I (ntok entries). */
int orc_cert_table(int32_t nstates, int32_t q0, const int32_t *next, const int32_t *accept,
                   const uint8_t *discard, int32_t ntok, orc_cert_info *out);

/* Witness of Theorem 2 for a byte b that some live state consumes but that
 * is not certified: writes w = u b v into out (capacity cap) and the offset
 * |u| of the occurrence of b.  Returns the length of w, 0 if b is certified
 * or not consumed live, or a negative error. */
int64_t orc_witness(const orc_set *s, int b, uint8_t *out, uint64_t cap, uint64_t *b_offset);

/* Chunked scan (Theorems 1 and 3, Corollary 1): cuts[0..ncuts) are strictly
 * increasing interior offsets in (0, n).  Each slice is scanned as a whole
 * input; the per-slice streams are concatenated in order and truncated after
 * the first slice that does not consume its whole length, whose halt offset
 * is reported in *err_off (n when every slice is consumed).  discard_filter
 * as in orc_lex. */
int orc_lex_chunked(const orc_set *s, const uint8_t *w, uint64_t n, const uint64_t *cuts,
                    uint64_t ncuts, int discard_filter, uint8_t *kinds, uint32_t *lens,
                    uint64_t cap, uint64_t *ntok, uint64_t *err_off);

/* Exhaustive check over every string of length 1..maxlen over the given
 * alphabet (Section 6.1's sweep, plus the lemmas and corollaries).  stats
 * receives ORC_BF_NSTATS counters, see ORC_BF_* below; every *_VIOL counter
 * must be zero. */
enum {
  ORC_BF_STRINGS = 0,       /* strings enumerated                                   */
  ORC_BF_TOKENIZABLE,       /* completely tokenizable strings                       */
  ORC_BF_LEMMA1_VIOL,       /* certified occurrence that is not a boundary          */
  ORC_BF_THM1_VIOL,         /* exact split differs from serial (tokenizable input)  */
  ORC_BF_COR1_VIOL,         /* exact split, malformed input, truncation rule fails  */
  ORC_BF_THM3_VIOL,         /* modulo-I split differs after pi_I (tokenizable)      */
  ORC_BF_MALFORMED_I_VIOL,  /* modulo-I split, malformed input, truncation rule     */
  ORC_BF_PROP3_VIOL,        /* exact-certified byte not certified modulo I          */
  ORC_BF_WITNESS_VIOL,      /* Theorem 2 witness does not lex as one token          */
  ORC_BF_NECESSITY_FOUND,   /* uncertified consumed bytes seen inside a token       */
  ORC_BF_NECESSITY_VIOL,    /* witness fits the bound but no such string was found  */
  ORC_BF_PAIRS_CONSUMED,    /* alphabet bytes some live state consumes              */
  ORC_BF_PAIRS_ADMITTED_I,  /* ... of which certified modulo I                      */
  ORC_BF_PAIRS_REFUSED_SAFE,/* consumed, refused modulo I, yet every split was safe */
  ORC_BF_MODE_SPLITS,       /* chunked scans compared                               */
  ORC_BF_NSTATS
};
int orc_bruteforce(const orc_set *s, const uint8_t *alphabet, uint32_t nalpha, uint32_t maxlen,
                   uint64_t *stats);

#ifdef __cplusplus
}
#endif

#endif
