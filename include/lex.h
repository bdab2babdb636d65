/*
 * lex.h -- C ABI of the MI355X certified-split lexer (gfx950, HIP).
 *
 * What it computes.  A token set is a list of byte regexes with tie-break priorities and
 * a flag marking the kinds a caller discards (the set I).  lex_compile builds, once, the
 * longest-match DFA whose accepting map resolves same-length ties by lower priority and
 * then lower index (Section 3), and its two 256-bit certificate maps: the exact map of
 * Definition 2 and the modulo-I map of Definition 3, each intersected with the bytes q0
 * consumes live (the useful sets of Corollary 2 and Proposition 2).  lex_run then scans a
 * device-resident byte buffer: it cuts the buffer only immediately before certified bytes,
 * scans every slice independently from q0 with the longest-match loop of Section 3, and
 * concatenates the per-slice (kind, length) streams in order.  By Theorem 1 (exact mode)
 * and Theorem 3 (modulo-I mode) the result equals the serial scan of the whole buffer,
 * after deleting discarded kinds in modulo-I mode.
 *
 * Malformed input.  The scan reports con(w), the final committed offset (Section 3), as
 * error_offset; error_offset == n exactly when the input is completely tokenizable.  The
 * tokens returned are those the serial scan emits before con(w): the output is truncated
 * after the first slice that does not consume its whole length (Corollary 1; the same
 * rule is applied in modulo-I mode, where the paper states no corollary -- see the
 * reading recorded with the design).
 *
 * Conventions
 *   - All sizes are in bytes unless stated; kinds are u8, lengths u32, offsets u64.
 *   - "device pointer" = memory of the current HIP device (e.g. a torch CUDA tensor);
 *     "host pointer" = ordinary process memory.
 *   - A stream argument is a hipStream_t passed as void*; NULL = the default stream.
 *   - Return values: LEX_OK (0) or a negative LEX_E* code.  Errors are reported
 *     synchronously only for invalid arguments; device-side outcomes (overflow, the
 *     error offset) are written to the caller's lex_result in device memory.
 *   - A lex_dfa is immutable after lex_compile and may be used concurrently from
 *     several host threads and streams.
 */
#ifndef PAPER_LEX_H
#define PAPER_LEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LEX_OK = 0,
  LEX_EINVAL = -1,    /* bad argument (null pointer, bad mode, misaligned buffer, ...) */
  LEX_ESYNTAX = -2,   /* a pattern does not parse                                     */
  LEX_ENOMEM = -3,    /* host or device allocation failed                             */
  LEX_EOVERFLOW = -4, /* more tokens than the output capacity (device-side status)     */
  LEX_EDEVICE = -5,   /* a HIP call failed                                            */
  LEX_ELIMIT = -6     /* > 255 kinds, too many states, workspace too small, n > 2^32-16 */
};

enum {
  LEX_MODE_EXACT = 0,   /* cut at the exact map; output tok(w)                             */
  LEX_MODE_DISCARD = 1, /* cut at the modulo-I map; output pi_I(tok(w)) (kept kinds only)  */
  LEX_MODE_SERIAL = 2   /* one slice, one lane: the serial scan itself (testing, refusal)  */
};

typedef struct lex_dfa lex_dfa;

/* One token definition (Section 3).  pattern: NUL-terminated byte regex (literals, '.',
 * classes [..] [^..] with ranges, groups, '|', postfix * + ? {m} {m,} {m,n}, escapes
 * \n \t \r \f \v \b \0 \xHH and a backslash before any non-alphanumeric byte).
 * priority: lower wins a same-length tie, then the lower index.  discard: 1 if the kind is
 * in I (used by LEX_MODE_DISCARD and the modulo-I map, Section 6.1). */
typedef struct {
  const char *pattern;
  int32_t priority;
  uint8_t discard;
} lex_tokdef;

/* Result of one scan, written by the device into caller memory. */
typedef struct {
  uint64_t ntokens;      /* tokens written; if status == LEX_EOVERFLOW, tokens required     */
  uint64_t error_offset; /* con(w); == n iff the input is completely tokenizable             */
  int32_t status;        /* LEX_OK or LEX_EOVERFLOW                                          */
  uint32_t nslices;      /* non-empty slices the plan produced (1 for a serial scan)         */
} lex_result;

/* Compiled-automaton summary (host copy). */
typedef struct {
  int32_t nkinds;
  int32_t nstates;    /* states of the trimmed, minimised live automaton (Section 4.1) */
  int32_t nclasses;   /* byte classes of the transition table                         */
  int32_t nrows;      /* rows of the packed device table                              */
  int32_t reentrant;  /* Definition 1                                                 */
  int32_t monotone;   /* 1: no live edge leaves an accepting state for a non-accepting
                         one, so the walker never needs to fall back                  */
  int32_t q0_live;    /* 0: the token set accepts nothing                             */
  int32_t reserved;
} lex_info_t;

/* Compiles ndefs (1..255) definitions.  On success *out owns the host tables and their
 * device copy (uploaded to the current HIP device) until lex_free.  On failure returns
 * LEX_ESYNTAX/LEX_ELIMIT/LEX_EINVAL/LEX_EDEVICE and writes a message into err (errlen
 * bytes, may be NULL). */
int lex_compile(const lex_tokdef *defs, uint32_t ndefs, lex_dfa **out, char *err, size_t errlen);

/* Framing at the producer (Section 7.1): compiles the ndefs (1..254) definitions with the
 * byte `reserved` (0..255) taken out of every byte class of every pattern, so that no token
 * of theirs contains it at any position, and appends one more definition, kind ndefs, whose
 * only word is that byte (priority 0, discarded iff reserved_discard != 0).  The reserved
 * byte is then consumed live only from q0 and is certified by Definition 2 whatever the
 * set was; a producer that writes it only at token boundaries (escaping it elsewhere) gets
 * a document that splits at every occurrence with the serial token stream reproduced.  A
 * pattern whose language becomes empty stays valid (its kind never matches).  Ownership,
 * device upload and errors as for lex_compile. */
int lex_compile_framed(const lex_tokdef *defs, uint32_t ndefs, uint32_t reserved, int reserved_discard,
                       lex_dfa **out, char *err, size_t errlen);

/* Builds a lexer from a hand-built automaton (the examples of Section 4.1): next is a
 * host array of nstates*256 targets (-1 = undefined), accept[q] a token index in
 * [0, ntok) or -1, discard[t] flags t in I (ntok entries, may be NULL for I empty).  The
 * automaton is trimmed to Q+ and minimised exactly as a compiled one. */
int lex_compile_table(int32_t nstates, int32_t q0, const int32_t *next, const int32_t *accept,
                      const uint8_t *discard, int32_t ntok, lex_dfa **out, char *err, size_t errlen);

/* Releases a lexer (host and device tables).  Resource management, no operation of the
 * paper.  The caller must not have scans in flight. */
void lex_free(lex_dfa *dfa);

/* Useful certified set of a mode (host call): bits[b >> 3] bit (b & 7) is set iff byte b is
 * a useful certified split byte (mode EXACT: Definition 2 with Corollary 2; DISCARD:
 * Definition 3 with Proposition 2).  raw != 0 returns the maps before the useful filter
 * (vacuous bytes included).  LEX_MODE_SERIAL returns the empty set. */
int lex_cert(const lex_dfa *dfa, int mode, int raw, uint8_t bits[32]);

/* Summary of the compiled automaton (host call, into *out): its kinds, the states of the
 * trimmed and minimised live automaton (Section 4.1) and its byte classes, whether q0 is
 * re-entrant (Definition 1), whether it is monotone (no live edge from an accepting to a
 * non-accepting state: longest match then never falls back, Section 3) and whether q0 is
 * live at all.  Returns LEX_EINVAL for null arguments. */
int lex_info(const lex_dfa *dfa, lex_info_t *out);

/* Host copy of the packed transition table of a mode: the longest-match DFA of Section 3,
 * trimmed and minimised (Section 4.1), one u32 per (row, byte) holding the next row, the
 * accepting and token-end flags of the step and the kind it emits (layout documented in
 * the library source), plus nrows row-info and row-kind bytes.  Caller-owned host arrays of
 * at least nrows*256 and nrows entries (LEX_ELIMIT otherwise; NULL skips an array); for
 * host-side models and the autotuner's table digest. */
int lex_tables(const lex_dfa *dfa, int mode, uint32_t *table, size_t table_entries,
               uint8_t *rowinfo, uint8_t *rowkind, size_t nrows);

/* Tuning of one scan (NULL = defaults).  chunk_bytes: target length of the paper's
 * equal-division chunks (boundaries slide forward to the next certified byte); lane_bytes:
 * target length of the sub-slices one GPU lane walks (a multiple of 16 and a divisor of
 * chunk_bytes; 0 = chosen from n).  path: 1 = the five-step pipeline (bitmap, plan, count
 * walk, scan, emit walk); 2 = fused (each lane finds its own cut, no bitmap; count walk,
 * scan and emit walk as separate launches); 3 = fused in one pass (windowed scans only,
 * else as 2): 256-lane workgroups take their lanes in order, count-walk them, find their
 * first output slot by a look-back over the earlier workgroups' published totals, and
 * emit, all in one launch; 0 = default: 3 where it applies, else 2.  block_threads:
 * threads per walk workgroup, 256, 512 or 1024 (0 = the largest whose LDS fits; one pass
 * uses 256 and a default path given another value takes path 2).  emit: 0 = default,
 * 1 = lane emit only.  By default a scan of an automaton with at most 256 rows uses the
 * windowed emit: the count
 * walk records checkpoints every 64 bytes and the emit walk runs one thread per 64-byte
 * sub-slice; a scan with a halted slice or a slice of 2^24 bytes or more falls back to the
 * lane emit (one thread per slice) on the device, and so does a scan of a non-monotone
 * automaton (a live edge from an accepting to a non-accepting state) in which some slice
 * fell back to an earlier accepting position.  One pass needs a monotone automaton and
 * certified cuts.  All write the same outputs.  events:
 * optional array of LEX_NPHASES + 1 hipEvent_t (passed as void*, created by the caller)
 * recorded on the scan's stream at the phase boundaries: [0] start, [1] after planning
 * (steps a, b), [2] after the count walk (c), [3] after the scan (d), [4] after the emit
 * walk (e).  In one pass, [1] follows the reset of the look-back state, [2] the one-pass
 * launch (planning, count walk and windowed emit) and [4] the lane emit's fallback. */
enum { LEX_NPHASES = 4 };
enum { LEX_EMIT_DEFAULT = 0, LEX_EMIT_LANE = 1 };
typedef struct {
  uint64_t chunk_bytes;
  uint32_t lane_bytes;
  int32_t path;
  int32_t block_threads;
  int32_t emit;
  void *const *events;
} lex_run_opts;

/* The configuration lex_run would use for n bytes in this mode under opts (NULL =
 * defaults): no operation of the paper; for tools, the autotuner and benchmarks that
 * attribute time and bytes to kernels.  path is
 * 1, 2 or 3 as in lex_run_opts (never 0); windowed: the windowed emit applies; hybrid: the
 * hybrid plan splits a refused set (path is then 1: its count walk, scan and emit run on
 * the speculative cuts, lane_bytes is the speculative lane).  Returns what lex_run would
 * return for these arguments (LEX_EINVAL, LEX_ELIMIT) or LEX_OK. */
typedef struct {
  uint32_t lane_bytes;
  uint32_t block_threads;
  int32_t path;
  int32_t windowed;
  int32_t hybrid;
} lex_plan_info;
int lex_plan(const lex_dfa *dfa, uint64_t n, int mode, const lex_run_opts *opts, lex_plan_info *out);

/* Device workspace bytes lex_run needs for n input bytes under opts (NULL = defaults):
 * memory sizing, no operation of the paper.  0 for arguments lex_run would refuse. */
size_t lex_workspace_size(const lex_dfa *dfa, uint64_t n, int mode, const lex_run_opts *opts);

/* Scans d_bytes[0, n) (device pointer) and writes, on `stream`, at most cap tokens:
 * d_kinds[i] (device u8), d_lens[i] (device u32) and, when d_offsets is non-NULL,
 * d_offsets[i] (device u64 start offset of token i in d_bytes).  *d_result (device pointer)
 * receives the lex_result.  d_kinds and d_lens must be 16-byte aligned (outputs leave the
 * kernels in 16-byte chunks).  d_ws (device pointer, ws_bytes >= lex_workspace_size(...),
 * 256-byte aligned) is scratch owned by the caller for the duration of the scan.
 * cap = n is always sufficient.  The call only enqueues work; it returns LEX_EINVAL for
 * bad arguments, LEX_ELIMIT for an oversized n or a short workspace, LEX_EDEVICE if a launch
 * fails.  Outputs are unspecified when the result status is LEX_EOVERFLOW.  n must not
 * exceed 2^32 - 16 (lengths and offsets inside one buffer are 32-bit on the device). */
int lex_run(const lex_dfa *dfa, const uint8_t *d_bytes, uint64_t n, int mode, uint8_t *d_kinds,
            uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap, lex_result *d_result, void *d_ws,
            size_t ws_bytes, const lex_run_opts *opts, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lex_run with the workspace taken from
 * scratch memory the library holds itself, LEX_STATIC_WS_BYTES on each device it runs on,
 * reserved when the library's device code is loaded there and held until the process
 * ends.  Arguments, outputs, asynchrony and results are those of lex_run (the same
 * kernels run); the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Returns LEX_ELIMIT when the scan needs more workspace than
 * LEX_STATIC_WS_BYTES (lex_workspace_size with the same arguments says how much; with
 * default options inputs up to about 200 MiB fit), and
 * LEX_EDEVICE when the lexer's tables are not yet on the current device (lex_compile
 * uploads them when a device is present; otherwise one ordinary lex_run on that device
 * does).  Every call on one device shares that device's scratch memory: calls whose
 * scans overlap on one device (different streams, or host threads without ordering)
 * race and give unspecified results; calls in order on one stream are safe. */
#define LEX_STATIC_WS_BYTES (64u << 20)
int lex_run_static(const lex_dfa *dfa, const uint8_t *d_bytes, uint64_t n, int mode, uint8_t *d_kinds,
                   uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap, lex_result *d_result,
                   const lex_run_opts *opts, void *stream);

/* ---- Batched documents (many independent scans in one launch sequence).
 *
 * A lex_batch holds up to 8 (lexer, mode) instances resident together on the current
 * device: their packed tables are combined into one LDS-resident table.  Each document of
 * a batch names its instance; it is scanned exactly as lex_run would scan it alone with
 * that lexer and mode (cut at its own useful certified bytes: Theorem 1, Theorem 3; a
 * document whose useful map is empty, or flagged serial, is one slice), and its result is
 * that scan's (Corollary 1 truncation, error offset relative to the document).  Documents
 * are independent: one's error does not affect another.  The launches use fixed grids,
 * reset their own work queues and never synchronise with the host, so a caller may
 * capture lex_run_batch in a hipGraph and replay it. */
typedef struct lex_batch lex_batch;

typedef struct {
  uint64_t offset;  /* first byte of the document in d_bytes */
  uint32_t length;  /* bytes */
  uint16_t inst;    /* instance index given to lex_batch_create */
  uint16_t flags;   /* bit 0: serial (one slice); other bits must be 0 */
} lex_doc;          /* 16 bytes */

typedef struct {
  uint64_t tok_offset;   /* the document's tokens are outputs [tok_offset, tok_offset + ntokens) */
  uint64_t ntokens;
  uint64_t error_offset; /* con of the document, relative to its first byte; == length if complete */
  int32_t status;        /* LEX_OK, or LEX_EOVERFLOW for every document when the batch overflows cap */
  uint32_t nslices;      /* non-empty slices the document was cut into */
} lex_doc_result;        /* 32 bytes */

/* Builds a batch from ninst lexers and modes (LEX_MODE_EXACT or LEX_MODE_DISCARD) on the
 * current device.  LEX_ELIMIT if more than 8 instances or the combined table does not fit
 * in LDS beside the emit stage. */
int lex_batch_create(const lex_dfa *const *dfas, const int32_t *modes, uint32_t ninst, lex_batch **out,
                     char *err, size_t errlen);
void lex_batch_free(lex_batch *batch);

/* Workspace for ndocs documents over nbytes bytes (opts: lane_bytes; NULL = defaults).  A
 * batch's default lane is 1 KiB, doubled while nbytes / lane exceeds 2^20, up to 4 KiB;
 * pass the same opts (or the same nbytes with defaults) to lex_run_batch. */
size_t lex_batch_workspace_size(const lex_batch *batch, uint32_t ndocs, uint64_t nbytes, const lex_run_opts *opts);

/* Scans the ndocs documents of d_docs (device array) over d_bytes[0, nbytes) (device).
 * Tokens go to d_kinds / d_lens (and d_offsets, relative to each document, if non-NULL),
 * document by document in d_docs order; d_res (device, ndocs entries) receives each
 * document's result and *d_total (device) the batch's: ntokens = total tokens,
 * error_offset = the number of documents that did not tokenize completely, status,
 * nslices.  nbytes must be below 2^32 (output offsets are 32-bit on the device); every
 * document must lie inside [0, nbytes).  Only enqueues work, on `stream`. */
int lex_run_batch(const lex_batch *batch, const uint8_t *d_bytes, uint64_t nbytes, const lex_doc *d_docs,
                  uint32_t ndocs, uint8_t *d_kinds, uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap,
                  lex_doc_result *d_res, lex_result *d_total, void *d_ws, size_t ws_bytes,
                  const lex_run_opts *opts, void *stream);

/* ---- Host baseline (not a GPU path, and never called by one).
 *
 * The paper's CPU executor (Section 6) on the host's cores, for timing the GPU scans
 * against: an equal-division plan cuts bytes[0, n) (host memory) before the first useful
 * certified byte of `mode` at or after each multiple of chunk_bytes (0 = 64 KiB; none in
 * LEX_MODE_SERIAL or when the useful map is empty); nthreads worker threads (0 = one per
 * hardware thread) take the chunks from a shared counter and scan each one alone with
 * the longest-match loop of Section 3 over this lexer's packed table; the per-chunk
 * streams are concatenated in order up to the first chunk that halts (Corollary 1).  By
 * Theorem 1 and Theorem 3 the result is the serial scan's, exactly as lex_run's.
 * kinds and lens are host arrays of cap >= n entries (chunks stage their tokens at their
 * own byte offsets before the concatenation compacts them); *result (host) receives the
 * token count, con(w) as error_offset, LEX_OK and the number of chunks as nslices.  Runs
 * synchronously; returns LEX_EINVAL on bad arguments (cap < n included), LEX_ELIMIT for
 * n > 2^32 - 16.  Failed lookahead is not bounded here (plain re-scans from the last
 * accepting position). */
int lex_cpu_chunked(const lex_dfa *dfa, const uint8_t *bytes, uint64_t n, int mode, uint8_t *kinds, uint32_t *lens,
                    uint64_t cap, uint64_t chunk_bytes, uint32_t nthreads, lex_result *result);

/* Certificate bitmap of step (a) on its own (device pointers): d_bits[i >> 6] bit (i & 63)
 * is set iff byte d_bytes[i] is in the useful map of `mode`; ceil(n / 64) u64 words. */
int lex_cert_bitmap(const lex_dfa *dfa, const uint8_t *d_bytes, uint64_t n, int mode, uint64_t *d_bits,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_LEX_H */
