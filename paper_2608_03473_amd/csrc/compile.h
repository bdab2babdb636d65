// compile.h -- host-side token-set compiler of the certified-split lexer.
//
// Builds, once per token set and discarded set I (Section 6.1: the modulo-I map depends
// on I, so I is fixed at build time):
//   * the longest-match DFA with tau resolved by (priority, index) (Section 3),
//     restricted to its live subautomaton and minimised (Section 4.1);
//   * the exact and modulo-I certificate maps, useful sets only (Definitions 2, 3,
//     Corollary 2, Proposition 2), derived in O(|Q| |Sigma|) (Section 6);
//   * the packed transition tables the HIP kernels walk.
// Internal to the library; the public interface is include/lex.h.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lexc {

// Packed-table entry layout (one u32 per (row, byte)):
//   bit  0       COUNT: a token of a kind written in this mode ends before this byte
//   bit  1       EMIT: a token ends immediately before this byte; the byte then starts
//                the next token (the step has already moved to delta(q0, byte))
//   bits 2..6    swizzle of the next row, (row & 31)
//   bit  7       ACC: the next row is an accepting DFA state
//   bits 10..23  byte offset of the next row in the table (row index * 1024)
//   bits 24..31  token kind emitted by this step (valid when EMIT is set)
// The walk state is the entry masked to bits 2..6 and 10..23, and the entry for byte b
// of that row sits at LDS byte address state ^ (b << 2): row r stores byte b's entry at
// index r * 256 + (b ^ (r & 31)), so lanes reading the same byte in different rows hit
// different LDS banks.
// Rows: 0 = token start (q0 before any byte of the token), 1 + q = DFA state q,
//       then SINK (halted; absorbs everything) and, for non-monotone automata,
//       FAIL (a dead end after a non-accepting state: the walker must fall back to
//       the last accepting position).
constexpr uint32_t kCount = 1u << 0;
constexpr uint32_t kEmit = 1u << 1;
constexpr uint32_t kAcc = 1u << 7;
constexpr uint32_t kStateMask = 0x00FFFC7Cu;
constexpr int kRowShift = 10;
constexpr int kKindShift = 24;
constexpr int kMaxRows = 1 << 14;
inline uint32_t row_swizzle(int row) { return (uint32_t)row & 31u; }
inline uint32_t row_state(int row) { return ((uint32_t)row << kRowShift) | (row_swizzle(row) << 2); }
// rowinfo byte: bit 7 = accepting, bit 6 = counted in this mode; the accepting kind is
// in rowkind[].
constexpr uint8_t kInfoAcc = 0x80;
constexpr uint8_t kInfoCount = 0x40;

struct Dfa {
  int nstates = 0;                 // live, minimised states; q0 == 0
  int nclasses = 0;
  uint8_t cls[256] = {0};          // byte -> class
  std::vector<int32_t> next;       // nstates * nclasses, -1 undefined
  std::vector<int32_t> acc;        // nstates, accepting kind or -1
};

struct Compiled {
  int nkinds = 0;
  std::vector<uint8_t> discard;    // per kind: in I
  bool q0_live = true;             // the token set accepts some word
  Dfa dfa;                         // trimmed and minimised
  bool reentrant = false;          // Definition 1
  bool monotone = true;            // no live edge from an accepting to a non-accepting state
  uint8_t exact_raw[32] = {0}, discard_raw[32] = {0};
  uint8_t exact_useful[32] = {0}, discard_useful[32] = {0};
  uint8_t q0_live_bytes[32] = {0};
  // Packed tables (index 0 = exact mode, 1 = discard mode).
  int nrows = 0, row_sink = 0, row_fail = -1;
  std::vector<uint32_t> table[2];  // nrows * 256
  std::vector<uint8_t> rowinfo[2]; // nrows
  std::vector<uint8_t> rowkind;    // nrows, accepting kind or 0xFF
};

struct TokDef {
  std::string pattern;
  int32_t priority = 0;
  bool discard = false;
  // A byte taken out of every byte class of the pattern (-1: none), so that no word of
  // this kind contains it: the reservation of a framing byte (Section 7.1).
  int exclude = -1;
};

// Returns false and sets err on a syntax error or a limit violation.
bool compile_defs(const std::vector<TokDef> &defs, Compiled &out, std::string &err);
// Hand-built automaton (next: nstates*256, -1 undefined; accept: -1 or token index).
bool compile_table(int nstates, int q0, const int32_t *next, const int32_t *accept,
                   const std::vector<uint8_t> &discard, Compiled &out, std::string &err);

}  // namespace lexc
