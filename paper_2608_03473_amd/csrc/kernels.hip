// kernels.hip -- the certified-split scan on gfx950.
//
// Steps (one scan of one buffer):
//   (a) k_bitmap     coalesced 16-byte loads; each byte is tested against the useful
//                    certificate map of the mode (SWAR compares when the map holds at
//                    most 8 bytes, an LDS lookup otherwise); a wavefront ballot yields
//                    the first certified byte of every 4 KiB tile.
//   (b) k_tiles_* +  the equal-division planner of Section 6 in one pass: every lane
//       k_plan       target j*lane_bytes slides forward to the next certified byte
//                    (bitmap words inside its tile, then a two-level suffix minimum over
//                    tiles); duplicate slides give empty lanes and a target with nothing
//                    after it gives the end of the input.  An empty useful map gives one
//                    slice.
//   (c) k_count      every lane runs the longest-match loop of Section 3 on its slice
//                    [cut_j, cut_j+1) from the start row, treating the slice end as the end
//                    of the input; the packed transition table lives in LDS.  The fused
//                    path places each lane's cut inside this kernel (lane_slice).
//   (d) k_scan       exclusive prefix of the per-lane counts; the first lane whose walk
//                    halted fixes the output length and, by Corollary 1, truncates it.
//   (e) k_emit       every lane up to the first halted one walks again and writes its
//                    (kind, length[, offset]) triples at its prefix offset, skipping
//                    discarded kinds in modulo-I mode (the image pi_I of Section 5).
//                    Tokens are staged in a 96-byte per-lane LDS ring (16 packed length
//                    words, 32 kinds) and leave in whole, aligned 32-byte sectors (8
//                    lengths or 32 kinds at a time), so the emit walk issues few,
//                    full-width memory requests.
//       k_emit_win   the windowed emit: one thread per 64-byte window, restarted from
//                    the count walk's checkpoint, tokens staged per wave (their ends, or
//                    their lengths in a mode with discarded kinds) and written out
//                    coalesced.
//   k_onepass        (b)-(e) for windowed scans in one launch: 256-lane groups taken in
//                    order plan, count, find their first output slot by a decoupled
//                    look-back over the earlier groups' totals, and emit their windows.
//   Batches of documents (lex_run_batch) have kernels of their own, further below.
//
// Table entries (layout in compile.h): COUNT (bit 0), EMIT (bit 1), the next row's
// swizzle (bits 2..6), ACC (bit 7), the next row's byte offset in bits 10..23 and the
// emitted kind in bits 24..31.  The walk state is the entry masked to the row offset and
// swizzle, so the next entry's LDS address is (e & kRowMask) ^ (b << 2).
// Row 0 is the token start, SINK absorbs after a halt, FAIL (non-monotone automata only)
// marks a dead end that falls back to the last accepting position.
#include <algorithm>

#include "kernels.h"

namespace lexk {
namespace {

constexpr uint32_t kCountBit = 1u << 0;
constexpr uint32_t kEmitBit = 1u << 1;
constexpr uint32_t kAccBit = 1u << 7;
constexpr uint32_t kRowMask = 0x00FFFC7Cu;  // next row offset and its swizzle
constexpr int kRowShift = 10;
constexpr uint8_t kInfoAcc = 0x80;
constexpr uint8_t kInfoCount = 0x40;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kTile = 4096;        // bytes per bitmap tile (64 words)

// Unsigned division by a divisor d >= 2 fixed for a launch, by multiplication
// (Granlund and Montgomery, "Division by invariant integers using multiplication", 1994):
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, n / d = (t + ((n - t) >> 1))
// >> (l - 1) where t = mulhi(n, m), for every 32-bit n.
struct FastDiv {
  uint32_t m, l;
};
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  const uint32_t t = __umulhi(n, f.m);
  return (t + ((n - t) >> 1)) >> (f.l - 1);
}
constexpr uint32_t kTilesPerBlock = 1024;

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// ------------------------------------------------------------- (a) bitmap
// Per-byte zero test of a 32-bit word: bit 7 of each byte of the result is set iff
// that byte of x is zero (exact: no borrow crosses bytes).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x) {
  uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  return ~(y | x | 0x7F7F7F7Fu);
}
// Gathers bits 7, 15, 23, 31 of m into bits 0..3.
__device__ __forceinline__ uint32_t gather4(uint32_t m) {
  return ((m >> 7) & 1u) | ((m >> 14) & 2u) | ((m >> 21) & 4u) | ((m >> 28) & 8u);
}

__device__ __forceinline__ uint32_t match_word_swar(uint32_t w, const uint32_t *pat, int np) {
  uint32_t m = 0;
  for (int i = 0; i < np; ++i) m |= zero_bytes(w ^ pat[i]);
  return gather4(m);
}

__device__ __forceinline__ uint32_t match_word_lut(uint32_t w, const uint8_t *lut) {
  return (uint32_t)lut[w & 0xFF] | ((uint32_t)lut[(w >> 8) & 0xFF] << 1) |
         ((uint32_t)lut[(w >> 16) & 0xFF] << 2) | ((uint32_t)lut[w >> 24] << 3);
}

struct CertArg {
  uint32_t pat[8];   // byte broadcast to 4 lanes of a word
  int np;            // number of patterns (SWAR) or -1 (LUT)
  uint32_t words[8]; // 256-bit map
};

// One thread per 64-byte word of the bitmap; one wave per 4 KiB tile.
__global__ void __launch_bounds__(256) k_bitmap(const uint8_t *__restrict__ in, uint32_t n, CertArg ca,
                                                uint64_t *__restrict__ bits, uint64_t *__restrict__ tile_first) {
  __shared__ uint8_t lut[256];
  __shared__ uint32_t pat[8];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) lut[i] = (ca.words[i >> 5] >> (i & 31)) & 1u;
  if (threadIdx.x < 8) pat[threadIdx.x] = ca.pat[threadIdx.x];
  __syncthreads();
  const uint32_t nwords = (n + 63) / 64;
  const uint32_t wi = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t word = 0;
  if (wi < nwords) {
    const uint32_t base = wi * 64;
    if (base + 64 <= n && ((reinterpret_cast<uintptr_t>(in) & 15) == 0)) {
      const uint4 *v = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint4 x = v[q];
        uint32_t w4[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t m = ca.np >= 0 ? match_word_swar(w4[k], pat, ca.np) : match_word_lut(w4[k], lut);
          word |= (uint64_t)m << (q * 16 + k * 4);
        }
      }
    } else {
      for (uint32_t i = 0; i < 64 && base + i < n; ++i) word |= (uint64_t)lut[in[base + i]] << i;
    }
    bits[wi] = word;
  }
  if (!tile_first) return;
  // First certified byte of this wave's tile (tile index == global wave index).
  const uint64_t any = __ballot(word != 0);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t tile = wi >> 6;
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  if (any) {
    const uint32_t first = __ffsll((unsigned long long)any) - 1;
    if (lane == first) tile_first[tile] = (uint64_t)wi * 64 + (__ffsll((unsigned long long)word) - 1);
  } else if (lane == 0 && tile < ntiles) {
    tile_first[tile] = ~0ull;
  }
}

// --------------------------------------------------------------- (b) plan
// Two-level suffix minimum over tiles.  Level 1: in-block suffix minimum of each group
// of kTilesPerBlock tiles (in place) and the group minimum.  Level 2: one workgroup
// turns the group minima into exclusive suffix minima (min over later groups).
__global__ void __launch_bounds__(1024) k_tiles_blocks(uint64_t *__restrict__ t, uint32_t ntiles,
                                                       uint64_t *__restrict__ grp) {
  __shared__ uint64_t part[kTilesPerBlock];
  const uint32_t tid = threadIdx.x;
  const uint32_t i = blockIdx.x * kTilesPerBlock + tid;
  part[tid] = i < ntiles ? t[i] : ~0ull;
  __syncthreads();
  for (uint32_t d = 1; d < kTilesPerBlock; d <<= 1) {
    uint64_t v = tid + d < kTilesPerBlock ? part[tid + d] : ~0ull;
    __syncthreads();
    part[tid] = min(part[tid], v);
    __syncthreads();
  }
  if (i < ntiles) t[i] = part[tid];
  if (tid == 0) grp[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(1024) k_tiles_top(uint64_t *__restrict__ grp, uint32_t ngroups) {
  __shared__ uint64_t part[1024];
  const uint32_t tid = threadIdx.x;
  part[tid] = tid < ngroups ? grp[tid] : ~0ull;
  __syncthreads();
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    uint64_t v = tid + d < 1024 ? part[tid + d] : ~0ull;
    __syncthreads();
    part[tid] = min(part[tid], v);
    __syncthreads();
  }
  if (tid < ngroups) grp[tid] = tid + 1 < 1024 ? part[tid + 1] : ~0ull;  // exclusive
}

// First certified byte at or after the start of tile t (~0 if none).
__device__ __forceinline__ uint64_t tile_next(const uint64_t *tn, const uint64_t *grp, uint32_t t,
                                              uint32_t ntiles) {
  if (t >= ntiles) return ~0ull;
  return min(tn[t], grp[t / kTilesPerBlock]);
}

// cuts[j] = first certified byte at or after j*lane_bytes (n if none), cuts[0] = 0,
// cuts[M] = n.  Non-decreasing; equal neighbours make empty lanes.
__global__ void __launch_bounds__(256) k_plan(const uint64_t *__restrict__ bits, const uint64_t *__restrict__ tn,
                                              const uint64_t *__restrict__ grp, uint32_t n, uint32_t lane_bytes,
                                              uint32_t nlanes, uint32_t *__restrict__ cuts) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nlanes) return;
  if (j == 0 || j == nlanes) {
    cuts[j] = j ? n : 0;
    return;
  }
  const uint64_t x = (uint64_t)j * lane_bytes;
  uint64_t cut = n;
  if (x < n) {
    const uint32_t nwords = (n + 63) / 64;
    const uint32_t ntiles = (n + kTile - 1) / kTile;
    uint32_t w = (uint32_t)(x >> 6);
    uint64_t m = bits[w] & (~0ull << (x & 63));
    const uint32_t tile_end = min(nwords, (w | 63u) + 1);
    while (!m && ++w < tile_end) m = bits[w];
    if (m) cut = (uint64_t)w * 64 + (__ffsll((unsigned long long)m) - 1);
    else cut = min<uint64_t>(tile_next(tn, grp, (uint32_t)(x >> 12) + 1, ntiles), n);
  }
  cuts[j] = (uint32_t)min<uint64_t>(cut, n);
}

// ----------------------------------------------------------- (c), (e) walk
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

struct Tables {
  const lds_u8 *T;      // LDS table, byte-addressed (so that (e & mask) ^ (b << 2) is one
                        // bit operation and the table's LDS offset an immediate)
  const uint8_t *info;  // LDS
  const uint8_t *kind;  // LDS
  uint32_t sink, fail;  // row byte offsets (fail == sink when monotone)
  uint32_t start;       // row offset of the token-start row (0 unless several tables share LDS)
};

__device__ __forceinline__ uint32_t entry(const Tables &tb, uint32_t st, uint32_t b) {
  return *reinterpret_cast<const lds_u32 *>(tb.T + (st ^ (b << 2)));
}

// The same lookup from the previous entry itself (its row bits, masked in the same
// instruction): (e & kRowMask) ^ (b << 2) as one v_bitop3 (truth table 0x6C over the
// operands e, b << 2, kRowMask), used directly as the LDS address.  This relies on the
// table sitting at LDS address 0: the walk kernels declare no static LDS, so their
// dynamic LDS, whose first bytes carve_lds gives the table, starts there.  (Adding the
// table's address instead costs a v_add per byte: it is only known to be 0 after
// instruction selection.)
__device__ __forceinline__ uint32_t entry_from(const Tables &, uint32_t e, uint32_t b) {
  return *(const lds_u32 *)(size_t)__builtin_amdgcn_bitop3_b32(e, b << 2, kRowMask, 0x6C);
}

__device__ __forceinline__ const lds_u8 *lds_bytes_of(const void *p) { return (const lds_u8 *)p; }

// Emit-side per-lane state.  The lane owns output slots [first, first + count).
//
// Packed path (lanes shorter than 2^24 bytes, so every length fits 24 bits): each byte
// step writes one word (length << 8 | kind) into a 16-slot LDS ring whether or not a
// token ends there, and a kept token advances the slot.  Chunks of 8 kept tokens are
// split off at most once per 8 bytes: the 8 lengths leave as one whole 32-byte sector
// (two 16-byte stores) and the 8 kinds go to a 32-byte LDS stage that leaves as one
// sector every 32 tokens.  A chunk that reaches below `first` (the lane's head) is
// written slot by slot, as are the lane's incomplete last chunks.  Between two splits
// at most 15 words are pending, so the 16 slots never overrun.
//
// Direct path (lanes of 2^24 bytes or more): every kept token is stored on the spot.
constexpr int kSlots = 16;      // packed words in the ring
constexpr int kChunk = 8;       // lengths per 32-byte sector
constexpr int kKindSlots = 32;  // kinds per 32-byte sector
// The workgroup's rings are stored slot-major: dword d of lane t sits at
// (d * blockDim + t) * 4, so the lanes of a wave touch consecutive banks whatever
// slots they write.  Per lane: 16 words, then 8 dwords of staged kinds.
constexpr int kRingDwords = kSlots + kKindSlots / 4;  // 24
constexpr int kRingBytes = 4 * kRingDwords;

struct Ring {
  uint32_t *w;        // LDS: dword d of this lane's ring is w[d * stride]
  uint32_t stride;    // blockDim
  uint8_t *kinds;     // global outputs (16-byte aligned)
  uint32_t *lens;
  uint64_t *offs;     // optional
  uint32_t o;         // next output slot
  uint32_t fl;        // slots below fl have been split off (a multiple of kChunk)
  uint32_t first;     // the lane's first slot
  bool write;
  bool direct;
};

__device__ __forceinline__ uint32_t &ring_at(Ring &r, uint32_t d) { return r.w[d * r.stride]; }

__device__ __forceinline__ uint32_t pack_word(uint32_t e, uint32_t len) {
  // byte 0 <- byte 3 of e (the kind), bytes 1..3 <- bytes 0..2 of len
  return __builtin_amdgcn_perm(e, len, 0x02010007u);
}

// Splits the chunk [r.fl, r.fl + 8) off the ring.
__device__ __forceinline__ void ring_split(Ring &r) {
  const uint32_t c0 = r.fl;
  const uint32_t base = c0 & (kSlots - 1);
  uint32_t wd[kChunk];
#pragma unroll
  for (int i = 0; i < kChunk; ++i) wd[i] = ring_at(r, base + i);
  // kinds: byte 0 of each word, packed 4 to a dword, staged after the words
  const uint32_t k0 = __builtin_amdgcn_perm(__builtin_amdgcn_perm(wd[3], wd[2], 0x0c0c0400u),
                                            __builtin_amdgcn_perm(wd[1], wd[0], 0x0c0c0400u), 0x05040100u);
  const uint32_t k1 = __builtin_amdgcn_perm(__builtin_amdgcn_perm(wd[7], wd[6], 0x0c0c0400u),
                                            __builtin_amdgcn_perm(wd[5], wd[4], 0x0c0c0400u), 0x05040100u);
  ring_at(r, kSlots + (c0 & (kKindSlots - 1)) / 4) = k0;
  ring_at(r, kSlots + (c0 & (kKindSlots - 1)) / 4 + 1) = k1;
  const uint4 la = make_uint4(wd[0] >> 8, wd[1] >> 8, wd[2] >> 8, wd[3] >> 8);
  const uint4 lb = make_uint4(wd[4] >> 8, wd[5] >> 8, wd[6] >> 8, wd[7] >> 8);
  if (c0 >= r.first) {
    uint4 *dst = reinterpret_cast<uint4 *>(r.lens + c0);
    dst[0] = la;
    dst[1] = lb;
  } else {  // the lane's head: only slots >= first are the lane's
#pragma unroll
    for (int i = 0; i < kChunk; ++i)
      if (c0 + i >= r.first) r.lens[c0 + i] = wd[i] >> 8;
  }
  r.fl = c0 + kChunk;
  if ((r.fl & (kKindSlots - 1)) == 0) {
    const uint32_t k32 = r.fl - kKindSlots;
    uint32_t kd[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) kd[i] = ring_at(r, kSlots + i);
    if (k32 >= r.first) {
      uint4 *dst = reinterpret_cast<uint4 *>(r.kinds + k32);
      dst[0] = make_uint4(kd[0], kd[1], kd[2], kd[3]);
      dst[1] = make_uint4(kd[4], kd[5], kd[6], kd[7]);
    } else {
      for (uint32_t i = r.first - k32; i < kKindSlots; ++i) r.kinds[k32 + i] = (uint8_t)(kd[i / 4] >> (8 * (i & 3)));
    }
  }
}

__device__ __forceinline__ void ring_maybe_split(Ring &r) {
  if (r.write && r.o - r.fl >= kChunk) ring_split(r);
}

// Records the token whose word is in slot r.o as kept.
__device__ __forceinline__ void ring_commit(Ring &r, uint32_t kind, uint32_t len, uint32_t start) {
  if (r.write) {
    if (r.direct) {
      r.kinds[r.o] = (uint8_t)kind;
      r.lens[r.o] = len;
    }
    if (r.offs) r.offs[r.o] = start;
  }
  ++r.o;
  if (!r.direct) ring_maybe_split(r);
}

// The lane's incomplete last chunks, slot by slot (slots below first are skipped).
__device__ __forceinline__ void ring_flush_tail(Ring &r) {
  if (!r.write || r.direct) return;
  for (uint32_t i = max(r.fl & ~(uint32_t)(kKindSlots - 1), r.first); i < max(r.fl, r.first); ++i) {
    const uint32_t q = i & (kKindSlots - 1);
    r.kinds[i] = (uint8_t)(ring_at(r, kSlots + q / 4) >> (8 * (q & 3)));
  }
  for (uint32_t i = max(r.fl, r.first); i < r.o; ++i) {
    const uint32_t wd = ring_at(r, i & (kSlots - 1));
    r.kinds[i] = (uint8_t)(wd & 0xFF);
    r.lens[i] = wd >> 8;
  }
}

__device__ __forceinline__ void ring_put(Ring &r, uint32_t kind, uint32_t len, uint32_t start) {
  if (!r.direct) ring_at(r, r.o & (kSlots - 1)) = (len << 8) | kind;
  ring_commit(r, kind, len, start);
}

struct LaneState {
  uint32_t st;    // current row byte offset
  uint32_t tok;   // start of the current token
  uint32_t lacc;  // position after the last accepting step (non-monotone)
  uint32_t lrow;  // row byte offset of that accepting state
  uint32_t cnt;   // counted tokens (count walk)
  uint32_t fb;    // the walk fell back at least once (non-monotone)
  // non-monotone count walk: lrow is left as kLazyRow and recomputed when a fallback needs
  // it, by walking from lst0, the row at block start lblk, up to lacc
  uint32_t lblk, lst0;
};
constexpr uint32_t kLazyRow = 0xFFFFFFFFu;

// The row after the accepting step at lacc - 1, walked from row st at position blk.
__device__ __forceinline__ uint32_t rewalk_row(const Tables &tb, const uint8_t *in, uint32_t st, uint32_t blk,
                                               uint32_t lacc) {
  for (uint32_t p = blk; p < lacc; ++p) st = entry(tb, st, in[p]) & kRowMask;
  return st;
}

// One transition on byte b at position p.  Emit walk: the step writes the candidate
// token into the next ring slot unconditionally (a later step overwrites it unless the
// token is kept), so only the chunk write-out is a branch.
template <bool EMIT, bool MONO>
__device__ __forceinline__ void step(LaneState &L, Ring &r, const Tables &tb, uint32_t b, uint32_t p) {
  const uint32_t e = entry(tb, L.st, b);
  if (EMIT) {
    const uint32_t len = p - L.tok;
    if (!r.direct) ring_at(r, r.o & (kSlots - 1)) = pack_word(e, len);
    if (e & kCountBit) ring_commit(r, e >> 24, len, L.tok);
  } else {
    L.cnt += e & kCountBit;
  }
  L.tok = (e & kEmitBit) ? p : L.tok;
  L.st = e & kRowMask;
  if (!MONO && (e & kAccBit)) {
    L.lacc = p + 1;
    L.lrow = L.st;
  }
}

template <bool EMIT>
__device__ __forceinline__ void put(LaneState &L, Ring &r, uint32_t kind, uint32_t end) {
  if (EMIT) ring_put(r, kind, end - L.tok, L.tok);
  else ++L.cnt;
}

// Loads the 16-byte block starting at in + blk, reading only bytes inside [0, n).
__device__ __forceinline__ uint4 load_block(const uint8_t *in, int64_t blk, uint32_t n) {
  if (blk >= 0 && blk + 16 <= (int64_t)n) return *reinterpret_cast<const uint4 *>(in + blk);
  uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t q = blk + k;
    if (q >= 0 && q < (int64_t)n) w[k >> 2] |= (uint32_t)in[q] << (8 * (k & 3));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Non-monotone automata: the walk reached FAIL (a dead end after a non-accepting
// state).  Longest match takes the last accepting position of the current token if
// there is one: emit it and re-scan from there, byte by byte, up to `upto`; with no
// accepting position since the token start the scan halts there (SINK).  The guard on
// fail != sink keeps the loop finite should a monotone table ever reach it.
//
// Bounded failed lookahead (Section 9 names the Theta(N^2) cost of naive longest match and
// its removal by remembering failed (state, position) pairs, as Reps does).  A trace that
// failed visited, after its last accepting step, only pairs from which no accepting state
// is reached before FAIL or the end of the re-scan; a re-scan that meets one of them fails
// the same way, so it stops there.  Up to kMemo failed traces are kept as cursors (position,
// row), advanced in step with the re-scan and compared at equal positions; cursors that
// meet merge, a dead one is dropped, and a new trace pushes out the oldest.  On a^N over
// {a, a+b, ;} a re-scan then stops two bytes in: linear work instead of quadratic.
constexpr int kMemo = 4;

template <bool EMIT>
__device__ __forceinline__ void recover(LaneState &L, Ring &r, const Tables &tb, const uint8_t *in, uint32_t upto) {
  uint32_t cp[kMemo], cr[kMemo];  // cursor positions (kNone: empty) and rows
#pragma unroll
  for (int k = 0; k < kMemo; ++k) cp[k] = kNone, cr[k] = 0;
  const uintptr_t base = reinterpret_cast<uintptr_t>(in);
  int64_t cb = INT64_MIN;  // position of the cached block (16-aligned in memory)
  uint4 cv = make_uint4(0, 0, 0, 0);
  L.fb = 1;
  while (L.st == tb.fail && tb.fail != tb.sink) {
    if (L.lacc > L.tok) {
      if (L.lrow == kLazyRow) L.lrow = rewalk_row(tb, in, L.lst0, L.lblk, L.lacc);
#pragma unroll
      for (int k = kMemo - 1; k > 0; --k) cp[k] = cp[k - 1], cr[k] = cr[k - 1];
      cp[0] = L.lacc;  // the trace that just failed, from its last accepting step on
      cr[0] = L.lrow;
      const uint32_t row = L.lrow >> kRowShift;
      if (tb.info[row] & kInfoCount) put<EMIT>(L, r, tb.kind[row], L.lacc);
      L.tok = L.lacc;
      L.st = tb.start;
      for (uint32_t p = L.tok; p < upto; ++p) {
        // bytes through a 16-byte block held in registers (one load per block, not per byte)
        const int64_t blk = (int64_t)p - (int64_t)((base + p) & 15);
        if (blk != cb) {
          cb = blk;
          cv = load_block(in, blk, upto);
        }
        const uint32_t q = (uint32_t)((int64_t)p - blk);
        const uint32_t w4 = q < 4 ? cv.x : q < 8 ? cv.y : q < 12 ? cv.z : cv.w;
        const uint32_t b = (w4 >> (8 * (q & 3))) & 0xFFu;
        step<EMIT, false>(L, r, tb, b, p);
        bool join = false;
#pragma unroll
        for (int k = 0; k < kMemo; ++k) {
          if (cp[k] == p) {
            cr[k] = entry(tb, cr[k], b) & kRowMask;
            cp[k] = cr[k] == tb.fail ? kNone : p + 1;
          }
          join |= cp[k] == p + 1 && cr[k] == L.st;
        }
#pragma unroll
        for (int k = 1; k < kMemo; ++k)
#pragma unroll
          for (int j = 0; j < k; ++j)
            if (cp[k] == cp[j] && cr[k] == cr[j]) cp[k] = kNone;
        if (L.st == tb.fail) break;
        if (join) {
          L.st = tb.fail;  // a failed pair: this trace fails as that one did
          break;
        }
      }
    } else {
      L.st = tb.sink;
    }
  }
}

// End of the slice: an accepting state emits its token; a non-accepting one halts
// (monotone) or falls back (non-monotone).  Returns true if the slice halted.
template <bool EMIT, bool MONO>
__device__ __forceinline__ bool finish(LaneState &L, Ring &r, const Tables &tb, const uint8_t *in, uint32_t end) {
  for (;;) {
    if (!MONO && L.st == tb.fail) {
      recover<EMIT>(L, r, tb, in, end);
      continue;
    }
    if (L.st == tb.start) return false;
    if (L.st == tb.sink) return true;
    const uint32_t row = L.st >> kRowShift;
    if (tb.info[row] & kInfoAcc) {
      if (tb.info[row] & kInfoCount) put<EMIT>(L, r, tb.kind[row], end);
      L.tok = end;
      L.st = tb.start;
      return false;
    }
    if (MONO) {
      L.st = tb.sink;
      return true;
    }
    L.st = tb.fail;  // end of input after a non-accepting state: fall back
  }
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &v, int k) {
  const uint32_t w = k < 4 ? v.x : k < 8 ? v.y : k < 12 ? v.z : v.w;
  return (w >> (8 * (k & 3))) & 0xFFu;
}

// The 128-byte memory line at position P of in[0, n) (in + P is 128-aligned; bytes
// outside [0, n) read as 0).
__device__ __forceinline__ void load_line(const uint8_t *in, int64_t P, uint32_t n, uint4 (&v)[8]) {
  if (P >= 0 && P + 128 <= (int64_t)n) {
    const uint4 *src = reinterpret_cast<const uint4 *>(in + P);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = src[i];
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = load_block(in, P + 16 * i, n);
  }
}

// Bits [lo, hi) of the 32-bit word that covers bits [32 w, 32 w + 32) of a longer mask.
__device__ __forceinline__ uint32_t range_word(int64_t lo, int64_t hi, int w) {
  const int64_t a = min<int64_t>(32, max<int64_t>(0, lo - 32 * w));
  const int64_t b = min<int64_t>(32, max<int64_t>(0, hi - 32 * w));
  const uint32_t below_b = b >= 32 ? ~0u : (1u << (uint32_t)b) - 1u;
  const uint32_t below_a = a >= 32 ? ~0u : (1u << (uint32_t)a) - 1u;
  return below_b & ~below_a;
}

// Checkpoints of the count walk for the windowed emit.  Windows are the kWin-aligned
// stretches of the input's address space: window i starts at position i * kWin - mis0
// (mis0 = the input's address modulo kWin).  When a lane's walk reaches a window start
// strictly inside its slice it records, for that window, the row it is in before reading
// the byte, the tokens it has counted so far and the start of the token in progress.
//
// Storage: a window whose start lies k = (start - j l) / kWin windows into lane j's nominal
// range [j l, (j + 1) l) keeps its checkpoint in main when k < kslots, in blocks of kCkB
// consecutive windows per lane with the lanes interleaved block by block (ck_index): the
// lanes of a wave, which cross their k-th windows at about the same step, write nearly
// contiguous bytes, and the emit, whose 64-window tiles cover one or two lanes, uses kCkB
// checkpoints of every cache line it reads.  The rare windows further out (a slice running
// far past its lane) go to over[window index].
constexpr uint32_t kCkB = 2;
__host__ __device__ inline size_t ck_index(uint32_t k, uint32_t j, uint32_t nlanes) {
  return ((size_t)(k / kCkB) * nlanes + j) * kCkB + k % kCkB;
}
struct CkSink {
  uint2 *main;      // null: off
  uint2 *over;
  uint32_t nlanes, kslots, j, jl;  // jl = j * lane_bytes
  uint32_t mis0;
  uintptr_t base;   // address of the input
};

__device__ __forceinline__ uint2 ck_value(const LaneState &L) {
  return make_uint2(((L.st >> kRowShift) << 24) | L.cnt, L.tok);
}

__device__ __forceinline__ void ck_store(const CkSink &c, uint2 v, uint32_t blk) {
  const uint32_t k = (blk - c.jl) / kWin;
  if (k < c.kslots) c.main[ck_index(k, c.j, c.nlanes)] = v;
  else c.over[(blk + c.mis0) / kWin] = v;
}

__device__ __forceinline__ void ck_record(const CkSink &c, const LaneState &L, uint32_t blk) {
  ck_store(c, ck_value(L), blk);
}

// The two window starts of a 128-byte line at blk (a line start, so both lie strictly inside
// the slice when the first does, r0, or only the second): both checkpoints in one 16-byte
// store when they form one block of ck_index, else one by one.
__device__ __forceinline__ void ck_pair(const CkSink &c, bool r0, uint2 c0, const LaneState &L, uint32_t blk) {
  const uint2 c1 = ck_value(L);
  const uint32_t k0 = (blk - c.jl) / kWin;
  if (r0 && k0 % 2 == 0 && k0 + 1 < c.kslots) {  // kCkB is even: k0 and k0 + 1 share a block
    *reinterpret_cast<uint4 *>(c.main + ck_index(k0, c.j, c.nlanes)) = make_uint4(c0.x, c0.y, c1.x, c1.y);
    return;
  }
  if (r0) ck_store(c, c0, blk);
  ck_store(c, c1, blk + kWin);
}

__device__ __forceinline__ void ck_maybe(const CkSink &c, const LaneState &L, uint32_t blk) {
  if (c.main && ((c.base + blk) & (kWin - 1)) == 0) ck_record(c, L, blk);
}

// A full 16-byte block, unmasked.  FAST: the lane uses the packed ring and writes no
// offsets (see Ring), so the emit steps need no branch.
template <bool EMIT, bool MONO, bool FAST>
__device__ __forceinline__ void block16(LaneState &L, Ring &r, const Tables &tb, const uint4 &v, uint32_t blk) {
  if (!EMIT && !MONO) {
    // count walk of a non-monotone automaton: each step shifts its COUNT and EMIT bits into
    // m (step k's pair lands in bits 2k, 2k + 1) and its ACC bit into a (bit 16 + k); the
    // last accepting step's row is recomputed only if a fallback needs it (kLazyRow)
    uint32_t m = 0, ac = 0, e = L.st;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      e = entry_from(tb, e, byte_of(v, k));
      m = __builtin_amdgcn_alignbit(e, m, 2);
      ac = __builtin_amdgcn_alignbit(e >> 7, ac, 1);
    }
    const uint32_t st0 = L.st;
    L.st = e & kRowMask;
    L.cnt += __builtin_popcount(m & 0x55555555u);
    const uint32_t me = m & 0xAAAAAAAAu;  // bit 2k + 1: step k emitted
    L.tok = me ? blk + ((31 - __clz(me)) >> 1) : L.tok;
    if (ac) {
      L.lacc = blk + (31 - __clz(ac)) - 15;  // one past the last accepting step
      L.lrow = kLazyRow;
      L.lblk = blk;
      L.lst0 = st0;
    }
    return;
  }
  if (!EMIT && MONO) {
    // count walk of a monotone automaton: the COUNT and EMIT bits of the 16 steps are
    // shifted into m (step k's pair lands in bits 2k, 2k + 1) and the COUNT bits popcounted
    // once.
    uint32_t m = 0, e = L.st;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      e = entry_from(tb, e, byte_of(v, k));
      m = __builtin_amdgcn_alignbit(e, m, 2);
    }
    L.st = e & kRowMask;
    L.cnt += __builtin_popcount(m & 0x55555555u);
    // start of the token in progress: the last step at which a token ended, kept or
    // discarded (only read by checkpoints)
    const uint32_t me = m & 0xAAAAAAAAu;
    L.tok = me ? blk + ((31 - __clz(me)) >> 1) : L.tok;
    return;
  }
  if (EMIT && FAST) {
    {
      // packed emit walk: no branch per byte; chunks are split off after 8 and 16 bytes.
      // Non-monotone automata also track the last accepting step; a FAIL reached inside
      // the block stays in the FAIL row (no flags) to the block's end, and the caller's
      // fallback re-scans from that step.
      uint32_t st = L.st, tok = L.tok, o = r.o, lacc = L.lacc, lrow = L.lrow;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t p = blk + k;
        const uint32_t e = entry(tb, st, byte_of(v, k));
        ring_at(r, o & (kSlots - 1)) = pack_word(e, p - tok);
        o += e & kCountBit;
        tok = (e & kEmitBit) ? p : tok;
        st = e & kRowMask;
        if (!MONO) {
          lacc = (e & kAccBit) ? p + 1 : lacc;
          lrow = (e & kAccBit) ? st : lrow;
        }
        if (k == 7 || k == 15) {
          r.o = o;
          ring_maybe_split(r);
        }
      }
      L.st = st;
      L.tok = tok;
      if (!MONO) {
        L.lacc = lacc;
        L.lrow = lrow;
      }
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) step<EMIT, MONO>(L, r, tb, byte_of(v, k), blk + k);
}

// Walks the slice [s, e) of in[0, n); returns true if it halted (error inside).
// Input is read in whole 128-byte lines (eight 16-byte loads issued together and
// consumed from registers), so each cache line is fetched once and used at once
// instead of staying half-read in L2 while thousands of other lanes stream past it.
// The slice's unaligned head and tail go through 16-byte blocks, masked per byte at
// the slice ends.
template <bool EMIT, bool MONO, bool FAST, bool CK = false>
__device__ __forceinline__ bool walk(LaneState &L, Ring &r, const Tables &tb, const uint8_t *in, uint32_t n, uint32_t s,
                     uint32_t e, const CkSink &ck = CkSink{}) {
  L.st = tb.start;
  L.tok = s;
  L.lacc = s;
  L.lrow = tb.start;
  L.fb = 0;
  if (s >= e) return false;
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(in + s) & 15);
  int64_t b0 = (int64_t)s - mis;
  {  // first (masked) block
    const uint4 v = load_block(in, b0, n);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t p = b0 + k;
      if (p >= (int64_t)s && p < (int64_t)e) step<EMIT, MONO>(L, r, tb, byte_of(v, k), (uint32_t)p);
    }
    b0 += 16;
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, r, tb, in, (uint32_t)min<int64_t>(b0, e));
  }
  if (b0 >= (int64_t)e) return finish<EMIT, MONO>(L, r, tb, in, e);
  uint32_t blk = (uint32_t)b0;  // > s and 16-aligned in memory from here on
  // Lines of kBlocks blocks: whole 128-byte lines for the count walk and the packed
  // emit walk, single blocks for the generic emit walk.
  constexpr int kBlocks = EMIT ? (FAST && MONO ? 8 : 1) : 8;
  // full blocks up to a line boundary
  while (blk + 16 <= e && (reinterpret_cast<uintptr_t>(in + blk) & (16 * kBlocks - 1))) {
    const uint4 v = *reinterpret_cast<const uint4 *>(in + blk);
    if (CK) ck_maybe(ck, L, blk);
    block16<EMIT, MONO, FAST>(L, r, tb, v, blk);
    blk += 16;
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, r, tb, in, blk);
  }
  while (blk + 16 * kBlocks <= e) {
    uint4 v[kBlocks];
    const uint4 *src = reinterpret_cast<const uint4 *>(in + blk);
#pragma unroll
    for (int i = 0; i < kBlocks; ++i) v[i] = src[i];
#pragma unroll
    for (int i = 0; i < kBlocks; ++i) {
      // a line starts on a 128-byte boundary, so its blocks 0 and 4 start windows
      if (CK && ck.main && (i * 16) % kWin == 0) ck_record(ck, L, blk);
      block16<EMIT, MONO, FAST>(L, r, tb, v[i], blk);
      blk += 16;
      if (!MONO && L.st == tb.fail) recover<EMIT>(L, r, tb, in, blk);
    }
  }
  // remaining full blocks, then the masked last block
  while (blk + 16 <= e) {
    const uint4 v = *reinterpret_cast<const uint4 *>(in + blk);
    if (CK) ck_maybe(ck, L, blk);
    block16<EMIT, MONO, FAST>(L, r, tb, v, blk);
    blk += 16;
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, r, tb, in, blk);
  }
  if (blk < e) {
    if (CK) ck_maybe(ck, L, blk);
    const uint4 v = load_block(in, blk, n);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t p = blk + k;
      if (p < e) step<EMIT, MONO>(L, r, tb, byte_of(v, k), p);
    }
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, r, tb, in, e);
  }
  return finish<EMIT, MONO>(L, r, tb, in, e);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int d = 32; d; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d));
  return v;
}

// Certified bytes of a 16-byte block as a 16-bit mask (bit k = byte k).
__device__ __forceinline__ uint32_t match16(const uint4 &v, const CertArg &ca, const uint8_t *lut) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t x = 0;
    if (ca.np >= 0) {
      uint32_t z = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i)  // fixed trip count: the patterns stay in registers
        if (i < ca.np) z |= zero_bytes(w[q] ^ ca.pat[i]);
      x = gather4(z);
    } else {
      x = match_word_lut(w[q], lut);
    }
    m |= x << (4 * q);
  }
  return m;
}

// Count walk of a monotone automaton over the slice [s, e) in whole 128-byte memory lines,
// the lanes of a wave stepping through their lines together (same result as
// walk<false, true, false>; a per-lane head, body and tail would leave most lanes idle while
// the others finish theirs).  A line inside the slice of every lane still walking takes the
// plain path; otherwise every lane takes the masked path, where the row is held at the start
// before s, frozen from e on, and count bits outside [s, e) are dropped.  Lanes past their
// last line walk along and keep nothing.  CK records the checkpoints of walk<..., CK>: the
// window starts of each line that lie strictly inside the slice.  Every lane of the wave
// must call this in the same control flow; `live` is false for lanes without a slice.
// Returns true if the slice halted.
template <bool CK>
__device__ __forceinline__ bool walk_lines(LaneState &L, Ring &r, const Tables &tb, const uint8_t *in, uint32_t n,
                                           uint32_t s, uint32_t e, bool live, const CkSink &ck) {
  L.st = tb.start;
  L.tok = s;
  L.lacc = s;
  L.lrow = tb.start;
  L.cnt = 0;
  L.fb = 0;
  live = live && s < e;
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(in) & 127);
  const int64_t P0 = (((int64_t)s + mis) & ~int64_t(127)) - mis;  // the line holding s
  const uint32_t nl = live ? (uint32_t)(((int64_t)e - P0 + 127) >> 7) : 0;
  const uint32_t maxl = wave_max(nl);
  for (uint32_t li = 0; li < maxl; ++li) {
    const int64_t P = P0 + 128 * (int64_t)li;
    const bool mine = li < nl;
    const bool full = !mine || (P >= (int64_t)s && P + 128 <= (int64_t)e);
    uint4 v[8];  // a lane past its last line reloads that line (any defined bytes do)
    load_line(in, mine ? P : P0 + 128 * (int64_t)(nl ? nl - 1 : 0), n, v);
    const uint32_t st0 = L.st, cnt0 = L.cnt, tok0 = L.tok;
    const uint32_t blk = (uint32_t)P;  // positions blk + q modulo 2^32
    if (__all(full)) {
      // the line's two window starts: a pair of checkpoints for one lane (one 16-byte store
      // when they fill one block of ck_index)
      uint2 c0 = make_uint2(0, 0);
      bool r0 = false;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (CK && i == 0 && ck.main && mine && P > (int64_t)s) {
          c0 = ck_value(L);
          r0 = true;
        }
        if (CK && i == 4 && ck.main && mine) ck_pair(ck, r0, c0, L, blk);
        block16<false, true, false>(L, r, tb, v[i], blk + 16 * i);
      }
    } else {
      // steps q < lo are before s, q >= hi at or after e (clamped: q and 16 i lie in [0, 128))
      const int lo = (int)max<int64_t>(-1, min<int64_t>(128, (int64_t)s - P));
      const int hi = (int)max<int64_t>(0, min<int64_t>(129, (int64_t)e - P));
      uint32_t st = L.st;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (CK && i % 4 == 0 && ck.main && mine && 16 * i > lo && 16 * i < hi) {
          L.st = st & kRowMask;
          ck_record(ck, L, blk + 16 * i);
        }
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int q = 16 * i + k;
          const uint32_t y = entry_from(tb, st, byte_of(v[i], k));
          st = q < lo ? tb.start : q < hi ? y : st;
          m = __builtin_amdgcn_alignbit(y, m, 2);
        }
        // bits 2k, 2k + 1: COUNT and EMIT of step 16 i + k, kept for the steps in [lo, hi)
        m &= range_word(2 * (lo - 16 * i), 2 * (hi - 16 * i), 0);
        L.cnt += __builtin_popcount(m & 0x55555555u);
        const uint32_t me = m & 0xAAAAAAAAu;
        L.tok = me ? blk + 16 * i + ((31 - __clz(me)) >> 1) : L.tok;
      }
      L.st = st & kRowMask;
    }
    if (!mine) {
      L.st = st0;
      L.cnt = cnt0;
      L.tok = tok0;
    }
  }
  if (!live) return false;
  return finish<false, true>(L, r, tb, in, e);
}

struct WalkArgs {
  const uint32_t *table;  // global copies, staged into LDS
  const uint8_t *rowinfo;
  const uint8_t *rowkind;
  int nrows;
  uint32_t sink, fail;    // row byte offsets (fail == sink for monotone automata)
  const uint8_t *in;
  uint32_t n;
  uint32_t *cuts;         // lane boundaries (pipeline: planned; fused: recorded starts)
  uint32_t lane_bytes;    // fused path: targets
  uint32_t nlanes;
  const uint8_t *cert;    // fused path: global 256-byte LUT of the useful map
  CertArg ca;             // fused path: the useful map as SWAR patterns
  uint32_t *ends;         // fused path: slice ends recorded by the count walk
  uint32_t *counts;
  uint64_t *blk_sum;
  uint32_t *blk_fail;
  uint32_t *blk_nonempty;
  uint32_t *blk_big;
  uint32_t *lane_pre;     // exclusive prefix of counts inside the workgroup
  uint2 *ck;              // checkpoints (windowed emit), null when not recorded: main part
  uint2 *ck_over;         // and overflow (see CkSink)
  uint32_t kslots;
  int32_t *lnz;           // per lane: last non-empty lane at or before it in its workgroup, or -1
  int32_t *blk_lnz;       // per workgroup: last non-empty lane (count); before it (after the scan)
  uint32_t block;         // lanes per count workgroup (lane_pre's groups)
  uint32_t block_shift;   // log2(block)
  FastDiv lane_div;       // division by lane_bytes
  int fallback_only;      // one pass: the lane emit runs only for the scans the one-pass kernel left
  uint64_t *chunk_st;     // one pass: look-back status per workgroup of lanes
  uint32_t *chunk_ctr;    // one pass: next workgroup of lanes to take
  // emit
  const uint32_t *meta;
  ResultDev *res;
  uint8_t *kinds;
  uint32_t *lens;
  uint64_t *offs;
  uint64_t cap;
};

// Dynamic LDS layout of the walk kernels: table | rowinfo | rowkind | lut (256) |
// reduction scratch | ring or stage.  The walk kernels must declare no static LDS, so that
// the table sits at LDS address 0 (entry_from addresses it absolutely).
struct Lds {
  uint32_t *T;
  uint8_t *info, *kind, *lut;
  uint64_t *red64;   // 16
  uint32_t *red32;   // 32
  uint32_t *xchg;    // blockDim (count walk: slice starts)
  uint8_t *ring;     // blockDim * kRingBytes (emit walk)
};

__host__ __device__ inline size_t lds_ring_offset(int nrows) {
  return align16((size_t)nrows * 1024 + 2 * (size_t)nrows + 256) + 16 * 8 + 32 * 4;
}
__host__ __device__ inline size_t lds_bytes(int nrows, int block, bool emit) {
  return lds_ring_offset(nrows) + (size_t)block * (emit ? kRingBytes : 4);
}

__device__ __forceinline__ Lds carve_lds(int nrows) {
  extern __shared__ __align__(16) uint8_t smem[];
  Lds l;
  l.T = reinterpret_cast<uint32_t *>(smem);
  l.info = smem + (size_t)nrows * 1024;
  l.kind = l.info + nrows;
  l.lut = l.kind + nrows;
  uint8_t *p = smem + align16((size_t)nrows * 1024 + 2 * (size_t)nrows + 256);
  l.red64 = reinterpret_cast<uint64_t *>(p);
  l.red32 = reinterpret_cast<uint32_t *>(p + 16 * 8);
  l.ring = smem + lds_ring_offset(nrows);
  l.xchg = reinterpret_cast<uint32_t *>(l.ring);  // the count walk has no ring
  return l;
}

__device__ __forceinline__ void stage_tables(const WalkArgs &a, const Lds &l, bool fused) {
  const int words = a.nrows * 256;
  const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
  uint4 *dst = reinterpret_cast<uint4 *>(l.T);
  for (int i = threadIdx.x; i < words / 4; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < a.nrows; i += blockDim.x) {
    l.info[i] = a.rowinfo[i];
    l.kind[i] = a.rowkind[i];
  }
  if (fused)
    for (int i = threadIdx.x; i < 256; i += blockDim.x) l.lut[i] = a.cert[i];
  __syncthreads();
}

// Fused planning: the first certified byte in [x, x + span) (or `none`), 16 bytes at a
// time.
__device__ __forceinline__ uint32_t search_cert(const uint8_t *in, uint32_t n, const CertArg &ca, const uint8_t *lut, uint32_t x,
                                uint32_t span, uint32_t none) {
  const uint32_t end = (uint32_t)min<uint64_t>((uint64_t)x + span, n);
  int64_t blk = (int64_t)x - (int64_t)(reinterpret_cast<uintptr_t>(in + x) & 15);
  // four 16-byte blocks per step, loaded together: one load latency per 64 bytes searched
  for (; blk < (int64_t)end; blk += 64) {
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = load_block(in, blk + 16 * q, n);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t b = blk + 16 * q;
      if (b >= (int64_t)end) return none;
      uint32_t m = match16(v[q], ca, lut);
      if (b < (int64_t)x) m &= ~0u << (uint32_t)((int64_t)x - b);       // bytes before x (first block only)
      if (b + 16 > (int64_t)end) m &= (1u << (uint32_t)(end - b)) - 1;  // bytes at or after end
      if (m) return (uint32_t)b + (__ffs(m) - 1);
    }
  }
  return none;
}

// Lane j's slice.  Pipeline: [cuts[j], cuts[j+1]).  Fused: [c(j l), c((j+1) l)) with c(x)
// = first certified byte at or after x.  The start search is bounded by one lane length
// (no certified byte there means the slice is empty, because then c(j l) = c((j+1) l));
// the end is the next lane's start when that lane found one, which the lanes of a
// workgroup exchange through LDS, and a search of its own otherwise.  Every lane of the
// workgroup must call this (it holds a barrier).
template <bool FUSED>
__device__ __forceinline__ void lane_slice(const WalkArgs &a, uint32_t j, const uint8_t *lut, uint32_t *xchg,
                                           uint32_t &s, uint32_t &e) {
  if (!FUSED) {
    if (j < a.nlanes) {
      s = a.cuts[j];
      e = a.cuts[j + 1];
    }
    return;
  }
  const uint64_t x = (uint64_t)j * a.lane_bytes, x1 = x + a.lane_bytes;
  uint32_t start = kNone;  // kNone: no certified byte in [x, x1)
  if (j < a.nlanes) {
    if (j == 0) start = 0;
    else if (x < a.n) start = search_cert(a.in, a.n, a.ca, lut, (uint32_t)x, a.lane_bytes, kNone);
  }
  xchg[threadIdx.x] = start;
  __syncthreads();
  if (j >= a.nlanes) return;
  if (start == kNone) {  // empty slice
    s = e = (uint32_t)min<uint64_t>(x, a.n);
    return;
  }
  s = start;
  if (j + 1 == a.nlanes || x1 >= a.n) {
    e = a.n;
    return;
  }
  const uint32_t next = threadIdx.x + 1 < blockDim.x ? xchg[threadIdx.x + 1] : kNone;
  e = next != kNone ? next : search_cert(a.in, a.n, a.ca, lut, (uint32_t)x1, a.n - (uint32_t)x1, a.n);
}

__device__ __forceinline__ CkSink ck_sink(const WalkArgs &a, uint32_t j) {
  CkSink ck{};
  ck.base = reinterpret_cast<uintptr_t>(a.in);
  ck.main = a.ck;
  ck.over = a.ck_over;
  ck.nlanes = a.nlanes;
  ck.kslots = a.kslots;
  ck.j = j;
  ck.jl = j * a.lane_bytes;
  ck.mis0 = (uint32_t)(ck.base & (kWin - 1));
  return ck;
}

// CK: record checkpoints for the windowed emit.
template <bool MONO, bool FUSED, bool CK>
__global__ void __launch_bounds__(1024) k_count(WalkArgs a) {
  const Lds l = carve_lds(a.nrows);
  stage_tables(a, l, FUSED);
  const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t cnt = 0, fail = kNone, nonempty = 0, big = 0;
  uint32_t s = 0, e = 0;
  const bool active = j < a.nlanes;
  lane_slice<FUSED>(a, j, l.lut, l.xchg, s, e);
  LaneState L;
  L.cnt = 0;
  Ring r{};
  bool halted = false;
  if (MONO) {
    // every lane of the wave walks its lines together (walk_lines holds wave votes)
    CkSink ck{};
    if (CK) ck = ck_sink(a, j);
    // the younger half of each SIMD's waves (slots 2 and 3 of 4) issue first: the SIMD's
    // arbiter otherwise favours the older waves, and a CU's walk ends with its youngest
    const uint32_t slot = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 4) & 3;  // HW_ID wave slot
    if (slot >= 2) __builtin_amdgcn_s_setprio(1);
    halted = walk_lines<CK>(L, r, tb, a.in, a.n, s, e, active, ck);
    __builtin_amdgcn_s_setprio(0);
    // checkpoints hold the count in 24 bits: after a longer slice the windowed emit
    // stands down for the whole scan
    if (CK) big = active && e - s >= (1u << 24);
  } else {
    // non-monotone automata: checkpoints as above; they describe the serial scan only while
    // the lane never fell back (a re-scan revisits positions whose checkpoints the first
    // pass wrote), so a fallback stands the windowed emit down like a long slice
    CkSink ck{};
    if (CK) ck = ck_sink(a, j);
    if (active) halted = walk<false, false, false, CK>(L, r, tb, a.in, a.n, s, e, ck);
    if (CK) big = active && (e - s >= (1u << 24) || L.fb);
  }
  if (active && FUSED) {
    a.cuts[j] = s;
    a.ends[j] = e;
  }
  if (active) {
    cnt = L.cnt;
    a.counts[j] = cnt;
    if (halted) fail = j;
    nonempty = s < e;
  }
  // block reductions: exclusive prefix and sum of counts, min failing lane, non-empty
  // count, any long slice
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t incl = cnt;
  int32_t lnz = j < a.nlanes && nonempty ? (int32_t)j : -1;  // last non-empty lane so far
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(incl, d);
    const int32_t z = __shfl_up(lnz, d);
    if (lane >= d) {
      incl += v;
      lnz = max(lnz, z);
    }
  }
  for (int d = 32; d; d >>= 1) {
    fail = min(fail, (uint32_t)__shfl_xor((int)fail, d));
    nonempty += __shfl_xor(nonempty, d);
    big |= __shfl_xor(big, d);
  }
  // red64[w]: the wave's count sum (low half) and last non-empty lane (high half)
  if (lane == 63) l.red64[wid] = ((uint64_t)(uint32_t)lnz << 32) | incl;
  if (lane == 0) {
    l.red32[wid] = fail;
    l.red32[16 + wid] = nonempty | (big << 31);
  }
  __syncthreads();
  uint32_t pre = 0;
  for (int w = 0; w < wid; ++w) {
    pre += (uint32_t)l.red64[w];
    lnz = max(lnz, (int32_t)(l.red64[w] >> 32));
  }
  if (j < a.nlanes) {
    a.lane_pre[j] = pre + incl - cnt;
    a.lnz[j] = lnz;
  }
  if (threadIdx.x == 0) {
    uint64_t sum = 0;
    uint32_t f = kNone, ne = 0, bg = 0;
    for (int w = 0; w < nw; ++w) {
      sum += (uint32_t)l.red64[w];
      f = min(f, l.red32[w]);
      ne += l.red32[16 + w] & 0x7FFFFFFFu;
      bg |= l.red32[16 + w] >> 31;
    }
    a.blk_sum[blockIdx.x] = sum;
    a.blk_fail[blockIdx.x] = f;
    a.blk_nonempty[blockIdx.x] = ne;
    a.blk_big[blockIdx.x] = bg;
    int32_t z = -1;
    for (int w = 0; w < nw; ++w) z = max(z, (int32_t)(l.red64[w] >> 32));
    a.blk_lnz[blockIdx.x] = z;
  }
}

// (d) One workgroup: exclusive scan of block sums (in place), first halted lane,
// output length, status.
__global__ void __launch_bounds__(1024) k_scan(uint64_t *__restrict__ blk_sum, const uint32_t *__restrict__ blk_fail,
                                               const uint32_t *__restrict__ blk_nonempty,
                                               const uint32_t *__restrict__ blk_big,
                                               int32_t *__restrict__ blk_lnz, uint32_t nblocks,
                                               uint32_t block, const uint32_t *__restrict__ counts,
                                               uint32_t *__restrict__ meta, ResultDev *__restrict__ res, uint64_t cap,
                                               uint32_t n) {
  // each thread folds a contiguous range of workgroups; the ranges' sums, minima and maxima
  // are scanned inclusively within each wave by shuffles, across the waves through LDS
  __shared__ uint64_t wsum[16];
  __shared__ uint32_t wf[16], wn[16], any_big;
  __shared__ int32_t wz[16];
  const uint32_t tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t per = (nblocks + nt - 1) / nt;
  const uint32_t lo = min(nblocks, tid * per), hi = min(nblocks, lo + per);
  if (tid == 0) any_big = 0;
  __syncthreads();
  uint64_t s = 0;
  uint32_t f = kNone, ne = 0, bg = 0;
  int32_t z = -1;
  for (uint32_t i = lo; i < hi; ++i) {
    s += blk_sum[i];
    f = min(f, blk_fail[i]);
    ne += blk_nonempty[i];
    bg |= blk_big[i];
    z = max(z, blk_lnz[i]);
  }
  if (bg) atomicOr(&any_big, 1u);
  // inclusive scans within the wave
  uint64_t is = s;
  uint32_t iff = f, in = ne;
  int32_t iz = z;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t v = __shfl_up(is, d);
    const uint32_t vf = __shfl_up(iff, d), vn = __shfl_up(in, d);
    const int32_t vz = __shfl_up(iz, d);
    if (lane >= (uint32_t)d) {
      is += v;
      iff = min(iff, vf);
      in += vn;
      iz = max(iz, vz);
    }
  }
  if (lane == 63) {
    wsum[wid] = is;
    wf[wid] = iff;
    wn[wid] = in;
    wz[wid] = iz;
  }
  __syncthreads();
  // the earlier waves' totals
  uint64_t ps = 0;
  uint32_t pf = kNone, pn = 0;
  int32_t pz = -1;
  for (uint32_t w = 0; w < wid; ++w) {
    ps += wsum[w];
    pf = min(pf, wf[w]);
    pn += wn[w];
    pz = max(pz, wz[w]);
  }
  // exclusive prefixes of this thread's range, written back in place
  uint64_t run = ps + is - s;
  int32_t zrun = max(pz, (int32_t)__shfl_up(iz, 1));
  if (lane == 0) zrun = pz;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint64_t x = blk_sum[i];
    blk_sum[i] = run;
    run += x;
    const int32_t y = blk_lnz[i];
    blk_lnz[i] = zrun;  // last non-empty lane of the earlier workgroups
    zrun = max(zrun, y);
  }
  __syncthreads();
  if (tid == nt - 1) {
    const uint64_t total = ps + is;
    const uint32_t first = min(pf, iff);
    uint64_t ntok = total;
    if (first != kNone) {
      // tokens before the halted lane plus those it emitted before halting
      const uint32_t b = first / block;
      uint64_t pre = 0;
      for (uint32_t l = b * block; l < first; ++l) pre += counts[l];
      ntok = blk_sum[b] + pre + counts[first];
    }
    meta[0] = first;
    meta[1] = any_big;
    res->ntokens = ntok;
    res->error_offset = n;  // replaced by the halted lane in the emit pass
    res->status = ntok > cap ? -4 : 0;
    res->nslices = pn + in;
  }
}

// The lane emit of lane j: its slice walked again from its certified start, its tokens
// written from its first output slot through the thread's ring (column threadIdx.x of
// `ring`, blockDim.x columns).  The scan's first halted lane also reports the halt offset.
template <bool MONO, bool FUSED>
__device__ __forceinline__ void emit_lane(const WalkArgs &a, const Tables &tb, uint8_t *ring, uint32_t j,
                                          uint32_t first) {
  const uint64_t off = a.blk_sum[j >> a.block_shift] + a.lane_pre[j];
  const uint32_t s = a.cuts[j], e = FUSED ? a.ends[j] : a.cuts[j + 1];
  Ring r;
  r.w = reinterpret_cast<uint32_t *>(ring) + threadIdx.x;
  r.stride = blockDim.x;
  r.kinds = a.kinds;
  r.lens = a.lens;
  r.offs = a.offs;
  r.o = (uint32_t)off;
  r.fl = (uint32_t)off & ~(uint32_t)(kChunk - 1);
  r.first = (uint32_t)off;
  r.write = a.res->status == 0;
  r.direct = e - s >= (1u << 24);
  LaneState L;
  L.cnt = 0;
  if (!r.direct && !r.offs) walk<true, MONO, true>(L, r, tb, a.in, a.n, s, e);
  else walk<true, MONO, false>(L, r, tb, a.in, a.n, s, e);
  ring_flush_tail(r);
  if (j == first) a.res->error_offset = L.tok;  // the halt offset: start of the failed token
}

// The lane emit of every lane up to the first halted one, a thread per lane.
template <bool MONO, bool FUSED>
__global__ void __launch_bounds__(1024) k_emit(WalkArgs a) {
  const uint32_t first = a.meta[0];
  // beside the one-pass kernel, this kernel takes the scans that one cannot
  if (a.fallback_only && first == kNone && a.meta[1] == 0) return;
  const uint32_t j0 = blockIdx.x * blockDim.x;
  if (j0 > first) return;  // the whole block lies after the first halted lane
  const Lds l = carve_lds(a.nrows);
  stage_tables(a, l, FUSED);
  const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
  const uint32_t j = j0 + threadIdx.x;
  if (j >= a.nlanes || j > first) return;
  emit_lane<MONO, FUSED>(a, tb, l.ring, j, first);
}


// ---------------------------------------------------------- (e) windowed emit
// For a monotone automaton whose token ends are all counted, and a scan with no halted
// slice, the emit needs no lane-long walks.  Every lane starts at a certified byte, where
// the serial lexer also starts a token (Theorem 1), so the lanes' states, counts and token
// starts agree with the serial lexer's everywhere; the count walk left them at every
// window start.  One thread walks one kWin-byte window from its checkpoint, straight
// through any lane start inside it (for a monotone automaton the serial step there is
// the token end the lane walk took at its slice end), and finishes the input's last token.
//
// Windows in order, 64 to a wave: a wave's windows are a contiguous 4 KiB of input and own
// a contiguous range of output slots.  The wave stages that range in LDS as words
// (end - P) << 8 | kind, P being the start of the range's first token, and writes it out
// with 16-byte stores; lengths are the differences of consecutive ends.  A range longer
// than the stage (less its 64 spill words, which come first), or spanning 2^24 bytes or
// more, is written token by token instead.
//
// A window's output offset comes from the lane that owns its first byte: lane j0 =
// start / lane_bytes when that lane is not empty and starts at or before it, otherwise
// the last non-empty lane before j0 (slices tile the input, and a non-empty lane j starts
// inside [j l, (j + 1) l)).
constexpr int kWinWaves = 4;             // waves per workgroup of the one-pass kernel
constexpr uint32_t kStageWords = 1280;   // staged words per wave

__host__ __device__ inline size_t win_lds_bytes(int nrows, uint32_t waves = kWinWaves) {
  return lds_ring_offset(nrows) + (size_t)waves * kStageWords * 4;
}
// k_emit_win: a stage per wave, or a ring per thread when the scan takes the lane emit.
__host__ __device__ inline size_t emit_win_lds_bytes(int nrows, uint32_t waves) {
  const size_t stage = win_lds_bytes(nrows, waves), ring = lds_bytes(nrows, (int)waves * 64, true);
  return stage > ring ? stage : ring;
}
// Waves of a windowed-emit workgroup: 16, 8 or 4, the most whose LDS fits in a CU.
__host__ __device__ inline uint32_t win_waves(int nrows) {
  for (uint32_t w = 16; w > 4; w >>= 1)
    if (emit_win_lds_bytes(nrows, w) <= 160 * 1024) return w;
  return 4;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t row_state(uint32_t row) { return (row << kRowShift) | ((row & 31u) << 2); }

// First-round loads for window i (owner candidates).
struct WinR1 {
  uint32_t ws, j0, s0, e0;
  int32_t lz, bz;  // last non-empty lane at or before j0 - 1: in its workgroup; before it
};

template <bool FUSED>
__device__ __forceinline__ WinR1 win_r1(const WalkArgs &a, uint32_t i, uint32_t mis0, uint32_t nwin) {
  WinR1 r{};
  if (i >= nwin) return r;
  r.ws = i ? i * kWin - mis0 : 0;
  r.j0 = min(fdiv(r.ws, a.lane_div), a.nlanes - 1);
  r.s0 = a.cuts[r.j0];
  r.e0 = FUSED ? a.ends[r.j0] : a.cuts[r.j0 + 1];
  r.lz = r.j0 ? a.lnz[r.j0 - 1] : -1;
  r.bz = r.j0 ? a.blk_lnz[(r.j0 - 1) >> a.block_shift] : -1;
  return r;
}

// Second round: the state at the window's start and its first output slot (offsets fit
// 32 bits: a scan has fewer than 2^32 tokens).  Window nwin (past the end) gives ntok.
struct WinMeta {
  uint32_t st, tok, out;
  uint32_t fresh;  // a lane starts at the window's first byte
};

__device__ __forceinline__ WinMeta win_meta(const WalkArgs &a, const WinR1 &r, uint32_t i, uint32_t nwin,
                                            uint32_t ntok) {
  WinMeta m{0, 0, ntok, 0};
  if (i >= nwin) return m;
  const bool here = r.s0 < r.e0 && r.s0 <= r.ws;
  const uint32_t owner = here ? r.j0 : (uint32_t)(r.lz >= 0 ? r.lz : r.bz);
  const uint32_t base = (uint32_t)a.blk_sum[owner >> a.block_shift] + a.lane_pre[owner];
  if (here && r.s0 == r.ws) {  // the owner starts here: a fresh token
    m.tok = r.ws;
    m.out = base;
    m.fresh = 1;
    return m;
  }
  const uint32_t k = (r.ws - owner * a.lane_bytes) / kWin;
  const uint2 c = k < a.kslots ? a.ck[ck_index(k, owner, a.nlanes)] : a.ck_over[i];
  m.st = row_state(c.x >> 24);
  m.tok = c.y;
  m.out = base + (c.x & 0xFFFFFFu);
  return m;
}

// Output of the staged and the direct walk.
struct WinOut {
  uint32_t D, G;       // staged: LDS address of the lane's spill word G, and D such that
                       // G + D is the address of the next slot
  uint32_t base;       // staged: P
  uint32_t tok;        // direct: start of the token in progress
  uint32_t o, lim;     // direct: next output slot, end of the thread's range
};

// st carries the previous entry unmasked (or a row state); mask it before reading a row.
// DISC: some token ends are not counted (discarded kinds), so a staged word holds the kept
// token's length, p - tok, instead of its end (a length is then no difference of ends).
template <bool STAGED, bool DISC>
__device__ __forceinline__ void win_step(const Tables &tb, const WalkArgs &a, uint32_t &st, WinOut &w, uint32_t b,
                                         uint32_t p) {
  const uint32_t e = entry_from(tb, st, b);
  if (STAGED) {
    // every step writes its word: to the next slot when a counted token ends here (the
    // slot then advances), else to the lane's spill word.  G + c * D with c in {0, 1} is
    // one 24-bit multiply-add, and the write needs no branch.  (Writing only on token
    // ends saves LDS traffic but costs more in exec-mask handling than it saves.)
    const uint32_t c = e & kCountBit;
    __builtin_assume(w.D < 4 * kStageWords);  // the slots lie above the spill words
    *(lds_u32 *)(size_t)(__umul24(c, w.D) + w.G) =
        __builtin_amdgcn_perm(e, p - (DISC ? w.tok : w.base), 0x02010007u);
    w.D += c << 2;
    if (DISC) w.tok = (e & kEmitBit) ? p : w.tok;
  } else {
    if ((e & kCountBit) && w.o < w.lim) {
      a.kinds[w.o] = (uint8_t)(e >> 24);
      a.lens[w.o] = p - w.tok;
      if (a.offs) a.offs[w.o] = w.tok;
      ++w.o;
    }
    w.tok = (e & kEmitBit) ? p : w.tok;
  }
  st = e;
}

// The window's 64 bytes at position wp (its kWin-aligned start, possibly before 0).
struct Win64 {
  uint4 v[4];
};

template <bool EDGE>
__device__ __forceinline__ Win64 win_load(const uint8_t *in, int64_t wp, uint32_t n) {
  Win64 d;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t p = wp + 16 * q;
    if (EDGE) d.v[q] = (p >= 0 && p + 16 <= (int64_t)n) ? *reinterpret_cast<const uint4 *>(in + p) : load_block(in, p, n);
    else d.v[q] = *reinterpret_cast<const uint4 *>(in + p);
  }
  return d;
}

// Walks the window [wp, wp + 64) ∩ [0, n).  EDGE: some positions may lie outside.
template <bool STAGED, bool EDGE, bool DISC>
__device__ __forceinline__ void win_walk(const Tables &tb, const WalkArgs &a, const Win64 &d, int64_t wp,
                                         uint32_t n, uint32_t &st, WinOut &w) {
  const uint32_t p0 = (uint32_t)wp;  // positions p0 + k modulo 2^32; only those in [0, n) are walked
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t p = wp + 16 * q + k;
      if (!EDGE || (p >= 0 && p < (int64_t)n))
        win_step<STAGED, DISC>(tb, a, st, w, byte_of(d.v[q], k), p0 + 16 * q + k);
    }
  }
}

// One tile of 64 windows, window i on this lane (valid: i is one of the tile's windows;
// edge: some of its positions may lie outside [0, n)).  o_first: the tile's first output
// slot; o_end: one past its last output when `exact`, else a bound on it (the walk then
// counts the outputs); out_end: bound on this window's outputs (the next window's first
// slot when known); next_fresh: a lane starts at the next window's first byte; P: start of
// the token in progress at the tile's start; span_end: end of the tile's bytes; lim: no
// output at or above it.  Staged when the range fits the stage (see the kernel notes),
// else each token goes straight to global memory.  DISC (a mode with discarded kinds):
// staged words hold lengths, and a scan that asks for offsets goes straight to memory.
template <bool DISC>
__device__ __forceinline__ void win_tile(const Tables &tb, const WalkArgs &a, uint32_t *stage, uint32_t lane,
                                         const WinMeta &cur, uint32_t i, bool valid, bool edge, const Win64 &dat,
                                         int64_t wp, uint32_t nwin, uint32_t o_first, uint32_t o_end, bool exact,
                                         uint32_t out_end, uint32_t next_fresh, uint32_t P, uint32_t span_end,
                                         uint32_t lim) {
  const uint32_t stage_addr = (uint32_t)(size_t)(lds_u32 *)stage;
  // slot q holds output o_first - pad + q; pad >= 4 leaves slot pad - 1 free to hold end
  // 0, the start of the tile's first token (so every length is a difference of ends)
  const uint32_t pad = (o_first & 3) + 4;
  const bool staged = o_first <= o_end && o_end <= lim && o_end - o_first + pad + 3 <= kStageWords - 64 &&
                      span_end - P < (1u << 24) && !(DISC && a.offs);
  uint32_t st = cur.st;
  WinOut w;
  w.tok = cur.tok;
  uint32_t d0 = 0;
  if (staged) {
    // the spill word: one for the whole wave (the stage's first word; 64 are reserved), so
    // the lanes whose step ends no token all write one address and take no LDS bank from a
    // lane writing a slot; slots follow, so 0 < D < 4 * kStageWords
    w.G = stage_addr;
    w.D = d0 = 4 * (64 + pad + (cur.out - o_first));
    w.base = P;
    if (lane == 0) stage[64 + pad - 1] = 0;
    if (valid) {
      if (edge) win_walk<true, true, DISC>(tb, a, dat, wp, a.n, st, w);
      else win_walk<true, false, DISC>(tb, a, dat, wp, a.n, st, w);
    }
  } else {
    w.o = cur.out;
    w.lim = valid ? min(out_end, lim) : cur.out;
    if (valid) {
      if (edge) win_walk<false, true, DISC>(tb, a, dat, wp, a.n, st, w);
      else win_walk<false, false, DISC>(tb, a, dat, wp, a.n, st, w);
    }
  }
  // The input's end, or a lane starting at the next window's first byte: the token in
  // progress ends here, as the lane walk's slice end made it (the next window starts
  // afresh and does not see it).
  st &= kRowMask;
  if (valid && (i + 1 == nwin || next_fresh) && st != tb.start) {
    const uint32_t end = i + 1 == nwin ? a.n : (i + 1) * kWin - (uint32_t)(reinterpret_cast<uintptr_t>(a.in) & (kWin - 1));
    const uint32_t row = st >> kRowShift;
    if ((tb.info[row] & kInfoAcc) && (tb.info[row] & kInfoCount)) {
      if (staged) {
        *(lds_u32 *)(size_t)(w.G + w.D) = (uint32_t)tb.kind[row] | ((end - (DISC ? w.tok : P)) << 8);
        w.D += 4;
      } else if (w.o < w.lim) {
        a.kinds[w.o] = tb.kind[row];
        a.lens[w.o] = end - w.tok;
        if (a.offs) a.offs[w.o] = w.tok;
      }
    }
  }
  if (!staged) return;  // wave-uniform
  // the range's length: known, or counted by the walk (the last valid window's end slot)
  const uint32_t total = exact ? o_end - o_first
                               : wave_max(valid ? cur.out - o_first + (w.D - d0) / 4 : 0);
  wave_sync();
  // write the range out, four slots per lane and step: lengths are differences of
  // consecutive ends (slot pad - 1 holds 0) or, DISC, the words themselves; kinds the low
  // bytes
  const uint32_t o0 = o_first - pad;
  const uint32_t *slots = stage + 64;
  for (uint32_t q = 4 + lane * 4; q < pad + total; q += 256) {
    const uint4 v = *reinterpret_cast<const uint4 *>(slots + q);
    const uint32_t e0 = DISC ? 0 : slots[q - 1] >> 8, e1 = v.x >> 8, e2 = v.y >> 8, e3 = v.z >> 8, e4 = v.w >> 8;
    const uint4 len = DISC ? make_uint4(e1, e2, e3, e4) : make_uint4(e1 - e0, e2 - e1, e3 - e2, e4 - e3);
    const uint32_t kd = __builtin_amdgcn_perm(__builtin_amdgcn_perm(v.w, v.z, 0x0C0C0400u),
                                              __builtin_amdgcn_perm(v.y, v.x, 0x0C0C0400u), 0x05040100u);
    const uint32_t o = o0 + q;
    if (q >= pad && q + 4 <= pad + total) {
      *reinterpret_cast<uint4 *>(a.lens + o) = len;
      *reinterpret_cast<uint32_t *>(a.kinds + o) = kd;
      if (a.offs) {
        a.offs[o] = P + e0;
        a.offs[o + 1] = P + e1;
        a.offs[o + 2] = P + e2;
        a.offs[o + 3] = P + e3;
      }
    } else {
      const uint32_t lv[4] = {len.x, len.y, len.z, len.w}, sv[4] = {e0, e1, e2, e3};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (q + k >= pad && q + k < pad + total) {
          a.lens[o + k] = lv[k];
          a.kinds[o + k] = (uint8_t)(kd >> (8 * k));
          if (a.offs) a.offs[o + k] = P + sv[k];
        }
      }
    }
  }
  wave_sync();
}

// A tile is 64 windows.  A workgroup takes a contiguous range of tiles, and its waves
// draw single tiles from it in order through a counter in LDS until the range runs dry:
// the waves that the CU's arbitration lets run ahead take more tiles, so that they finish
// together instead of the oldest first (with fixed runs per wave the youngest waves of a
// CU finished 15% after its mean).  Software pipeline: the next tile's bytes and the
// state of the tile after it load while a tile walks.  A tile's last window ends where
// the first window of the tile after it (in the input) begins; that window's start is
// read for every tile, uniformly across the wave, since a wave's next tile is seldom the
// adjacent one.
//
// A scan with a halted slice, or a slice too long for the checkpoints, takes the lane emit
// instead, in the same launch: each thread emits lanes j, j + the grid's threads, ... up
// to the first halted lane.
template <bool FUSED, bool DISC, bool MONO>
__global__ void __launch_bounds__(1024) k_emit_win(WalkArgs a) {
  const uint32_t first = a.meta[0];
  const Lds l = carve_lds(a.nrows);
  if (first != kNone || a.meta[1] != 0) {  // uniform
    stage_tables(a, l, false);
    const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < a.nlanes && j <= first; j += gridDim.x * blockDim.x)
      emit_lane<MONO, FUSED>(a, tb, l.ring, j, first);
    return;
  }
  if (a.res->status != 0 || a.n == 0) return;
  uint32_t *ctr = l.red32;  // the workgroup's tile counter
  if (threadIdx.x == 0) *ctr = 0;
  stage_tables(a, l, false);  // its barrier publishes the zeroed counter
  const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t *stage = reinterpret_cast<uint32_t *>(l.ring) + wid * kStageWords;
  const uintptr_t base = reinterpret_cast<uintptr_t>(a.in);
  const uint32_t mis0 = (uint32_t)(base & (kWin - 1));
  const uint32_t nwin = (uint32_t)(((uint64_t)a.n + mis0 + kWin - 1) / kWin);
  const uint32_t ntiles = (nwin + 63) / 64;
  const uint32_t ntok = (uint32_t)a.res->ntokens;  // every store below stays under it
  const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t g_lo = min(ntiles, blockIdx.x * per), g_hi = min(ntiles, g_lo + per);
  bool more = true;
  auto take = [&]() -> uint32_t {  // the wave's next tile (wave-uniform), kNone at the end
    if (!more) return kNone;
    uint32_t k = 0;
    if (lane == 0) k = atomicAdd(ctr, 1u);
    const uint32_t t = g_lo + (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)k, 0));
    if (t >= g_hi) {
      more = false;
      return kNone;
    }
    return t;
  };
  uint32_t id0 = take(), id1 = take(), id2 = take();
  if (id0 == kNone) return;  // wave-uniform, and no workgroup barrier follows
  auto win_of = [&](uint32_t t) { return t == kNone ? nwin : t * 64 + lane; };
  auto after = [&](uint32_t t) { return t == kNone ? nwin : min(nwin, (t + 1) * 64); };  // uniform
  auto meta_of = [&](uint32_t i) { return win_meta(a, win_r1<FUSED>(a, i, mis0, nwin), i, nwin, ntok); };
  WinMeta cur = meta_of(win_of(id0)), cx = meta_of(after(id0));
  WinMeta nxt = meta_of(win_of(id1)), nx = meta_of(after(id1));
  WinR1 r1 = win_r1<FUSED>(a, win_of(id2), mis0, nwin), r1x = win_r1<FUSED>(a, after(id2), mis0, nwin);
  auto wpos = [&](uint32_t t) { return (int64_t)t * 64 * kWin + (int64_t)lane * kWin - mis0; };
  auto is_edge = [&](uint32_t t) { return t == 0 || t + 1 == ntiles; };
  Win64 dat = is_edge(id0) ? win_load<true>(a.in, wpos(id0), a.n) : win_load<false>(a.in, wpos(id0), a.n);
  while (id0 != kNone) {
    const uint32_t i = id0 * 64 + lane;
    Win64 ndat = dat;
    if (id1 != kNone)
      ndat = is_edge(id1) ? win_load<true>(a.in, wpos(id1), a.n) : win_load<false>(a.in, wpos(id1), a.n);
    // the state of the tile after next, and the first-round loads of the one after that:
    // issued here, they complete while this tile walks
    const WinMeta n2 = win_meta(a, r1, win_of(id2), nwin, ntok), n2x = win_meta(a, r1x, after(id2), nwin, ntok);
    const uint32_t id3 = take();
    r1 = win_r1<FUSED>(a, win_of(id3), mis0, nwin);
    r1x = win_r1<FUSED>(a, after(id3), mis0, nwin);
    // this window's range of output slots ends where the next window's begins
    // (every shuffle runs with the whole wave active: a lane reading from an inactive
    // lane gets no defined value)
    const uint32_t o_first = __shfl(cur.out, 0), o_next = cx.out;
    const uint32_t down = __shfl_down(cur.out, 1), fdown = __shfl_down(cur.fresh, 1);
    const uint32_t f_next = cx.fresh;
    const uint32_t P = __shfl(cur.tok, 0);  // start of the token in progress at the tile's start
    const uint32_t span_end = (uint32_t)min<int64_t>((int64_t)(id0 + 1) * 64 * kWin - mis0, a.n);
    win_tile<DISC>(tb, a, stage, lane, cur, i, i < nwin, is_edge(id0), dat, wpos(id0), nwin, o_first, o_next,
                   true, lane < 63 ? down : o_next, lane < 63 ? fdown : f_next, P, span_end, ntok);
    cur = nxt;
    cx = nx;
    nxt = n2;
    nx = n2x;
    dat = ndat;
    id0 = id1;
    id1 = id2;
    id2 = id3;
  }
}

// ------------------------------------------------- (b)-(e) in one pass over lane groups
// Windowed scans in one launch.  Each workgroup takes groups of 256 consecutive lanes in
// order from a counter and, for each group: plans and count-walks its lanes (as k_count,
// recording checkpoints); publishes the group's token total; finds the group's first output
// slot by a decoupled look-back over the earlier groups' published totals and prefixes
// (the counter hands groups out in order, so every earlier group is already running); then
// emits the windows whose first byte lies in its own lanes' slices [S, E) exactly as the
// windowed emit does.  The group's bytes are read a second time while still in the caches,
// and groups in different phases overlap the count walk's table lookups with the emit's
// stores.  Owners, prefixes and checkpoints all come from the group itself: the one thing a
// group needs about later ones is whether a lane starts at the first window after E, which
// it decides from the bytes there (a lane starts at y exactly when y is the first certified
// byte at or after the lane's target and lies before the next target).
//
// Each group also writes what k_count writes (slices, counts, prefixes, block totals and
// flags), so k_scan and the lane emit's fallback run after it unchanged: a halted slice, a
// slice too long for the checkpoints, or a look-back that did not finish (bounded spin)
// leaves the emit to them, and a group emits only when no earlier group halted.
constexpr uint64_t kStAgg = 1ull << 62, kStIncl = 2ull << 62, kStPoison = 1ull << 61;
constexpr uint64_t kStValue = (1ull << 61) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

__host__ __device__ inline size_t one_lds_bytes(int nrows) {
  return lds_ring_offset(nrows) + (size_t)kChunkLanes * 13 + 16 + (size_t)kWinWaves * kStageWords * 4;
}

// First window whose first byte is at or after position x (window 0 starts at 0, window
// i >= 1 at i * kWin - mis0).
__device__ __forceinline__ uint32_t win_from(uint32_t x, uint32_t mis0) {
  return x ? (uint32_t)(((uint64_t)x + mis0 + kWin - 1) / kWin) : 0;
}

struct GroupLds {
  const uint32_t *s, *e, *pre;  // per lane of the group: slice, exclusive prefix of counts
  const uint8_t *lnz;           // last non-empty lane at or before it (0xFF: none)
};

// Window i of a group's range [i_lo, i_hi): owner, state, token start and output slot.
// Past the range: out = bound, fresh = whether a lane starts at window i_hi.
__device__ __forceinline__ WinMeta group_meta(const WalkArgs &a, const GroupLds &g, uint32_t i, uint32_t i_hi,
                                              uint32_t c0, uint32_t last, uint32_t Pc, uint32_t mis0,
                                              uint32_t fresh_after, uint32_t bound) {
  WinMeta m{0, 0, bound, fresh_after};
  if (i >= i_hi) return m;
  const uint32_t W = i ? i * kWin - mis0 : 0;
  const uint32_t j0 = fdiv(W, a.lane_div);
  uint32_t o = last;  // a window past the group's nominal range lies in its last slice
  bool here = false;
  if (j0 < c0 + kChunkLanes) {
    const uint32_t q = j0 - c0;  // W >= S >= c0 * lane_bytes, so j0 >= c0
    here = g.s[q] < g.e[q] && g.s[q] <= W;
    o = here ? q : (q && g.lnz[q - 1] != 0xFF ? g.lnz[q - 1] : last);
  }
  const uint32_t base = Pc + g.pre[o];
  if (here && g.s[o] == W) {  // the owner starts here: a fresh token
    m.st = 0;
    m.tok = W;
    m.out = base;
    m.fresh = 1;
    return m;
  }
  const uint32_t j = c0 + o;
  const uint32_t k = (W - j * a.lane_bytes) / kWin;
  const uint2 c = k < a.kslots ? a.ck[ck_index(k, j, a.nlanes)] : a.ck_over[i];
  m.st = row_state(c.x >> 24);
  m.tok = c.y;
  m.out = base + (c.x & 0xFFFFFFu);
  m.fresh = 0;
  return m;
}

template <bool DISC>
__global__ void __launch_bounds__(256, 4) k_onepass(WalkArgs a) {  // four waves per SIMD: at most 128 VGPRs
  const Lds l = carve_lds(a.nrows);
  stage_tables(a, l, true);
  const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
  uint32_t *ls = reinterpret_cast<uint32_t *>(l.ring), *le = ls + kChunkLanes, *lpre = le + kChunkLanes;
  uint8_t *llnz = reinterpret_cast<uint8_t *>(lpre + kChunkLanes);
  uint32_t *bc = reinterpret_cast<uint32_t *>(llnz + kChunkLanes);  // group index, prefix, emit flag, fresh
  const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint32_t *stage = bc + 4 + wid * kStageWords;
  const uint32_t mis0 = (uint32_t)(reinterpret_cast<uintptr_t>(a.in) & (kWin - 1));
  const uint32_t nwin = (uint32_t)(((uint64_t)a.n + mis0 + kWin - 1) / kWin);
  const uint32_t ngroups = (a.nlanes + kChunkLanes - 1) / kChunkLanes;
  const uint32_t cap = (uint32_t)min<uint64_t>(a.cap, 0xFFFFFFFFu);
  const GroupLds g{ls, le, lpre, llnz};
  for (;;) {
    if (tid == 0) bc[0] = atomicAdd(a.chunk_ctr, 1u);
    __syncthreads();
    const uint32_t c = bc[0];
    if (c >= ngroups) break;  // the same for the whole workgroup
    const uint32_t c0 = c * kChunkLanes, j = c0 + tid;
    const bool active = j < a.nlanes;
    // ---- plan and count (as k_count); the slice exchange borrows le
    uint32_t s = 0, e = 0;
    lane_slice<true>(a, j, l.lut, le, s, e);
    LaneState L;
    L.cnt = 0;
    Ring r{};
    const bool halted = walk_lines<true>(L, r, tb, a.in, a.n, s, e, active, ck_sink(a, j));
    const uint32_t cnt = active ? L.cnt : 0;
    const bool nonempty = active && s < e;
    if (active) {
      a.cuts[j] = s;
      a.ends[j] = e;
      a.counts[j] = cnt;
    }
    uint32_t incl = cnt, fail = active && halted ? j : kNone, ne = nonempty, big = active && e - s >= (1u << 24);
    uint32_t smin = nonempty ? s : 0xFFFFFFFFu;
    int32_t lz = nonempty ? (int32_t)tid : -1;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d);
      const int32_t z = __shfl_up(lz, d);
      if (lane >= d) {
        incl += v;
        lz = max(lz, z);
      }
    }
    for (int d = 32; d; d >>= 1) {
      fail = min(fail, (uint32_t)__shfl_xor((int)fail, d));
      smin = min(smin, (uint32_t)__shfl_xor((int)smin, d));
      ne += __shfl_xor(ne, d);
      big |= __shfl_xor(big, d);
    }
    __syncthreads();  // every lane has read its neighbour's slice start from le
    if (lane == 63) l.red64[wid] = ((uint64_t)(uint32_t)lz << 32) | incl;
    if (lane == 0) {
      l.red32[wid] = fail;
      l.red32[4 + wid] = smin;
      l.red32[16 + wid] = ne | (big << 31);
    }
    __syncthreads();
    uint32_t pre = 0, T = 0, F = kNone, S = 0xFFFFFFFFu, NE = 0, BG = 0;
    int32_t zmax = -1;
    for (int w = 0; w < kWinWaves; ++w) {
      if (w < (int)wid) {
        pre += (uint32_t)l.red64[w];
        lz = max(lz, (int32_t)(l.red64[w] >> 32));
      }
      T += (uint32_t)l.red64[w];
      zmax = max(zmax, (int32_t)(l.red64[w] >> 32));
      F = min(F, l.red32[w]);
      S = min(S, l.red32[4 + w]);
      NE += l.red32[16 + w] & 0x7FFFFFFFu;
      BG |= l.red32[16 + w] >> 31;
    }
    const uint32_t epre = pre + incl - cnt;
    if (active) {
      a.lane_pre[j] = epre;
      a.lnz[j] = lz >= 0 ? (int32_t)(c0 + lz) : -1;
    }
    ls[tid] = s;
    le[tid] = e;
    lpre[tid] = epre;
    llnz[tid] = lz >= 0 ? (uint8_t)lz : 0xFF;
    if (tid == 0) {
      a.blk_sum[c] = T;
      a.blk_fail[c] = F;
      a.blk_nonempty[c] = NE;
      a.blk_lnz[c] = zmax >= 0 ? (int32_t)(c0 + zmax) : -1;
      // ---- publish the total, then look back for the prefix
      const bool poison = F != kNone || BG;
      __hip_atomic_store(&a.chunk_st[c], kStAgg | (poison ? kStPoison : 0) | T, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      uint64_t prefix = 0;
      bool any_poison = poison, ok = true;
      for (uint32_t q = c; q-- > 0;) {
        uint64_t w = 0;
        for (uint32_t spins = 0;; ++spins) {
          w = __hip_atomic_load(&a.chunk_st[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if ((w >> 62) != 0 || spins >= kSpinLimit) break;
          __builtin_amdgcn_s_sleep(2);
        }
        if ((w >> 62) == 0) {  // not published in time: leave this group to the fallback
          ok = false;
          break;
        }
        prefix += w & kStValue;
        any_poison = any_poison || (w & kStPoison);
        if ((w >> 62) == 2) break;
      }
      if (ok)
        __hip_atomic_store(&a.chunk_st[c], kStIncl | (any_poison ? kStPoison : 0) | (prefix + T), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      a.blk_big[c] = BG | !ok;  // an unfinished look-back hands the scan to the fallback emit
      bc[1] = (uint32_t)prefix;
      bc[2] = ok && !any_poison && NE && prefix + T <= cap;
      // whether a lane starts at the first window after the group's last slice
      uint32_t fresh_after = 0;
      const uint32_t E = NE ? le[llnz[kChunkLanes - 1]] : 0;
      if (NE && E < a.n) {
        const uint32_t i_hi = win_from(E, mis0);
        const uint32_t W = i_hi * kWin - mis0;
        if (W == E) {
          fresh_after = 1;
        } else if (W < a.n) {
          const uint32_t t = fdiv(W, a.lane_div) * a.lane_bytes;  // the last target at or before W
          if (t > E && l.lut[a.in[W]]) {
            fresh_after = 1;
            for (uint32_t y = t; y < W; ++y) fresh_after &= !l.lut[a.in[y]];
          }
        }
      }
      bc[3] = fresh_after;
    }
    __syncthreads();
    // ---- emit the windows starting in [S, E)
    if (bc[2]) {
      const uint32_t Pc = bc[1], fresh_after = bc[3];
      const uint32_t last = llnz[kChunkLanes - 1], E = le[last];
      const uint32_t i_lo = win_from(S, mis0), i_hi = E >= a.n ? nwin : win_from(E, mis0);
      const uint32_t nt = (i_hi - i_lo + 63) / 64;
      const uint32_t per = (nt + kWinWaves - 1) / kWinWaves;
      const uint32_t t_lo = min(nt, wid * per), t_hi = min(nt, t_lo + per);
      if (t_lo < t_hi) {  // wave-uniform
        auto meta = [&](uint32_t t) {
          return group_meta(a, g, i_lo + t * 64 + lane, i_hi, c0, last, Pc, mis0, fresh_after, cap);
        };
        auto wpos = [&](uint32_t t) { return (int64_t)(i_lo + t * 64 + lane) * kWin - mis0; };
        auto is_edge = [&](uint32_t t) { return i_lo + t * 64 == 0 || i_lo + t * 64 + 64 >= nwin; };
        WinMeta cur = meta(t_lo), nxt = meta(t_lo + 1);
        Win64 dat = is_edge(t_lo) ? win_load<true>(a.in, wpos(t_lo), a.n) : win_load<false>(a.in, wpos(t_lo), a.n);
        for (uint32_t t = t_lo; t < t_hi; ++t) {
          const uint32_t i = i_lo + t * 64 + lane;
          Win64 ndat = dat;
          if (t + 1 < t_hi)
            ndat = is_edge(t + 1) ? win_load<true>(a.in, wpos(t + 1), a.n) : win_load<false>(a.in, wpos(t + 1), a.n);
          const WinMeta n2 = meta(t + 2);
          const uint32_t o_first = __shfl(cur.out, 0), o_next = __shfl(nxt.out, 0);
          const uint32_t down = __shfl_down(cur.out, 1), fdown = __shfl_down(cur.fresh, 1);
          const uint32_t f_next = __shfl(nxt.fresh, 0);
          const uint32_t P = __shfl(cur.tok, 0);
          // the group's last tile ends past E: its outputs are counted by the walk, within a
          // bound (the last window ends at most 64 tokens and finishes one)
          const bool exact = t + 1 < nt;
          const uint32_t lastv = min(63u, i_hi - 1 - (i_lo + t * 64));
          const uint32_t o_end = exact ? o_next : __shfl(cur.out, lastv) + 65;
          const uint32_t span_end = (uint32_t)min<uint64_t>((uint64_t)(i_lo + t * 64 + 64) * kWin - mis0, a.n);
          win_tile<DISC>(tb, a, stage, lane, cur, i, i < i_hi, is_edge(t), dat, wpos(t), nwin, o_first, o_end,
                         exact, lane < 63 ? down : o_next, lane < 63 ? fdown : f_next, P, span_end, cap);
          cur = nxt;
          nxt = n2;
          dat = ndat;
        }
      }
    }
    __syncthreads();  // the group's LDS is rewritten by the next one
  }
}

__global__ void k_onepass_reset(uint64_t *st, uint32_t n, uint32_t *ctr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) st[i] = 0;
  if (i == 0) *ctr = 0;
}

// ------------------------------------------------------------- B. batched documents
// Many documents, each with its own (lexer, mode) instance, in one sequence of launches
// that a hipGraph can capture (fixed grids, no host synchronisation, work queues reset by
// the first kernel).  The instances' packed tables are rebased into one combined table
// (rows renumbered, so walk() and its absolute LDS addressing are unchanged) and all of
// them sit in LDS.  Each document is split into lanes exactly as a single scan would split
// it (Theorem 1, Theorem 3): lane jj of a document targets jj * lane_bytes inside it, and a
// document whose useful map is empty, or that asks for a serial scan, is one lane.  Lanes
// are numbered long single-lane documents first, so the longest walks start first; the
// count workgroups take 64-lane tiles from an atomic queue (work stealing) after a first
// tile fixed per wave, and the windowed emit gives each wave a contiguous range of tiles.
// Each document's result is its own scan's: its tokens up to and including its first
// halted slice, error offset relative to the document.
//
// Hybrid plan for refused token sets: a document of such a set (no useful certified byte),
// not flagged serial and longer than one speculative lane (kSpecX bytes) and than the batch
// lane is split speculatively.  Lane k starts at k * S in the start row as if a token
// began there, walks its range and kSpecX bytes on, and restarts one byte further on after
// a halt, recording the token starts of its first kSpecX bytes (head) and of the kSpecX
// bytes after its range (tail).  Lane 0 is the serial scan.  If lane k - 1's walk is the
// serial scan by the end of its range, the first position where its tail and lane k's head
// both start a token is a token start of the serial scan, and from there both walks agree
// (both restart in the start row on the same bytes).  By induction the cuts found this
// way are serial token boundaries, and the slices between them are counted and emitted
// like certified slices.  The last lane's window reaches the document's end; when it finds
// no common start (a token runs from before its start to the end), lane k - 1, which is the
// serial scan up to the end, takes the rest.  A document falls back to one lane when another
// boundary finds no common start within kSpecX bytes, or when a lane restarted at or after
// its own cut (the serial scan halts there: the one-lane scan then reports the error as
// usual).
constexpr int kMaxInst = 8;
constexpr uint32_t kSpecX = 2048;  // the sync window; at most the speculative lane
constexpr uint32_t kSpecWords = kSpecX / 32;

struct BatchInst {
  uint32_t start, sink, fail;  // row byte offsets in the combined table
  uint32_t mono, refused;      // refused: empty useful map (one lane per document)
  uint32_t disc;               // the mode discards some kind (windowed emit stages lengths)
  CertArg ca;
};

struct DocDev {  // mirrors lex_doc
  uint64_t offset;
  uint32_t length;
  uint16_t inst, flags;
};

struct DocResDev {  // mirrors lex_doc_result
  uint64_t tok_offset, ntokens, error_offset;
  int32_t status;
  uint32_t nslices;
};

// meta words: work queues (count, lane emit; kQWin is reset but no kernel takes from it),
// lane / speculative-lane / tile totals, a stopped batch, no windowed emit for this batch,
// some document for the lane emit
enum { kQCount = 0, kQEmit = 1, kNLanes = 2, kBad = 3, kNSpec = 4, kQWin = 5, kNTiles = 6, kNoWin = 7,
       kAnyLane = 8, kBatchMeta = 16 };

struct BatchArgs {
  const uint32_t *table;
  const uint8_t *rowinfo, *rowkind, *luts;  // luts: ninst * 256 certificate bytes
  int nrows;
  uint32_t ninst;
  BatchInst inst[kMaxInst];
  const uint8_t *bytes;
  uint64_t nbytes;
  const DocDev *docs;
  uint32_t ndocs, lane_bytes, max_lanes;
  uint32_t *meta;  // kBatchMeta words: queues, lane count
  uint64_t *part;  // kDocGroups x kPartWords: per-group sums of the planning and result kernels
  uint32_t *lanes_of, *lane_base, *lane_doc, *cuts, *ends, *counts, *halted, *lane_pre, *doc_halt;
  uint32_t *doc_ntok, *doc_nsl;
  // hybrid plan: per document the first speculative lane's index and the fall-back flag;
  // per speculative lane its document, cut, last restart, and head then tail token starts
  uint32_t spec_bytes, max_spec;
  uint32_t *spec_base, *spec_fail, *spec_doc, *spec_cut, *spec_rst, *spec_bits;
  uint4 *spec_part, *spec_pre;  // per speculative lane: its parts' starts and count prefixes (k_bsplit)
  // windowed emit: count-walk checkpoints (main slots per lane, kslots of them, and an
  // overflow region of 64 windows per tile of each document), tiles of 64 windows per
  // document (prefix and tile -> document map), per lane the last non-empty lane at or
  // before it in its document, per document whether it takes the windowed emit
  uint2 *ck_main, *ck_over;
  uint32_t kslots, max_tiles, win_ok;  // win_ok: the combined table's rows fit a checkpoint
  uint32_t *tile_base, *tile_doc, *lnz, *doc_win;
  uint8_t *kinds;
  uint32_t *lens;
  uint64_t *offs;
  uint64_t cap;
  DocResDev *res;
  ResultDev *total;
};

// Windows of a document of `length` bytes at address `addr`: the kWin-aligned windows of the
// address space it touches (window 0 starts at the document's first byte), and tiles of 64.
__device__ __forceinline__ uint32_t doc_windows(uintptr_t addr, uint32_t length) {
  return length ? (uint32_t)(((uint64_t)length + (addr & (kWin - 1)) + kWin - 1) / kWin) : 0;
}
__device__ __forceinline__ uint32_t doc_tiles(uintptr_t addr, uint32_t length) {
  return (doc_windows(addr, length) + 63) / 64;
}

__host__ __device__ inline size_t batch_lds_offset(int nrows, uint32_t ninst) {
  return align16((size_t)nrows * 1024 + 2 * (size_t)nrows + (size_t)ninst * 256);
}

// The batch windowed emit: the combined table and a stage per wave.
__host__ __device__ inline size_t batch_win_lds_bytes(int nrows, uint32_t ninst, uint32_t waves) {
  return batch_lds_offset(nrows, ninst) + waves * (size_t)kStageWords * 4 + 16;  // + the tile counter
}
// Waves of a windowed-emit workgroup: 16, 8 or 4, the most whose LDS fits; 0: none fits.
__host__ __device__ inline uint32_t batch_win_waves(int nrows, uint32_t ninst) {
  for (uint32_t w = 16; w >= 4; w >>= 1)
    if (batch_win_lds_bytes(nrows, ninst, w) <= 160 * 1024) return w;
  return 0;
}

struct BatchLds {
  const lds_u8 *T;  // the combined table (LDS address 0)
  const uint8_t *info, *kind, *luts;
  uint8_t *ring;
};

// Stages the combined table (at LDS address 0), row info, kinds and LUTs.
__device__ __forceinline__ BatchLds batch_stage(const BatchArgs &a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int words = a.nrows * 256;
  const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
  uint4 *dst = reinterpret_cast<uint4 *>(smem);
  for (int i = threadIdx.x; i < words / 4; i += blockDim.x) dst[i] = src[i];
  uint8_t *info = smem + (size_t)a.nrows * 1024, *kind = info + a.nrows, *luts = kind + a.nrows;
  for (int i = threadIdx.x; i < a.nrows; i += blockDim.x) {
    info[i] = a.rowinfo[i];
    kind[i] = a.rowkind[i];
  }
  for (uint32_t i = threadIdx.x; i < a.ninst * 256; i += blockDim.x) luts[i] = a.luts[i];
  __syncthreads();
  return BatchLds{lds_bytes_of(smem), info, kind, luts, smem + batch_lds_offset(a.nrows, a.ninst)};
}

// Bit k: instance k's set is refused.  Built from uniform loads, so the per-document tests
// below index no kernel argument by a per-lane value (that compiles to a dependent vector
// load from argument memory).
__device__ __forceinline__ uint32_t refused_mask(const BatchArgs &a) {
  uint32_t m = 0;
  for (uint32_t k = 0; k < a.ninst; ++k) m |= (a.inst[k].refused ? 1u : 0u) << k;
  return m;
}

// A refused set's document longer than a speculative lane and than the batch lane is split
// by the hybrid plan; a shorter one is one lane among the certified documents' lanes.
__device__ __forceinline__ bool spec_split(const BatchArgs &a, uint32_t rm, const DocDev &d) {
  return d.inst < a.ninst && ((rm >> d.inst) & 1) && !(d.flags & 1) && d.length > max(a.spec_bytes, a.lane_bytes);
}

__device__ __forceinline__ bool one_lane(const BatchArgs &a, uint32_t rm, const DocDev &d) {
  // (an unknown instance stops the batch)
  return !spec_split(a, rm, d) &&
         (d.length <= a.lane_bytes || (d.flags & 1) || d.inst >= a.ninst || ((rm >> d.inst) & 1));
}

__device__ __forceinline__ uint32_t ceil_div(uint32_t x, uint32_t y) { return x / y + (x % y != 0); }

__device__ __forceinline__ uint32_t doc_lanes(const BatchArgs &a, uint32_t rm, const DocDev &d) {
  if (spec_split(a, rm, d)) return ceil_div(d.length, a.spec_bytes);
  return one_lane(a, rm, d) ? 1 : ceil_div(d.length, a.lane_bytes);
}

// The planning and result kernels (k_bplan_*, k_bscan_*) split the document table into at
// most kDocGroups contiguous groups, one workgroup of 256 threads each, a document per
// thread at a time (coalesced loads).  A first kernel writes each group's sums to part[],
// a second adds the earlier groups' sums (every workgroup reads all of them) and scans its
// own documents.  (One workgroup for the whole table left the chip idle for 0.2 ms at
// 50 000 documents.)
constexpr uint32_t kDocGroups = 256;
constexpr uint32_t kPartWords = 8;  // per group: plan sums (0-4), result sums (5-7)

__host__ __device__ inline uint32_t doc_groups(uint32_t ndocs) {
  return ndocs > 256u * kDocGroups ? kDocGroups : ndocs ? (ndocs + 255) / 256 : 1;
}

__device__ __forceinline__ void group_range(uint32_t ndocs, uint32_t &lo, uint32_t &hi) {
  const uint32_t per = (ndocs + gridDim.x - 1) / gridDim.x;
  lo = min(ndocs, blockIdx.x * per);
  hi = min(ndocs, lo + per);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
  for (int k = 32; k; k >>= 1) v += __shfl_xor(v, k);
  return v;
}

__device__ __forceinline__ uint64_t wave_incl64(uint64_t v, uint32_t lane) {
  for (int k = 1; k < 64; k <<= 1) {
    const uint64_t t = __shfl_up(v, k);
    if ((int)lane >= k) v += t;
  }
  return v;
}

// Sums of Q values over the workgroup (256 threads); red: Q x 4 words of LDS.
template <int Q>
__device__ __forceinline__ void block_sum(uint64_t (&v)[Q], uint64_t (*red)[4]) {
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = wave_sum64(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < Q; ++q) red[q][wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  __syncthreads();
}

// Inclusive scan of Q values over the workgroup (256 threads), and their totals.
template <int Q>
__device__ __forceinline__ void block_incl(uint64_t (&v)[Q], uint64_t (&tot)[Q], uint64_t (*red)[4]) {
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = wave_incl64(v[q], lane);
  if (lane == 63)
#pragma unroll
    for (int q = 0; q < Q; ++q) red[q][wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    uint64_t pre = 0, t = 0;
    for (uint32_t w = 0; w < 4; ++w) {
      pre += w < wid ? red[q][w] : 0;
      t += red[q][w];
    }
    v[q] += pre;
    tot[q] = t;
  }
  __syncthreads();
}

// Sums of words [q0, q0 + Q) of part[] over the groups before this one (pre) and over all
// groups (tot).
template <int Q>
__device__ __forceinline__ void group_prefix(const uint64_t *part, uint32_t q0, uint64_t (&pre)[Q],
                                             uint64_t (&tot)[Q], uint64_t (*red)[4]) {
  const uint32_t t = threadIdx.x;
  uint64_t v[2 * Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint64_t x = t < gridDim.x ? part[(size_t)t * kPartWords + q0 + q] : 0;
    v[q] = t < blockIdx.x ? x : 0;
    v[Q + q] = x;
  }
  block_sum<2 * Q>(v, red);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    pre[q] = v[q];
    tot[q] = v[Q + q];
  }
}

// Planning, first half: lanes per document, each group's lane, speculative-lane and tile
// sums and whether it holds a bad record; the queues reset.  The document table is the
// caller's device data: a document outside the bytes, an unknown instance or flag, or more
// lanes than the workspace holds stops the batch.
__global__ void __launch_bounds__(256) k_bplan_a(BatchArgs a) {
  __shared__ uint64_t red[5][4];
  const uint32_t rm = refused_mask(a);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.meta[kQCount] = 0;
    a.meta[kQEmit] = 0;
    a.meta[kQWin] = 0;
    a.meta[kAnyLane] = 0;
  }
  const uintptr_t base = reinterpret_cast<uintptr_t>(a.bytes);
  uint32_t lo, hi;
  group_range(a.ndocs, lo, hi);
  uint64_t v[5] = {0, 0, 0, 0, 0};  // single-lane long documents, other lanes, speculative lanes, tiles, bad
  for (uint32_t d = lo + threadIdx.x; d < hi; d += blockDim.x) {
    const DocDev x = a.docs[d];
    const bool fits = x.offset <= a.nbytes && x.length <= a.nbytes - x.offset;
    v[4] |= !fits || x.inst >= a.ninst || x.flags > 1;
    const uint32_t nl = doc_lanes(a, rm, x);
    a.lanes_of[d] = nl;
    a.spec_fail[d] = 0;
    const bool first = nl == 1 && x.length > a.lane_bytes;
    v[0] += first ? nl : 0;
    v[1] += first ? 0 : nl;
    if (spec_split(a, rm, x)) v[2] += nl;
    if (fits) v[3] += doc_tiles(base + x.offset, x.length);
  }
  block_sum<5>(v, red);
  if (threadIdx.x < 5) a.part[(size_t)blockIdx.x * kPartWords + threadIdx.x] = v[threadIdx.x];
}

// Planning, second half: lane numbering (long single-lane documents first, then the rest,
// each in document order), speculative-lane and tile numbering; the first group writes the
// totals and the stop flags.
__global__ void __launch_bounds__(256) k_bplan_b(BatchArgs a) {
  __shared__ uint64_t red[10][4];
  const uint32_t rm = refused_mask(a);
  const uintptr_t base = reinterpret_cast<uintptr_t>(a.bytes);
  uint64_t pre[5], tot[5];
  group_prefix<5>(a.part, 0, pre, tot, red);
  uint64_t r[4] = {pre[0], tot[0] + pre[1], pre[2], pre[3]};  // 64-bit: a hostile table may ask for 2^32 lanes
  uint32_t lo, hi;
  group_range(a.ndocs, lo, hi);
  for (uint32_t d0 = lo; d0 < hi; d0 += blockDim.x) {  // workgroup-uniform: the scans see every thread
    const uint32_t d = d0 + threadIdx.x;
    const bool in = d < hi;
    const DocDev x = a.docs[in ? d : lo];
    const uint32_t nl = in ? a.lanes_of[d] : 0;
    const bool first = nl == 1 && x.length > a.lane_bytes;
    const bool fits = in && x.offset <= a.nbytes && x.length <= a.nbytes - x.offset;
    uint64_t v[4] = {first ? nl : 0, first ? 0 : nl, in && spec_split(a, rm, x) ? nl : 0,
                     fits ? doc_tiles(base + x.offset, x.length) : 0};
    const uint64_t v0[4] = {v[0], v[1], v[2], v[3]};
    uint64_t t[4];
    block_incl<4>(v, t, red);
    if (in) {
      const uint64_t lb = first ? r[0] + v[0] - v0[0] : r[1] + v[1] - v0[1];
      a.lane_base[d] = (uint32_t)min<uint64_t>(lb, 0xFFFFFFFFu);  // unused when stopped
      a.spec_base[d] = (uint32_t)min<uint64_t>(r[2] + v[2] - v0[2], 0xFFFFFFFFu);
      a.tile_base[d] = (uint32_t)min<uint64_t>(r[3] + v[3] - v0[3], 0xFFFFFFFFu);  // unused without tiles
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] += t[q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t nlanes = tot[0] + tot[1], nspec = tot[2];
    const bool stop = tot[4] || nlanes > a.max_lanes || nspec > a.max_spec;
    a.meta[kBad] = stop;
    a.meta[kNLanes] = stop ? 0 : (uint32_t)nlanes;
    a.meta[kNSpec] = stop ? 0 : (uint32_t)nspec;
    // the windowed emit needs its checkpoints' rows in 8 bits and its tiles in the workspace
    // (overlapping documents may ask for more tiles than the bytes hold)
    const bool nowin = stop || !a.win_ok || tot[3] > a.max_tiles;
    a.meta[kNoWin] = nowin;
    a.meta[kNTiles] = nowin ? 0 : (uint32_t)tot[3];
  }
}

// A wave per document: the lane -> document map.
__global__ void __launch_bounds__(256) k_bmap(BatchArgs a) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
  if (a.meta[kBad]) return;
  const bool win = !a.meta[kNoWin];
  const uintptr_t base = reinterpret_cast<uintptr_t>(a.bytes);
  for (uint32_t d = wave; d < a.ndocs; d += nwaves) {
    const uint32_t lb = a.lane_base[d], nl = a.lanes_of[d];
    const DocDev doc = a.docs[d];
    for (uint32_t k = lane; k < nl; k += 64) a.lane_doc[lb + k] = d;
    if (spec_split(a, refused_mask(a), doc))
      for (uint32_t k = lane; k < nl; k += 64) a.spec_doc[a.spec_base[d] + k] = d;
    if (win) {
      const uint32_t tb = a.tile_base[d], nt = doc_tiles(base + doc.offset, doc.length);
      for (uint32_t k = lane; k < nt; k += 64) a.tile_doc[tb + k] = d;
    }
  }
}

// Speculative walk of [b, end) (hybrid plan): from the start row as if a token began at b,
// restarting one byte further on after a halt (a halt at the start of a token that cannot
// be matched), so the walk never stops.  Token starts in [b, b + kSpecX) go to head, those
// in [b2, b2 + kSpecX) to tail (bit i: position base + i); rst: the last restart position
// or kNone.  Token starts come in increasing order, so each bitmap is built a word at a
// time.  Bytes are read through a 16-byte block held in registers.
template <bool MONO>
__device__ void walk_spec(const Tables &tb, const uint8_t *in, uint32_t n, uint32_t b, uint32_t end, uint32_t b2,
                          uint32_t *head, uint32_t *tail, uint32_t &rst) {
  uint32_t hw = 0, hv = 0, tw = 0, tv = 0;  // current word index and bits of head and tail
  auto mark = [&](uint32_t t) {
    if (t - b < kSpecX) {
      const uint32_t w = (t - b) >> 5;
      if (w != hw) {
        head[hw] = hv;
        hw = w;
        hv = 0;
      }
      hv |= 1u << ((t - b) & 31);
    }
    if (t - b2 < kSpecX) {
      const uint32_t w = (t - b2) >> 5;
      if (w != tw) {
        tail[tw] = tv;
        tw = w;
        tv = 0;
      }
      tv |= 1u << ((t - b2) & 31);
    }
  };
  for (uint32_t w = 0; w < kSpecWords; ++w) head[w] = tail[w] = 0;
  const uintptr_t base = reinterpret_cast<uintptr_t>(in);
  int64_t cb = INT64_MIN;  // position of the cached block (16-aligned in memory)
  uint4 cv = make_uint4(0, 0, 0, 0);
  // Aligned blocks are loaded four ahead of the walk (a speculative walk runs at a few
  // waves per CU, so nothing else hides a load's latency): q0..q3 hold the blocks at qp,
  // qp + 16, qp + 32, qp + 48.  A load past the last aligned block that fits reads that
  // block instead (n >= 32 here), and its bytes are never walked.
  const int64_t qlast = (int64_t)(((base + n - 16) & ~(uintptr_t)15) - base);
  auto qload = [&](int64_t x) { return *reinterpret_cast<const uint4 *>(in + min(x, qlast)); };
  int64_t qp = INT64_MIN;
  uint4 q0 = cv, q1 = cv, q2 = cv, q3 = cv;
  // the token starts of one aligned 16-byte block (bit k: position P + k) into both bitmaps,
  // a word at a time (positions come in increasing order, as for mark)
  auto mark_bits = [&](uint32_t mk, uint32_t P) {
    auto put = [&](uint32_t bits, int64_t off, uint32_t *words, uint32_t &cw, uint32_t &cv) {
      if (off <= -16 || off >= (int64_t)kSpecX) return;
      if (off < 0) {
        bits >>= (uint32_t)(-off);
        off = 0;
      }
      const uint32_t wi = (uint32_t)off >> 5, sh = (uint32_t)off & 31;
      const uint32_t lo = bits << sh, hi = sh > 16 ? bits >> (32 - sh) : 0;
      if (lo) {
        if (wi != cw) {
          words[cw] = cv;
          cw = wi;
          cv = 0;
        }
        cv |= lo;
      }
      if (hi && wi + 1 < kSpecWords) {
        words[cw] = cv;
        cw = wi + 1;
        cv = hi;
      }
    };
    put(mk, (int64_t)P - b, head, hw, hv);
    put(mk, (int64_t)P - b2, tail, tw, tv);
  };
  uint32_t st = tb.start, tok = b, lacc = b, lrow = 0, lblk = b, lst0 = 0;
  // non-monotone automata: failed traces as cursors, as the lane walk's fallback keeps them
  uint32_t cp[kMemo], cr[kMemo];
#pragma unroll
  for (int k = 0; k < kMemo; ++k) cp[k] = kNone, cr[k] = 0;
  bool live = false;  // some cursor is set
  rst = kNone;
  mark(b);
  for (uint32_t p = b; p < end;) {
    if (!live && ((base + p) & 15) == 0 && p + 16 <= end) {
      // an aligned block without cursors: 16 steps, their EMIT and ACC bits as masks (bit
      // 16 + k: step k); a halt or FAIL inside leaves the row there, flagless, to the
      // block's end, and the restart below acts on it as after the step that caused it
      if (qp != (int64_t)p) {
        q0 = qload(p);
        q1 = qload((int64_t)p + 16);
        q2 = qload((int64_t)p + 32);
        q3 = qload((int64_t)p + 48);
      }
      const uint4 v = q0;
      q0 = q1;
      q1 = q2;
      q2 = q3;
      q3 = qload((int64_t)p + 64);
      qp = (int64_t)p + 16;
      uint32_t e = st, me = 0, ma = 0;
      const uint32_t st0 = st;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        e = entry_from(tb, e, byte_of(v, k));
        me = __builtin_amdgcn_alignbit(e >> 1, me, 1);
        if (!MONO) ma = __builtin_amdgcn_alignbit(e >> 7, ma, 1);
      }
      st = e & kRowMask;
      if (me) {
        tok = p + (31 - __clz(me)) - 16;
        mark_bits(me >> 16, p);
      }
      if (!MONO && ma) {
        lacc = p + (31 - __clz(ma)) - 15;
        lrow = kLazyRow;  // rebuilt from lst0 at lblk if a restart needs it
        lblk = p;
        lst0 = st0;
      }
      p += 16;
      if (st == tb.sink || (!MONO && st == tb.fail)) {
        if (!MONO && st == tb.fail && lacc > tok) {
          if (lrow == kLazyRow) lrow = rewalk_row(tb, in, lst0, lblk, lacc);
#pragma unroll
          for (int k = kMemo - 1; k > 0; --k) cp[k] = cp[k - 1], cr[k] = cr[k - 1];
          cp[0] = lacc;  // the failed trace, from its last accepting step on
          cr[0] = lrow;
          live = true;
          tok = lacc;
        } else {
          rst = tok;  // no token starts at tok: restart one byte on
          tok = tok + 1;
        }
        p = tok;
        lacc = tok;
        st = tb.start;
        if (p < end) mark(p);
      }
      continue;
    }
    const int64_t blk = (int64_t)p - (int64_t)((base + p) & 15);
    if (blk != cb) {
      cb = blk;
      cv = load_block(in, blk, n);
    }
    const uint32_t q = (uint32_t)((int64_t)p - blk);
    const uint32_t w4 = q < 4 ? cv.x : q < 8 ? cv.y : q < 12 ? cv.z : cv.w;
    const uint32_t by = (w4 >> (8 * (q & 3))) & 0xFFu;
    const uint32_t e = entry(tb, st, by);
    if (e & kEmitBit) {
      tok = p;
      mark(p);
    }
    st = e & kRowMask;
    if (!MONO && (e & kAccBit)) {
      lacc = p + 1;
      lrow = st;
    }
    if (!MONO && live) {
      bool join = false;
      live = false;
#pragma unroll
      for (int k = 0; k < kMemo; ++k) {
        if (cp[k] == p) {
          cr[k] = entry(tb, cr[k], by) & kRowMask;
          cp[k] = cr[k] == tb.fail ? kNone : p + 1;
        }
        join |= cp[k] == p + 1 && cr[k] == st;
      }
#pragma unroll
      for (int k = 1; k < kMemo; ++k)
#pragma unroll
        for (int j = 0; j < k; ++j)
          if (cp[k] == cp[j] && cr[k] == cr[j]) cp[k] = kNone;
#pragma unroll
      for (int k = 0; k < kMemo; ++k) live |= cp[k] != kNone;
      if (join && st != tb.sink) st = tb.fail;  // a failed pair: fail as that trace did
    }
    ++p;
    if (st == tb.sink || (!MONO && st == tb.fail)) {
      if (!MONO && st == tb.fail && lacc > tok) {
        if (lrow == kLazyRow) lrow = rewalk_row(tb, in, lst0, lblk, lacc);
#pragma unroll
        for (int k = kMemo - 1; k > 0; --k) cp[k] = cp[k - 1], cr[k] = cr[k - 1];
        cp[0] = lacc;  // the failed trace, from its last accepting step on
        cr[0] = lrow;
        live = true;
        tok = lacc;  // longest match: the token ends at its last accepting position
      } else {
        rst = tok;  // no token starts at tok: restart one byte on
        tok = tok + 1;
      }
      p = tok;
      lacc = tok;
      st = tb.start;
      if (p < end) mark(p);
    }
  }
  head[hw] = hv;
  tail[tw] = tv;
}

// The speculative walk of speculative lane i (< the batch's count of them).
__device__ __forceinline__ void spec_lane(const BatchArgs &a, const BatchLds &l, uint32_t i) {
  const uint32_t d = a.spec_doc[i];
  const DocDev doc = a.docs[d];
  const BatchInst &in = a.inst[doc.inst];
  const uint32_t k = i - a.spec_base[d], S = a.spec_bytes;
  const uint32_t b = k * S;  // < length
  // the tail window; past the document's end it can hold no token start
  const uint32_t b2 = (uint32_t)min<uint64_t>((uint64_t)(k + 1) * S, doc.length);
  const uint32_t end = (uint32_t)min<uint64_t>((uint64_t)b2 + kSpecX, doc.length);
  const Tables tb{l.T, l.info, l.kind, in.sink, in.fail, in.start};
  uint32_t *bits = a.spec_bits + (size_t)i * 2 * kSpecWords;
  uint32_t rst;
  if (in.mono) walk_spec<true>(tb, a.bytes + doc.offset, doc.length, b, end, b2, bits, bits + kSpecWords, rst);
  else walk_spec<false>(tb, a.bytes + doc.offset, doc.length, b, end, b2, bits, bits + kSpecWords, rst);
  a.spec_rst[i] = rst;
}

// Cuts of the hybrid plan: one thread per speculative lane k; lane k's cut is the first
// common token start of lane k - 1's tail and lane k's head (lane 0: the document start).
// A missing cut, or a restart at or after the lane's cut, sends the document to one lane.
__global__ void __launch_bounds__(256) k_bsync(BatchArgs a) {
  if (a.meta[kBad]) return;
  const uint32_t ns = a.meta[kNSpec];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
    const uint32_t d = a.spec_doc[i];
    const uint32_t k = i - a.spec_base[d];
    uint32_t cut = 0;
    bool ok = true;
    if (k) {
      const uint32_t *head = a.spec_bits + (size_t)i * 2 * kSpecWords;
      const uint32_t *tail = a.spec_bits + (size_t)(i - 1) * 2 * kSpecWords + kSpecWords;
      cut = kNone;
      for (uint32_t w = 0; w < kSpecWords && cut == kNone; ++w) {
        const uint32_t x = head[w] & tail[w];
        if (x) cut = k * a.spec_bytes + 32 * w + (__ffs(x) - 1);
      }
      // the last lane's window reaches the end: with no common token start, lane k - 1
      // (the serial scan up to the end) takes the rest
      if (cut == kNone && k + 1 == a.lanes_of[d]) cut = a.docs[d].length;
      ok = cut != kNone;
    }
    const uint32_t rst = a.spec_rst[i];
    if (ok && rst != kNone && rst >= cut) ok = false;
    a.spec_cut[i] = cut;
    if (!ok) a.spec_fail[d] = 1;
  }
}

// Pulls the next 64-lane tile for this wave (lane 0 takes it, the wave shares it).
__device__ __forceinline__ uint32_t next_tile(uint32_t *q) {
  uint32_t t = 0;
  if ((threadIdx.x & 63) == 0) t = atomicAdd(q, 1u);
  return (uint32_t)__shfl((int)t, 0);
}

// Count walk of the batch: each lane places its own slice inside its document (the fused
// planner) and counts it with its document's table.  One queue hands out, first, the
// hybrid plan's speculative walks (few and serial, they would leave the chip idle in a
// launch of their own), then the lanes of every document the hybrid plan does not split,
// which keep the chip busy meanwhile.  The split documents are counted after the cuts
// (k_bsplit).
__global__ void __launch_bounds__(1024) k_bcount(BatchArgs a) {
  const BatchLds l = batch_stage(a);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nlanes = a.meta[kNLanes], nspec = a.meta[kNSpec];
  const uint32_t nst = (nspec + 63) / 64;  // speculative tiles first
  const bool ck_on = !a.meta[kNoWin];
  // every wave's first tile is fixed (all waves taking it from the queue at once would
  // queue on its atomic counter); later ones come from the queue, past the fixed ones
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6, gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  for (uint32_t tile = gw;; tile = next_tile(&a.meta[kQCount]) + nwaves) {
    if (tile < nst) {  // wave-uniform
      const uint32_t i = tile * 64 + lane;
      if (i < nspec) spec_lane(a, l, i);
      continue;
    }
    const uint32_t t = tile - nst;
    if ((uint64_t)t * 64 >= nlanes) break;  // wave-uniform exit
    const uint32_t j = t * 64 + lane;
    const bool valid = j < nlanes;
    uint32_t d = 0, jj = 0, nl = 1, start = kNone;
    DocDev doc{0, 0, 0, 0};
    if (valid) {
      d = a.lane_doc[j];
      doc = a.docs[d];
      jj = j - a.lane_base[d];
      nl = a.lanes_of[d];
    }
    const BatchInst &in = a.inst[valid ? doc.inst : 0];
    const uint8_t *src = a.bytes + doc.offset;
    const uint8_t *lut = l.luts + 256 * (valid ? doc.inst : 0);
    const bool spec = valid && spec_split(a, refused_mask(a), doc);
    if (valid && !spec) {
      if (jj == 0) start = 0;
      else start = search_cert(src, doc.length, in.ca, lut, jj * a.lane_bytes, a.lane_bytes, kNone);
    }
    // the next lane's start, when that lane is this document's and this tile's
    const uint32_t nstart = (uint32_t)__shfl_down((int)start, 1);
    if (!valid || spec) continue;
    const bool same = lane < 63 && jj + 1 < nl;
    uint32_t s, e;
    if (start == kNone) {
      s = e = min(jj * a.lane_bytes, doc.length);
    } else {
      s = start;
      if (jj + 1 == nl) e = doc.length;
      else if (same && nstart != kNone) e = nstart;
      else {
        const uint32_t x1 = (jj + 1) * a.lane_bytes;
        e = search_cert(src, doc.length, in.ca, lut, x1, doc.length - x1, doc.length);
      }
    }
    a.cuts[j] = s;
    a.ends[j] = e;
    const Tables tb{l.T, l.info, l.kind, in.sink, in.fail, in.start};
    LaneState L;
    L.cnt = 0;
    Ring r{};
    // checkpoints for the windowed emit: main slots by the window's place in the lane's
    // nominal range, else the document's overflow region (its 64 windows per tile)
    CkSink ck{};
    if (ck_on) {
      ck.base = reinterpret_cast<uintptr_t>(src);
      ck.main = a.ck_main;
      ck.over = a.ck_over + (size_t)a.tile_base[d] * 64;
      ck.nlanes = a.max_lanes;
      ck.kslots = a.kslots;
      ck.j = j;
      ck.jl = jj * a.lane_bytes;
      ck.mis0 = (uint32_t)(ck.base & (kWin - 1));
    }
    const bool halted = in.mono ? walk<false, true, false, true>(L, r, tb, src, doc.length, s, e, ck)
                                : walk<false, false, false, true>(L, r, tb, src, doc.length, s, e, ck);
    a.counts[j] = L.cnt;
    // bit 0: the slice halted; bit 1: no windowed emit for its document (a fallback
    // re-scanned positions the checkpoints describe, or counts overflow 24 bits)
    a.halted[j] = (halted ? 1u : 0u) | ((L.fb || e - s >= (1u << 24)) ? 2u : 0u);
  }
}

// The first token start of speculative lane i's walk at or after x and before e (else e):
// lane k = i's place in its document walked [k S, (k+1) S + kSpecX) and marked its token
// starts in head ([k S, k S + kSpecX), kSpecX = S) and tail ([b2, b2 + kSpecX)).  Past the
// lane's cut they are serial token starts (its walk is the serial scan from there on).
__device__ __forceinline__ uint32_t spec_next_start(const BatchArgs &a, uint32_t i, uint32_t k, uint32_t len,
                                                    uint32_t x, uint32_t e) {
  const uint32_t *head = a.spec_bits + (size_t)i * 2 * kSpecWords, *tail = head + kSpecWords;
  const uint32_t b = k * a.spec_bytes;
  const uint32_t b2 = (uint32_t)min<uint64_t>((uint64_t)(k + 1) * a.spec_bytes, len);
  // four bitmap words (128 positions) per load: the search is a chain of dependent loads
  for (uint32_t pos = x; pos < e;) {
    const bool h = pos < b2;
    const uint32_t base = h ? b : b2, off = pos - base;
    if (off >= kSpecX) break;  // past the bitmaps
    const uint32_t w0 = (off >> 5) & ~3u;  // 16-byte aligned: the bitmaps start 256-byte aligned
    const uint4 v = *reinterpret_cast<const uint4 *>((h ? head : tail) + w0);
    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t at = 32 * (w0 + u);  // bitmap position of the word's bit 0
      const uint32_t m = at + 32 <= off ? 0u : at >= off ? wv[u] : wv[u] & (~0u << (off - at));
      if (m) return min(e, base + at + (uint32_t)(__ffs(m) - 1));
    }
    pos = base + 32 * (w0 + 4);
  }
  return e;
}

// Count walks of the documents the hybrid plan splits, after the cuts.  A split document's
// lane is its speculative lane's slice [s, e).  kParts threads walk it, in parts cut at the
// speculative walk's token starts (serial ones past the cut): part q starts at the first at
// or after s + q (e - s) / kParts, so each walk is about a quarter of a slice (these walks are
// few, and one walk's length sets the kernel's time).  A part's checkpoints count from the
// part's own start, and the windowed emit adds the counts of the parts before it
// (spec_part: the parts' starts, spec_pre: their inclusive count prefixes).  A document
// that falls back to one lane is not split further: its walk may restart where the serial
// scan halts, so its token starts are not all serial.
constexpr uint32_t kParts = 4;
__global__ void __launch_bounds__(256) k_bsplit(BatchArgs a) {
  const BatchLds l = batch_stage(a);
  const uint32_t lane = threadIdx.x & 63, q = lane % kParts, g0 = lane - q;
  const uint32_t nspec = a.meta[kNSpec];
  const bool ck_on = !a.meta[kNoWin];
  constexpr uint32_t kPer = 64 / kParts;  // speculative lanes per 64-thread tile
  // a tile per wave, in a fixed order: the walks are about one per wave, and a queue's
  // atomic counter, which every wave would hit at once, costs more than the walks
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6, gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  for (uint32_t t = gw; (uint64_t)t * kPer < nspec; t += nwaves) {  // wave-uniform
    const uint32_t i = t * kPer + lane / kParts;
    const bool valid = i < nspec;
    uint32_t s = 0, e = 0, k = 0, j = 0, d = 0;
    bool fail = true;
    DocDev doc{0, 0, 0, 0};
    if (valid) {
      d = a.spec_doc[i];
      doc = a.docs[d];
      k = i - a.spec_base[d];
      j = a.lane_base[d] + k;
      fail = a.spec_fail[d] != 0;
      if (fail) {
        s = k ? doc.length : 0;
        e = doc.length;
      } else {
        s = a.spec_cut[i];
        e = k + 1 < a.lanes_of[d] ? a.spec_cut[i + 1] : doc.length;
      }
    }
    uint32_t p = s;  // this part's start
    if (q) p = valid && !fail ? spec_next_start(a, i, k, doc.length, s + (uint32_t)((uint64_t)(e - s) * q / kParts), e) : e;
    const uint32_t pn = (uint32_t)__shfl_down((int)p, 1);
    const uint32_t pe = q + 1 < kParts ? pn : e;  // this part's end
    const BatchInst &in = a.inst[valid ? doc.inst : 0];
    const uint8_t *src = a.bytes + doc.offset;
    const Tables tb{l.T, l.info, l.kind, in.sink, in.fail, in.start};
    LaneState L;
    L.cnt = 0;
    L.fb = 0;
    Ring r{};
    bool halted = false;
    if (valid) {
      CkSink ck{};
      if (ck_on) {
        ck.base = reinterpret_cast<uintptr_t>(src);
        ck.main = a.ck_main;
        ck.over = a.ck_over + (size_t)a.tile_base[d] * 64;
        ck.nlanes = a.max_lanes;
        ck.kslots = a.kslots;
        ck.j = j;
        ck.jl = k * a.spec_bytes;
        ck.mis0 = (uint32_t)(ck.base & (kWin - 1));
      }
      halted = in.mono ? walk<false, true, false, true>(L, r, tb, src, doc.length, p, pe, ck)
                       : walk<false, false, false, true>(L, r, tb, src, doc.length, p, pe, ck);
    }
    // the lane's count: its parts' up to the first that halted; inclusive prefixes in the group
    uint32_t pre = valid ? L.cnt : 0;
    for (uint32_t dd = 1; dd < kParts; dd <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)pre, dd);
      if (q >= dd) pre += v;
    }
    const unsigned long long hb = __ballot(valid && halted), fb = __ballot(valid && L.fb);
    const uint32_t gh = (uint32_t)(hb >> g0) & ((1u << kParts) - 1), gf = (uint32_t)(fb >> g0) & ((1u << kParts) - 1);
    const uint32_t qh = gh ? (uint32_t)__ffs(gh) - 1 : kParts - 1;
    const uint32_t tot = (uint32_t)__shfl((int)pre, g0 + qh);
    const uint32_t pre0 = (uint32_t)__shfl((int)pre, g0), pre1 = (uint32_t)__shfl((int)pre, g0 + 1),
                   pre2 = (uint32_t)__shfl((int)pre, g0 + 2);
    const uint32_t p1 = (uint32_t)__shfl((int)p, g0 + 1), p2 = (uint32_t)__shfl((int)p, g0 + 2),
                   p3 = (uint32_t)__shfl((int)p, g0 + 3);
    if (valid && q == 0) {
      a.cuts[j] = s;
      a.ends[j] = e;
      a.counts[j] = tot;
      a.halted[j] = (gh ? 1u : 0u) | ((gf || e - s >= (1u << 24)) ? 2u : 0u);
      a.spec_part[i] = make_uint4(p1, p2, p3, 0);
      a.spec_pre[i] = make_uint4(pre0, pre1, pre2, 0);
    }
  }
}

// A wave per document: its first halted lane, the token count up to and including it,
// in-document prefixes of the lane counts, non-empty slices.
__global__ void __launch_bounds__(256) k_bdoc(BatchArgs a) {
  if (a.meta[kBad]) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
  const bool win = !a.meta[kNoWin];
  bool any_lane = false;  // some document of this wave's takes the lane emit
  // the next document's lane range and the next chunk's lanes load while the current ones
  // are scanned (a document of thousands of lanes would otherwise wait on every chunk)
  uint32_t n_lb = 0, n_nl = 1;
  if (wave < a.ndocs) {
    n_lb = a.lane_base[wave];
    n_nl = a.lanes_of[wave];
  }
  for (uint32_t d = wave; d < a.ndocs; d += nwaves) {
    const uint32_t lb = n_lb, nl = n_nl;  // nl >= 1
    if (d + nwaves < a.ndocs) {
      n_lb = a.lane_base[d + nwaves];
      n_nl = a.lanes_of[d + nwaves];
    }
    uint32_t run = 0, nsl = 0, halt = kNone;
    bool nowin = !win;
    int32_t zrun = -1;  // last non-empty lane of the earlier chunks
    // lanes past the document's last reload that lane (any defined value does)
    auto load = [&](uint32_t c, uint32_t &cn, uint32_t &hf, uint32_t &cu, uint32_t &en) {
      const uint32_t jc = lb + min(c + lane, nl - 1);
      cn = a.counts[jc];
      hf = a.halted[jc];
      cu = a.cuts[jc];
      en = a.ends[jc];
    };
    uint32_t q_cn, q_hf, q_cu, q_en;
    load(0, q_cn, q_hf, q_cu, q_en);
    for (uint32_t c = 0; c < nl; c += 64) {
      const uint32_t cn0 = q_cn, hf0 = q_hf, cu0 = q_cu, en0 = q_en;
      if (c + 64 < nl) load(c + 64, q_cn, q_hf, q_cu, q_en);  // wave-uniform
      const bool ok = c + lane < nl;
      const uint32_t j = lb + c + lane;
      const uint32_t cnt = ok ? cn0 : 0;
      const uint32_t hf = ok ? hf0 : 0;
      const bool h = hf & 1;
      const bool ne = ok && cu0 < en0;
      uint32_t incl = cnt;
      int32_t z = ne ? (int32_t)j : zrun;
      for (int k = 1; k < 64; k <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, k);
        const int32_t zz = __shfl_up(z, k);
        if ((int)lane >= k) {
          incl += v;
          z = max(z, zz);
        }
      }
      if (ok) {
        a.lane_pre[j] = run + incl - cnt;
        if (win) a.lnz[j] = (uint32_t)z;
      }
      nowin = nowin || __any(hf & 2);
      zrun = __shfl(z, 63);
      const unsigned long long hb = __ballot(h), nb = __ballot(ne);
      if (hb) {  // wave-uniform
        const int f = __ffsll(hb) - 1;
        run += (uint32_t)__shfl((int)incl, f);
        nsl += __popcll(nb & ((2ull << f) - 1));
        halt = lb + c + f;
        break;
      }
      run += (uint32_t)__shfl((int)incl, 63);
      nsl += __popcll(nb);
    }
    if (lane == 0) {
      a.doc_ntok[d] = run;
      a.doc_halt[d] = halt;
      a.doc_nsl[d] = nsl;
      // a halted document, a fallback or a long slice: the lane emit writes it
      const bool w = !nowin && halt == kNone;
      a.doc_win[d] = w;
      any_lane |= !w;
    }
  }
  if (lane == 0 && any_lane) a.meta[kAnyLane] = 1;  // every writer stores the same value
}

// Results, first half: each group's token, halted-document and slice sums.
__global__ void __launch_bounds__(256) k_bscan_a(BatchArgs a) {
  __shared__ uint64_t red[3][4];
  if (a.meta[kBad]) return;  // uniform: no barrier follows
  uint32_t lo, hi;
  group_range(a.ndocs, lo, hi);
  uint64_t v[3] = {0, 0, 0};
  for (uint32_t d = lo + threadIdx.x; d < hi; d += blockDim.x) {
    v[0] += a.doc_ntok[d];
    v[1] += a.doc_halt[d] != kNone;
    v[2] += a.doc_nsl[d];
  }
  block_sum<3>(v, red);
  if (threadIdx.x < 3) a.part[(size_t)blockIdx.x * kPartWords + 5 + threadIdx.x] = v[threadIdx.x];
}

// Results, second half: output offsets of the documents (exclusive scan), results, status;
// the first group writes the batch's totals.
__global__ void __launch_bounds__(256) k_bscan_b(BatchArgs a) {
  __shared__ uint64_t red[6][4];
  if (a.meta[kBad]) {  // nothing was counted: report the bad table
    for (uint32_t d = blockIdx.x * blockDim.x + threadIdx.x; d < a.ndocs; d += gridDim.x * blockDim.x)
      a.res[d] = DocResDev{0, 0, 0, -1, 0};
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.total->ntokens = 0;
      a.total->error_offset = 0;
      a.total->status = -1;
      a.total->nslices = 0;
    }
    return;
  }
  uint64_t pre[3], tot[3];
  group_prefix<3>(a.part, 5, pre, tot, red);
  const uint64_t total = tot[0];
  const int32_t status = total > a.cap ? -4 : 0;
  uint64_t run = pre[0];
  uint32_t lo, hi;
  group_range(a.ndocs, lo, hi);
  for (uint32_t d0 = lo; d0 < hi; d0 += blockDim.x) {  // workgroup-uniform: the scan sees every thread
    const uint32_t d = d0 + threadIdx.x;
    const bool in = d < hi;
    const uint32_t nt = in ? a.doc_ntok[d] : 0;
    uint64_t v[1] = {nt}, t[1];
    block_incl<1>(v, t, red);
    if (in) {
      DocResDev r;
      r.tok_offset = run + v[0] - nt;
      r.ntokens = nt;
      r.error_offset = a.docs[d].length;  // a halted document's emit replaces it
      r.status = status;
      r.nslices = a.doc_nsl[d];
      a.res[d] = r;
    }
    run += t[0];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.total->ntokens = total;
    a.total->error_offset = tot[1];  // documents that did not tokenize completely
    a.total->status = status;
    a.total->nslices = (uint32_t)tot[2];
  }
}

// Emit walk of the batch: the lane emit of each lane up to its document's first halted one.
__global__ void __launch_bounds__(256) k_bemit(BatchArgs a) {
  if (!a.meta[kAnyLane]) return;  // every document takes the windowed emit (uniform)
  const BatchLds l = batch_stage(a);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nlanes = a.meta[kNLanes];
  const bool write = a.total->status == 0;
  for (;;) {
    const uint32_t tile = next_tile(&a.meta[kQEmit]);
    if ((uint64_t)tile * 64 >= nlanes) break;  // wave-uniform exit
    const uint32_t j = tile * 64 + lane;
    if (j >= nlanes) continue;
    const uint32_t d = a.lane_doc[j];
    const uint32_t halt = a.doc_halt[d];
    if ((halt != kNone && j > halt) || a.doc_win[d]) continue;
    const DocDev doc = a.docs[d];
    const BatchInst &in = a.inst[doc.inst];
    const uint8_t *src = a.bytes + doc.offset;
    const uint32_t s = a.cuts[j], e = a.ends[j];
    const uint32_t off = (uint32_t)a.res[d].tok_offset + a.lane_pre[j];
    Ring r;
    r.w = reinterpret_cast<uint32_t *>(l.ring) + threadIdx.x;
    r.stride = blockDim.x;
    r.kinds = a.kinds;
    r.lens = a.lens;
    r.offs = a.offs;
    r.o = off;
    r.fl = off & ~(uint32_t)(kChunk - 1);
    r.first = off;
    r.write = write;
    r.direct = e - s >= (1u << 24);
    const Tables tb{l.T, l.info, l.kind, in.sink, in.fail, in.start};
    LaneState L;
    L.cnt = 0;
    if (in.mono) {
      if (!r.direct && !r.offs) walk<true, true, true>(L, r, tb, src, doc.length, s, e);
      else walk<true, true, false>(L, r, tb, src, doc.length, s, e);
    } else {
      if (!r.direct && !r.offs) walk<true, false, true>(L, r, tb, src, doc.length, s, e);
      else walk<true, false, false>(L, r, tb, src, doc.length, s, e);
    }
    ring_flush_tail(r);
    if (j == halt) a.res[d].error_offset = L.tok;  // the halt offset, relative to the document
  }
}

// The windowed emit over a batch's documents.  Work items are tiles of 64 windows of one
// document (windows: the kWin-aligned stretches of the address space, clipped to the
// document), in contiguous ranges per wave; each wave walks one tile at a time, a window per thread,
// from the count walk's checkpoint, stages the tile's tokens and writes them out coalesced,
// exactly as the single-buffer windowed emit does with the document as its input (its
// slices, cut at certified bytes or at the hybrid plan's serial token starts, are the
// lanes; the document's end is the end of input).  Documents the count walk marked (a
// halt, a fallback of a non-monotone automaton, a slice of 2^24 bytes or more) are left to
// the lane emit.
// A document's windowed-emit context (wave-uniform).
struct BDoc {
  const uint8_t *src;
  uint32_t len, mis0, nwin, lb, nl, lnom, out0, lim;
  const uint2 *over;
  uint32_t inst;
  uint32_t sb;  // split by the hybrid plan: its first speculative lane, else kNone
};

// First-round loads for window i of the document (the candidate owner's slice and the last
// non-empty lane before it; all three addresses are known without a load).
struct BWinR1 {
  uint32_t ws, j0, s0, e0, lz;
};

__device__ __forceinline__ BWinR1 bwin_r1(const BatchArgs &a, const BDoc &c, uint32_t i) {
  BWinR1 r{};
  if (i >= c.nwin) return r;
  r.ws = i ? i * kWin - c.mis0 : 0;  // document-relative start
  r.j0 = c.lb + min(r.ws / c.lnom, c.nl - 1);
  r.s0 = a.cuts[r.j0];
  r.e0 = a.ends[r.j0];
  r.lz = r.j0 > c.lb ? a.lnz[r.j0 - 1] : r.j0;  // lane 0 starts at 0: it owns a window it misses
  return r;
}

// Second round: the owner's state at the window's start and its first output slot.  Past the
// document's windows: the document's output end.
__device__ __forceinline__ WinMeta bwin_meta(const BatchArgs &a, const BDoc &c, const BatchInst &in,
                                             const BWinR1 &r, uint32_t i) {
  WinMeta m{0, 0, c.lim, 0};
  if (i >= c.nwin) return m;
  const bool here = r.s0 < r.e0 && r.s0 <= r.ws;
  const uint32_t j = here ? r.j0 : r.lz;
  const uint32_t base = c.out0 + a.lane_pre[j];
  if (here && r.s0 == r.ws) {  // the lane starts here: a fresh token
    m.st = in.start;
    m.tok = r.ws;
    m.out = base;
    m.fresh = 1;
    return m;
  }
  // A split document's slice was counted in parts (k_bsplit): the counts of the parts before
  // this window's come on top of its checkpoint's, and a window starting a part starts a
  // token, as at a lane start (the window before it then ends the token in progress).
  uint32_t add = 0;
  if (c.sb != kNone) {
    const uint4 pp = a.spec_part[c.sb + (j - c.lb)], pr = a.spec_pre[c.sb + (j - c.lb)];
    const uint32_t q = (r.ws >= pp.x) + (r.ws >= pp.y) + (r.ws >= pp.z);
    add = q == 3 ? pr.z : q == 2 ? pr.y : q == 1 ? pr.x : 0;
    if (r.ws == pp.x || r.ws == pp.y || r.ws == pp.z) {
      m.st = in.start;
      m.tok = r.ws;
      m.out = base + add;
      m.fresh = 1;
      return m;
    }
  }
  const uint32_t k = (r.ws - (j - c.lb) * c.lnom) / kWin;
  const uint2 ck = k < a.kslots ? a.ck_main[ck_index(k, j, a.max_lanes)] : c.over[i];
  m.st = row_state(ck.x >> 24);
  m.tok = ck.y;
  m.out = base + (ck.x & 0xFFFFFFu) + add;
  return m;
}

// Each workgroup takes a contiguous range of tiles, and its waves claim runs of it through
// a counter in LDS, guided: a run is a (2 × waves)-th of what remains, at least one tile,
// so that runs are long at first and single tiles at the end, and the waves of a CU finish
// together (a device-scope atomic per tile would cost more than the tile).  A wave walks a
// run document segment by document segment; within a segment the next tile's bytes and
// the following tiles' window states load while a tile walks, as in the single-buffer
// windowed emit.
__global__ void __launch_bounds__(1024) k_bemit_win(BatchArgs a) {
  if (a.meta[kNoWin] || a.total->status != 0) return;  // uniform: no barrier follows
  extern __shared__ __align__(16) uint8_t smem_w[];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  uint32_t *ctr = reinterpret_cast<uint32_t *>(smem_w + batch_win_lds_bytes(a.nrows, a.ninst, wpb) - 16);
  if (threadIdx.x == 0) *ctr = 0;
  const BatchLds l = batch_stage(a);  // its barrier publishes the zeroed counter
  uint32_t *stage = reinterpret_cast<uint32_t *>(l.ring) + wid * kStageWords;
  const uint32_t ntiles = a.meta[kNTiles];
  const uint32_t rm = refused_mask(a);
  const uint32_t per_g = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t g_lo = min(ntiles, blockIdx.x * per_g), g_hi = min(ntiles, g_lo + per_g), span = g_hi - g_lo;
  for (;;) {
    uint32_t c0 = 0, len = 0;
    if (lane == 0) {
      const uint32_t done = *reinterpret_cast<volatile uint32_t *>(ctr);
      len = max(1u, (span > done ? span - done : 0u) / (2 * wpb));
      c0 = atomicAdd(ctr, len);
    }
    c0 = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)c0, 0));
    len = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)len, 0));
    if (c0 >= span) break;
    const uint32_t t_lo = g_lo + c0, t_hi = g_lo + min(span, c0 + len);
  for (uint32_t t = t_lo; t < t_hi;) {
    const uint32_t d = a.tile_doc[t];
    const DocDev doc = a.docs[d];
    const uint32_t tb0 = a.tile_base[d];
    BDoc c;
    c.src = a.bytes + doc.offset;
    c.len = doc.length;
    c.mis0 = (uint32_t)(reinterpret_cast<uintptr_t>(c.src) & (kWin - 1));
    c.nwin = doc_windows(reinterpret_cast<uintptr_t>(c.src), doc.length);
    const uint32_t nt = (c.nwin + 63) / 64;
    const uint32_t tt_lo = t - tb0, tt_hi = min(t_hi, tb0 + nt) - tb0;
    t = tb0 + tt_hi;  // the next segment
    if (!a.doc_win[d]) continue;
    c.lb = a.lane_base[d];
    c.nl = a.lanes_of[d];
    const bool split = spec_split(a, rm, doc);
    c.lnom = split ? a.spec_bytes : a.lane_bytes;
    c.sb = split ? a.spec_base[d] : kNone;
    c.out0 = (uint32_t)a.res[d].tok_offset;
    c.lim = c.out0 + (uint32_t)a.res[d].ntokens;  // the document's outputs end here
    c.over = a.ck_over + (size_t)tb0 * 64;
    c.inst = doc.inst;
    const BatchInst &in = a.inst[doc.inst];
    const Tables tb{l.T, l.info, l.kind, in.sink, in.fail, in.start};
    WalkArgs wa{};
    wa.in = c.src;
    wa.n = c.len;
    wa.kinds = a.kinds;
    wa.lens = a.lens;
    wa.offs = a.offs;
    auto wpos = [&](uint32_t tt) { return (int64_t)(tt * 64 + lane) * kWin - c.mis0; };
    auto is_edge = [&](uint32_t tt) { return tt == 0 || tt + 1 == nt; };
    WinMeta cur = bwin_meta(a, c, in, bwin_r1(a, c, tt_lo * 64 + lane), tt_lo * 64 + lane);
    WinMeta nxt = bwin_meta(a, c, in, bwin_r1(a, c, (tt_lo + 1) * 64 + lane), (tt_lo + 1) * 64 + lane);
    BWinR1 r1 = bwin_r1(a, c, (tt_lo + 2) * 64 + lane);
    Win64 dat = is_edge(tt_lo) ? win_load<true>(c.src, wpos(tt_lo), c.len) : win_load<false>(c.src, wpos(tt_lo), c.len);
    for (uint32_t tt = tt_lo; tt < tt_hi; ++tt) {
      const uint32_t i = tt * 64 + lane;
      Win64 ndat = dat;
      if (tt + 1 < tt_hi)
        ndat = is_edge(tt + 1) ? win_load<true>(c.src, wpos(tt + 1), c.len)
                               : win_load<false>(c.src, wpos(tt + 1), c.len);
      const WinMeta n2 = bwin_meta(a, c, in, r1, (tt + 2) * 64 + lane);
      r1 = bwin_r1(a, c, (tt + 3) * 64 + lane);
      const uint32_t o_first = __shfl(cur.out, 0), o_next = __shfl(nxt.out, 0);
      const uint32_t down = __shfl_down(cur.out, 1), fdown = __shfl_down(cur.fresh, 1);
      const uint32_t f_next = __shfl(nxt.fresh, 0);
      const uint32_t P = __shfl(cur.tok, 0);
      const uint32_t span_end = (uint32_t)min<int64_t>((int64_t)(tt + 1) * 64 * kWin - c.mis0, c.len);
      if (in.disc)
        win_tile<true>(tb, wa, stage, lane, cur, i, i < c.nwin, is_edge(tt), dat, wpos(tt), c.nwin, o_first, o_next,
                       true, lane < 63 ? down : o_next, lane < 63 ? fdown : f_next, P, span_end, c.lim);
      else
        win_tile<false>(tb, wa, stage, lane, cur, i, i < c.nwin, is_edge(tt), dat, wpos(tt), c.nwin, o_first, o_next,
                        true, lane < 63 ? down : o_next, lane < 63 ? fdown : f_next, P, span_end, c.lim);
      cur = nxt;
      nxt = n2;
      dat = ndat;
    }
  }
  }
}

// ------------------------------------------------- hybrid plan for a single buffer
// The hybrid plan (see the batch notes above) for one buffer of a refused set: lane k walks
// [k S, (k+1) S + kSpecX) speculatively (k_hspec), k_hsync finds the cuts, and k_hcuts
// writes them as the planned lane boundaries, or {0, n, ..., n} (one slice) when the plan
// falls back.  The count walk, scan and emit of the pipeline path then run unchanged.
struct HybridArgs {
  const uint8_t *in;
  uint32_t n, nlanes, S;
  uint32_t *cut, *rst, *bits, *fail;  // per lane: cut, last restart, head then tail; one flag
  uint32_t *cuts;                     // nlanes + 1 lane boundaries
};

__global__ void __launch_bounds__(256) k_hspec(WalkArgs a, HybridArgs h) {
  const Lds l = carve_lds(a.nrows);
  stage_tables(a, l, false);
  const Tables tb{lds_bytes_of(l.T), l.info, l.kind, a.sink, a.fail, 0};
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) *h.fail = 0;
  for (uint32_t k = gid; k < h.nlanes; k += gridDim.x * blockDim.x) {
    const uint32_t b = k * h.S;
    const uint32_t b2 = (uint32_t)min<uint64_t>((uint64_t)(k + 1) * h.S, h.n);
    const uint32_t end = (uint32_t)min<uint64_t>((uint64_t)b2 + kSpecX, h.n);
    uint32_t *bits = h.bits + (size_t)k * 2 * kSpecWords;
    uint32_t rst;
    if (a.fail == a.sink) walk_spec<true>(tb, h.in, h.n, b, end, b2, bits, bits + kSpecWords, rst);
    else walk_spec<false>(tb, h.in, h.n, b, end, b2, bits, bits + kSpecWords, rst);
    h.rst[k] = rst;
  }
}

__global__ void __launch_bounds__(256) k_hsync(HybridArgs h) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < h.nlanes; k += gridDim.x * blockDim.x) {
    uint32_t cut = 0;
    bool ok = true;
    if (k) {
      const uint32_t *head = h.bits + (size_t)k * 2 * kSpecWords;
      const uint32_t *tail = h.bits + (size_t)(k - 1) * 2 * kSpecWords + kSpecWords;
      cut = kNone;
      for (uint32_t w = 0; w < kSpecWords && cut == kNone; ++w) {
        const uint32_t x = head[w] & tail[w];
        if (x) cut = k * h.S + 32 * w + (__ffs(x) - 1);
      }
      if (cut == kNone && k + 1 == h.nlanes) cut = h.n;  // as in k_bsync
      ok = cut != kNone;
    }
    if (ok && h.rst[k] != kNone && h.rst[k] >= cut) ok = false;
    h.cut[k] = cut;
    if (!ok) *h.fail = 1;
  }
}

__global__ void __launch_bounds__(256) k_hcuts(HybridArgs h) {
  const bool fail = *h.fail != 0;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= h.nlanes; k += gridDim.x * blockDim.x)
    h.cuts[k] = k == h.nlanes ? h.n : fail ? (k ? h.n : 0) : h.cut[k];
}

}  // namespace

// ------------------------------------------------------------------ host side
uint32_t windows_max(uint32_t n) { return (uint32_t)(((uint64_t)n + 2 * kWin - 1) / kWin); }
// A lane's nominal range plus four windows of slack (slices usually end within a line
// of their lane's end).
uint32_t ck_slots(uint32_t lane_bytes) { return (lane_bytes / kWin + 4 + kCkB - 1) / kCkB * kCkB; }

static size_t carve_layout(uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, int windowed, int hybrid,
                           size_t *offs) {
  const uint32_t nlanes = n ? (n + lane_bytes - 1) / lane_bytes : 1;
  const uint32_t nblocks = (nlanes + block - 1) / block;
  const uint32_t nwords = (n + 63) / 64;
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  const uint32_t ngroups = (ntiles + kTilesPerBlock - 1) / kTilesPerBlock;
  size_t at = 0;
  offs[0] = at;
  at += align256(pipeline ? (size_t)(nwords ? nwords : 1) * 8 : 0);
  offs[1] = at;
  at += align256(pipeline ? (size_t)(ntiles + 1) * 8 : 0);
  offs[2] = at;
  at += align256(pipeline ? (size_t)(ngroups + 1) * 8 : 0);
  offs[3] = at;
  at += align256((size_t)(nlanes + 1) * 4);
  offs[4] = at;
  at += align256((size_t)nlanes * 4);
  offs[9] = at;  // slice ends (fused path)
  at += align256((size_t)nlanes * 4);
  offs[5] = at;
  at += align256((size_t)nblocks * 8);
  offs[6] = at;
  at += align256((size_t)nblocks * 4);
  offs[7] = at;
  at += align256((size_t)nblocks * 4);
  offs[8] = at;
  at += align256(16);
  offs[10] = at;  // per-block long-slice flags
  at += align256((size_t)nblocks * 4);
  offs[11] = at;  // in-block count prefixes
  at += align256((size_t)nlanes * 4);
  offs[12] = at;  // checkpoints: main part, then overflow (one spare window for any alignment)
  if (windowed) at += align256((size_t)ck_slots(lane_bytes) * nlanes * 8) + align256((size_t)windows_max(n) * 8);
  offs[13] = at;  // per lane: last non-empty lane in the workgroup so far
  at += align256((size_t)nlanes * 4);
  offs[14] = at;  // per workgroup: last non-empty lane
  at += align256((size_t)nblocks * 4);
  offs[15] = at;  // one pass: look-back status per workgroup
  if (windowed) at += align256((size_t)nblocks * 8);
  offs[16] = at;  // one pass: workgroup counter
  if (windowed) at += align256(4);
  offs[17] = at;  // hybrid plan: per lane cut, last restart, head and tail token starts; a flag
  if (hybrid) at += 2 * align256((size_t)nlanes * 4) + align256((size_t)nlanes * 2 * kSpecWords * 4) + align256(4);
  return at;
}

size_t workspace_bytes(uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, int windowed, int hybrid) {
  size_t offs[18];
  return carve_layout(n, lane_bytes, block, pipeline, windowed, hybrid, offs);
}

bool carve(void *ws, size_t ws_bytes, uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, int windowed,
           int hybrid, Plan &p) {
  size_t offs[18];
  const size_t need = carve_layout(n, lane_bytes, block, pipeline, windowed, hybrid, offs);
  if (ws_bytes < need || !ws) return false;
  uint8_t *b = static_cast<uint8_t *>(ws);
  p.n = n;
  p.lane_bytes = lane_bytes;
  p.nlanes = n ? (n + lane_bytes - 1) / lane_bytes : 1;
  p.block = block;
  p.nblocks = (p.nlanes + block - 1) / block;
  p.ntiles = (n + kTile - 1) / kTile;
  p.bitmap = pipeline ? reinterpret_cast<uint64_t *>(b + offs[0]) : nullptr;
  p.tile_next = pipeline ? reinterpret_cast<uint64_t *>(b + offs[1]) : nullptr;
  p.tile_group = pipeline ? reinterpret_cast<uint64_t *>(b + offs[2]) : nullptr;
  p.cuts = reinterpret_cast<uint32_t *>(b + offs[3]);
  p.counts = reinterpret_cast<uint32_t *>(b + offs[4]);
  p.ends = reinterpret_cast<uint32_t *>(b + offs[9]);
  p.blk_sum = reinterpret_cast<uint64_t *>(b + offs[5]);
  p.blk_fail = reinterpret_cast<uint32_t *>(b + offs[6]);
  p.blk_nonempty = reinterpret_cast<uint32_t *>(b + offs[7]);
  p.meta = reinterpret_cast<uint32_t *>(b + offs[8]);
  p.blk_big = reinterpret_cast<uint32_t *>(b + offs[10]);
  p.lane_pre = reinterpret_cast<uint32_t *>(b + offs[11]);
  p.windowed = windowed;
  p.kslots = ck_slots(lane_bytes);
  p.ck = windowed ? reinterpret_cast<uint2 *>(b + offs[12]) : nullptr;
  p.ck_over = windowed ? reinterpret_cast<uint2 *>(b + offs[12] + align256((size_t)p.kslots * p.nlanes * 8)) : nullptr;
  p.lnz = reinterpret_cast<int32_t *>(b + offs[13]);
  p.blk_lnz = reinterpret_cast<int32_t *>(b + offs[14]);
  p.chunk_st = windowed ? reinterpret_cast<uint64_t *>(b + offs[15]) : nullptr;
  p.chunk_ctr = windowed ? reinterpret_cast<uint32_t *>(b + offs[16]) : nullptr;
  p.hybrid = hybrid;
  if (hybrid) {
    uint8_t *h = b + offs[17];
    p.spec_cut = reinterpret_cast<uint32_t *>(h), h += align256((size_t)p.nlanes * 4);
    p.spec_rst = reinterpret_cast<uint32_t *>(h), h += align256((size_t)p.nlanes * 4);
    p.spec_bits = reinterpret_cast<uint32_t *>(h), h += align256((size_t)p.nlanes * 2 * kSpecWords * 4);
    p.spec_fail = reinterpret_cast<uint32_t *>(h);
  } else {
    p.spec_cut = p.spec_rst = p.spec_bits = p.spec_fail = nullptr;
  }
  return true;
}

size_t walk_lds_bytes(int nrows, uint32_t block, bool emit) { return lds_bytes(nrows, (int)block, emit); }
size_t window_lds_bytes(int nrows) { return emit_win_lds_bytes(nrows, 4); }
size_t onepass_lds_bytes(int nrows) { return one_lds_bytes(nrows); }

static CertArg cert_arg(const CertMap &cm) {
  CertArg ca{};
  for (int i = 0; i < 8; ++i) ca.words[i] = cm.words[i];
  if (cm.nbytes <= 8) {
    ca.np = cm.nbytes;
    for (int i = 0; i < cm.nbytes; ++i) ca.pat[i] = 0x01010101u * cm.bytes[i];
  } else {
    ca.np = -1;
  }
  return ca;
}

hipError_t launch_bitmap(const uint8_t *in, uint32_t n, const CertMap &cm, uint64_t *bits, hipStream_t s) {
  const uint32_t nwords = (n + 63) / 64;
  if (!nwords) return hipSuccess;
  k_bitmap<<<(nwords + 255) / 256, 256, 0, s>>>(in, n, cert_arg(cm), bits, nullptr);
  return hipGetLastError();
}

static WalkArgs walk_args(const DevTable &t, const CertMap &cm, const uint8_t *in, const Plan &p, uint8_t *kinds,
                          uint32_t *lens, uint64_t *offs, uint64_t cap, ResultDev *res, const uint8_t *cert_lut) {
  WalkArgs a{};
  a.ca = cert_arg(cm);
  a.ends = p.ends;
  a.table = t.table;
  a.rowinfo = t.rowinfo;
  a.rowkind = t.rowkind;
  a.nrows = t.nrows;
  a.sink = ((uint32_t)t.row_sink << kRowShift) | (((uint32_t)t.row_sink & 31u) << 2);
  a.fail = t.row_fail >= 0 ? ((uint32_t)t.row_fail << kRowShift) | (((uint32_t)t.row_fail & 31u) << 2) : a.sink;
  a.in = in;
  a.n = p.n;
  a.cuts = p.cuts;
  a.lane_bytes = p.lane_bytes;
  a.nlanes = p.nlanes;
  a.cert = cert_lut;
  a.counts = p.counts;
  a.blk_sum = p.blk_sum;
  a.blk_fail = p.blk_fail;
  a.blk_nonempty = p.blk_nonempty;
  a.blk_big = p.blk_big;
  a.lane_pre = p.lane_pre;
  a.ck = p.ck;
  a.ck_over = p.ck_over;
  a.kslots = p.kslots;
  a.lnz = p.lnz;
  a.blk_lnz = p.blk_lnz;
  a.chunk_st = p.chunk_st;
  a.chunk_ctr = p.chunk_ctr;
  a.block = p.block;
  a.block_shift = (uint32_t)__builtin_ctz(p.block);
  {
    const uint32_t d = p.lane_bytes;  // >= 16
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    a.lane_div.l = l;
    a.lane_div.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  }
  a.meta = p.meta;
  a.res = res;
  a.kinds = kinds;
  a.lens = lens;
  a.offs = offs;
  a.cap = cap;
  return a;
}

static inline void mark(hipEvent_t const *ev, int i, hipStream_t s) {
  if (ev && ev[i]) (void)hipEventRecord(ev[i], s);
}

// Workgroups of the windowed emit: 16 waves per CU in workgroups of `waves`, fewer for a
// short input (about one tile per wave).
static uint32_t win_grid(uint32_t waves, uint32_t ntiles) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t want = (ntiles + waves - 1) / waves;
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(want, (uint32_t)cus * (16 / waves)));
  return g >= 8 ? g & ~7u : g;  // whole rounds of the 8 XCDs
}

template <bool FUSED>
static hipError_t count_scan_emit(const DevTable &t, const WalkArgs &a0, const Plan &p, uint64_t cap,
                                  ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  WalkArgs a = a0;
  const size_t smem_c = lds_bytes(t.nrows, (int)p.block, false);
  const size_t smem_e = lds_bytes(t.nrows, (int)p.block, true);
  const bool win = p.windowed;
  mark(ev, 1, s);
  if (win && t.monotone) k_count<true, FUSED, true><<<p.nblocks, p.block, smem_c, s>>>(a);
  else if (win) k_count<false, FUSED, true><<<p.nblocks, p.block, smem_c, s>>>(a);
  else if (t.monotone) k_count<true, FUSED, false><<<p.nblocks, p.block, smem_c, s>>>(a);
  else k_count<false, FUSED, false><<<p.nblocks, p.block, smem_c, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 2, s);
  k_scan<<<1, 1024, 0, s>>>(p.blk_sum, p.blk_fail, p.blk_nonempty, p.blk_big, p.blk_lnz, p.nblocks, p.block,
                            p.counts, p.meta, res, cap, p.n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 3, s);
  if (win) {  // the windowed emit, or the lane emit in the same launch
    const uint32_t ntiles = (windows_max(p.n) + 63) / 64, w = win_waves(t.nrows);
    const uint32_t g = win_grid(w, ntiles);
    const size_t lds = emit_win_lds_bytes(t.nrows, w);
    if (t.all_counted && t.monotone) k_emit_win<FUSED, false, true><<<g, w * 64, lds, s>>>(a);
    else if (t.all_counted) k_emit_win<FUSED, false, false><<<g, w * 64, lds, s>>>(a);
    else if (t.monotone) k_emit_win<FUSED, true, true><<<g, w * 64, lds, s>>>(a);
    else k_emit_win<FUSED, true, false><<<g, w * 64, lds, s>>>(a);
  } else if (t.monotone) {
    k_emit<true, FUSED><<<p.nblocks, p.block, smem_e, s>>>(a);
  } else {
    k_emit<false, FUSED><<<p.nblocks, p.block, smem_e, s>>>(a);
  }
  e = hipGetLastError();
  mark(ev, 4, s);
  return e;
}

hipError_t run_pipeline(const DevTable &t, const CertMap &cm, const uint8_t *in, const Plan &p, bool serial,
                        uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap, ResultDev *res,
                        hipStream_t s, hipEvent_t const *ev) {
  mark(ev, 0, s);
  // One slice (serial mode, an empty useful map, or an input shorter than one lane):
  // cuts = {0, n}; otherwise bitmap, tile suffix minimum, then one target per lane.
  const bool one = serial || p.nlanes == 1 || cm.nbytes == 0;
  if (one && p.nlanes != 1) return hipErrorInvalidValue;  // the host plans one lane then
  if (!one) {
    const uint32_t nwords = (p.n + 63) / 64;
    const uint32_t ngroups = (p.ntiles + kTilesPerBlock - 1) / kTilesPerBlock;
    if (ngroups > 1024) return hipErrorInvalidValue;
    k_bitmap<<<(nwords + 255) / 256, 256, 0, s>>>(in, p.n, cert_arg(cm), p.bitmap, p.tile_next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tiles_blocks<<<ngroups, kTilesPerBlock, 0, s>>>(p.tile_next, p.ntiles, p.tile_group);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tiles_top<<<1, 1024, 0, s>>>(p.tile_group, ngroups);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  k_plan<<<(p.nlanes + 1 + 255) / 256, 256, 0, s>>>(p.bitmap, p.tile_next, p.tile_group, p.n, p.lane_bytes,
                                                    p.nlanes, p.cuts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const WalkArgs a = walk_args(t, cm, in, p, kinds, lens, offs, cap, res, nullptr);
  return count_scan_emit<false>(t, a, p, cap, res, s, ev);
}

// ------------------------------------------------------------------ batches
// A batch's speculative lane is kSpecX bytes, the shortest the sync window allows: the
// speculative walks ([k S, (k + 1) S + kSpecX)) are serial and few (refused documents
// only), so their length, not their number, sets the walk kernel's time.
static uint32_t batch_spec_bytes(uint32_t) { return kSpecX; }

// a document of n bytes has ceil(n / L) <= n / L + 1 lanes, L its lane length
static uint32_t batch_max_lanes(uint32_t ndocs, uint64_t nbytes, uint32_t lane_bytes) {
  const uint32_t shortest = std::min(lane_bytes, batch_spec_bytes(lane_bytes));
  return (uint32_t)std::min<uint64_t>(0xFFFFFFF0ull, (uint64_t)ndocs + nbytes / shortest + 1);
}

// speculative lanes: a split document of n bytes has ceil(n / S) <= n / S + 1 of them
static uint32_t batch_max_spec(uint32_t ndocs, uint64_t nbytes, uint32_t lane_bytes) {
  return (uint32_t)std::min<uint64_t>(0xFFFFFFF0ull, (uint64_t)ndocs + nbytes / batch_spec_bytes(lane_bytes) + 1);
}

// tiles of 64 windows: a document of n bytes touches at most n / kWin + 2 windows
static uint32_t batch_max_tiles(uint32_t ndocs, uint64_t nbytes) {
  return (uint32_t)std::min<uint64_t>(0xFFFFFFF0ull, 2ull * ndocs + nbytes / (64 * kWin) + 1);
}

size_t batch_workspace_bytes(uint32_t ndocs, uint64_t nbytes, uint32_t lane_bytes) {
  const uint64_t nl = batch_max_lanes(ndocs, nbytes, lane_bytes);
  const uint64_t ns = batch_max_spec(ndocs, nbytes, lane_bytes);
  const uint64_t nt = batch_max_tiles(ndocs, nbytes);
  const size_t per_doc = align256((size_t)std::max<uint32_t>(ndocs, 1) * 4);
  return align256(kBatchMeta * 4) + align256((size_t)kDocGroups * kPartWords * 8) + 9 * per_doc + 7 * align256((size_t)nl * 4) + 3 * align256((size_t)ns * 4) +
         align256((size_t)ns * 2 * kSpecWords * 4) + 2 * align256((size_t)ns * 16) +
         align256((size_t)ck_slots(lane_bytes) * nl * 8) +
         align256((size_t)nt * 64 * 8) + align256((size_t)nt * 4);
}

size_t batch_emit_lds_bytes(int nrows, uint32_t ninst) {
  const size_t b = batch_lds_offset(nrows, ninst) + 256 * (size_t)kRingBytes;
  return b <= 160 * 1024 ? b : 0;
}

hipError_t run_batch(const BatchTables &bt, const uint8_t *bytes, uint64_t nbytes, const void *docs, uint32_t ndocs,
                     uint32_t lane_bytes, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap, void *res,
                     ResultDev *total, void *ws, size_t ws_bytes, hipStream_t s, hipEvent_t const *ev) {
  if (ws_bytes < batch_workspace_bytes(ndocs, nbytes, lane_bytes)) return hipErrorInvalidValue;
  const size_t lds_e = batch_emit_lds_bytes(bt.nrows, bt.ninst);
  if (!lds_e || bt.ninst == 0 || bt.ninst > (uint32_t)kMaxInst) return hipErrorInvalidValue;
  BatchArgs a{};
  a.table = bt.table;
  a.rowinfo = bt.rowinfo;
  a.rowkind = bt.rowkind;
  a.luts = bt.luts;
  a.nrows = bt.nrows;
  a.ninst = bt.ninst;
  for (uint32_t k = 0; k < bt.ninst; ++k) {
    a.inst[k].start = bt.inst[k].start;
    a.inst[k].sink = bt.inst[k].sink;
    a.inst[k].fail = bt.inst[k].fail;
    a.inst[k].mono = bt.inst[k].mono;
    a.inst[k].refused = bt.inst[k].refused;
    a.inst[k].disc = bt.inst[k].disc;
    a.inst[k].ca = cert_arg(bt.inst[k].cm);
  }
  a.bytes = bytes;
  a.nbytes = nbytes;
  a.docs = static_cast<const DocDev *>(docs);
  a.ndocs = ndocs;
  a.lane_bytes = lane_bytes;
  a.max_lanes = batch_max_lanes(ndocs, nbytes, lane_bytes);
  // workspace: the per-lane arrays are sized for the most lanes the byte count allows
  uint8_t *w = static_cast<uint8_t *>(ws);
  a.meta = reinterpret_cast<uint32_t *>(w);
  w += align256(kBatchMeta * 4);
  a.part = reinterpret_cast<uint64_t *>(w);
  w += align256((size_t)kDocGroups * kPartWords * 8);
  const size_t dsz = align256((size_t)std::max<uint32_t>(ndocs, 1) * 4);
  a.lanes_of = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.lane_base = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.doc_halt = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.doc_ntok = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.doc_nsl = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.spec_base = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.spec_fail = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.tile_base = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.doc_win = reinterpret_cast<uint32_t *>(w), w += dsz;
  a.spec_bytes = batch_spec_bytes(lane_bytes);
  a.max_spec = batch_max_spec(ndocs, nbytes, lane_bytes);
  const size_t per_spec = align256((size_t)a.max_spec * 4);
  a.spec_doc = reinterpret_cast<uint32_t *>(w), w += per_spec;
  a.spec_cut = reinterpret_cast<uint32_t *>(w), w += per_spec;
  a.spec_rst = reinterpret_cast<uint32_t *>(w), w += per_spec;
  a.spec_bits = reinterpret_cast<uint32_t *>(w), w += align256((size_t)a.max_spec * 2 * kSpecWords * 4);
  a.spec_part = reinterpret_cast<uint4 *>(w), w += align256((size_t)a.max_spec * 16);
  a.spec_pre = reinterpret_cast<uint4 *>(w), w += align256((size_t)a.max_spec * 16);
  const size_t per_lane = align256((size_t)batch_max_lanes(ndocs, nbytes, lane_bytes) * 4);
  a.lane_doc = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.cuts = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.ends = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.counts = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.halted = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.lane_pre = reinterpret_cast<uint32_t *>(w), w += per_lane;
  a.lnz = reinterpret_cast<uint32_t *>(w), w += per_lane;
  // windowed emit: checkpoints (main slots per lane, overflow per document tile), tile map
  a.kslots = ck_slots(lane_bytes);
  a.max_tiles = batch_max_tiles(ndocs, nbytes);
  a.ck_main = reinterpret_cast<uint2 *>(w), w += align256((size_t)a.kslots * a.max_lanes * 8);
  a.ck_over = reinterpret_cast<uint2 *>(w), w += align256((size_t)a.max_tiles * 64 * 8);
  a.tile_doc = reinterpret_cast<uint32_t *>(w), w += align256((size_t)a.max_tiles * 4);
  const uint32_t win_waves = batch_win_waves(bt.nrows, bt.ninst);
  a.win_ok = bt.nrows <= 256 && win_waves;  // checkpoints keep the row in 8 bits
  a.kinds = kinds;
  a.lens = lens;
  a.offs = offs;
  a.cap = cap;
  a.res = static_cast<DocResDev *>(res);
  a.total = total;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds_c = batch_lds_offset(bt.nrows, bt.ninst);
  // The count walk: workgroups of 16 waves, so that one copy of the combined table in LDS
  // serves the waves per SIMD the kernel's registers allow (workgroups of 4 waves, each with
  // its own copy, ran out of LDS at three per CU when the table is large).  The split
  // documents' walks, a few serial ones, spread over more CUs in workgroups of 4 waves.
  // Both grids are what the CUs hold at once: each wave's first tile is fixed, and a
  // workgroup that waited for a free CU would take its fixed tiles last.
  auto resident = [&](const void *k, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, lds_c) != hipSuccess || nb < 1) nb = 1;
    return (uint32_t)nb;
  };
  const uint32_t per_cu_c = resident(reinterpret_cast<const void *>(k_bcount), 1024);
  const uint32_t per_cu_c4 = resident(reinterpret_cast<const void *>(k_bsplit), 256);
  const uint32_t per_cu_e = (uint32_t)std::min<size_t>(8, 160 * 1024 / lds_e);
  const uint32_t gdoc = std::max<uint32_t>(1, std::min<uint32_t>(4096, (ndocs + 3) / 4));
  const uint32_t ngroups = doc_groups(ndocs);
  mark(ev, 0, s);
  k_bplan_a<<<ngroups, 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_bplan_b<<<ngroups, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_bmap<<<gdoc, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  mark(ev, 1, s);
  if (e == hipSuccess) {  // speculative walks, then the lanes of documents not split by them
    k_bcount<<<(uint32_t)cus * per_cu_c, 1024, lds_c, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {  // the hybrid plan's cuts
    k_bsync<<<(uint32_t)cus * 4, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {  // the lanes of the split documents
    k_bsplit<<<(uint32_t)cus * per_cu_c4, 256, lds_c, s>>>(a);
    e = hipGetLastError();
  }
  mark(ev, 2, s);
  if (e == hipSuccess) {
    k_bdoc<<<gdoc, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_bscan_a<<<ngroups, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_bscan_b<<<ngroups, 256, 0, s>>>(a);
    e = hipGetLastError();
  }
  mark(ev, 3, s);
  if (e == hipSuccess) {  // the lane emit: documents the windowed emit does not take
    k_bemit<<<(uint32_t)cus * per_cu_e, 256, lds_e, s>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess && win_waves) {  // the windowed emit: 16 waves per CU as LDS allows
    k_bemit_win<<<(uint32_t)cus * (16 / win_waves), win_waves * 64, batch_win_lds_bytes(bt.nrows, bt.ninst, win_waves),
                  s>>>(a);
    e = hipGetLastError();
  }
  mark(ev, 4, s);
  return e;
}

hipError_t run_fused(const DevTable &t, const CertMap &cm, const uint8_t *cert_lut, const uint8_t *in,
                     const Plan &p, bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                     ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  mark(ev, 0, s);
  const bool one = serial || p.nlanes == 1 || cm.nbytes == 0;
  if (one && p.nlanes != 1) return hipErrorInvalidValue;
  const WalkArgs a = walk_args(t, cm, in, p, kinds, lens, offs, cap, res, cert_lut);
  return count_scan_emit<true>(t, a, p, cap, res, s, ev);
}

hipError_t run_hybrid(const DevTable &t, const CertMap &cm, const uint8_t *in, const Plan &p, uint8_t *kinds,
                      uint32_t *lens, uint64_t *offs, uint64_t cap, ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  if (!p.hybrid || !p.spec_cut || p.nlanes < 2 || p.lane_bytes < kSpecX) return hipErrorInvalidValue;
  WalkArgs a = walk_args(t, cm, in, p, kinds, lens, offs, cap, res, nullptr);
  HybridArgs h{in, p.n, p.nlanes, p.lane_bytes, p.spec_cut, p.spec_rst, p.spec_bits, p.spec_fail, p.cuts};
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((p.nlanes + 255) / 256, (uint32_t)cus * 4));
  mark(ev, 0, s);
  k_hspec<<<g, 256, lds_bytes(t.nrows, 256, false), s>>>(a, h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_hsync<<<g, 256, 0, s>>>(h);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_hcuts<<<std::max<uint32_t>(1, std::min<uint32_t>((p.nlanes + 256) / 256, (uint32_t)cus * 4)), 256, 0, s>>>(h);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return count_scan_emit<false>(t, a, p, cap, res, s, ev);
}

hipError_t run_onepass(const DevTable &t, const CertMap &cm, const uint8_t *cert_lut, const uint8_t *in,
                       const Plan &p, bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                       ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  const bool one = serial || p.nlanes == 1 || cm.nbytes == 0;
  if (one && p.nlanes != 1) return hipErrorInvalidValue;
  if (p.block != kChunkLanes || !p.windowed || !t.monotone || !p.chunk_st) return hipErrorInvalidValue;
  const size_t lds = one_lds_bytes(t.nrows);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  WalkArgs a = walk_args(t, cm, in, p, kinds, lens, offs, cap, res, cert_lut);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t per_cu = std::max<uint32_t>(1, std::min<uint32_t>(8, (uint32_t)(160 * 1024 / lds)));
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(p.nblocks, (uint32_t)cus * per_cu));
  mark(ev, 0, s);
  k_onepass_reset<<<(p.nblocks + 255) / 256, 256, 0, s>>>(p.chunk_st, p.nblocks, p.chunk_ctr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 1, s);
  if (t.all_counted) k_onepass<false><<<grid, kChunkLanes, lds, s>>>(a);
  else k_onepass<true><<<grid, kChunkLanes, lds, s>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 2, s);
  k_scan<<<1, 1024, 0, s>>>(p.blk_sum, p.blk_fail, p.blk_nonempty, p.blk_big, p.blk_lnz, p.nblocks, p.block,
                            p.counts, p.meta, res, cap, p.n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 3, s);
  a.fallback_only = 1;  // halted scans, long slices, an unfinished look-back
  k_emit<true, true><<<p.nblocks, p.block, lds_bytes(t.nrows, (int)p.block, true), s>>>(a);
  e = hipGetLastError();
  mark(ev, 4, s);
  return e;
}

}  // namespace lexk
