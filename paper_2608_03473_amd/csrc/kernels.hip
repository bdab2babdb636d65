// kernels.hip -- the certified-split scan on gfx950.
//
// Steps (one scan of one buffer):
//   (a) k_bitmap     coalesced 16-byte loads; each byte is tested against the useful
//                    certificate map of the mode (SWAR compares when the map holds at
//                    most 8 bytes, an LDS lookup otherwise); a wavefront ballot yields
//                    the first certified byte of every 4 KiB tile.
//   (b) k_tiles +    the equal-division planner of Section 6, one pass: every lane
//       k_plan       target j*lane_bytes slides forward to the next certified byte
//                    (bitmap words inside its tile, then a suffix minimum over tiles);
//                    duplicate slides give empty lanes, a target with nothing after it
//                    gives the end of the input.  An empty useful map gives one slice.
//   (c) k_walk<COUNT> every lane runs the longest-match loop of Section 3 on its slice
//                    [cut_j, cut_j+1) from the start row, treating the slice end as the end
//                    of the input; the packed transition table lives in LDS.
//   (d) k_scan       exclusive prefix of the per-lane counts; the first lane whose walk
//                    halted fixes the output length and, by Corollary 1, truncates it.
//   (e) k_walk<EMIT> every lane up to the first halted one walks again and writes its
//                    (kind, length[, offset]) triples at its prefix offset, skipping
//                    discarded kinds in modulo-I mode (the image pi_I of Section 5).
//
// Table entries (see compile.h): next row index * 256 in bits 0..19, kind in 20..27,
// ACC (28), EMIT (30), COUNT (31).  Row 0 is the token start, SINK absorbs after a halt,
// FAIL (non-monotone automata only) marks a dead end that must fall back to the last
// accepting position.
#include "kernels.h"

namespace lexk {
namespace {

constexpr uint32_t kNextMask = 0xFFFFFu;
constexpr uint32_t kAcc = 1u << 28;
constexpr uint32_t kEmit = 1u << 30;
constexpr uint8_t kInfoAcc = 0x80;
constexpr uint8_t kInfoCount = 0x40;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kTile = 4096;  // bytes per bitmap tile (64 words)

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

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
  // First certified byte of this wave's tile (tile index == global wave index).
  if (!tile_first) return;
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
// Suffix minimum over tiles: tile_next[t] = first certified byte at or after tile t
// (~0 if none); tile_next[ntiles] = ~0.  One workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_tiles(uint64_t *__restrict__ t, uint32_t ntiles) {
  __shared__ uint64_t part[1024];
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (ntiles + nt - 1) / nt;
  const uint32_t lo = min(ntiles, tid * per), hi = min(ntiles, lo + per);
  uint64_t m = ~0ull;
  for (uint32_t i = lo; i < hi; ++i) m = min(m, t[i]);
  part[tid] = m;
  __syncthreads();
  // inclusive suffix-min scan over part[] (Hillis-Steele)
  for (uint32_t d = 1; d < nt; d <<= 1) {
    uint64_t v = tid + d < nt ? part[tid + d] : ~0ull;
    __syncthreads();
    part[tid] = min(part[tid], v);
    __syncthreads();
  }
  uint64_t run = tid + 1 < nt ? part[tid + 1] : ~0ull;
  for (uint32_t i = hi; i > lo; --i) {
    run = min(run, t[i - 1]);
    t[i - 1] = run;
  }
  if (tid == 0) t[ntiles] = ~0ull;
}

// cuts[j] = first certified byte at or after j*lane_bytes (n if none), cuts[0] = 0,
// cuts[M] = n.  Non-decreasing; equal neighbours make empty lanes.
__global__ void __launch_bounds__(256) k_plan(const uint64_t *__restrict__ bits, const uint64_t *__restrict__ tile_next,
                                              uint32_t n, uint32_t lane_bytes, uint32_t nlanes,
                                              uint32_t *__restrict__ cuts) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nlanes) return;
  if (j == 0) {
    cuts[0] = 0;
    return;
  }
  if (j == nlanes) {
    cuts[nlanes] = n;
    return;
  }
  const uint64_t x = (uint64_t)j * lane_bytes;
  uint64_t cut = n;
  if (x < n) {
    const uint32_t nwords = (n + 63) / 64;
    uint32_t w = (uint32_t)(x >> 6);
    uint64_t m = bits[w] & (~0ull << (x & 63));
    const uint32_t tile_end = min(nwords, (w | 63u) + 1);
    while (!m && ++w < tile_end) m = bits[w];
    if (m) {
      cut = (uint64_t)w * 64 + (__ffsll((unsigned long long)m) - 1);
    } else {
      const uint64_t t = tile_next[(x >> 12) + 1];
      cut = t < n ? t : n;
    }
  }
  cuts[j] = (uint32_t)min<uint64_t>(cut, n);
}

// ----------------------------------------------------------- (c), (e) walk
struct Tables {
  const uint32_t *T;      // LDS
  const uint8_t *info;    // LDS
  const uint8_t *kind;    // LDS
  uint32_t sink, fail;    // row index * 256
};

struct Out {
  uint8_t *kinds;
  uint32_t *lens;
  uint64_t *offs;
  uint64_t o, lim;        // next slot, end of this lane's slots
  bool write;
};

struct LaneState {
  uint32_t st;    // current row * 256
  uint32_t tok;   // start of the current token
  uint32_t lacc;  // position after the last accepting step (non-monotone)
  uint32_t lrow;  // row * 256 of that accepting state
  uint64_t cnt;   // counted tokens
};

template <bool EMIT>
__device__ __forceinline__ void put(LaneState &L, Out &o, uint32_t kind, uint32_t end) {
  if (EMIT) {
    if (o.write && o.o < o.lim) {
      o.kinds[o.o] = (uint8_t)kind;
      o.lens[o.o] = end - L.tok;
      if (o.offs) o.offs[o.o] = L.tok;
    }
    ++o.o;
  }
  ++L.cnt;
}

// One transition on byte b at position p.
template <bool EMIT, bool MONO>
__device__ __forceinline__ void step(LaneState &L, Out &o, const Tables &tb, uint32_t b, uint32_t p) {
  const uint32_t e = tb.T[L.st + b];
  if (EMIT || !MONO) {
    if (e & kEmit) {
      if ((int32_t)e < 0) put<EMIT>(L, o, (e >> 20) & 0xFF, p);
      L.tok = p;
    }
  } else {
    L.cnt += e >> 31;
  }
  L.st = e & kNextMask;
  if (!MONO && (e & kAcc)) {
    L.lacc = p + 1;
    L.lrow = L.st;
  }
}

// Non-monotone automata: the walk reached FAIL (a dead end after a non-accepting
// state).  Longest match takes the last accepting position of the current token if
// there is one: emit it and re-scan from there, byte by byte, up to `upto`; with no
// accepting position since the token start the scan halts there (SINK).
template <bool EMIT>
__device__ void recover(LaneState &L, Out &o, const Tables &tb, const uint8_t *in, uint32_t upto) {
  // Only instantiated for non-monotone automata, whose FAIL row differs from SINK; the
  // guard keeps the loop finite even if a monotone table ever reached here.
  while (L.st == tb.fail && tb.fail != tb.sink) {
    if (L.lacc > L.tok) {
      const uint32_t r = L.lrow >> 8;
      if (tb.info[r] & kInfoCount) put<EMIT>(L, o, tb.kind[r], L.lacc);
      L.tok = L.lacc;
      L.st = 0;
      for (uint32_t p = L.tok; p < upto; ++p) {
        step<EMIT, false>(L, o, tb, in[p], p);
        if (L.st == tb.fail) break;
      }
    } else {
      L.st = tb.sink;
    }
  }
}

// End of the slice: an accepting state emits its token; a non-accepting one halts
// (monotone) or falls back (non-monotone).  Returns true if the slice halted.
template <bool EMIT, bool MONO>
__device__ bool finish(LaneState &L, Out &o, const Tables &tb, const uint8_t *in, uint32_t end) {
  for (;;) {
    if (!MONO && L.st == tb.fail) {
      recover<EMIT>(L, o, tb, in, end);
      continue;
    }
    if (L.st == 0) return false;
    if (L.st == tb.sink) return true;
    const uint32_t r = L.st >> 8;
    if (tb.info[r] & kInfoAcc) {
      if (tb.info[r] & kInfoCount) put<EMIT>(L, o, tb.kind[r], end);
      L.tok = end;
      L.st = 0;
      return false;
    }
    if (MONO) {
      L.st = tb.sink;
      return true;
    }
    L.st = tb.fail;  // end of input after a non-accepting state: fall back
  }
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

__device__ __forceinline__ uint32_t byte_of(const uint4 &v, int k) {
  const uint32_t w = k < 4 ? v.x : k < 8 ? v.y : k < 12 ? v.z : v.w;
  return (w >> (8 * (k & 3))) & 0xFFu;
}

// Walks the slice [s, e) of in[0, n); returns true if it halted (error inside).
template <bool EMIT, bool MONO>
__device__ bool walk(LaneState &L, Out &o, const Tables &tb, const uint8_t *in, uint32_t n, uint32_t s,
                     uint32_t e) {
  L.st = 0;
  L.tok = s;
  L.lacc = s;
  L.lrow = 0;
  if (s >= e) return false;
  // 16-byte blocks aligned on the absolute address; the first and last blocks of the
  // slice are processed with a per-byte mask.
  const int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(in + s) & 15);
  int64_t blk = (int64_t)s - mis;
  {
    const uint4 v = load_block(in, blk, n);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t p = blk + k;
      if (p >= (int64_t)s && p < (int64_t)e) step<EMIT, MONO>(L, o, tb, byte_of(v, k), (uint32_t)p);
    }
    blk += 16;
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, o, tb, in, (uint32_t)min<int64_t>(blk, e));
  }
  if (blk + 16 <= (int64_t)e) {
    uint4 v = *reinterpret_cast<const uint4 *>(in + blk);
    for (;;) {
      const int64_t nb = blk + 16;
      const bool more = nb + 16 <= (int64_t)e;
      uint4 nv = v;
      if (more) nv = *reinterpret_cast<const uint4 *>(in + nb);  // prefetch the next block
#pragma unroll
      for (int k = 0; k < 16; ++k) step<EMIT, MONO>(L, o, tb, byte_of(v, k), (uint32_t)(blk + k));
      if (!MONO && L.st == tb.fail) recover<EMIT>(L, o, tb, in, (uint32_t)nb);
      blk = nb;
      if (!more) break;
      v = nv;
    }
  }
  if (blk < (int64_t)e) {
    const uint4 v = load_block(in, blk, n);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t p = blk + k;
      if (p < (int64_t)e) step<EMIT, MONO>(L, o, tb, byte_of(v, k), (uint32_t)p);
    }
    if (!MONO && L.st == tb.fail) recover<EMIT>(L, o, tb, in, e);
  }
  return finish<EMIT, MONO>(L, o, tb, in, e);
}

struct WalkArgs {
  const uint32_t *table;  // global copies, staged into LDS
  const uint8_t *rowinfo;
  const uint8_t *rowkind;
  int nrows;
  uint32_t sink, fail;    // row * 256 (fail == sink for monotone automata)
  const uint8_t *in;
  uint32_t n;
  const uint32_t *cuts;   // pipeline path: lane boundaries
  uint32_t lane_bytes;    // fused path: targets
  uint32_t nlanes;
  const uint8_t *cert;    // fused path: global 256-byte LUT of the useful map
  uint64_t *counts;
  uint64_t *blk_sum;
  uint32_t *blk_fail;
  uint32_t *blk_nonempty;
  // emit
  const uint32_t *meta;
  ResultDev *res;
  uint8_t *kinds;
  uint32_t *lens;
  uint64_t *offs;
  uint64_t cap;
};

__device__ __forceinline__ void stage_tables(const WalkArgs &a, uint32_t *T, uint8_t *info, uint8_t *kind) {
  const int words = a.nrows * 256;
  const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
  uint4 *dst = reinterpret_cast<uint4 *>(T);
  for (int i = threadIdx.x; i < words / 4; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < a.nrows; i += blockDim.x) {
    info[i] = a.rowinfo[i];
    kind[i] = a.rowkind[i];
  }
  __syncthreads();
}

// Fused planning: the first certified byte in [x, x + span) (or `none`).
__device__ uint32_t search_cert(const uint8_t *in, uint32_t n, const uint8_t *lut, uint32_t x, uint32_t span,
                                uint32_t none) {
  const uint32_t end = (uint32_t)min<uint64_t>((uint64_t)x + span, n);
  int64_t blk = (int64_t)x - (int64_t)(reinterpret_cast<uintptr_t>(in + x) & 15);
  for (; blk < (int64_t)end; blk += 16) {
    const uint4 v = load_block(in, blk, n);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t p = blk + k;
      if (p >= (int64_t)x && p < (int64_t)end && lut[byte_of(v, k)]) return (uint32_t)p;
    }
  }
  return none;
}

// Lane j's slice.  Pipeline: [cuts[j], cuts[j+1]).  Fused: [c(j l), c((j+1) l)) with c(x)
// = first certified byte at or after x; the start search is bounded by one lane length
// (no certified byte there means the slice is empty, because then c(j l) = c((j+1) l)).
template <bool FUSED>
__device__ __forceinline__ void lane_slice(const WalkArgs &a, uint32_t j, const uint8_t *lut, uint32_t &s,
                                           uint32_t &e) {
  if (!FUSED) {
    s = a.cuts[j];
    e = a.cuts[j + 1];
    return;
  }
  const uint64_t x = (uint64_t)j * a.lane_bytes, x1 = x + a.lane_bytes;
  if (j == 0) s = 0;
  else if (x >= a.n) s = a.n;
  else s = search_cert(a.in, a.n, lut, (uint32_t)x, a.lane_bytes, a.n);
  if (s >= x1 || s >= a.n) {  // no certified byte in [x, x1): empty slice
    e = s = (uint32_t)min<uint64_t>(s, a.n);
    return;
  }
  e = (j + 1 == a.nlanes || x1 >= a.n) ? a.n : search_cert(a.in, a.n, lut, (uint32_t)x1, a.n - (uint32_t)x1, a.n);
}

template <bool MONO, bool FUSED>
__global__ void __launch_bounds__(256) k_count(WalkArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t *T = reinterpret_cast<uint32_t *>(smem);
  uint8_t *info = smem + (size_t)a.nrows * 1024;
  uint8_t *kind = info + a.nrows;
  uint8_t *lut = kind + a.nrows;
  __shared__ uint64_t wsum[16];
  __shared__ uint32_t wfail[16], wne[16];
  if (FUSED)
    for (int i = threadIdx.x; i < 256; i += blockDim.x) lut[i] = a.cert[i];
  stage_tables(a, T, info, kind);
  const Tables tb{T, info, kind, a.sink, a.fail};
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t cnt = 0;
  uint32_t fail = kNone, nonempty = 0;
  if (j < a.nlanes) {
    uint32_t s, e;
    lane_slice<FUSED>(a, j, lut, s, e);
    LaneState L;
    L.cnt = 0;
    Out o{nullptr, nullptr, nullptr, 0, 0, false};
    const bool halted = walk<false, MONO>(L, o, tb, a.in, a.n, s, e);
    cnt = L.cnt;
    a.counts[j] = cnt;
    if (halted) fail = j;
    nonempty = s < e;
  }
  // block reductions: sum, min failing lane, non-empty count
  for (int d = 32; d; d >>= 1) {
    cnt += __shfl_xor(cnt, d);
    fail = min(fail, (uint32_t)__shfl_xor((int)fail, d));
    nonempty += __shfl_xor(nonempty, d);
  }
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wsum[wid] = cnt;
    wfail[wid] = fail;
    wne[wid] = nonempty;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    uint32_t f = kNone, ne = 0;
    for (int w = 0; w < nw; ++w) {
      s += wsum[w];
      f = min(f, wfail[w]);
      ne += wne[w];
    }
    a.blk_sum[blockIdx.x] = s;
    a.blk_fail[blockIdx.x] = f;
    a.blk_nonempty[blockIdx.x] = ne;
  }
}

// (d) One workgroup: exclusive scan of block sums (in place), first halted lane,
// output length, status.
__global__ void __launch_bounds__(1024) k_scan(uint64_t *__restrict__ blk_sum, const uint32_t *__restrict__ blk_fail,
                                               const uint32_t *__restrict__ blk_nonempty, uint32_t nblocks,
                                               uint32_t block, const uint64_t *__restrict__ counts,
                                               uint32_t *__restrict__ meta, ResultDev *__restrict__ res, uint64_t cap,
                                               uint32_t n) {
  __shared__ uint64_t part[1024];
  __shared__ uint32_t pf[1024], pn[1024];
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (nblocks + nt - 1) / nt;
  const uint32_t lo = min(nblocks, tid * per), hi = min(nblocks, lo + per);
  uint64_t s = 0;
  uint32_t f = kNone, ne = 0;
  for (uint32_t i = lo; i < hi; ++i) {
    s += blk_sum[i];
    f = min(f, blk_fail[i]);
    ne += blk_nonempty[i];
  }
  part[tid] = s;
  pf[tid] = f;
  pn[tid] = ne;
  __syncthreads();
  for (uint32_t d = 1; d < nt; d <<= 1) {  // inclusive prefix sums, min, sum
    uint64_t v = tid >= d ? part[tid - d] : 0;
    uint32_t vf = tid >= d ? pf[tid - d] : kNone;
    uint32_t vn = tid >= d ? pn[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    pf[tid] = min(pf[tid], vf);
    pn[tid] += vn;
    __syncthreads();
  }
  uint64_t run = tid ? part[tid - 1] : 0;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint64_t x = blk_sum[i];
    blk_sum[i] = run;
    run += x;
  }
  __syncthreads();
  if (tid == 0) {
    const uint64_t total = part[nt - 1];
    const uint32_t first = pf[nt - 1];
    uint64_t ntok = total;
    if (first != kNone) {
      // tokens before the halted lane plus those it emitted before halting
      const uint32_t b = first / block;
      uint64_t pre = 0;
      for (uint32_t l = b * block; l < first; ++l) pre += counts[l];
      ntok = blk_sum[b] + pre + counts[first];
    }
    meta[0] = first;
    res->ntokens = ntok;
    res->error_offset = n;  // replaced by the halted lane in the emit pass
    res->status = ntok > cap ? -4 : 0;
    res->nslices = pn[nt - 1];
  }
}

template <bool MONO, bool FUSED>
__global__ void __launch_bounds__(256) k_emit(WalkArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t *T = reinterpret_cast<uint32_t *>(smem);
  uint8_t *info = smem + (size_t)a.nrows * 1024;
  uint8_t *kind = info + a.nrows;
  uint8_t *lut = kind + a.nrows;
  __shared__ uint64_t wpre[16];
  const uint32_t first = a.meta[0];
  const uint32_t j0 = blockIdx.x * blockDim.x;
  if (j0 > first) return;  // the whole block lies after the first halted lane
  if (FUSED)
    for (int i = threadIdx.x; i < 256; i += blockDim.x) lut[i] = a.cert[i];
  stage_tables(a, T, info, kind);
  const Tables tb{T, info, kind, a.sink, a.fail};
  const uint32_t j = j0 + threadIdx.x;
  // exclusive prefix of this block's lane counts
  uint64_t c = j < a.nlanes ? a.counts[j] : 0;
  uint64_t incl = c;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t v = __shfl_up(incl, d);
    if (lane >= d) incl += v;
  }
  if (lane == 63) wpre[wid] = incl;
  __syncthreads();
  uint64_t base = a.blk_sum[blockIdx.x];
  for (int w = 0; w < wid; ++w) base += wpre[w];
  const uint64_t off = base + incl - c;
  if (j >= a.nlanes || j > first) return;
  uint32_t s, e;
  lane_slice<FUSED>(a, j, lut, s, e);
  const bool write = a.res->status == 0;
  Out o{a.kinds, a.lens, a.offs, off, off + c, write};
  LaneState L;
  L.cnt = 0;
  walk<true, MONO>(L, o, tb, a.in, a.n, s, e);
  if (j == first) a.res->error_offset = L.tok;  // the halt offset: start of the failed token
  (void)nw;
}

}  // namespace

// ------------------------------------------------------------------ host side
static size_t carve_layout(uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, size_t *offs) {
  const uint32_t nlanes = n ? (n + lane_bytes - 1) / lane_bytes : 1;
  const uint32_t nblocks = (nlanes + block - 1) / block;
  const uint32_t nwords = (n + 63) / 64;
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  size_t at = 0;
  offs[0] = at;
  at += align256(pipeline ? (size_t)(nwords ? nwords : 1) * 8 : 0);
  offs[1] = at;
  at += align256(pipeline ? (size_t)(ntiles + 1) * 8 : 0);
  offs[2] = at;
  at += align256((size_t)(nlanes + 1) * 4);
  offs[3] = at;
  at += align256((size_t)nlanes * 8);
  offs[4] = at;
  at += align256((size_t)nblocks * 8);
  offs[5] = at;
  at += align256((size_t)nblocks * 4);
  offs[6] = at;
  at += align256((size_t)nblocks * 4);
  offs[7] = at;
  at += align256(16);
  return at;
}

size_t workspace_bytes(uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline) {
  size_t offs[8];
  return carve_layout(n, lane_bytes, block, pipeline, offs);
}

bool carve(void *ws, size_t ws_bytes, uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, Plan &p) {
  size_t offs[8];
  const size_t need = carve_layout(n, lane_bytes, block, pipeline, offs);
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
  p.cuts = reinterpret_cast<uint32_t *>(b + offs[2]);
  p.counts = reinterpret_cast<uint64_t *>(b + offs[3]);
  p.blk_sum = reinterpret_cast<uint64_t *>(b + offs[4]);
  p.blk_fail = reinterpret_cast<uint32_t *>(b + offs[5]);
  p.blk_nonempty = reinterpret_cast<uint32_t *>(b + offs[6]);
  p.meta = reinterpret_cast<uint32_t *>(b + offs[7]);
  return true;
}

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

static WalkArgs walk_args(const DevTable &t, const uint8_t *in, const Plan &p, uint8_t *kinds, uint32_t *lens,
                          uint64_t *offs, uint64_t cap, ResultDev *res, const uint8_t *cert_lut) {
  WalkArgs a{};
  a.table = t.table;
  a.rowinfo = t.rowinfo;
  a.rowkind = t.rowkind;
  a.nrows = t.nrows;
  a.sink = (uint32_t)t.row_sink * 256u;
  a.fail = t.row_fail >= 0 ? (uint32_t)t.row_fail * 256u : a.sink;
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

template <bool FUSED>
static hipError_t count_scan_emit(const DevTable &t, const WalkArgs &a, const Plan &p, uint64_t cap,
                                  ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  const size_t smem = (size_t)t.nrows * 1024 + 2 * (size_t)t.nrows + 256;
  mark(ev, 1, s);
  if (t.monotone) {
    k_count<true, FUSED><<<p.nblocks, p.block, smem, s>>>(a);
  } else {
    k_count<false, FUSED><<<p.nblocks, p.block, smem, s>>>(a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 2, s);
  k_scan<<<1, 1024, 0, s>>>(p.blk_sum, p.blk_fail, p.blk_nonempty, p.nblocks, p.block, p.counts, p.meta, res, cap,
                            p.n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark(ev, 3, s);
  if (t.monotone) {
    k_emit<true, FUSED><<<p.nblocks, p.block, smem, s>>>(a);
  } else {
    k_emit<false, FUSED><<<p.nblocks, p.block, smem, s>>>(a);
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
    k_bitmap<<<(nwords + 255) / 256, 256, 0, s>>>(in, p.n, cert_arg(cm), p.bitmap, p.tile_next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tiles<<<1, 1024, 0, s>>>(p.tile_next, p.ntiles);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  k_plan<<<(p.nlanes + 1 + 255) / 256, 256, 0, s>>>(p.bitmap, p.tile_next, p.n, p.lane_bytes, p.nlanes, p.cuts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const WalkArgs a = walk_args(t, in, p, kinds, lens, offs, cap, res, nullptr);
  return count_scan_emit<false>(t, a, p, cap, res, s, ev);
}

hipError_t run_fused(const DevTable &t, const CertMap &cm, const uint8_t *cert_lut, const uint8_t *in,
                     const Plan &p, bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                     ResultDev *res, hipStream_t s, hipEvent_t const *ev) {
  mark(ev, 0, s);
  const bool one = serial || p.nlanes == 1 || cm.nbytes == 0;
  if (one && p.nlanes != 1) return hipErrorInvalidValue;
  const WalkArgs a = walk_args(t, in, p, kinds, lens, offs, cap, res, cert_lut);
  return count_scan_emit<true>(t, a, p, cap, res, s, ev);
}

}  // namespace lexk
