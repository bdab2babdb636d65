// kernels.h -- launchers of the HIP kernels (gfx950).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lexk {

// Device-resident, read-only description of one compiled lexer in one mode.
struct DevTable {
  const uint32_t *table;   // nrows * 256 packed entries
  const uint8_t *rowinfo;  // nrows
  const uint8_t *rowkind;  // nrows
  int nrows;
  int row_sink;            // index
  int row_fail;            // index, -1 if the automaton is monotone
  int monotone;
  int all_counted;         // every token end of this mode is counted (no discarded kind)
};

// The useful certificate map of the scan's mode, in a form the bitmap kernel uses.
struct CertMap {
  uint32_t words[8];   // bit b: byte b is a useful certified byte
  int nbytes;          // popcount
  uint8_t bytes[8];    // the certified bytes themselves when nbytes <= 8
};

// Workspace carve-up for one scan (all device pointers).
struct Plan {
  uint32_t n;              // input bytes (< 2^32)
  uint32_t lane_bytes;     // lane target length (multiple of 16)
  uint32_t nlanes;         // M = ceil(n / lane_bytes), at least 1
  uint32_t nblocks;        // walk workgroups
  uint32_t block;          // threads per walk workgroup
  uint64_t *bitmap;        // ceil(n / 64) words            (pipeline path)
  uint64_t *tile_next;     // ntiles + 1 entries            (pipeline path)
  uint64_t *tile_group;    // one per 1024 tiles             (pipeline path)
  uint32_t ntiles;         // ceil(n / 4096)
  uint32_t *cuts;          // nlanes + 1 lane boundaries
  uint32_t *counts;        // nlanes tokens per lane (counted kinds)
  uint32_t *ends;          // nlanes slice ends (fused path; cuts holds the starts)
  uint64_t *blk_sum;       // nblocks
  uint32_t *blk_fail;      // nblocks: first halted lane of the block or ~0u
  uint32_t *blk_nonempty;  // nblocks
  uint32_t *blk_big;       // nblocks: a slice of 2^24 bytes or more (no checkpoints)
  uint32_t *meta;          // [0] = first halted lane or ~0u, [1] = checkpoints unusable
  uint32_t *lane_pre;      // nlanes: exclusive prefix of counts inside the workgroup
  // Windowed emit (monotone automata whose token ends are all counted): the count walk
  // records its state at every 64-byte-aligned address strictly inside a slice; the emit
  // walk then runs one thread per 64-byte window of the input.
  int windowed;
  uint2 *ck;               // checkpoints: kslots * nlanes, two-window blocks per lane (ck_index)
  uint2 *ck_over;          // window-indexed checkpoints beyond a lane's kslots
  uint32_t kslots;
  int32_t *lnz;            // nlanes: last non-empty lane at or before it in its workgroup, or -1
  int32_t *blk_lnz;        // nblocks: last non-empty lane of the earlier workgroups, or -1
  // One pass (windowed scans, 256-lane workgroups): per workgroup of lanes, the status word
  // of the decoupled look-back, and the counter that hands the workgroups out in order.
  uint64_t *chunk_st;      // nblocks
  uint32_t *chunk_ctr;
  // Hybrid plan (a refused set split speculatively; lane_bytes is the speculative lane):
  // per lane its cut, last restart and head/tail token starts, and the fall-back flag.
  int hybrid;
  uint32_t *spec_cut, *spec_rst, *spec_bits, *spec_fail;
};
constexpr uint32_t kHybridLane = 4096;  // speculative lane bytes (at least)

constexpr uint32_t kWin = 64;  // window of the windowed emit
// Windows of n bytes at any alignment of the input, plus one.
uint32_t windows_max(uint32_t n);
uint32_t ck_slots(uint32_t lane_bytes);

size_t workspace_bytes(uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline, int windowed, int hybrid);
// Dynamic LDS of a walk workgroup: the table, its row info and, for the emit walk, a
// 96-byte token ring per lane.
size_t walk_lds_bytes(int nrows, uint32_t block, bool emit);
// Dynamic LDS of a windowed-emit workgroup (the table and four wave stages).
size_t window_lds_bytes(int nrows);
// Dynamic LDS of a one-pass workgroup (256 lanes: the table, the lanes' slices and
// prefixes, and four wave stages).
size_t onepass_lds_bytes(int nrows);
constexpr uint32_t kChunkLanes = 256;  // lanes per one-pass workgroup
bool carve(void *ws, size_t ws_bytes, uint32_t n, uint32_t lane_bytes, uint32_t block, int pipeline,
           int windowed, int hybrid, Plan &p);

struct ResultDev {  // mirrors lex_result
  uint64_t ntokens;
  uint64_t error_offset;
  int32_t status;
  uint32_t nslices;
};

hipError_t launch_bitmap(const uint8_t *in, uint32_t n, const CertMap &cm, uint64_t *bits, hipStream_t s);

// Five-step pipeline: (a) bitmap, (b) plan, (c) count walk, (d) scan, (e) emit walk.
// When the plan has one lane (serial mode, empty useful map) steps (a) and the tile
// scan are skipped: the plan kernel then writes cuts = {0, n}.
// ev: optional 5 events recorded at the phase boundaries (start, planned, counted,
// scanned, emitted).
hipError_t run_pipeline(const DevTable &t, const CertMap &cm, const uint8_t *in, const Plan &p,
                        bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                        ResultDev *res, hipStream_t s, hipEvent_t const *ev);
// Fused: each lane places its own cut by a bounded search (no bitmap, no plan kernel).
// cert_lut: device 256-byte 0/1 table of the useful map (the lanes search with it).
hipError_t run_fused(const DevTable &t, const CertMap &cm, const uint8_t *cert_lut, const uint8_t *in,
                     const Plan &p, bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                     ResultDev *res, hipStream_t s, hipEvent_t const *ev);

// Hybrid plan for a refused set: speculative walks and their cuts, then the pipeline's count
// walk, scan and emit over those cuts.
hipError_t run_hybrid(const DevTable &t, const CertMap &cm, const uint8_t *in, const Plan &p, uint8_t *kinds,
                      uint32_t *lens, uint64_t *offs, uint64_t cap, ResultDev *res, hipStream_t s, hipEvent_t const *ev);
// One pass (windowed scans, block == kChunkLanes): plan, count walk, look-back and windowed
// emit in one launch, then the scan and the lane emit's fallback.
hipError_t run_onepass(const DevTable &t, const CertMap &cm, const uint8_t *cert_lut, const uint8_t *in,
                       const Plan &p, bool serial, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap,
                       ResultDev *res, hipStream_t s, hipEvent_t const *ev);

// Batched documents.  The instances' tables are rebased into one combined table (rows of
// instance k follow those of instances 0..k-1); start/sink/fail are row byte offsets in it.
constexpr int kBatchMaxInst = 8;
struct BatchInstHost {
  uint32_t start, sink, fail;
  uint32_t mono, refused;
  uint32_t disc;  // the mode discards some kind
  CertMap cm;
};
struct BatchTables {
  const uint32_t *table;   // device, nrows * 256
  const uint8_t *rowinfo;  // device, nrows
  const uint8_t *rowkind;  // device, nrows
  const uint8_t *luts;     // device, ninst * 256
  int nrows;
  uint32_t ninst;
  BatchInstHost inst[kBatchMaxInst];
};
// Workspace of a batch of ndocs documents over nbytes bytes with lane target lane_bytes.
size_t batch_workspace_bytes(uint32_t ndocs, uint64_t nbytes, uint32_t lane_bytes);
// LDS of the batched lane-emit workgroup (the count walk needs less): 0 if it does not fit.
// (The windowed emit takes as many waves as fit beside the table, or stands down.)
size_t batch_emit_lds_bytes(int nrows, uint32_t ninst);
// docs: device array of 16-byte lex_doc; res: device array of 32-byte lex_doc_result.
hipError_t run_batch(const BatchTables &bt, const uint8_t *bytes, uint64_t nbytes, const void *docs, uint32_t ndocs,
                     uint32_t lane_bytes, uint8_t *kinds, uint32_t *lens, uint64_t *offs, uint64_t cap, void *res,
                     ResultDev *total, void *ws, size_t ws_bytes, hipStream_t s, hipEvent_t const *ev);

}  // namespace lexk
