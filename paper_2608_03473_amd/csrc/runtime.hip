// runtime.hip -- C ABI of the certified-split lexer (declared in include/lex.h).
//
// Host responsibilities: compile the token set (compile.cc), upload the packed tables
// once per lexer, validate arguments, size and carve the caller's workspace, and enqueue
// the kernels of kernels.hip on the caller's stream.  Nothing here touches the input
// bytes: every step of a scan runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lex.h"
#include "compile.h"
#include "kernels.h"

// Device copy of a lexer's tables on one HIP device.
struct DevCopy {
  int device = -1;
  uint32_t *d_table[2] = {nullptr, nullptr};
  uint8_t *d_rowinfo[2] = {nullptr, nullptr};
  uint8_t *d_rowkind = nullptr;
  uint8_t *d_cert_lut[2] = {nullptr, nullptr};  // 256-byte 0/1 useful maps
};

struct lex_batch {
  int device = -1;
  lexk::BatchTables bt{};
};

struct lex_dfa {
  lexc::Compiled c;
  lexk::CertMap cm[2];
  bool all_counted[2];  // every token end of the mode is counted (no discarded kind)
  std::vector<uint8_t> lut[2];
  // Tables are uploaded once per device: eagerly by lex_compile when a device is
  // present, otherwise by the first scan on that device.
  std::mutex mu;
  std::vector<DevCopy *> copies;
};

namespace {

void set_err(char *err, size_t errlen, const std::string &m) {
  if (err && errlen) snprintf(err, errlen, "%s", m.c_str());
}

bool bit(const uint8_t *m, int b) { return (m[b >> 3] >> (b & 7)) & 1; }

template <class T>
hipError_t upload(T **dst, const T *src, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
}

void free_copy(DevCopy *c) {
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (c->device >= 0) (void)hipSetDevice(c->device);
  for (int m = 0; m < 2; ++m) {
    if (c->d_table[m]) (void)hipFree(c->d_table[m]);
    if (c->d_rowinfo[m]) (void)hipFree(c->d_rowinfo[m]);
    if (c->d_cert_lut[m]) (void)hipFree(c->d_cert_lut[m]);
  }
  if (c->d_rowkind) (void)hipFree(c->d_rowkind);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete c;
}

void release(lex_dfa *d) {
  if (!d) return;
  for (DevCopy *c : d->copies) free_copy(c);
  delete d;
}

// Device copy of d's tables on device dev if one was uploaded, else nullptr (no upload).
DevCopy *find_copy(const lex_dfa *d, int dev) {
  std::lock_guard<std::mutex> g(const_cast<lex_dfa *>(d)->mu);
  for (DevCopy *c : d->copies)
    if (c->device == dev) return c;
  return nullptr;
}

// Device copy of d's tables on the current device, uploading them on first use.
DevCopy *device_copy(lex_dfa *d) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(d->mu);
  for (DevCopy *c : d->copies)
    if (c->device == dev) return c;
  DevCopy *c = new DevCopy;
  c->device = dev;
  const lexc::Compiled &k = d->c;
  hipError_t e = hipSuccess;
  for (int m = 0; m < 2 && e == hipSuccess; ++m) {
    e = upload(&c->d_table[m], k.table[m].data(), k.table[m].size());
    if (e == hipSuccess) e = upload(&c->d_rowinfo[m], k.rowinfo[m].data(), k.rowinfo[m].size());
    if (e == hipSuccess) e = upload(&c->d_cert_lut[m], d->lut[m].data(), d->lut[m].size());
  }
  if (e == hipSuccess) e = upload(&c->d_rowkind, k.rowkind.data(), k.rowkind.size());
  if (e != hipSuccess) {
    free_copy(c);
    return nullptr;
  }
  d->copies.push_back(c);
  return c;
}

uint32_t default_block(int nrows);

int finish_compile(lex_dfa *d, lex_dfa **out, char *err, size_t errlen) {
  const lexc::Compiled &c = d->c;
  if (default_block(c.nrows) == 0) {
    set_err(err, errlen, "automaton too large for the LDS-resident table (" + std::to_string(c.nrows) + " rows)");
    release(d);
    return LEX_ELIMIT;
  }
  for (int m = 0; m < 2; ++m) {
    d->all_counted[m] = true;
    for (uint32_t e : c.table[m])
      if ((e & lexc::kEmit) && !(e & lexc::kCount)) d->all_counted[m] = false;
  }
  for (int m = 0; m < 2; ++m) {
    const uint8_t *map = m == 0 ? c.exact_useful : c.discard_useful;
    lexk::CertMap &cm = d->cm[m];
    memset(&cm, 0, sizeof cm);
    d->lut[m].assign(256, 0);
    for (int b = 0; b < 256; ++b) {
      d->lut[m][b] = bit(map, b);
      if (d->lut[m][b]) {
        cm.words[b >> 5] |= 1u << (b & 31);
        if (cm.nbytes < 8) cm.bytes[cm.nbytes] = (uint8_t)b;
        ++cm.nbytes;
      }
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && !device_copy(d)) {
    set_err(err, errlen, "device upload failed");
    release(d);
    return LEX_EDEVICE;
  }
  (void)hipGetLastError();  // a CPU-only host leaves a no-device error behind
  *out = d;
  return LEX_OK;
}

struct Resolved {
  uint32_t lane_bytes;
  uint32_t block;
  int path;  // 1 pipeline, 2 fused (one pass or separate launches)
  bool serial;
  int table;  // 0 exact, 1 discard
  bool windowed;
  bool onepass;  // fused, in one pass
  bool hybrid;   // a refused set split speculatively (pipeline's count, scan and emit)
};

uint32_t default_lane_bytes(uint64_t n, bool onepass) {
  // Aim for about 512k lanes (2048 resident lanes on each of 256 CUs), or in one pass
  // about 256k (one 256-lane group for each of the ~1024 resident one-pass workgroups),
  // between 64 B and 4 KiB.
  const uint64_t want = onepass ? 256u << 10 : 512u << 10;
  uint64_t l = 64;
  while (l < 4096 && n / l > want) l <<= 1;
  return (uint32_t)l;
}

// Largest workgroup (1024, 512 or 256 lanes) whose emit-walk LDS fits the CU's 160 KiB.
uint32_t default_block(int nrows) {
  for (uint32_t b = 1024; b >= 256; b >>= 1)
    if (lexk::walk_lds_bytes(nrows, b, true) <= 160 * 1024) return b;
  return 0;
}

int resolve(const lex_dfa *d, uint64_t n, int mode, const lex_run_opts *o, Resolved &r) {
  if (mode < 0 || mode > 3) return LEX_EINVAL;
  r.table = mode & 1;
  // A refused set (no useful certified byte) is split by the hybrid plan when the buffer is
  // longer than one speculative lane and the mode does not ask for a serial scan.
  const bool refused = d->cm[r.table].nbytes == 0;
  const uint32_t spec = std::max<uint32_t>(lexk::kHybridLane, o && o->lane_bytes ? o->lane_bytes : 0);
  r.hybrid = refused && !(mode & 2) && n > spec;
  r.serial = (mode & 2) != 0 || (refused && !r.hybrid);
  const int asked = o && o->path ? o->path : 0;
  if (asked < 0 || asked > 3) return LEX_EINVAL;
  const int32_t bt = o ? o->block_threads : 0;
  if (asked == 3 && bt && bt != (int32_t)lexk::kChunkLanes) return LEX_EINVAL;
  const int emit = o ? o->emit : LEX_EMIT_DEFAULT;
  if (emit != LEX_EMIT_DEFAULT && emit != LEX_EMIT_LANE) return LEX_EINVAL;
  // The windowed emit: a non-monotone automaton needs a scan without fallbacks, which the
  // count walk reports (the lane emit then runs instead).  In a mode with discarded kinds
  // its staged words carry lengths, not ends.
  r.windowed = emit == LEX_EMIT_DEFAULT && d->c.nrows <= 256 && lexk::window_lds_bytes(d->c.nrows) <= 160 * 1024;
  // By default (and as path 3) a monotone windowed scan runs in one pass when its workgroup
  // fits; every other scan takes the fused path unless the pipeline is asked for.
  r.onepass = (asked == 0 || asked == 3) && r.windowed && d->c.monotone && (!bt || bt == (int32_t)lexk::kChunkLanes) &&
              lexk::onepass_lds_bytes(d->c.nrows) <= 160 * 1024;
  r.path = asked == 1 ? 1 : 2;
  r.block = r.onepass ? lexk::kChunkLanes : bt ? (uint32_t)bt : default_block(d->c.nrows);
  if (r.hybrid) {  // speculative lanes and cuts, then the pipeline's count, scan and emit
    r.onepass = false;
    r.path = 1;
    if (r.block != 256u && r.block != 512u && r.block != 1024u) return LEX_EINVAL;
    if (lexk::walk_lds_bytes(d->c.nrows, r.block, true) > 160 * 1024) return LEX_ELIMIT;
    if (o && o->lane_bytes && (o->lane_bytes < 16 || (o->lane_bytes & 15))) return LEX_EINVAL;
    r.lane_bytes = spec;
    return LEX_OK;
  }
  if (r.block != 256u && r.block != 512u && r.block != 1024u) return LEX_EINVAL;
  if (lexk::walk_lds_bytes(d->c.nrows, r.block, true) > 160 * 1024) return LEX_ELIMIT;
  uint32_t lb = o && o->lane_bytes ? o->lane_bytes : default_lane_bytes(n, r.onepass);
  if (lb < 16 || (lb & 15)) return LEX_EINVAL;
  if (o && o->chunk_bytes) {
    if (o->chunk_bytes % lb) return LEX_EINVAL;  // lanes subdivide the paper's chunks
  }
  if (r.serial || n <= lb) lb = (uint32_t)std::max<uint64_t>(16, (n + 15) & ~15ull);  // one lane
  if (r.serial && n > 0xFFFFFFF0ull) return LEX_ELIMIT;
  r.lane_bytes = lb;
  return LEX_OK;
}

// Definitions of the C-ABI into the compiler's form; exclude is the reserved byte or -1.
int compile_into(const lex_tokdef *defs, uint32_t ndefs, int exclude, const lexc::TokDef *extra,
                 lex_dfa **out, char *err, size_t errlen) {
  std::vector<lexc::TokDef> v(ndefs);
  for (uint32_t i = 0; i < ndefs; ++i) {
    if (!defs[i].pattern) {
      set_err(err, errlen, "null pattern");
      return LEX_EINVAL;
    }
    v[i].pattern = defs[i].pattern;
    v[i].priority = defs[i].priority;
    v[i].discard = defs[i].discard != 0;
    v[i].exclude = exclude;
  }
  if (extra) v.push_back(*extra);
  lex_dfa *d = new lex_dfa;
  std::string msg;
  if (!lexc::compile_defs(v, d->c, msg)) {
    set_err(err, errlen, msg);
    delete d;
    return msg.find("exceeds") != std::string::npos || msg.find("too") != std::string::npos ? LEX_ELIMIT
                                                                                            : LEX_ESYNTAX;
  }
  return finish_compile(d, out, err, errlen);
}

}  // namespace

extern "C" {

int lex_compile(const lex_tokdef *defs, uint32_t ndefs, lex_dfa **out, char *err, size_t errlen) {
  if (!defs || !out || ndefs == 0) {
    set_err(err, errlen, "null argument or no definitions");
    return LEX_EINVAL;
  }
  *out = nullptr;
  if (ndefs > 255) {
    set_err(err, errlen, "at most 255 token definitions");
    return LEX_ELIMIT;
  }
  return compile_into(defs, ndefs, -1, nullptr, out, err, errlen);
}

int lex_compile_framed(const lex_tokdef *defs, uint32_t ndefs, uint32_t reserved, int reserved_discard,
                       lex_dfa **out, char *err, size_t errlen) {
  if (!defs || !out || ndefs == 0 || reserved > 255) {
    set_err(err, errlen, "null argument, no definitions or a reserved byte above 255");
    return LEX_EINVAL;
  }
  *out = nullptr;
  if (ndefs > 254) {
    set_err(err, errlen, "at most 254 token definitions besides the reserved byte's");
    return LEX_ELIMIT;
  }
  char pat[8];
  snprintf(pat, sizeof pat, "\\x%02X", reserved);
  lexc::TokDef rs;
  rs.pattern = pat;
  rs.discard = reserved_discard != 0;
  return compile_into(defs, ndefs, (int)reserved, &rs, out, err, errlen);
}

int lex_compile_table(int32_t nstates, int32_t q0, const int32_t *next, const int32_t *accept,
                      const uint8_t *discard, int32_t ntok, lex_dfa **out, char *err, size_t errlen) {
  if (!next || !accept || !out || ntok < 0 || ntok > 255) {
    set_err(err, errlen, "bad argument");
    return LEX_EINVAL;
  }
  *out = nullptr;
  std::vector<uint8_t> disc((size_t)ntok, 0);
  for (int t = 0; t < ntok; ++t) disc[t] = discard && discard[t] ? 1 : 0;
  lex_dfa *d = new lex_dfa;
  std::string msg;
  if (!lexc::compile_table(nstates, q0, next, accept, disc, d->c, msg)) {
    set_err(err, errlen, msg);
    delete d;
    return LEX_EINVAL;
  }
  return finish_compile(d, out, err, errlen);
}

void lex_free(lex_dfa *dfa) { release(dfa); }

int lex_cert(const lex_dfa *d, int mode, int raw, uint8_t bits[32]) {
  if (!d || !bits || mode < 0 || mode > 3) return LEX_EINVAL;
  if (mode & 2) {
    memset(bits, 0, 32);
    return LEX_OK;
  }
  const lexc::Compiled &c = d->c;
  const uint8_t *src = (mode & 1) ? (raw ? c.discard_raw : c.discard_useful) : (raw ? c.exact_raw : c.exact_useful);
  memcpy(bits, src, 32);
  return LEX_OK;
}

int lex_info(const lex_dfa *d, lex_info_t *o) {
  if (!d || !o) return LEX_EINVAL;
  const lexc::Compiled &c = d->c;
  o->nkinds = c.nkinds;
  o->nstates = c.q0_live ? c.dfa.nstates : 0;
  o->nclasses = c.dfa.nclasses;
  o->nrows = c.nrows;
  o->reentrant = c.reentrant;
  o->monotone = c.monotone;
  o->q0_live = c.q0_live;
  o->reserved = 0;
  return LEX_OK;
}

int lex_tables(const lex_dfa *d, int mode, uint32_t *table, size_t table_entries, uint8_t *rowinfo,
               uint8_t *rowkind, size_t nrows) {
  if (!d || mode < 0 || mode > 1) return LEX_EINVAL;
  const lexc::Compiled &c = d->c;
  if (table_entries < c.table[mode].size() || nrows < (size_t)c.nrows) return LEX_ELIMIT;
  if (table) memcpy(table, c.table[mode].data(), c.table[mode].size() * 4);
  if (rowinfo) memcpy(rowinfo, c.rowinfo[mode].data(), c.nrows);
  if (rowkind) memcpy(rowkind, c.rowkind.data(), c.nrows);
  return LEX_OK;
}

size_t lex_workspace_size(const lex_dfa *d, uint64_t n, int mode, const lex_run_opts *opts) {
  Resolved r;
  if (!d || n > 0xFFFFFFF0ull || resolve(d, n, mode, opts, r) != LEX_OK) return 0;
  return lexk::workspace_bytes((uint32_t)n, r.lane_bytes, r.block, r.path == 1 && !r.hybrid, r.windowed, r.hybrid);
}

int lex_plan(const lex_dfa *d, uint64_t n, int mode, const lex_run_opts *opts, lex_plan_info *out) {
  if (!d || !out) return LEX_EINVAL;
  if (n > 0xFFFFFFF0ull) return LEX_ELIMIT;
  Resolved r;
  const int rc = resolve(d, n, mode, opts, r);
  if (rc != LEX_OK) return rc;
  out->lane_bytes = r.lane_bytes;
  out->block_threads = r.block;
  out->path = r.onepass ? 3 : r.path;
  out->windowed = r.windowed ? 1 : 0;
  out->hybrid = r.hybrid ? 1 : 0;
  return LEX_OK;
}

}  // extern "C"

namespace {

// Argument checks of a scan (host only).
int check_scan_args(const lex_dfa *d, const uint8_t *d_bytes, uint64_t n, uint8_t *d_kinds, uint32_t *d_lens,
                    uint64_t cap, lex_result *d_result) {
  if (!d || !d_result || (!d_bytes && n)) return LEX_EINVAL;
  if (cap && (!d_kinds || !d_lens)) return LEX_EINVAL;
  // outputs leave the kernels in 16-byte chunks
  if ((reinterpret_cast<uintptr_t>(d_kinds) | reinterpret_cast<uintptr_t>(d_lens)) & 15) return LEX_EINVAL;
  if (n > 0xFFFFFFF0ull) return LEX_ELIMIT;
  return LEX_OK;
}

// Carves the workspace and enqueues one scan on the device copy dc of d's tables.
int enqueue_scan(const lex_dfa *d, DevCopy *dc, const Resolved &r, const uint8_t *d_bytes, uint64_t n,
                 uint8_t *d_kinds, uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap, lex_result *d_result,
                 void *d_ws, size_t ws_bytes, const lex_run_opts *opts, void *stream) {
  lexk::Plan p;
  if (!lexk::carve(d_ws, ws_bytes, (uint32_t)n, r.lane_bytes, r.block, r.path == 1 && !r.hybrid, r.windowed, r.hybrid,
                   p))
    return LEX_ELIMIT;
  const int m = r.table;
  lexk::DevTable t{dc->d_table[m], dc->d_rowinfo[m], dc->d_rowkind, d->c.nrows, d->c.row_sink, d->c.row_fail,
                   d->c.monotone ? 1 : 0, d->all_counted[m] ? 1 : 0};
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto *res = reinterpret_cast<lexk::ResultDev *>(d_result);
  hipEvent_t const *ev = opts && opts->events ? reinterpret_cast<hipEvent_t const *>(opts->events) : nullptr;
  hipError_t e = r.hybrid      ? lexk::run_hybrid(t, d->cm[m], d_bytes, p, d_kinds, d_lens, d_offsets, cap, res, s, ev)
                 : r.path == 1 ? lexk::run_pipeline(t, d->cm[m], d_bytes, p, r.serial, d_kinds, d_lens, d_offsets,
                                                    cap, res, s, ev)
                 : r.onepass ? lexk::run_onepass(t, d->cm[m], dc->d_cert_lut[m], d_bytes, p, r.serial, d_kinds,
                                                 d_lens, d_offsets, cap, res, s, ev)
                             : lexk::run_fused(t, d->cm[m], dc->d_cert_lut[m], d_bytes, p, r.serial, d_kinds,
                                               d_lens, d_offsets, cap, res, s, ev);
  return e == hipSuccess ? LEX_OK : LEX_EDEVICE;
}

}  // namespace

// The host tables of a compiled lexer, for the host-side chunked baseline (cpu_chunked.cc).
const lexc::Compiled &lex_compiled(const lex_dfa *d) { return d->c; }

// Workspace of lex_run_static: one copy of this array on every device the library runs on
// (the device globals of a code object are instantiated per device), held until the
// process ends.  Host code never uses the name itself as an address: it is a host-side
// stand-in, so each device's address is looked up once with that device current and kept.
static __device__ __align__(256) uint8_t scratch[LEX_STATIC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};  // scratch's address on each device, once looked up

void *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

int lex_run(const lex_dfa *d, const uint8_t *d_bytes, uint64_t n, int mode, uint8_t *d_kinds, uint32_t *d_lens,
            uint64_t *d_offsets, uint64_t cap, lex_result *d_result, void *d_ws, size_t ws_bytes,
            const lex_run_opts *opts, void *stream) {
  int rc = check_scan_args(d, d_bytes, n, d_kinds, d_lens, cap, d_result);
  if (rc != LEX_OK) return rc;
  if (!d_ws) return LEX_EINVAL;
  Resolved r;
  rc = resolve(d, n, mode, opts, r);
  if (rc != LEX_OK) return rc;
  DevCopy *dc = device_copy(const_cast<lex_dfa *>(d));
  if (!dc) return LEX_EDEVICE;
  return enqueue_scan(d, dc, r, d_bytes, n, d_kinds, d_lens, d_offsets, cap, d_result, d_ws, ws_bytes, opts, stream);
}

int lex_run_static(const lex_dfa *d, const uint8_t *d_bytes, uint64_t n, int mode, uint8_t *d_kinds,
                   uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap, lex_result *d_result,
                   const lex_run_opts *opts, void *stream) {
  int rc = check_scan_args(d, d_bytes, n, d_kinds, d_lens, cap, d_result);
  if (rc != LEX_OK) return rc;
  Resolved r;
  rc = resolve(d, n, mode, opts, r);
  if (rc != LEX_OK) return rc;
  const size_t need =
      lexk::workspace_bytes((uint32_t)n, r.lane_bytes, r.block, r.path == 1 && !r.hybrid, r.windowed, r.hybrid);
  if (need > (size_t)LEX_STATIC_WS_BYTES) return LEX_ELIMIT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LEX_EDEVICE;
  DevCopy *dc = find_copy(d, dev);  // never uploads: that would allocate
  if (!dc) return LEX_EDEVICE;
  void *ws = scratch_on(dev);
  if (!ws) return LEX_EDEVICE;
  return enqueue_scan(d, dc, r, d_bytes, n, d_kinds, d_lens, d_offsets, cap, d_result, ws, (size_t)LEX_STATIC_WS_BYTES,
                      opts, stream);
}

int lex_batch_create(const lex_dfa *const *dfas, const int32_t *modes, uint32_t ninst, lex_batch **out, char *err,
                     size_t errlen) {
  if (!dfas || !modes || !out || ninst == 0) {
    set_err(err, errlen, "null argument or no instances");
    return LEX_EINVAL;
  }
  *out = nullptr;
  if (ninst > (uint32_t)lexk::kBatchMaxInst) {
    set_err(err, errlen, "at most 8 instances");
    return LEX_ELIMIT;
  }
  int total_rows = 0;
  for (uint32_t k = 0; k < ninst; ++k) {
    if (!dfas[k] || (modes[k] != LEX_MODE_EXACT && modes[k] != LEX_MODE_DISCARD)) {
      set_err(err, errlen, "bad instance " + std::to_string(k));
      return LEX_EINVAL;
    }
    total_rows += dfas[k]->c.nrows;
  }
  if (total_rows >= lexc::kMaxRows || lexk::batch_emit_lds_bytes(total_rows, ninst) == 0) {
    set_err(err, errlen, "combined tables too large for LDS (" + std::to_string(total_rows) + " rows)");
    return LEX_ELIMIT;
  }
  // Rebase every instance's packed table into one: rows of instance k follow those of the
  // earlier instances; each entry's next-row field and swizzle are renumbered, and each
  // row's columns are re-permuted for its new swizzle.
  std::vector<uint32_t> table((size_t)total_rows * 256);
  std::vector<uint8_t> info(total_rows), kind(total_rows), luts((size_t)ninst * 256);
  lexk::BatchTables bt{};
  bt.nrows = total_rows;
  bt.ninst = ninst;
  auto state = [](uint32_t row) { return (row << lexc::kRowShift) | (lexc::row_swizzle((int)row) << 2); };
  uint32_t base = 0;
  for (uint32_t k = 0; k < ninst; ++k) {
    const lexc::Compiled &c = dfas[k]->c;
    const int m = modes[k];
    for (int r = 0; r < c.nrows; ++r) {
      const uint32_t nr = base + (uint32_t)r;
      for (int b = 0; b < 256; ++b) {
        const uint32_t e = c.table[m][(size_t)r * 256 + ((uint32_t)b ^ lexc::row_swizzle(r))];
        const uint32_t next = (e & lexc::kStateMask) >> lexc::kRowShift;
        const uint32_t flags = e & ~lexc::kStateMask;
        table[(size_t)nr * 256 + ((uint32_t)b ^ lexc::row_swizzle((int)nr))] = flags | state(base + next);
      }
      info[nr] = c.rowinfo[m][r];
      kind[nr] = c.rowkind[r];
    }
    memcpy(&luts[(size_t)k * 256], dfas[k]->lut[m].data(), 256);
    lexk::BatchInstHost &in = bt.inst[k];
    in.start = state(base);
    in.sink = state(base + (uint32_t)c.row_sink);
    in.fail = c.row_fail >= 0 ? state(base + (uint32_t)c.row_fail) : in.sink;
    in.mono = c.monotone ? 1 : 0;
    in.refused = dfas[k]->cm[m].nbytes == 0;
    in.disc = dfas[k]->all_counted[m] ? 0 : 1;
    in.cm = dfas[k]->cm[m];
    base += (uint32_t)c.nrows;
  }
  lex_batch *bb = new lex_batch;
  (void)hipGetDevice(&bb->device);
  uint32_t *d_table = nullptr;
  uint8_t *d_info = nullptr, *d_kind = nullptr, *d_luts = nullptr;
  hipError_t e = upload(&d_table, table.data(), table.size());
  if (e == hipSuccess) e = upload(&d_info, info.data(), info.size());
  if (e == hipSuccess) e = upload(&d_kind, kind.data(), kind.size());
  if (e == hipSuccess) e = upload(&d_luts, luts.data(), luts.size());
  bt.table = d_table;
  bt.rowinfo = d_info;
  bt.rowkind = d_kind;
  bt.luts = d_luts;
  bb->bt = bt;
  if (e != hipSuccess) {
    lex_batch_free(bb);
    set_err(err, errlen, "device upload failed");
    return LEX_EDEVICE;
  }
  *out = bb;
  return LEX_OK;
}

void lex_batch_free(lex_batch *b) {
  if (!b) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  if (b->bt.table) (void)hipFree(const_cast<uint32_t *>(b->bt.table));
  if (b->bt.rowinfo) (void)hipFree(const_cast<uint8_t *>(b->bt.rowinfo));
  if (b->bt.rowkind) (void)hipFree(const_cast<uint8_t *>(b->bt.rowkind));
  if (b->bt.luts) (void)hipFree(const_cast<uint8_t *>(b->bt.luts));
  if (cur >= 0) (void)hipSetDevice(cur);
  delete b;
}

// Default batch lane: 1 KiB, doubled while the batch would have more than about 2M lanes,
// up to 4 KiB.  Below that count a lane's fixed costs (plan entry, count, scan slot, emit
// start) are small beside its walk; above it they dominate, and longer lanes pay.  (On the
// 50 000-document, 2.5 GB batch, 2 KiB lanes measured 3.15 ms against 3.24 ms at 4 KiB.)
static uint32_t batch_default_lane_bytes(uint64_t nbytes) {
  uint32_t l = 1024;
  while (l < 4096 && nbytes / l > (2u << 20)) l <<= 1;
  return l;
}

static int batch_lane_bytes(const lex_run_opts *o, uint64_t nbytes, uint32_t &lb) {
  lb = o && o->lane_bytes ? o->lane_bytes : batch_default_lane_bytes(nbytes);
  if (lb < 16 || (lb & 15)) return LEX_EINVAL;
  if (o && (o->emit || (o->path && o->path != 2))) return LEX_EINVAL;  // the batch plans like path 2
  return LEX_OK;
}

size_t lex_batch_workspace_size(const lex_batch *b, uint32_t ndocs, uint64_t nbytes, const lex_run_opts *opts) {
  uint32_t lb = 0;
  if (!b || nbytes > 0xFFFFFFF0ull || batch_lane_bytes(opts, nbytes, lb) != LEX_OK) return 0;
  return lexk::batch_workspace_bytes(ndocs, nbytes, lb);
}

int lex_run_batch(const lex_batch *b, const uint8_t *d_bytes, uint64_t nbytes, const lex_doc *d_docs, uint32_t ndocs,
                  uint8_t *d_kinds, uint32_t *d_lens, uint64_t *d_offsets, uint64_t cap, lex_doc_result *d_res,
                  lex_result *d_total, void *d_ws, size_t ws_bytes, const lex_run_opts *opts, void *stream) {
  if (!b || !d_total || !d_ws || (ndocs && (!d_docs || !d_res)) || (!d_bytes && nbytes)) return LEX_EINVAL;
  if (cap && (!d_kinds || !d_lens)) return LEX_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_kinds) | reinterpret_cast<uintptr_t>(d_lens)) & 15) return LEX_EINVAL;
  if (nbytes > 0xFFFFFFF0ull || cap > 0xFFFFFFF0ull) return LEX_ELIMIT;
  uint32_t lb = 0;
  int rc = batch_lane_bytes(opts, nbytes, lb);
  if (rc != LEX_OK) return rc;
  if (ws_bytes < lexk::batch_workspace_bytes(ndocs, nbytes, lb)) return LEX_ELIMIT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return LEX_EDEVICE;
  hipEvent_t const *ev = opts && opts->events ? reinterpret_cast<hipEvent_t const *>(opts->events) : nullptr;
  hipError_t e = lexk::run_batch(b->bt, d_bytes, nbytes, d_docs, ndocs, lb, d_kinds, d_lens, d_offsets, cap, d_res,
                                 reinterpret_cast<lexk::ResultDev *>(d_total), d_ws, ws_bytes,
                                 static_cast<hipStream_t>(stream), ev);
  return e == hipSuccess ? LEX_OK : LEX_EDEVICE;
}

int lex_cert_bitmap(const lex_dfa *d, const uint8_t *d_bytes, uint64_t n, int mode, uint64_t *d_bits,
                    void *stream) {
  if (!d || (!d_bytes && n) || (!d_bits && n) || mode < 0 || mode > 1) return LEX_EINVAL;
  if (n > 0xFFFFFFF0ull) return LEX_ELIMIT;
  hipError_t e = lexk::launch_bitmap(d_bytes, (uint32_t)n, d->cm[mode], d_bits, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LEX_OK : LEX_EDEVICE;
}

}  // extern "C"
