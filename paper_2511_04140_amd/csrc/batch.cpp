// batch.cpp -- many series in one launch: batch calls, reusable plans with
// an autotuned launch geometry, captured as a HIP graph.
//
// Every chunk of every series gets a launch chunk index t: the float64
// series come first, then the float32 ones, each series' chunks
// consecutive.  A launch hands chunks out in t order (compression tickets,
// decompression striding); each series' look-back stops at its own first
// chunk, so series are independent and each output is byte-identical to a
// one-series call.  Two launch forms exist: split (one launch per dtype,
// each over its own contiguous range of t) and mixed (one launch over all
// of t, the wave branching on the dtype of the chunk's series).
//
// A plan keeps its own scratch (status words, control block, length and
// error words), so the launch sequence it records never depends on host
// state: the status words are cleared by a fill kernel at the start of
// every run (no memset nodes), and the launch epoch is fixed.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "context.hpp"

using namespace falcon_dev;
using namespace falcon_host;

struct falcon_plan {
  falcon_ctx* ctx = nullptr;
  int op = 0;                // FALCON_OP_COMPRESS / FALCON_OP_DECOMPRESS
  size_t count = 0;
  std::vector<falcon_series> series;  // caller's descriptors (by caller index)
  uint64_t total = 0;        // launch chunks
  uint64_t t64 = 0;          // chunks of the float64 series (they come first)
  bool has64 = false, has32 = false;
  CompressSeries one_c{};    // the descriptor when count == 1
  DecompressSeries one_d{};
  void* many = nullptr;      // device descriptors, launch order
  uint64_t* status = nullptr;
  size_t status_words = 0;
  uint64_t* gstatus = nullptr;
  size_t gstatus_words = 0;
  uint32_t* sizes = nullptr;  // decompression: gathered chunk sizes
  Ctl* ctl = nullptr;
  uint64_t* lens = nullptr;   // device, one per series (compression)
  uint64_t* h_lens = nullptr; // pinned: count lengths, then the error word
  hipStream_t stream = nullptr;
  // geometry
  int split = 1;
  int nw = kCompressWaves;
  int grid_pct = 100;
  // tuning record
  int candidates = 0;
  float best_ms = 0.f, default_ms = 0.f;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t kPlanEpoch = 1;

int grid_of(falcon_plan* p, int form, uint64_t chunks, bool compress) {
  const int maxg = compress ? max_grid_c(p->ctx, form, p->nw) : max_grid_d(p->ctx, form);
  int g = (int)((int64_t)maxg * p->grid_pct / 100);
  if (g < 1) g = 1;
  const int per = compress ? p->nw : kDecompressWaves;
  const uint64_t want = (chunks + per - 1) / per;
  if (want < (uint64_t)g) g = (int)(want ? want : 1);
  return g;
}

// Launches of one run, in stream order.
falcon_status enqueue_plan(falcon_plan* p, hipStream_t s) {
  falcon_status st;
  // clear status words and the control block (ticket, exit counter, error)
  if ((st = dev_err(launch_fill_u64(p->status, p->status_words, 0, s))) != FALCON_OK ||
      (st = dev_err(launch_fill_u64(p->gstatus, p->gstatus_words, 0, s))) != FALCON_OK ||
      (st = dev_err(launch_fill_u64(reinterpret_cast<uint64_t*>(p->ctl), 2, 0, s))) != FALCON_OK)
    return st;
  struct Part { int form; uint64_t t0, chunks; };
  Part parts[2];
  int np = 0;
  if (p->has64 && p->has32 && !p->split) {
    parts[np++] = {kFormMixed, 0, p->total};
  } else {
    if (p->has64) parts[np++] = {2, 0, p->t64};
    if (p->has32) parts[np++] = {1, p->t64, p->total - p->t64};
  }
  if (np == 0) parts[np++] = {2, 0, 0};  // only empty series: one launch writes their headers
  if (p->op == FALCON_OP_COMPRESS) {
    for (int i = 0; i < np; ++i) {
      CompressArgs a{};
      a.one = p->one_c;
      a.many = static_cast<const CompressSeries*>(p->many);
      a.nseries = (uint32_t)p->count;
      a.total_chunks = parts[i].chunks;
      a.t0 = parts[i].t0;
      a.status = p->status;
      a.gstatus = p->gstatus;
      a.ctl = p->ctl;
      a.lens = p->lens;
      a.epoch = kPlanEpoch;
      const int grid = grid_of(p, parts[i].form, parts[i].chunks, true);
      a.total_waves = (uint32_t)(grid * p->nw);
      if ((st = dev_err(launch_compress(a, parts[i].form, p->nw, grid, s))) != FALCON_OK) return st;
    }
    return dev_err(hipMemcpyAsync(p->h_lens, p->lens, p->count * 8, hipMemcpyDeviceToHost, s));
  }
  // decompression: headers and sizes, one scan over all chunks, kernels
  DecompressSeries* many = static_cast<DecompressSeries*>(p->many);
  if ((st = dev_err(launch_batch_dprep(many, (uint32_t)p->count, p->total, p->sizes, p->ctl, kPlanEpoch, s))) !=
          FALCON_OK ||
      (st = dev_err(launch_scan_sizes(p->sizes, p->total, 7, (uint32_t)kF64Chunk, ~0ull, p->gstatus, p->status,
                                      p->ctl, kPlanEpoch, s))) != FALCON_OK)
    return st;
  for (int i = 0; i < np; ++i) {
    if (parts[i].chunks == 0) continue;
    DecompressArgs a{};
    a.one = p->one_d;
    a.many = many;
    a.nseries = (uint32_t)p->count;
    a.total_chunks = parts[i].chunks;
    a.t0 = parts[i].t0;
    a.status = p->status;
    a.ctl = p->ctl;
    a.epoch = kPlanEpoch;
    a.relative = 1;
    const int grid = grid_of(p, parts[i].form, parts[i].chunks, false);
    a.total_waves = (uint32_t)(grid * kDecompressWaves);
    if ((st = dev_err(launch_decompress(a, parts[i].form, grid, s))) != FALCON_OK) return st;
  }
  return dev_err(hipMemcpyAsync(p->h_lens + p->count, &p->ctl->error, 4, hipMemcpyDeviceToHost, s));
}

// Checks a series descriptor on the host.
falcon_status check_series(int op, const falcon_series& d) {
  const size_t es = elem_size(d.dtype);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  const uint64_t nc = chunks_of(d.n);
  // a decompression output may be null only when there is nothing to write
  if (nc >= 0xFFFFFFF0ull || (!d.d_out && (op == FALCON_OP_COMPRESS || d.n != 0)) ||
      ((uintptr_t)d.d_out % (op == FALCON_OP_COMPRESS ? 4 : es)))
    return FALCON_ERR_INVALID_ARG;
  if (op == FALCON_OP_COMPRESS) {
    if (d.n && (!d.d_in || ((uintptr_t)d.d_in % es))) return FALCON_ERR_INVALID_ARG;
    if (d.out_cap < falcon_compress_bound(d.n, d.dtype)) return FALCON_ERR_BUFFER_TOO_SMALL;
  } else {
    if (!d.d_in || ((uintptr_t)d.d_in % 4)) return FALCON_ERR_INVALID_ARG;
    if (d.in_len < 32 + 4 * nc) return FALCON_ERR_CORRUPT_STREAM;
    if (d.out_cap / es < d.n) return FALCON_ERR_BUFFER_TOO_SMALL;
  }
  return FALCON_OK;
}

void plan_free(falcon_plan* p) {
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->many) (void)hipFree(p->many);
  if (p->status) (void)hipFree(p->status);
  if (p->gstatus) (void)hipFree(p->gstatus);
  if (p->sizes) (void)hipFree(p->sizes);
  if (p->ctl) (void)hipFree(p->ctl);
  if (p->lens) (void)hipFree(p->lens);
  if (p->h_lens) (void)hipHostFree(p->h_lens);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// Times one run of the plan's current geometry: best of reps runs.
falcon_status time_runs(falcon_plan* p, int reps, float* best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FALCON_ERR_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FALCON_ERR_DEVICE;
  }
  falcon_status st = FALCON_OK;
  *best = 1e30f;
  for (int r = 0; r < reps && st == FALCON_OK; ++r) {
    float ms = 0.f;
    if ((st = dev_err(hipEventRecord(e0, p->stream))) != FALCON_OK || (st = enqueue_plan(p, p->stream)) != FALCON_OK ||
        (st = dev_err(hipEventRecord(e1, p->stream))) != FALCON_OK ||
        (st = dev_err(hipEventSynchronize(e1))) != FALCON_OK ||
        (st = dev_err(hipEventElapsedTime(&ms, e0, e1))) != FALCON_OK)
      break;
    if (r > 0 || reps == 1) *best = std::min(*best, ms);  // the first run warms up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Autotuner: tries every launch form x workgroup size x grid fraction on
// the plan's own series and keeps the fastest.  All candidates produce the
// same bytes (the launch geometry never changes the stream).
falcon_status autotune(falcon_plan* p) {
  struct Cand { int split, nw, pct; };
  std::vector<Cand> cands;
  const bool both = p->has64 && p->has32;
  for (int split = 1; split >= (both ? 0 : 1); --split)
    for (int nw : {16, 8})
      for (int pct : {100, 50}) {
        if (p->op == FALCON_OP_DECOMPRESS && nw != 16) continue;  // no workgroup size choice there
        cands.push_back({split, nw, pct});
      }
  float best = 1e30f;
  Cand pick = cands[0];
  for (size_t i = 0; i < cands.size(); ++i) {
    p->split = cands[i].split;
    p->nw = cands[i].nw;
    p->grid_pct = cands[i].pct;
    float ms;
    falcon_status st = time_runs(p, 3, &ms);
    if (st != FALCON_OK) return st;
    if (i == 0) p->default_ms = ms;
    if (ms < best) {
      best = ms;
      pick = cands[i];
    }
  }
  p->split = pick.split;
  p->nw = pick.nw;
  p->grid_pct = pick.pct;
  p->best_ms = best;
  p->candidates = (int)cands.size();
  return FALCON_OK;
}

falcon_status plan_finish(falcon_plan* p, falcon_series* s) {
  if (p->op == FALCON_OP_DECOMPRESS) {
    uint32_t err;
    memcpy(&err, p->h_lens + p->count, 4);
    if (err == kPlanEpoch) return FALCON_ERR_CORRUPT_STREAM;
  }
  if (s)
    for (size_t i = 0; i < p->count; ++i) s[i].out_len = p->op == FALCON_OP_COMPRESS ? p->h_lens[i] : p->series[i].n;
  return FALCON_OK;
}

}  // namespace

extern "C" {

falcon_status falcon_plan_create(falcon_ctx* ctx, falcon_op op, const falcon_series* s, size_t count,
                                 unsigned flags, falcon_plan** out) {
  if (!ctx || !out || (count && !s) || (op != FALCON_OP_COMPRESS && op != FALCON_OP_DECOMPRESS) ||
      count == 0 || count > 0x7FFFFFFFull)
    return FALCON_ERR_INVALID_ARG;
  *out = nullptr;
  for (size_t i = 0; i < count; ++i) {
    falcon_status st = check_series(op, s[i]);
    if (st != FALCON_OK) return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  falcon_plan* p = new (std::nothrow) falcon_plan();
  if (!p) return FALCON_ERR_OUT_OF_MEMORY;
  p->ctx = ctx;
  p->op = op;
  p->count = count;
  p->series.assign(s, s + count);
  // launch order: float64 series, then float32, each in caller order
  std::vector<uint32_t> order;
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 0; i < count; ++i)
      if ((s[i].dtype == FALCON_FLOAT64) == (pass == 0)) order.push_back((uint32_t)i);
  std::vector<CompressSeries> cs;
  std::vector<DecompressSeries> ds;
  uint64_t t = 0, g = 0;
  for (uint32_t i : order) {
    const falcon_series& d = s[i];
    const uint64_t nc = chunks_of(d.n);
    if (op == FALCON_OP_COMPRESS) {
      CompressSeries c{};
      c.in = d.d_in;
      c.out = static_cast<uint8_t*>(d.d_out);
      c.n = d.n;
      c.chunk0 = t;
      c.group0 = g;
      c.dtype = (uint32_t)d.dtype;
      c.idx = i;
      cs.push_back(c);
    } else {
      DecompressSeries c{};
      c.in = static_cast<const uint8_t*>(d.d_in);
      c.out = static_cast<uint8_t*>(d.d_out);
      c.n = d.n;
      c.chunk0 = t;
      c.group0 = g;
      c.in_len = d.in_len;
      c.dtype = (uint32_t)d.dtype;
      c.idx = i;
      ds.push_back(c);
    }
    if (d.dtype == FALCON_FLOAT64) {
      p->t64 += nc;
      p->has64 |= nc > 0;
    } else {
      p->has32 |= nc > 0;
    }
    t += nc;
    g += groups_of(nc);
  }
  p->total = t;
  if (!cs.empty()) p->one_c = cs[0];
  if (!ds.empty()) p->one_d = ds[0];
  const size_t desc_bytes = op == FALCON_OP_COMPRESS ? cs.size() * sizeof(CompressSeries)
                                                     : ds.size() * sizeof(DecompressSeries);
  p->status_words = t ? t : 1;
  p->gstatus_words = (op == FALCON_OP_COMPRESS ? g : scan_tiles(t)) + 1;
  falcon_status st = FALCON_OK;
  if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) st = FALCON_ERR_DEVICE;
  if (st == FALCON_OK &&
      (hipMalloc(&p->many, desc_bytes) != hipSuccess || hipMalloc(&p->status, p->status_words * 8) != hipSuccess ||
       hipMalloc(&p->gstatus, p->gstatus_words * 8) != hipSuccess || hipMalloc(&p->ctl, 64) != hipSuccess ||
       hipMalloc(&p->lens, count * 8) != hipSuccess ||
       hipHostMalloc(&p->h_lens, (count + 1) * 8, hipHostMallocDefault) != hipSuccess ||
       (op == FALCON_OP_DECOMPRESS && hipMalloc(&p->sizes, (t ? t : 1) * 4) != hipSuccess)))
    st = FALCON_ERR_OUT_OF_MEMORY;
  if (st == FALCON_OK &&
      (hipMemcpy(p->many, op == FALCON_OP_COMPRESS ? (const void*)cs.data() : (const void*)ds.data(), desc_bytes,
                 hipMemcpyHostToDevice) != hipSuccess ||
       hipMemset(p->ctl, 0, 64) != hipSuccess))
    st = FALCON_ERR_DEVICE;
  if (st == FALCON_OK && (flags & FALCON_PLAN_TUNE)) st = autotune(p);
  if (st == FALCON_OK && (flags & FALCON_PLAN_GRAPH)) {
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = FALCON_ERR_DEVICE;
    } else {
      falcon_status est = enqueue_plan(p, p->stream);
      const hipError_t ce = hipStreamEndCapture(p->stream, &p->graph);
      if (est != FALCON_OK) st = est;
      else if (ce != hipSuccess || hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        st = FALCON_ERR_DEVICE;
    }
  }
  if (st != FALCON_OK) {
    plan_free(p);
    return st;
  }
  *out = p;
  return FALCON_OK;
}

falcon_status falcon_plan_run(falcon_plan* p, falcon_series* s, void* stream) {
  if (!p) return FALCON_ERR_INVALID_ARG;
  if (hipSetDevice(p->ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  hipStream_t st_ = stream ? static_cast<hipStream_t>(stream) : p->stream;
  falcon_status st = p->exec ? dev_err(hipGraphLaunch(p->exec, st_)) : enqueue_plan(p, st_);
  if (st != FALCON_OK) return st;
  if ((st = dev_err(hipStreamSynchronize(st_))) != FALCON_OK) return st;
  return plan_finish(p, s);
}

falcon_status falcon_plan_describe(const falcon_plan* p, falcon_plan_info* info) {
  if (!p || !info) return FALCON_ERR_INVALID_ARG;
  info->split = p->split;
  info->waves_per_group = p->op == FALCON_OP_COMPRESS ? p->nw : kDecompressWaves;
  info->grid_percent = p->grid_pct;
  info->candidates = p->candidates;
  info->best_ms = p->best_ms;
  info->default_ms = p->default_ms;
  info->graph = p->exec != nullptr;
  info->total_chunks = p->total;
  return FALCON_OK;
}

void falcon_plan_destroy(falcon_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  plan_free(p);
}

falcon_status falcon_compress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream) {
  if (count == 0) return ctx ? FALCON_OK : FALCON_ERR_INVALID_ARG;
  falcon_plan* p = nullptr;
  falcon_status st = falcon_plan_create(ctx, FALCON_OP_COMPRESS, s, count, 0, &p);
  if (st != FALCON_OK) return st;
  st = falcon_plan_run(p, s, stream);
  falcon_plan_destroy(p);
  return st;
}

falcon_status falcon_decompress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream) {
  if (count == 0) return ctx ? FALCON_OK : FALCON_ERR_INVALID_ARG;
  falcon_plan* p = nullptr;
  falcon_status st = falcon_plan_create(ctx, FALCON_OP_DECOMPRESS, s, count, 0, &p);
  if (st != FALCON_OK) return st;
  st = falcon_plan_run(p, s, stream);
  falcon_plan_destroy(p);
  return st;
}

}  // extern "C"
