// batch.cpp -- many series in one launch: batch calls, reusable plans with
// an autotuned launch geometry, captured as a HIP graph.
//
// Every chunk of every series gets a launch chunk index t: the float64
// series come first, then the float32 ones, each series' chunks
// consecutive.  Waves take chunks by static striding over t; each series'
// offsets are the scan of all chunk sizes minus the offset of its own first
// chunk, so series are independent and each output is byte-identical to a
// one-series call.  Two launch forms exist: split (one launch per dtype,
// each over its own contiguous range of t) and mixed (one launch over all
// of t, the wave branching on the dtype of the chunk's series).
//
// Compression runs in two passes over all series (size pass, one scan of
// all chunk sizes, write pass; see codec_kernels.hpp), so no chunk waits on
// another, or, when the autotuner finds it faster, in the single pass with a
// work queue over all chunks and a look-back that stops at each series'
// first chunk.  A run never depends on host state beyond its descriptors: the
// control block is cleared by a fill kernel at the start of a decompression
// run (no memset nodes in a recorded graph) and the launch epoch is fixed.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "context.hpp"

using namespace falcon_dev;

namespace falcon_host {

namespace {

constexpr uint32_t kBatchEpoch = 1;

// Grows a device (pinned = false) or pinned host array to at least need
// elements, waiting for stream s before freeing the old one.
template <class P>
falcon_status grow(P** p, size_t* cap, size_t need, size_t elem, bool pinned, hipStream_t s) {
  if (need <= *cap && *p) return FALCON_OK;
  size_t c = *cap ? *cap : 64;
  while (c < need) c *= 2;
  if (*p) {
    if (hipStreamSynchronize(s) != hipSuccess) return FALCON_ERR_DEVICE;
    if (pinned) (void)hipHostFree(*p);
    else (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
  }
  void* q = nullptr;
  const hipError_t e = pinned ? hipHostMalloc(&q, c * elem, hipHostMallocDefault) : hipMalloc(&q, c * elem);
  if (e != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
  *p = static_cast<P*>(q);
  *cap = c;
  return FALCON_OK;
}

int grid_of(const falcon_ctx* ctx, const BatchGeom& g, int form, int pass, uint64_t chunks, bool compress) {
  const int maxg = !compress ? max_grid_d(ctx, form) : g.form ? max_grid_q(ctx, form, g.nw) : max_grid_c(ctx, form, pass, g.nw);
  int grid = (int)((int64_t)maxg * g.grid_pct / 100);
  if (grid < 1) grid = 1;
  const int per = compress ? g.nw : kDecompressWaves;
  const uint64_t want = (chunks + per - 1) / per;
  if (want < (uint64_t)grid) grid = (int)(want ? want : 1);
  return grid;
}

}  // namespace

falcon_status batch_check(int op, const falcon_series& d) {
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

falcon_status batch_layout(BatchScratch& b, int op, const falcon_series* s, size_t count, BatchLayout& L,
                           hipStream_t st) {
  L = BatchLayout();
  L.op = op;
  L.count = count;
  const size_t dsz = op == FALCON_OP_COMPRESS ? sizeof(CompressSeries) : sizeof(DecompressSeries);
  L.desc_bytes = count * dsz;
  falcon_status r = grow(&b.h_desc, &b.h_desc_cap, L.desc_bytes, 1, true, st);
  if (r != FALCON_OK) return r;
  uint64_t t = 0;
  size_t k = 0;
  for (int pass = 0; pass < 2; ++pass) {  // float64 series first, then float32
    for (size_t i = 0; i < count; ++i) {
      const falcon_series& d = s[i];
      if ((d.dtype == FALCON_FLOAT64) != (pass == 0)) continue;
      const uint64_t nc = chunks_of(d.n);
      if (op == FALCON_OP_COMPRESS) {
        CompressSeries c{};
        c.in = d.d_in;
        c.out = static_cast<uint8_t*>(d.d_out);
        c.n = d.n;
        c.chunk0 = t;
        c.dtype = (uint32_t)d.dtype;
        c.idx = (uint32_t)i;
        memcpy(b.h_desc + k * dsz, &c, dsz);
        if (k == 0) L.one_c = c;
      } else {
        DecompressSeries c{};
        c.in = static_cast<const uint8_t*>(d.d_in);
        c.out = static_cast<uint8_t*>(d.d_out);
        c.n = d.n;
        c.chunk0 = t;
        c.in_len = d.in_len;
        c.dtype = (uint32_t)d.dtype;
        c.idx = (uint32_t)i;
        memcpy(b.h_desc + k * dsz, &c, dsz);
        if (k == 0) L.one_d = c;
      }
      ++k;
      if (d.dtype == FALCON_FLOAT64) {
        L.t64 += nc;
        L.has64 |= nc > 0;
      } else {
        L.has32 |= nc > 0;
      }
      t += nc;
    }
  }
  L.total = t;
  const size_t gwords = scan_tiles(t) + 1;
  if ((r = grow(&b.many, &b.many_cap, L.desc_bytes, 1, false, st)) != FALCON_OK ||
      (r = grow(&b.offsets, &b.offsets_cap, t ? t : 1, 8, false, st)) != FALCON_OK ||
      (r = grow(&b.tiles, &b.tiles_cap, gwords, 8, false, st)) != FALCON_OK ||
      (r = grow(&b.lens, &b.lens_cap, count, 8, false, st)) != FALCON_OK ||
      (r = grow(&b.h_lens, &b.h_lens_cap, count + 1, 8, true, st)) != FALCON_OK)
    return r;
  if ((r = grow(&b.sizes, &b.sizes_cap, t ? t : 1, 4, false, st)) != FALCON_OK) return r;
  if (op == FALCON_OP_COMPRESS && (r = grow(&b.meta, &b.meta_cap, t ? t : 1, sizeof(ChunkMeta), false, st)) !=
                                      FALCON_OK)
    return r;
  if (op == FALCON_OP_COMPRESS &&
      (r = grow(&b.status, &b.status_cap, (size_t)kQueueGroups * kQueueStride + (t ? t : 1), 8, false, st)) !=
          FALCON_OK)
    return r;
  if (!b.ctl) {
    if (hipMalloc(&b.ctl, 64) != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
    if (launch_fill_u64(reinterpret_cast<uint64_t*>(b.ctl), 8, 0, st) != hipSuccess) return FALCON_ERR_DEVICE;
  }
  return FALCON_OK;
}

falcon_status batch_enqueue(const falcon_ctx* ctx, BatchScratch& b, const BatchLayout& L, const BatchGeom& g,
                            hipStream_t s, bool upload) {
  falcon_status st;
  if (upload && (st = dev_err(hipMemcpyAsync(b.many, b.h_desc, L.desc_bytes, hipMemcpyHostToDevice, s))) !=
                    FALCON_OK)
    return st;
  struct Part { int form; uint64_t t0, chunks; };
  Part parts[2];
  int np = 0;
  if (L.has64 && L.has32 && !g.split) {
    parts[np++] = {kFormMixed, 0, L.total};
  } else {
    if (L.has64) parts[np++] = {2, 0, L.t64};
    if (L.has32) parts[np++] = {1, L.t64, L.total - L.t64};
  }
  if (L.op == FALCON_OP_COMPRESS) {
    if (np == 0) parts[np++] = {2, 0, 0};  // only empty series: the last launch writes their headers
    CompressArgs a{};
    a.one = L.one_c;
    a.many = static_cast<const CompressSeries*>(b.many);
    a.nseries = (uint32_t)L.count;
    a.lens = b.lens;
    a.meta = b.meta;
    a.gsizes = b.sizes;
    a.offsets = b.offsets;
    a.relative = 1;
    if (g.form == 1) {
      // single pass: a work queue and a per-series look-back; counters,
      // status words and the error word cleared by fill kernels (a recorded
      // graph replays them), so every run uses the same tag
      const size_t nq = (size_t)kQueueGroups * kQueueStride;
      if ((st = dev_err(launch_fill_u64(b.status, nq + (L.total ? L.total : 1), 0, s))) != FALCON_OK ||
          (st = dev_err(launch_fill_u64(reinterpret_cast<uint64_t*>(b.ctl), 1, 0, s))) != FALCON_OK)
        return st;
      a.qctr = b.status;
      a.status = b.status + nq;
      a.ctl = b.ctl;
      a.qtag = kBatchEpoch;
      for (int i = 0; i < np; ++i) {
        // launches run one after the other on s: each starts with cleared counters
        if (i > 0 && (st = dev_err(launch_fill_u64(b.status, nq, 0, s))) != FALCON_OK) return st;
        a.total_chunks = parts[i].chunks;
        a.t0 = parts[i].t0;
        const int grid = grid_of(ctx, g, parts[i].form, 0, parts[i].chunks, true);
        a.total_waves = (uint32_t)(grid * g.nw);
        a.qgroups = (uint32_t)(grid < kQueueGroups ? grid : kQueueGroups);
        if ((st = dev_err(launch_compress_queue(a, parts[i].form, g.nw, grid, s))) != FALCON_OK) return st;
      }
      if ((st = dev_err(hipMemcpyAsync(b.h_lens, b.lens, L.count * 8, hipMemcpyDeviceToHost, s))) != FALCON_OK)
        return st;
      return dev_err(hipMemcpyAsync(b.h_lens + L.count, b.ctl, 8, hipMemcpyDeviceToHost, s));
    }
    // two passes over all series: sizes, one scan over all chunks, writes
    for (int pass = 1; pass <= 2; ++pass) {
      for (int i = 0; i < np; ++i) {
        if (pass == 1 && parts[i].chunks == 0) continue;
        a.total_chunks = parts[i].chunks;
        a.t0 = parts[i].t0;
        const int grid = grid_of(ctx, g, parts[i].form, pass, parts[i].chunks, true);
        a.total_waves = (uint32_t)(grid * g.nw);
        if ((st = dev_err(launch_compress(a, parts[i].form, pass, g.nw, grid, s))) != FALCON_OK) return st;
      }
      if (pass == 1 && L.total &&
          (st = dev_err(launch_scan_sizes(b.sizes, L.total, 0, ~0u, ~0ull, b.tiles, b.offsets, b.ctl, kBatchEpoch,
                                          s))) != FALCON_OK)
        return st;
    }
    if ((st = dev_err(hipMemcpyAsync(b.h_lens, b.lens, L.count * 8, hipMemcpyDeviceToHost, s))) != FALCON_OK)
      return st;
    return dev_err(hipMemcpyAsync(b.h_lens + L.count, b.ctl, 8, hipMemcpyDeviceToHost, s));
  }
  // clear the control block (error word) of decompression
  if ((st = dev_err(launch_fill_u64(reinterpret_cast<uint64_t*>(b.ctl), 2, 0, s))) != FALCON_OK) return st;
  // decompression: headers and sizes, one scan over all chunks, kernels
  DecompressSeries* many = static_cast<DecompressSeries*>(b.many);
  if ((st = dev_err(launch_batch_dprep(many, (uint32_t)L.count, L.total, b.sizes, b.ctl, kBatchEpoch, s))) !=
          FALCON_OK ||
      (st = dev_err(launch_scan_sizes(b.sizes, L.total, 7, (uint32_t)kF64Chunk, ~0ull, b.tiles, b.offsets, b.ctl,
                                      kBatchEpoch, s))) != FALCON_OK)
    return st;
  for (int i = 0; i < np; ++i) {
    DecompressArgs a{};
    a.one = L.one_d;
    a.many = many;
    a.nseries = (uint32_t)L.count;
    a.total_chunks = parts[i].chunks;
    a.t0 = parts[i].t0;
    a.offsets = b.offsets;
    a.ctl = b.ctl;
    a.epoch = kBatchEpoch;
    a.relative = 1;
    const int grid = grid_of(ctx, g, parts[i].form, 0, parts[i].chunks, false);
    a.total_waves = (uint32_t)(grid * kDecompressWaves);
    if ((st = dev_err(launch_decompress(a, parts[i].form, grid, s))) != FALCON_OK) return st;
  }
  return dev_err(hipMemcpyAsync(b.h_lens + L.count, &b.ctl->error, 4, hipMemcpyDeviceToHost, s));
}

falcon_status batch_result(const BatchScratch& b, const BatchLayout& L, const falcon_series* src,
                           falcon_series* dst) {
  uint32_t err[2];
  memcpy(err, b.h_lens + L.count, 8);
  if (L.op == FALCON_OP_DECOMPRESS && err[0] == kBatchEpoch) return FALCON_ERR_CORRUPT_STREAM;
  // a single-pass look-back that gave up (never in a correct run)
  if (L.op == FALCON_OP_COMPRESS && err[1] != 0) return FALCON_ERR_DEVICE;
  if (dst)
    for (size_t i = 0; i < L.count; ++i) dst[i].out_len = L.op == FALCON_OP_COMPRESS ? b.h_lens[i] : src[i].n;
  return FALCON_OK;
}

void batch_free(BatchScratch& b) {
  if (b.many) (void)hipFree(b.many);
  if (b.h_desc) (void)hipHostFree(b.h_desc);
  if (b.offsets) (void)hipFree(b.offsets);
  if (b.tiles) (void)hipFree(b.tiles);
  if (b.sizes) (void)hipFree(b.sizes);
  if (b.meta) (void)hipFree(b.meta);
  if (b.ctl) (void)hipFree(b.ctl);
  if (b.lens) (void)hipFree(b.lens);
  if (b.h_lens) (void)hipHostFree(b.h_lens);
  if (b.status) (void)hipFree(b.status);
  b = BatchScratch();
}

}  // namespace falcon_host

using namespace falcon_host;

struct falcon_plan {
  falcon_ctx* ctx = nullptr;
  std::vector<falcon_series> series;  // caller's descriptors (by caller index)
  BatchLayout layout;
  BatchScratch scratch;               // never grows after creation (the graph holds its pointers)
  BatchGeom geom;
  hipStream_t stream = nullptr;
  int candidates = 0;
  bool from_cache = false;
  float best_ms = 0.f, default_ms = 0.f;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free(falcon_plan* p) {
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  batch_free(p->scratch);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// Times the plan's current geometry: best of reps - 1 runs after a warm-up.
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
    if ((st = dev_err(hipEventRecord(e0, p->stream))) != FALCON_OK ||
        (st = batch_enqueue(p->ctx, p->scratch, p->layout, p->geom, p->stream, false)) != FALCON_OK ||
        (st = dev_err(hipEventRecord(e1, p->stream))) != FALCON_OK ||
        (st = dev_err(hipEventSynchronize(e1))) != FALCON_OK ||
        (st = dev_err(hipEventElapsedTime(&ms, e0, e1))) != FALCON_OK)
      break;
    if (r > 0 || reps == 1) *best = std::min(*best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Shape class of a plan for the tuning record: operation, dtypes present,
// log2 of the chunk count and of the series count.
uint64_t shape_class(const BatchLayout& L) {
  auto lg = [](uint64_t v) {
    uint64_t k = 0;
    while (v > 1) {
      v >>= 1;
      ++k;
    }
    return k;
  };
  return (uint64_t)L.op | (uint64_t)L.has64 << 1 | (uint64_t)L.has32 << 2 | lg(L.total + 1) << 3 |
         lg(L.count) << 16;
}

// Autotuner: times every candidate geometry on the plan's own series and
// keeps the fastest.  Compression: launch form (split / mixed) x 16 or 8
// waves per workgroup x full or half grid x two passes (static striding) or
// single pass (work queue); decompression: launch form x grid.  All
// candidates produce the same bytes (the launch geometry never changes a
// stream).  The choice is recorded in the context by shape class, and a
// later plan of the same class takes it without timing.
falcon_status autotune(falcon_plan* p) {
  const uint64_t key = shape_class(p->layout);
  auto hit = p->ctx->tuned.find(key);
  if (hit != p->ctx->tuned.end()) {
    p->geom = hit->second;
    p->from_cache = true;
    return FALCON_OK;
  }
  std::vector<BatchGeom> cands;
  const bool both = p->layout.has64 && p->layout.has32;
  const bool comp = p->layout.op == FALCON_OP_COMPRESS;
  for (int form = 0; form <= (comp ? 1 : 0); ++form)
    for (int split = 1; split >= (both ? 0 : 1); --split)
      for (int nw : {16, 8})
        for (int pct : {100, 50}) {
          if (!comp && nw != 16) continue;  // no workgroup size choice there
          BatchGeom g;
          g.split = split;
          g.nw = nw;
          g.grid_pct = pct;
          g.form = form;
          cands.push_back(g);
        }
  float best = 1e30f;
  BatchGeom pick = cands[0];
  for (size_t i = 0; i < cands.size(); ++i) {
    p->geom = cands[i];
    float ms;
    falcon_status st = time_runs(p, 3, &ms);
    if (st != FALCON_OK) return st;
    if (i == 0) p->default_ms = ms;
    if (ms < best) {
      best = ms;
      pick = cands[i];
    }
  }
  p->geom = pick;
  p->best_ms = best;
  p->candidates = (int)cands.size();
  p->ctx->tuned[key] = pick;
  return FALCON_OK;
}

// One-shot batch calls run with the context's batch scratch (grown on
// demand) and the default geometry.
falcon_status batch_call(falcon_ctx* ctx, int op, falcon_series* s, size_t count, void* stream) {
  if (!ctx || (count && !s)) return FALCON_ERR_INVALID_ARG;
  if (count == 0) return FALCON_OK;
  if (count > 0x7FFFFFFFull) return FALCON_ERR_INVALID_ARG;
  for (size_t i = 0; i < count; ++i) {
    falcon_status st = batch_check(op, s[i]);
    if (st != FALCON_OK) return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  hipStream_t hs = stream ? static_cast<hipStream_t>(stream) : ctx->main.stream;
  BatchLayout L;
  BatchGeom g;
  g.form = op == FALCON_OP_COMPRESS ? ctx->compress_form : 0;
  falcon_status st = batch_layout(ctx->batch, op, s, count, L, hs);
  if (st == FALCON_OK) st = batch_enqueue(ctx, ctx->batch, L, g, hs, true);
  if (st == FALCON_OK) st = dev_err(hipStreamSynchronize(hs));
  if (st == FALCON_OK) st = batch_result(ctx->batch, L, s, s);
  return st;
}

}  // namespace

extern "C" {

falcon_status falcon_plan_create(falcon_ctx* ctx, falcon_op op, const falcon_series* s, size_t count,
                                 unsigned flags, falcon_plan** out) {
  if (!ctx || !out || !s || (op != FALCON_OP_COMPRESS && op != FALCON_OP_DECOMPRESS) || count == 0 ||
      count > 0x7FFFFFFFull)
    return FALCON_ERR_INVALID_ARG;
  *out = nullptr;
  for (size_t i = 0; i < count; ++i) {
    falcon_status st = batch_check(op, s[i]);
    if (st != FALCON_OK) return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  falcon_plan* p = new (std::nothrow) falcon_plan();
  if (!p) return FALCON_ERR_OUT_OF_MEMORY;
  p->ctx = ctx;
  p->series.assign(s, s + count);
  falcon_status st = FALCON_OK;
  if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) st = FALCON_ERR_DEVICE;
  if (st == FALCON_OK) st = batch_layout(p->scratch, op, s, count, p->layout, p->stream);
  // descriptors go up once; runs reuse them
  if (st == FALCON_OK)
    st = dev_err(hipMemcpyAsync(p->scratch.many, p->scratch.h_desc, p->layout.desc_bytes, hipMemcpyHostToDevice,
                                p->stream));
  if (st == FALCON_OK) st = dev_err(hipStreamSynchronize(p->stream));
  if (op == FALCON_OP_COMPRESS && (flags & FALCON_PLAN_SINGLE_PASS)) p->geom.form = 1;
  if (st == FALCON_OK && (flags & FALCON_PLAN_TUNE)) st = autotune(p);
  if (st == FALCON_OK && (flags & FALCON_PLAN_GRAPH)) {
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = FALCON_ERR_DEVICE;
    } else {
      const falcon_status est = batch_enqueue(ctx, p->scratch, p->layout, p->geom, p->stream, false);
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
  hipStream_t hs = stream ? static_cast<hipStream_t>(stream) : p->stream;
  falcon_status st = p->exec ? dev_err(hipGraphLaunch(p->exec, hs))
                             : batch_enqueue(p->ctx, p->scratch, p->layout, p->geom, hs, false);
  if (st != FALCON_OK) return st;
  if ((st = dev_err(hipStreamSynchronize(hs))) != FALCON_OK) return st;
  return batch_result(p->scratch, p->layout, p->series.data(), s);
}

falcon_status falcon_plan_describe(const falcon_plan* p, falcon_plan_info* info) {
  if (!p || !info) return FALCON_ERR_INVALID_ARG;
  info->split = p->geom.split;
  info->waves_per_group = p->layout.op == FALCON_OP_COMPRESS ? p->geom.nw : kDecompressWaves;
  info->grid_percent = p->geom.grid_pct;
  info->candidates = p->candidates;
  info->best_ms = p->best_ms;
  info->default_ms = p->default_ms;
  info->graph = p->exec != nullptr;
  info->total_chunks = p->layout.total;
  info->form = p->layout.op == FALCON_OP_COMPRESS ? p->geom.form : 0;
  info->from_cache = p->from_cache ? 1 : 0;
  return FALCON_OK;
}

void falcon_plan_destroy(falcon_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  plan_free(p);
}

falcon_status falcon_compress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream) {
  return batch_call(ctx, FALCON_OP_COMPRESS, s, count, stream);
}

falcon_status falcon_decompress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream) {
  return batch_call(ctx, FALCON_OP_DECOMPRESS, s, count, stream);
}

}  // extern "C"
