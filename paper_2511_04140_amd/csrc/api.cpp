// api.cpp -- C ABI of the Falcon codec (declared in include/falcon.h):
// context life cycle and the device-resident compress / decompress calls.
//
// A context owns a main lane (a HIP stream, a small pinned staging buffer
// for the few bytes read back per call, the chunk offsets and size-pass
// results of its launches, and the control block) and, once the host
// pipeline is used, one lane per pipeline stream.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "context.hpp"

using namespace falcon_dev;

namespace falcon_host {

void write_header(uint8_t* h, falcon_dtype dt, uint64_t n, uint64_t payload) {
  memset(h, 0, 32);
  memcpy(h, "FLCN", 4);
  h[4] = 1;
  h[5] = (uint8_t)dt;
  const uint32_t cn = (uint32_t)kChunkN;
  memcpy(h + 8, &cn, 4);
  memcpy(h + 16, &n, 8);
  memcpy(h + 24, &payload, 8);
}

falcon_status lane_init(Lane& l) {
  if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&l.ctl, 64) != hipSuccess || hipMemset(l.ctl, 0, 64) != hipSuccess ||
      hipMalloc(&l.qctr, 8 * kQueueGroups * kQueueStride) != hipSuccess ||
      hipHostMalloc(&l.stage, kStageBytes, hipHostMallocDefault) != hipSuccess) {
    lane_free(l);
    return FALCON_ERR_DEVICE;
  }
  memset(l.stage, 0, kStageBytes);
  return FALCON_OK;
}

void lane_free(Lane& l) {
  if (l.stream) (void)hipStreamSynchronize(l.stream);
  if (l.offsets) (void)hipFree(l.offsets);
  if (l.tiles) (void)hipFree(l.tiles);
  if (l.meta) (void)hipFree(l.meta);
  if (l.gsizes) (void)hipFree(l.gsizes);
  if (l.status) (void)hipFree(l.status);
  if (l.qctr) (void)hipFree(l.qctr);
  if (l.ctl) (void)hipFree(l.ctl);
  if (l.stage) (void)hipHostFree(l.stage);
  if (l.stream) (void)hipStreamDestroy(l.stream);
  l = Lane();
}

namespace {

// Grows a device array to at least n elements (contents undefined).
template <class P>
falcon_status grow_raw(P** arr, size_t* cap, uint64_t n, hipStream_t s) {
  if (n <= *cap && *arr) return FALCON_OK;
  size_t c = *cap ? *cap : 1024;
  while (c < n) c *= 2;
  if (*arr) {
    if (hipStreamSynchronize(s) != hipSuccess) return FALCON_ERR_DEVICE;
    (void)hipFree(*arr);
  }
  *arr = nullptr;
  *cap = 0;
  if (hipMalloc(reinterpret_cast<void**>(arr), c * sizeof(P)) != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
  *cap = c;
  return FALCON_OK;
}

// Makes the lane's arrays hold nchunks chunk offsets and ntiles scan tile
// sums, and advances the launch epoch (the value a failing decompression
// launch leaves in the error word).
falcon_status prepare_launch(Lane& l, uint64_t nchunks, uint64_t ntiles, hipStream_t s) {
  falcon_status st = grow_raw(&l.offsets, &l.offsets_cap, nchunks, s);
  if (st == FALCON_OK) st = grow_raw(&l.tiles, &l.tiles_cap, ntiles, s);
  if (st != FALCON_OK) return st;
  l.epoch += 1;
  if (l.epoch == 0) l.epoch = 1;
  return FALCON_OK;
}

int grid_for(int max_grid, uint64_t nchunks, int waves_per_block) {
  uint64_t want = (nchunks + waves_per_block - 1) / waves_per_block;
  if (want < 1) want = 1;
  return (int)(want < (uint64_t)max_grid ? want : (uint64_t)max_grid);
}

}  // namespace

// Makes the lane's status array hold nchunks words, picks the tag of the
// next single-pass launch and clears the ticket counters.  The status array
// is cleared when it is (re)allocated and whenever the 16-bit tag wraps, so
// a word left by an earlier launch never carries the current tag.
falcon_status prepare_queue(Lane& l, uint64_t nchunks, hipStream_t s) {
  const size_t old_cap = l.status_cap;
  const uint64_t* old = l.status;
  falcon_status st = grow_raw(&l.status, &l.status_cap, nchunks, s);
  if (st != FALCON_OK) return st;
  l.qtag = (l.qtag + 1) & 0xFFFFu;
  if (l.status != old || l.status_cap != old_cap || l.qtag == 0) {
    if (l.qtag == 0) l.qtag = 1;
    if ((st = dev_err(launch_fill_u64(l.status, l.status_cap, 0, s))) != FALCON_OK) return st;
  }
  return dev_err(launch_fill_u64(l.qctr, (size_t)kQueueGroups * kQueueStride, 0, s));
}

// Moves the timing ring to a fresh slot for a timed call and returns its
// four events; the slot counts as complete once the call has recorded all
// of them.
static hipEvent_t* begin_timed(falcon_ctx* ctx) {
  ctx->ev_slot = (ctx->ev_slot + 1) % FALCON_TIMED_CALLS;
  ctx->ev_ok[ctx->ev_slot] = false;
  return ctx->ev[ctx->ev_slot];
}

// Compression, in one of two forms.  Two passes (the default, and the
// only form of the ablation variants): a size pass, a scan of the chunk
// sizes into offsets, a write pass that redoes a4-a7 and writes each chunk
// at its offset.  Single pass: one launch in which waves take chunks from
// a work queue and find their offsets with a decoupled look-back (see
// codec_kernels.hpp).  Both give the same stream.
falcon_status enqueue_compress(falcon_ctx* ctx, Lane& l, const void* d_in, uint64_t n, falcon_dtype dt, void* d_out,
                               hipStream_t s, bool timed, int variant, int form, uint64_t* d_len) {
  const uint64_t nc = chunks_of(n);
  falcon_status st = FALCON_OK;
  CompressArgs a{};
  a.one.in = d_in;
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.dtype = (uint32_t)dt;
  a.one.idx = 0;
  a.many = nullptr;
  a.nseries = 1;
  a.total_chunks = nc;
  a.lens = d_len;
  a.relative = 0;
  hipEvent_t* ev = timed ? begin_timed(ctx) : nullptr;
  auto mark = [&](int i) { return timed ? dev_err(hipEventRecord(ev[i], s)) : FALCON_OK; };
  if (variant == 0 && form == FALCON_FORM_SINGLE_PASS) {
    if ((st = mark(0)) != FALCON_OK || (st = prepare_queue(l, nc ? nc : 1, s)) != FALCON_OK) return st;
    const int nw = kCompressWaves;
    const int grid = grid_for(max_grid_q(ctx, dt, nw), nc, nw);
    a.total_waves = (uint32_t)(grid * nw);
    a.status = l.status;
    a.qctr = l.qctr;
    a.qgroups = (uint32_t)(grid < kQueueGroups ? grid : kQueueGroups);
    a.ctl = l.ctl;
    a.qtag = l.qtag;
    if ((st = dev_err(launch_compress_queue(a, (int)dt, nw, grid, s))) != FALCON_OK) return st;
    if ((st = mark(1)) != FALCON_OK || (st = mark(2)) != FALCON_OK || (st = mark(3)) != FALCON_OK) return st;
  } else {
    st = prepare_launch(l, nc ? nc : 1, scan_tiles(nc) + 1, s);
    if (st == FALCON_OK) st = grow_raw(&l.meta, &l.meta_cap, nc ? nc : 1, s);
    if (st == FALCON_OK) st = grow_raw(&l.gsizes, &l.gsizes_cap, nc ? nc : 1, s);
    if (st != FALCON_OK) return st;
    a.meta = l.meta;
    a.gsizes = l.gsizes;
    a.offsets = l.offsets;
    const int nw = variant ? kVariantWaves : compress_waves((int)dt);
    const int g1 = grid_for(variant ? ctx->grid_v[dt][variant][1] : max_grid_c(ctx, dt, 1, nw), nc, nw);
    const int g2 = grid_for(variant ? ctx->grid_v[dt][variant][2] : max_grid_c(ctx, dt, 2, nw), nc, nw);
    auto launch = [&](int pass, int grid) {
      a.total_waves = (uint32_t)(grid * nw);
      return dev_err(variant ? launch_compress_variant(a, (int)dt, variant, pass, grid, s)
                             : launch_compress(a, (int)dt, pass, nw, grid, s));
    };
    if ((st = mark(0)) != FALCON_OK) return st;
    if (nc && (st = launch(1, g1)) != FALCON_OK) return st;
    if ((st = mark(1)) != FALCON_OK) return st;
    if (nc && (st = dev_err(launch_scan_sizes(l.gsizes, nc, 0, ~0u, ~0ull, l.tiles, l.offsets, l.ctl, l.epoch,
                                              s))) != FALCON_OK)
      return st;
    if ((st = mark(2)) != FALCON_OK) return st;
    if ((st = launch(2, g2)) != FALCON_OK) return st;
    if ((st = mark(3)) != FALCON_OK) return st;
  }
  if (timed) ctx->ev_ok[ctx->ev_slot] = true;
  return FALCON_OK;
}

falcon_status enqueue_decompress(falcon_ctx* ctx, Lane& l, const uint8_t* d_in, uint64_t in_len, uint64_t n,
                                 falcon_dtype dt, uint64_t payload, void* d_out, hipStream_t s, bool timed,
                                 bool copy_error) {
  const uint64_t nc = chunks_of(n);
  falcon_status st = prepare_launch(l, nc, scan_tiles(nc) + 1, s);
  if (st != FALCON_OK) return st;
  // chunk offsets: exclusive prefix of the size array (which the scan also
  // checks: every size in [lo, hi], and their sum equal to the payload byte
  // count when the host knows it; otherwise the last chunk's check does that)
  const uint32_t lo = dt == FALCON_FLOAT64 ? 11u : 7u;
  const uint32_t hi = (uint32_t)max_chunk_bytes(dt);
  hipEvent_t* ev = timed ? begin_timed(ctx) : nullptr;
  auto mark = [&](int i) { return timed ? dev_err(hipEventRecord(ev[i], s)) : FALCON_OK; };
  if ((st = mark(0)) != FALCON_OK || (st = mark(1)) != FALCON_OK) return st;
  if ((st = dev_err(launch_scan_sizes(reinterpret_cast<const uint32_t*>(d_in + 32), nc, lo, hi,
                                      payload == kPayloadFromHeader ? ~0ull : payload, l.tiles, l.offsets, l.ctl,
                                      l.epoch, s))) != FALCON_OK)
    return st;
  DecompressArgs a{};
  a.one.in = d_in;
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.payload_bytes = payload;
  a.one.in_len = in_len;
  a.one.dtype = (uint32_t)dt;
  a.many = nullptr;
  a.nseries = 1;
  a.total_chunks = nc;
  a.offsets = l.offsets;
  a.ctl = l.ctl;
  a.epoch = l.epoch;
  a.relative = 0;
  const int grid = grid_for(max_grid_d(ctx, dt), nc, kDecompressWaves);
  a.total_waves = (uint32_t)(grid * kDecompressWaves);
  if ((st = mark(2)) != FALCON_OK) return st;
  if ((st = dev_err(launch_decompress(a, (int)dt, grid, s))) != FALCON_OK) return st;
  if ((st = mark(3)) != FALCON_OK) return st;
  if (timed) ctx->ev_ok[ctx->ev_slot] = true;
  if (!copy_error) return FALCON_OK;
  return dev_err(hipMemcpyAsync(l.stage + 32, &l.ctl->error, 4, hipMemcpyDeviceToHost, s));
}

namespace {

// ---- asynchronous device calls --------------------------------------------
// A device call runs in three steps: begin_call (stream choice, ordering
// after the previous call), the enqueue, end_call (records the call's end,
// and with FALCON_OPT_BLOCKING synchronises and reports at once).

hipStream_t call_stream(falcon_ctx* ctx, void* stream) {
  return stream ? static_cast<hipStream_t>(stream) : ctx->main.stream;
}

falcon_status begin_call(falcon_ctx* ctx, hipStream_t s) {
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  if (ctx->last_stream && ctx->last_stream != s && hipStreamWaitEvent(s, ctx->ev_done, 0) != hipSuccess)
    return FALCON_ERR_DEVICE;
  return FALCON_OK;
}

falcon_status end_call(falcon_ctx* ctx, hipStream_t s, falcon_status st) {
  // the work enqueued so far is recorded even after an error, so that a
  // later call or falcon_sync still orders after it
  if (hipEventRecord(ctx->ev_done, s) != hipSuccess && st == FALCON_OK) st = FALCON_ERR_DEVICE;
  ctx->last_stream = s;
  ctx->unsynced = true;
  if (ctx->opt_flags & FALCON_OPT_BLOCKING) {
    const falcon_status sy = falcon_sync(ctx);
    if (st == FALCON_OK) st = sy;
  }
  return st;
}

// A device word that the kernels of one compression fill with its stream
// length, reported to *dst at falcon_sync.
falcon_status pending_length(falcon_ctx* ctx, size_t* dst, uint64_t** d_len) {
  const size_t slot = ctx->pending.size();
  const size_t b = slot / kLenBlock;
  if (b == ctx->len_blocks.size()) {
    void* p = nullptr;
    if (hipMalloc(&p, kLenBlock * 8) != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
    ctx->len_blocks.push_back(static_cast<uint64_t*>(p));
  }
  *d_len = ctx->len_blocks[b] + slot % kLenBlock;
  ctx->pending.push_back({dst, slot});
  return FALCON_OK;
}

// Writes 32 (the stream length of n = 0, which no kernel writes) to a
// device length word.
falcon_status empty_length(uint64_t* d_len, hipStream_t s) { return dev_err(launch_fill_u64(d_len, 1, 32, s)); }

}  // namespace

}  // namespace falcon_host

using namespace falcon_host;

extern "C" {

const char* falcon_status_str(falcon_status st) {
  switch (st) {
    case FALCON_OK: return "ok";
    case FALCON_ERR_INVALID_ARG: return "invalid argument";
    case FALCON_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case FALCON_ERR_CORRUPT_STREAM: return "corrupt stream";
    case FALCON_ERR_DEVICE: return "device error";
    case FALCON_ERR_OUT_OF_MEMORY: return "out of memory";
  }
  return "unknown status";
}

size_t falcon_compress_bound(size_t n, falcon_dtype dt) {
  const size_t per = max_chunk_bytes(dt);
  if (per == 0) return 0;
  return 32 + chunks_of(n) * (4 + per);
}

falcon_status falcon_create(int device, const falcon_opts* opts, falcon_ctx** out) {
  if (!out) return FALCON_ERR_INVALID_ARG;
  *out = nullptr;
  const unsigned flags = opts ? opts->flags : 0u;
  const int form = opts ? opts->compress_form : 0;
  if ((flags & ~(unsigned)(FALCON_OPT_BLOCKING | FALCON_OPT_DEVICE_LENGTHS)) ||
      (form != FALCON_FORM_TWO_PASS && form != FALCON_FORM_SINGLE_PASS))
    return FALCON_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FALCON_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FALCON_ERR_DEVICE;
  falcon_ctx* ctx = new (std::nothrow) falcon_ctx();
  if (!ctx) return FALCON_ERR_OUT_OF_MEMORY;
  ctx->device = device;
  ctx->opt_flags = flags;
  ctx->compress_form = form;
  bool ok = lane_init(ctx->main) == FALCON_OK &&
            hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming) == hipSuccess;
  for (int c = 0; ok && c < FALCON_TIMED_CALLS; ++c)
    for (int i = 0; ok && i < 4; ++i) ok = hipEventCreate(&ctx->ev[c][i]) == hipSuccess;
  if (!ok) {
    falcon_destroy(ctx);
    return FALCON_ERR_DEVICE;
  }
  for (int form_ = 1; form_ <= 3; ++form_) {
    for (int pass = 1; pass <= 2; ++pass) {
      ctx->grid_c[form_][pass][0] = max_grid_compress(device, form_, pass, 8);
      ctx->grid_c[form_][pass][1] = max_grid_compress(device, form_, pass, 16);
    }
    ctx->grid_d[form_] = max_grid_decompress(device, form_);
    ctx->grid_q[form_][0] = max_grid_compress_queue(device, form_, 8);
    ctx->grid_q[form_][1] = max_grid_compress_queue(device, form_, 16);
  }
  for (int f = 1; f <= 2; ++f)
    for (int v = 1; v <= 3; ++v)
      for (int pass = 1; pass <= 2; ++pass) ctx->grid_v[f][v][pass] = max_grid_compress_variant(device, f, v, pass);
  if (noalloc_setup(device) != FALCON_OK) {
    falcon_destroy(ctx);
    return FALCON_ERR_DEVICE;
  }
  *out = ctx;
  return FALCON_OK;
}

falcon_status falcon_sync(falcon_ctx* ctx) {
  if (!ctx) return FALCON_ERR_INVALID_ARG;
  if (!ctx->unsynced) return FALCON_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  Lane& l = ctx->main;
  hipStream_t s = ctx->last_stream;
  falcon_status st = FALCON_OK;
  const size_t np = ctx->pending.size();
  if (np > ctx->len_host_cap) {
    // grown only here, when no copy into it is in flight
    if (hipStreamSynchronize(s) != hipSuccess) st = FALCON_ERR_DEVICE;
    if (ctx->len_host) (void)hipHostFree(ctx->len_host);
    ctx->len_host = nullptr;
    ctx->len_host_cap = 0;
    size_t cap = kLenBlock;
    while (cap < np) cap *= 2;
    void* p = nullptr;
    if (hipHostMalloc(&p, cap * 8, hipHostMallocDefault) != hipSuccess) {
      st = FALCON_ERR_OUT_OF_MEMORY;
    } else {
      ctx->len_host = static_cast<uint64_t*>(p);
      ctx->len_host_cap = cap;
    }
  }
  for (size_t b = 0; st == FALCON_OK && b * kLenBlock < np; ++b) {
    const size_t k = np - b * kLenBlock < kLenBlock ? np - b * kLenBlock : kLenBlock;
    st = dev_err(hipMemcpyAsync(ctx->len_host + b * kLenBlock, ctx->len_blocks[b], k * 8, hipMemcpyDeviceToHost, s));
  }
  if (st == FALCON_OK) st = dev_err(hipMemcpyAsync(l.stage + 32, l.ctl, 8, hipMemcpyDeviceToHost, s));
  const falcon_status sy = dev_err(hipStreamSynchronize(s));
  if (st == FALCON_OK) st = sy;
  if (st == FALCON_OK) {
    for (const auto& p : ctx->pending) *p.dst = (size_t)ctx->len_host[p.slot];
    // the decompression error word holds the epoch of the last launch whose
    // chunk failed: a launch since the last sync has a larger one
    const uint32_t err = rd32(l.stage + 32);
    if (err != 0 && err > ctx->sync_epoch && err <= l.epoch) st = FALCON_ERR_CORRUPT_STREAM;
    if (rd32(l.stage + 36) != 0) {
      (void)launch_fill_u64(reinterpret_cast<uint64_t*>(l.ctl), 1, 0, s);
      (void)hipStreamSynchronize(s);
      st = FALCON_ERR_DEVICE;
    }
  }
  ctx->pending.clear();
  ctx->sync_epoch = l.epoch;
  ctx->unsynced = false;
  return st;
}

void falcon_destroy(falcon_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  pipe_release(ctx);
  if (ctx->main.stream) (void)hipStreamSynchronize(ctx->main.stream);
  if (ctx->last_stream) (void)hipStreamSynchronize(ctx->last_stream);
  batch_free(ctx->batch);
  lane_free(ctx->main);
  for (auto& call : ctx->ev)
    for (hipEvent_t e : call)
      if (e) (void)hipEventDestroy(e);
  if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
  for (uint64_t* b : ctx->len_blocks) (void)hipFree(b);
  if (ctx->len_host) (void)hipHostFree(ctx->len_host);
  delete ctx;
}

falcon_status falcon_stream_info(const void* h_hdr, size_t len, size_t* n, falcon_dtype* dt) {
  if (!h_hdr || !n || !dt) return FALCON_ERR_INVALID_ARG;
  const uint8_t* h = static_cast<const uint8_t*>(h_hdr);
  if (len < 32 || memcmp(h, "FLCN", 4) != 0 || h[4] != 1 || (h[5] != 1 && h[5] != 2) || h[6] || h[7] ||
      rd32(h + 8) != kChunkN || rd32(h + 12) != 0)
    return FALCON_ERR_CORRUPT_STREAM;
  *n = (size_t)rd64(h + 16);
  *dt = (falcon_dtype)h[5];
  return FALCON_OK;
}

falcon_status falcon_compress(falcon_ctx* ctx, const void* d_in, size_t n, falcon_dtype dt, void* d_out,
                              size_t out_cap, size_t* out_len, void* stream) {
  return falcon_compress_variant(ctx, d_in, n, dt, FALCON_VARIANT_FALCON, d_out, out_cap, out_len, stream);
}

size_t falcon_compress_bound_variant(size_t n, falcon_dtype dt, falcon_variant v) {
  if (v < FALCON_VARIANT_FALCON || v > FALCON_VARIANT_DENSE) return 0;
  if (v != FALCON_VARIANT_SPARSE) return falcon_compress_bound(n, dt);
  const size_t per = dt == FALCON_FLOAT64 ? 11 + 8 + 64 * 144 : dt == FALCON_FLOAT32 ? 7 + 4 + 32 * 144 : 0;
  if (per == 0) return 0;
  return 32 + chunks_of(n) * (4 + per);
}

falcon_status falcon_compress_variant(falcon_ctx* ctx, const void* d_in, size_t n, falcon_dtype dt, falcon_variant v,
                                      void* d_out, size_t out_cap, size_t* out_len, void* stream) {
  if (!ctx || !d_out || !out_len || (n && !d_in)) return FALCON_ERR_INVALID_ARG;
  if (v < FALCON_VARIANT_FALCON || v > FALCON_VARIANT_DENSE) return FALCON_ERR_INVALID_ARG;
  const size_t es = elem_size(dt);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  if (((uintptr_t)d_in % es) || ((uintptr_t)d_out % 4)) return FALCON_ERR_INVALID_ARG;
  const bool dev_len = (ctx->opt_flags & FALCON_OPT_DEVICE_LENGTHS) != 0;
  if (dev_len && ((uintptr_t)out_len % 8)) return FALCON_ERR_INVALID_ARG;
  if (out_cap < falcon_compress_bound_variant(n, dt, v)) return FALCON_ERR_BUFFER_TOO_SMALL;
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull) return FALCON_ERR_INVALID_ARG;
  hipStream_t s = call_stream(ctx, stream);
  falcon_status st = begin_call(ctx, s);
  if (st != FALCON_OK) return st;
  uint64_t* d_len = nullptr;
  if (dev_len) d_len = reinterpret_cast<uint64_t*>(out_len);
  else if (n) st = pending_length(ctx, out_len, &d_len);
  else *out_len = 32;
  if (st == FALCON_OK)
    st = enqueue_compress(ctx, ctx->main, d_in, n, dt, d_out, s, true, (int)v, ctx->compress_form, d_len);
  if (st == FALCON_OK && dev_len && n == 0) st = empty_length(d_len, s);
  return end_call(ctx, s, st);
}

falcon_status falcon_decompress_n(falcon_ctx* ctx, const void* d_in, size_t in_len, size_t n, falcon_dtype dt,
                                  void* d_out, size_t out_cap_bytes, void* stream) {
  if (!ctx || !d_in || ((uintptr_t)d_in % 4)) return FALCON_ERR_INVALID_ARG;
  const size_t es = elem_size(dt);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull || in_len < 32 || (in_len - 32) / 4 < nc) return FALCON_ERR_CORRUPT_STREAM;
  if (out_cap_bytes / es < n) return FALCON_ERR_BUFFER_TOO_SMALL;
  if (n && (!d_out || ((uintptr_t)d_out % es))) return FALCON_ERR_INVALID_ARG;
  hipStream_t s = call_stream(ctx, stream);
  falcon_status st = begin_call(ctx, s);
  if (st != FALCON_OK) return st;
  // an empty stream has no chunk to check its header: nothing to launch
  if (n) st = enqueue_decompress(ctx, ctx->main, static_cast<const uint8_t*>(d_in), in_len, n, dt,
                                 kPayloadFromHeader, d_out, s, true, false);
  return end_call(ctx, s, st);
}

falcon_status falcon_decompress(falcon_ctx* ctx, const void* d_in, size_t in_len, void* d_out, size_t out_cap_bytes,
                                size_t* n_out, void* stream) {
  if (!ctx || !d_in || !n_out || ((uintptr_t)d_in % 4)) return FALCON_ERR_INVALID_ARG;
  if (in_len < 32) return FALCON_ERR_CORRUPT_STREAM;
  Lane& l = ctx->main;
  hipStream_t s = call_stream(ctx, stream);
  falcon_status st = begin_call(ctx, s);
  if (st != FALCON_OK) return st;
  // the header, read after the work already on the stream
  if ((st = dev_err(hipMemcpyAsync(l.stage, d_in, 32, hipMemcpyDeviceToHost, s))) != FALCON_OK ||
      (st = dev_err(hipStreamSynchronize(s))) != FALCON_OK)
    return end_call(ctx, s, st);
  size_t n = 0;
  falcon_dtype dt;
  if ((st = falcon_stream_info(l.stage, 32, &n, &dt)) != FALCON_OK) return end_call(ctx, s, st);
  const uint64_t payload = rd64(l.stage + 24);
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull || (in_len - 32) / 4 < nc || payload > in_len - 32 - 4 * nc ||
      (n == 0 && payload != 0))
    return end_call(ctx, s, FALCON_ERR_CORRUPT_STREAM);
  *n_out = n;
  const size_t es = elem_size(dt);
  if (out_cap_bytes / es < n) return end_call(ctx, s, FALCON_ERR_BUFFER_TOO_SMALL);
  if (n && (!d_out || ((uintptr_t)d_out % es))) return end_call(ctx, s, FALCON_ERR_INVALID_ARG);
  if (n)
    st = enqueue_decompress(ctx, l, static_cast<const uint8_t*>(d_in), in_len, n, dt, payload, d_out, s, true, false);
  return end_call(ctx, s, st);
}

// The one-series-per-launch path over many series: one asynchronous call per
// series, lengths written by the kernels to a device array, one wait.
falcon_status falcon_compress_each(falcon_ctx* ctx, falcon_series* ss, size_t count, void* stream) {
  if (!ctx || (count && !ss)) return FALCON_ERR_INVALID_ARG;
  for (size_t i = 0; i < count; ++i) {
    const falcon_status st = batch_check(FALCON_OP_COMPRESS, ss[i]);
    if (st != FALCON_OK) return st;
  }
  if (count == 0) return FALCON_OK;
  hipStream_t s = call_stream(ctx, stream);
  falcon_status st = begin_call(ctx, s);
  if (st != FALCON_OK) return st;
  std::vector<uint64_t*> dl(count);
  for (size_t i = 0; i < count && st == FALCON_OK; ++i) {
    st = pending_length(ctx, &ss[i].out_len, &dl[i]);
    if (st == FALCON_OK)
      st = enqueue_compress(ctx, ctx->main, ss[i].d_in, ss[i].n, ss[i].dtype, ss[i].d_out, s, false, 0,
                            ctx->compress_form, dl[i]);
    if (st == FALCON_OK && ss[i].n == 0) st = empty_length(dl[i], s);
  }
  st = end_call(ctx, s, st);
  const falcon_status sy = falcon_sync(ctx);
  return st != FALCON_OK ? st : sy;
}

falcon_status falcon_decompress_each(falcon_ctx* ctx, falcon_series* ss, size_t count, void* stream) {
  if (!ctx || (count && !ss)) return FALCON_ERR_INVALID_ARG;
  for (size_t i = 0; i < count; ++i) {
    const falcon_status st = batch_check(FALCON_OP_DECOMPRESS, ss[i]);
    if (st != FALCON_OK) return st;
  }
  if (count == 0) return FALCON_OK;
  hipStream_t s = call_stream(ctx, stream);
  falcon_status st = begin_call(ctx, s);
  if (st != FALCON_OK) return st;
  for (size_t i = 0; i < count && st == FALCON_OK; ++i) {
    if (ss[i].n)
      st = enqueue_decompress(ctx, ctx->main, static_cast<const uint8_t*>(ss[i].d_in), ss[i].in_len, ss[i].n,
                              ss[i].dtype, kPayloadFromHeader, ss[i].d_out, s, false, false);
    ss[i].out_len = ss[i].n;
  }
  st = end_call(ctx, s, st);
  const falcon_status sy = falcon_sync(ctx);
  return st != FALCON_OK ? st : sy;
}

falcon_status falcon_call_stage_ms(falcon_ctx* ctx, unsigned back, float* ms) {
  if (!ctx || !ms || back >= FALCON_TIMED_CALLS) return FALCON_ERR_INVALID_ARG;
  const int slot = (ctx->ev_slot + FALCON_TIMED_CALLS - (int)back) % FALCON_TIMED_CALLS;
  if (!ctx->ev_ok[slot]) return FALCON_ERR_INVALID_ARG;
  hipEvent_t* ev = ctx->ev[slot];
  if (hipEventSynchronize(ev[3]) != hipSuccess) return FALCON_ERR_DEVICE;
  for (int i = 0; i < 3; ++i)
    if (hipEventElapsedTime(ms + i, ev[i], ev[i + 1]) != hipSuccess) return FALCON_ERR_DEVICE;
  return FALCON_OK;
}

falcon_status falcon_last_stage_ms(falcon_ctx* ctx, float* ms) { return falcon_call_stage_ms(ctx, 0, ms); }

falcon_status falcon_last_kernel_ms(falcon_ctx* ctx, float* ms) {
  if (!ms) return FALCON_ERR_INVALID_ARG;
  float st[3];
  const falcon_status s = falcon_call_stage_ms(ctx, 0, st);
  if (s == FALCON_OK) *ms = st[0] + st[1] + st[2];
  return s;
}

}  // extern "C"
