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

// Two-pass compression: size pass, scan of the sizes, write pass (see
// codec_kernels.hpp).  The lane's offset array receives the scan.
falcon_status enqueue_compress(falcon_ctx* ctx, Lane& l, const void* d_in, uint64_t n, falcon_dtype dt, void* d_out,
                               hipStream_t s, bool timed, int variant) {
  const uint64_t nc = chunks_of(n);
  falcon_status st = prepare_launch(l, nc ? nc : 1, scan_tiles(nc) + 1, s);
  if (st == FALCON_OK) st = grow_raw(&l.meta, &l.meta_cap, nc ? nc : 1, s);
  if (st == FALCON_OK) st = grow_raw(&l.gsizes, &l.gsizes_cap, nc ? nc : 1, s);
  if (st != FALCON_OK) return st;
  CompressArgs a{};
  a.one.in = d_in;
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.dtype = (uint32_t)dt;
  a.many = nullptr;
  a.nseries = 1;
  a.total_chunks = nc;
  a.lens = nullptr;
  a.meta = l.meta;
  a.gsizes = l.gsizes;
  a.offsets = l.offsets;
  a.relative = 0;
  const int nw = variant ? kVariantWaves : kCompressWaves;
  const int g1 = grid_for(variant ? ctx->grid_v[dt][variant][1] : max_grid_c(ctx, dt, 1, nw), nc, nw);
  const int g2 = grid_for(variant ? ctx->grid_v[dt][variant][2] : max_grid_c(ctx, dt, 2, nw), nc, nw);
  auto launch = [&](int pass, int grid) {
    a.total_waves = (uint32_t)(grid * nw);
    return dev_err(variant ? launch_compress_variant(a, (int)dt, variant, pass, grid, s)
                           : launch_compress(a, (int)dt, pass, nw, grid, s));
  };
  auto mark = [&](int i) { return timed ? dev_err(hipEventRecord(ctx->ev[i], s)) : FALCON_OK; };
  if (timed) ctx->timed = false;
  if ((st = mark(0)) != FALCON_OK) return st;
  if (nc && (st = launch(1, g1)) != FALCON_OK) return st;
  if ((st = mark(1)) != FALCON_OK) return st;
  if (nc && (st = dev_err(launch_scan_sizes(l.gsizes, nc, 0, ~0u, ~0ull, l.tiles, l.offsets, l.ctl, l.epoch, s))) !=
                FALCON_OK)
    return st;
  if ((st = mark(2)) != FALCON_OK) return st;
  if ((st = launch(2, g2)) != FALCON_OK) return st;
  if ((st = mark(3)) != FALCON_OK) return st;
  if (timed) {
    ctx->timed = true;
    ctx->timed_compress = true;
  }
  return FALCON_OK;
}

falcon_status enqueue_decompress(falcon_ctx* ctx, Lane& l, const uint8_t* d_in, uint64_t n, falcon_dtype dt,
                                 uint64_t payload, void* d_out, hipStream_t s, bool timed) {
  const uint64_t nc = chunks_of(n);
  falcon_status st = prepare_launch(l, nc, scan_tiles(nc) + 1, s);
  if (st != FALCON_OK) return st;
  // chunk offsets: exclusive prefix of the size array (which the scan also
  // checks: every size in [lo, hi], their sum equal to the payload bytes).
  const uint32_t lo = dt == FALCON_FLOAT64 ? 11u : 7u;
  const uint32_t hi = (uint32_t)max_chunk_bytes(dt);
  auto mark = [&](int i) { return timed ? dev_err(hipEventRecord(ctx->ev[i], s)) : FALCON_OK; };
  if (timed) ctx->timed = false;
  if ((st = mark(0)) != FALCON_OK || (st = mark(1)) != FALCON_OK) return st;
  if ((st = dev_err(launch_scan_sizes(reinterpret_cast<const uint32_t*>(d_in + 32), nc, lo, hi, payload, l.tiles,
                                      l.offsets, l.ctl, l.epoch, s))) != FALCON_OK)
    return st;
  DecompressArgs a{};
  a.one.in = d_in;
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.payload_bytes = payload;
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
  if (timed) {
    ctx->timed = true;
    ctx->timed_compress = false;
  }
  return dev_err(hipMemcpyAsync(l.stage + 32, &l.ctl->error, 4, hipMemcpyDeviceToHost, s));
}

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

falcon_status falcon_create(int device, falcon_ctx** out) {
  if (!out) return FALCON_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FALCON_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FALCON_ERR_DEVICE;
  falcon_ctx* ctx = new (std::nothrow) falcon_ctx();
  if (!ctx) return FALCON_ERR_OUT_OF_MEMORY;
  ctx->device = device;
  if (lane_init(ctx->main) != FALCON_OK || hipEventCreate(&ctx->ev[0]) != hipSuccess ||
      hipEventCreate(&ctx->ev[1]) != hipSuccess || hipEventCreate(&ctx->ev[2]) != hipSuccess ||
      hipEventCreate(&ctx->ev[3]) != hipSuccess) {
    falcon_destroy(ctx);
    return FALCON_ERR_DEVICE;
  }
  for (int form = 1; form <= 3; ++form) {
    for (int pass = 1; pass <= 2; ++pass) {
      ctx->grid_c[form][pass][0] = max_grid_compress(device, form, pass, 8);
      ctx->grid_c[form][pass][1] = max_grid_compress(device, form, pass, 16);
    }
    ctx->grid_d[form] = max_grid_decompress(device, form);
  }
  for (int form = 1; form <= 2; ++form)
    for (int v = 1; v <= 3; ++v)
      for (int pass = 1; pass <= 2; ++pass) ctx->grid_v[form][v][pass] = max_grid_compress_variant(device, form, v, pass);
  *out = ctx;
  return FALCON_OK;
}

void falcon_destroy(falcon_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  pipe_release(ctx);
  if (ctx->main.stream) (void)hipStreamSynchronize(ctx->main.stream);
  batch_free(ctx->batch);
  lane_free(ctx->main);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
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
  if (out_cap < falcon_compress_bound_variant(n, dt, v)) return FALCON_ERR_BUFFER_TOO_SMALL;
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull) return FALCON_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  Lane& l = ctx->main;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : l.stream;
  falcon_status st = enqueue_compress(ctx, l, d_in, n, dt, d_out, s, true, (int)v);
  if (st != FALCON_OK) return st;
  if ((st = dev_err(hipMemcpyAsync(l.stage + 40, static_cast<uint8_t*>(d_out) + 24, 8, hipMemcpyDeviceToHost, s))) !=
      FALCON_OK)
    return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  *out_len = 32 + 4 * nc + rd64(l.stage + 40);
  return FALCON_OK;
}

falcon_status falcon_decompress(falcon_ctx* ctx, const void* d_in, size_t in_len, void* d_out, size_t out_cap_bytes,
                                size_t* n_out, void* stream) {
  if (!ctx || !d_in || !n_out || ((uintptr_t)d_in % 4)) return FALCON_ERR_INVALID_ARG;
  if (in_len < 32) return FALCON_ERR_CORRUPT_STREAM;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  Lane& l = ctx->main;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : l.stream;
  falcon_status st;
  if ((st = dev_err(hipMemcpyAsync(l.stage, d_in, 32, hipMemcpyDeviceToHost, s))) != FALCON_OK) return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  size_t n = 0;
  falcon_dtype dt;
  if ((st = falcon_stream_info(l.stage, 32, &n, &dt)) != FALCON_OK) return st;
  const uint64_t payload = rd64(l.stage + 24);
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull || (in_len - 32) / 4 < nc || payload > in_len - 32 - 4 * nc)
    return FALCON_ERR_CORRUPT_STREAM;
  *n_out = n;
  const size_t es = elem_size(dt);
  if (out_cap_bytes / es < n) return FALCON_ERR_BUFFER_TOO_SMALL;
  if (n == 0) return payload == 0 ? FALCON_OK : FALCON_ERR_CORRUPT_STREAM;
  if (!d_out || ((uintptr_t)d_out % es)) return FALCON_ERR_INVALID_ARG;
  if ((st = enqueue_decompress(ctx, l, static_cast<const uint8_t*>(d_in), n, dt, payload, d_out, s, true)) !=
      FALCON_OK)
    return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  return decompress_failed(l) ? FALCON_ERR_CORRUPT_STREAM : FALCON_OK;
}

falcon_status falcon_last_kernel_ms(falcon_ctx* ctx, float* ms) {
  if (!ctx || !ms || !ctx->timed) return FALCON_ERR_INVALID_ARG;
  if (hipEventSynchronize(ctx->ev[3]) != hipSuccess) return FALCON_ERR_DEVICE;
  return dev_err(hipEventElapsedTime(ms, ctx->ev[ctx->timed_compress ? 0 : 2], ctx->ev[3]));
}

falcon_status falcon_last_stage_ms(falcon_ctx* ctx, float* ms) {
  if (!ctx || !ms || !ctx->timed) return FALCON_ERR_INVALID_ARG;
  if (hipEventSynchronize(ctx->ev[3]) != hipSuccess) return FALCON_ERR_DEVICE;
  for (int i = 0; i < 3; ++i)
    if (hipEventElapsedTime(ms + i, ctx->ev[i], ctx->ev[i + 1]) != hipSuccess) return FALCON_ERR_DEVICE;
  return FALCON_OK;
}

}  // extern "C"
