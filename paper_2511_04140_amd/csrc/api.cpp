// api.cpp -- C ABI of the Falcon codec (declared in include/falcon.h).
//
// A context owns one HIP stream, a small pinned staging buffer for the
// few bytes read back per call, the per-chunk status words of the
// decoupled look-back and the launch control block.  Status words carry a
// 16-bit launch epoch, so they are cleared only when the array grows or the
// epoch wraps.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "../../include/falcon.h"
#include "internal.hpp"

using namespace falcon_dev;

namespace {
constexpr uint64_t kChunkN = 1025;
constexpr size_t kF64Chunk = 8211, kF32Chunk = 4107;

size_t elem_size(falcon_dtype dt) { return dt == FALCON_FLOAT64 ? 8 : dt == FALCON_FLOAT32 ? 4 : 0; }

uint32_t rd32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
uint64_t rd64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }
}  // namespace

struct falcon_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t* status = nullptr;   // look-back status words, one per chunk
  size_t status_cap = 0;
  uint64_t* gstatus = nullptr;  // one per 64-chunk group
  size_t gstatus_cap = 0;
  Ctl* ctl = nullptr;           // device control block
  uint8_t* stage = nullptr;     // pinned host staging (64 bytes)
  uint32_t epoch = 0;
  int grid_c[3] = {0, 0, 0};   // co-resident workgroups per kernel, by dtype
  int grid_d[3] = {0, 0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the last kernel launch
  bool timed = false;
};

namespace {

falcon_status dev_err(hipError_t e) { return e == hipSuccess ? FALCON_OK : FALCON_ERR_DEVICE; }

// Grows a zeroed status array to at least n words.
falcon_status grow_zeroed(uint64_t** arr, size_t* cap, uint64_t n, hipStream_t s) {
  if (n <= *cap) return FALCON_OK;
  size_t c = *cap ? *cap : 1024;
  while (c < n) c *= 2;
  // the stream may still use the old array: wait before freeing it
  if (hipStreamSynchronize(s) != hipSuccess) return FALCON_ERR_DEVICE;
  if (*arr) (void)hipFree(*arr);
  *arr = nullptr;
  *cap = 0;
  if (hipMalloc(arr, c * sizeof(uint64_t)) != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
  *cap = c;
  return launch_fill_u64(*arr, c, 0, s) == hipSuccess ? FALCON_OK : FALCON_ERR_DEVICE;
}

// Makes the status arrays hold nchunks chunk words and ngroups group words,
// and advances the launch epoch.
falcon_status prepare_launch(falcon_ctx* ctx, uint64_t nchunks, uint64_t ngroups, hipStream_t s) {
  falcon_status st = grow_zeroed(&ctx->status, &ctx->status_cap, nchunks, s);
  if (st == FALCON_OK) st = grow_zeroed(&ctx->gstatus, &ctx->gstatus_cap, ngroups, s);
  if (st != FALCON_OK) return st;
  ctx->epoch += 1;
  if ((ctx->epoch & 0xFFFF) == 0) {  // epoch tag wrapped: clear old words
    ctx->epoch += 1;
    if (launch_fill_u64(ctx->status, ctx->status_cap, 0, s) != hipSuccess ||
        launch_fill_u64(ctx->gstatus, ctx->gstatus_cap, 0, s) != hipSuccess)
      return FALCON_ERR_DEVICE;
  }
  return FALCON_OK;
}

uint64_t groups_of(uint64_t nchunks) { return (nchunks + 63) / 64; }

int grid_for(int max_grid, uint64_t nchunks, int waves_per_block) {
  uint64_t want = (nchunks + waves_per_block - 1) / waves_per_block;
  if (want < 1) want = 1;
  return (int)(want < (uint64_t)max_grid ? want : (uint64_t)max_grid);
}

}  // namespace

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
  const size_t per = dt == FALCON_FLOAT64 ? kF64Chunk : dt == FALCON_FLOAT32 ? kF32Chunk : 0;
  if (per == 0) return 0;
  const size_t nc = (n + kChunkN - 1) / kChunkN;
  return 32 + nc * (4 + per);
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
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&ctx->ctl, 64) != hipSuccess || hipMemset(ctx->ctl, 0, 64) != hipSuccess ||
      hipHostMalloc(&ctx->stage, 64, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
    falcon_destroy(ctx);
    return FALCON_ERR_DEVICE;
  }
  for (int dt = 1; dt <= 2; ++dt) {
    ctx->grid_c[dt] = max_grid_compress(device, dt);
    ctx->grid_d[dt] = max_grid_decompress(device, dt);
  }
  *out = ctx;
  return FALCON_OK;
}

void falcon_destroy(falcon_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->status) (void)hipFree(ctx->status);
  if (ctx->gstatus) (void)hipFree(ctx->gstatus);
  if (ctx->ctl) (void)hipFree(ctx->ctl);
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
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
  if (!ctx || !d_out || !out_len || (n && !d_in)) return FALCON_ERR_INVALID_ARG;
  const size_t es = elem_size(dt);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  if (((uintptr_t)d_in % es) || ((uintptr_t)d_out % 4)) return FALCON_ERR_INVALID_ARG;
  if (out_cap < falcon_compress_bound(n, dt)) return FALCON_ERR_BUFFER_TOO_SMALL;
  const uint64_t nc = (n + kChunkN - 1) / kChunkN;
  if (nc >= 0xFFFFFFF0ull) return FALCON_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  falcon_status st = prepare_launch(ctx, nc ? nc : 1, groups_of(nc) + 1, s);
  if (st != FALCON_OK) return st;
  CompressArgs a{};
  a.one.in = d_in;
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.group0 = 0;
  a.one.dtype = (uint32_t)dt;
  a.many = nullptr;
  a.nseries = 1;
  a.total_chunks = nc;
  a.status = ctx->status;
  a.gstatus = ctx->gstatus;
  a.ctl = ctx->ctl;
  a.epoch = ctx->epoch;
  const int grid = grid_for(ctx->grid_c[dt], nc, kCompressWaves);
  a.total_waves = (uint32_t)(grid * kCompressWaves);
  ctx->timed = false;
  if ((st = dev_err(hipEventRecord(ctx->ev0, s))) != FALCON_OK) return st;
  if ((st = dev_err(launch_compress(a, (int)dt, grid, s))) != FALCON_OK) return st;
  if ((st = dev_err(hipEventRecord(ctx->ev1, s))) != FALCON_OK) return st;
  ctx->timed = true;
  if ((st = dev_err(hipMemcpyAsync(ctx->stage, static_cast<uint8_t*>(d_out) + 24, 8, hipMemcpyDeviceToHost, s))) !=
      FALCON_OK)
    return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  *out_len = 32 + 4 * nc + rd64(ctx->stage);
  return FALCON_OK;
}

falcon_status falcon_decompress(falcon_ctx* ctx, const void* d_in, size_t in_len, void* d_out, size_t out_cap_bytes,
                                size_t* n_out, void* stream) {
  if (!ctx || !d_in || !n_out || ((uintptr_t)d_in % 4)) return FALCON_ERR_INVALID_ARG;
  if (in_len < 32) return FALCON_ERR_CORRUPT_STREAM;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  falcon_status st;
  if ((st = dev_err(hipMemcpyAsync(ctx->stage, d_in, 32, hipMemcpyDeviceToHost, s))) != FALCON_OK) return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  size_t n = 0;
  falcon_dtype dt;
  if ((st = falcon_stream_info(ctx->stage, 32, &n, &dt)) != FALCON_OK) return st;
  const uint64_t payload = rd64(ctx->stage + 24);
  const uint64_t nc = (n + kChunkN - 1) / kChunkN;
  if (nc >= 0xFFFFFFF0ull || (in_len - 32) / 4 < nc || payload > in_len - 32 - 4 * nc)
    return FALCON_ERR_CORRUPT_STREAM;
  *n_out = n;
  const size_t es = elem_size(dt);
  if (out_cap_bytes / es < n) return FALCON_ERR_BUFFER_TOO_SMALL;
  if (n == 0) return payload == 0 ? FALCON_OK : FALCON_ERR_CORRUPT_STREAM;
  if (!d_out || ((uintptr_t)d_out % es)) return FALCON_ERR_INVALID_ARG;
  if ((st = prepare_launch(ctx, nc, groups_of(nc) + scan_tiles(nc) + 1, s)) != FALCON_OK) return st;
  // chunk offsets: exclusive prefix of the size array, written into the
  // status array (offsets carry a zero epoch tag, so a later compression
  // never mistakes them for look-back words); the tile sums go to gstatus.
  const uint32_t lo = dt == FALCON_FLOAT64 ? 11u : 7u;
  const uint32_t hi = (uint32_t)(dt == FALCON_FLOAT64 ? kF64Chunk : kF32Chunk);
  ctx->timed = false;
  if ((st = dev_err(launch_scan_sizes(reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(d_in) + 32), nc,
                                      lo, hi, payload, ctx->gstatus, ctx->status, ctx->ctl, ctx->epoch, s))) !=
      FALCON_OK)
    return st;
  DecompressArgs a{};
  a.one.in = static_cast<const uint8_t*>(d_in);
  a.one.out = static_cast<uint8_t*>(d_out);
  a.one.n = n;
  a.one.chunk0 = 0;
  a.one.group0 = 0;
  a.one.payload_bytes = payload;
  a.one.dtype = (uint32_t)dt;
  a.many = nullptr;
  a.nseries = 1;
  a.total_chunks = nc;
  a.status = ctx->status;
  a.ctl = ctx->ctl;
  a.epoch = ctx->epoch;
  const int grid = grid_for(ctx->grid_d[dt], nc, kDecompressWaves);
  a.total_waves = (uint32_t)(grid * kDecompressWaves);
  if ((st = dev_err(hipEventRecord(ctx->ev0, s))) != FALCON_OK) return st;
  if ((st = dev_err(launch_decompress(a, (int)dt, grid, s))) != FALCON_OK) return st;
  if ((st = dev_err(hipEventRecord(ctx->ev1, s))) != FALCON_OK) return st;
  ctx->timed = true;
  if ((st = dev_err(hipMemcpyAsync(ctx->stage + 32, &ctx->ctl->error, 4, hipMemcpyDeviceToHost, s))) != FALCON_OK)
    return st;
  if ((st = dev_err(hipStreamSynchronize(s))) != FALCON_OK) return st;
  if (rd32(ctx->stage + 32) == ctx->epoch) return FALCON_ERR_CORRUPT_STREAM;
  return FALCON_OK;
}

falcon_status falcon_last_kernel_ms(falcon_ctx* ctx, float* ms) {
  if (!ctx || !ms || !ctx->timed) return FALCON_ERR_INVALID_ARG;
  if (hipEventSynchronize(ctx->ev1) != hipSuccess) return FALCON_ERR_DEVICE;
  return dev_err(hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
}

}  // extern "C"
