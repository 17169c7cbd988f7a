// pipeline.cpp -- host <-> device pipeline of Sec. 3.1 (Alg. 1, the
// event-driven scheduler) on HIP streams.
//
// Compression: the input is cut into batches of whole chunks.  Each of N_s
// lanes (a stream with its own device buffers and launch scratch) runs
// H2D -> compression kernel -> copy of the batch's payload byte count
// (M-D2H), then, once the host has seen that count and every earlier batch
// has been placed, the copy of the batch's sizes and payload to their final
// place in the output (P-D2H).  Because the stream keeps one global size
// array after its header, a batch's sizes have a fixed place, and its
// payload goes right after the payload of the batch launched before it: the
// output is byte-identical to one device-resident compression of the whole
// array.
//
// Decompression: the size array is in host memory, so the host computes
// every batch's payload offset up front (the pre-allocation scheme, which
// the paper uses for decompression, Sec. 4); each lane runs H2D -> offsets
// scan -> decompression kernel -> D2H of the values to their place.
//
// Caller buffers that are pinned (hipHostMalloc'd) are transferred
// directly; pageable ones go through pinned staging buffers of the lane,
// copied on the host thread while the other lanes' transfers proceed.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <thread>
#include <vector>

#include "context.hpp"

namespace falcon_host {

namespace {

enum { kIdle = 0, kMPend = 1, kPPend = 2, kBusy = 3 };

size_t batch_buf_bytes(uint64_t batch_chunks) {
  const size_t a = 32 + batch_chunks * (4 + kF64Chunk);  // largest stream of one batch (>= its values)
  return (a + 255) & ~(size_t)255;
}

bool is_pinned(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory is not an error here
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

falcon_status pipe_ensure(falcon_ctx* ctx, bool staging) {
  const size_t bytes = batch_buf_bytes(ctx->pipe_batch_chunks);
  if (ctx->pipe.size() != (size_t)ctx->pipe_streams || ctx->pipe_buf_bytes != bytes) {
    pipe_release(ctx);
    ctx->pipe.resize((size_t)ctx->pipe_streams);
    ctx->pipe_buf_bytes = bytes;
    for (auto& p : ctx->pipe) {
      if (lane_init(p.lane) != FALCON_OK || hipEventCreateWithFlags(&p.ev, hipEventDisableTiming) != hipSuccess) {
        pipe_release(ctx);
        return FALCON_ERR_DEVICE;
      }
      if (hipMalloc(&p.g_in, bytes) != hipSuccess || hipMalloc(&p.g_out, bytes) != hipSuccess) {
        pipe_release(ctx);
        return FALCON_ERR_OUT_OF_MEMORY;
      }
    }
  }
  if (staging && !ctx->pipe_staging) {
    for (auto& p : ctx->pipe) {
      if (hipHostMalloc(&p.p_in, bytes, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc(&p.p_out, bytes, hipHostMallocDefault) != hipSuccess) {
        pipe_release(ctx);
        return FALCON_ERR_OUT_OF_MEMORY;
      }
    }
    ctx->pipe_staging = true;
  }
  return FALCON_OK;
}

// Waits for every lane (used before returning an error, so that no copy into
// a caller buffer is still pending).
void drain(falcon_ctx* ctx) {
  for (auto& p : ctx->pipe)
    if (p.lane.stream) (void)hipStreamSynchronize(p.lane.stream);
}

// Polls a lane's event: 1 = reached, 0 = pending, -1 = device error.
int poll(const PipeLane& p) {
  const hipError_t e = hipEventQuery(p.ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return -1;
}

}  // namespace

void pipe_release(falcon_ctx* ctx) {
  for (auto& p : ctx->pipe) {
    lane_free(p.lane);  // waits for the lane's stream first
    if (p.g_in) (void)hipFree(p.g_in);
    if (p.g_out) (void)hipFree(p.g_out);
    if (p.p_in) (void)hipHostFree(p.p_in);
    if (p.p_out) (void)hipHostFree(p.p_out);
    if (p.ev) (void)hipEventDestroy(p.ev);
  }
  ctx->pipe.clear();
  ctx->pipe_buf_bytes = 0;
  ctx->pipe_staging = false;
}

}  // namespace falcon_host

using namespace falcon_host;

extern "C" {

falcon_status falcon_set_pipeline(falcon_ctx* ctx, int n_streams, size_t batch_chunks) {
  if (!ctx || n_streams < 1 || n_streams > 64 || batch_chunks < 1 || batch_chunks > (1u << 20))
    return FALCON_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  if (n_streams != ctx->pipe_streams || batch_chunks != ctx->pipe_batch_chunks) pipe_release(ctx);
  ctx->pipe_streams = n_streams;
  ctx->pipe_batch_chunks = batch_chunks;
  return FALCON_OK;
}

falcon_status falcon_compress_host(falcon_ctx* ctx, const void* h_in, size_t n, falcon_dtype dt, void* h_out,
                                   size_t out_cap, size_t* out_len) {
  if (!ctx || !h_out || !out_len || (n && !h_in)) return FALCON_ERR_INVALID_ARG;
  const size_t es = elem_size(dt);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  const size_t bound = falcon_compress_bound(n, dt);
  if (out_cap < bound) {
    *out_len = bound;
    return FALCON_ERR_BUFFER_TOO_SMALL;
  }
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull) return FALCON_ERR_INVALID_ARG;
  uint8_t* out = static_cast<uint8_t*>(h_out);
  if (n == 0) {
    write_header(out, dt, 0, 0);
    *out_len = 32;
    return FALCON_OK;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  const bool in_pinned = is_pinned(h_in), out_pinned = is_pinned(h_out);
  falcon_status st = pipe_ensure(ctx, !(in_pinned && out_pinned));
  if (st != FALCON_OK) return st;
  const uint8_t* in = static_cast<const uint8_t*>(h_in);
  const uint64_t bc = ctx->pipe_batch_chunks;
  const uint64_t nbatch = (nc + bc - 1) / bc;
  const uint64_t payload_base = 32 + 4 * nc;
  const int ns = (int)ctx->pipe.size();
  // Lanes in launch order: a lane waiting for its batch's byte count may
  // place its payload only after every batch launched before it.
  std::vector<int> order(nbatch);
  uint64_t next = 0, placed = 0, done = 0, offset = 0;
  for (auto& p : ctx->pipe) p.state = kIdle;
  while (done < nbatch) {
    bool moved = false;
    for (int i = 0; i < ns; ++i) {
      PipeLane& p = ctx->pipe[i];
      hipStream_t s = p.lane.stream;
      if (p.state == kIdle) {
        if (next >= nbatch) continue;
        const uint64_t b = next++;
        p.c0 = b * bc;
        p.nchunks = nc - p.c0 < bc ? nc - p.c0 : bc;
        const uint64_t v0 = p.c0 * kChunkN;
        p.nvals = n - v0 < p.nchunks * kChunkN ? n - v0 : p.nchunks * kChunkN;
        const uint8_t* src = in + v0 * es;
        if (!in_pinned) {
          memcpy(p.p_in, src, p.nvals * es);
          src = p.p_in;
        }
        if ((st = dev_err(hipMemcpyAsync(p.g_in, src, p.nvals * es, hipMemcpyHostToDevice, s))) != FALCON_OK ||
            (st = enqueue_compress(ctx, p.lane, p.g_in, p.nvals, dt, p.g_out, s, false)) != FALCON_OK ||
            (st = dev_err(hipMemcpyAsync(p.lane.stage + 40, p.g_out + 24, 8, hipMemcpyDeviceToHost, s))) !=
                FALCON_OK ||
            (st = dev_err(hipEventRecord(p.ev, s))) != FALCON_OK)
          goto fail;
        order[b] = i;
        p.state = kMPend;
        moved = true;
      } else if (p.state == kMPend) {
        if (order[placed] != i) continue;  // not the current lane yet
        const int r = poll(p);
        if (r < 0) { st = FALCON_ERR_DEVICE; goto fail; }
        if (r == 0) continue;
        p.cs = rd64(p.lane.stage + 40);
        if (p.cs > p.nchunks * max_chunk_bytes(dt)) { st = FALCON_ERR_DEVICE; goto fail; }
        p.dst = offset;
        const uint8_t* sizes = p.g_out + 32;
        if (out_pinned) {
          if ((st = dev_err(hipMemcpyAsync(out + 32 + 4 * p.c0, sizes, 4 * p.nchunks, hipMemcpyDeviceToHost, s))) !=
                  FALCON_OK ||
              (st = dev_err(hipMemcpyAsync(out + payload_base + offset, sizes + 4 * p.nchunks, p.cs,
                                           hipMemcpyDeviceToHost, s))) != FALCON_OK)
            goto fail;
        } else if ((st = dev_err(hipMemcpyAsync(p.p_out, sizes, 4 * p.nchunks + p.cs, hipMemcpyDeviceToHost, s))) !=
                   FALCON_OK) {
          goto fail;
        }
        if ((st = dev_err(hipEventRecord(p.ev, s))) != FALCON_OK) goto fail;
        offset += p.cs;
        ++placed;
        p.state = kPPend;
        moved = true;
      } else {  // kPPend
        const int r = poll(p);
        if (r < 0) { st = FALCON_ERR_DEVICE; goto fail; }
        if (r == 0) continue;
        if (!out_pinned) {
          memcpy(out + 32 + 4 * p.c0, p.p_out, 4 * p.nchunks);
          memcpy(out + payload_base + p.dst, p.p_out + 4 * p.nchunks, p.cs);
        }
        ++done;
        p.state = kIdle;
        moved = true;
      }
    }
    if (!moved) std::this_thread::yield();
  }
  write_header(out, dt, n, offset);
  *out_len = payload_base + offset;
  return FALCON_OK;
fail:
  drain(ctx);
  return st;
}

falcon_status falcon_decompress_host(falcon_ctx* ctx, const void* h_in, size_t in_len, void* h_out,
                                     size_t out_cap_bytes, size_t* n_out) {
  if (!ctx || !h_in || !n_out) return FALCON_ERR_INVALID_ARG;
  if (in_len < 32) return FALCON_ERR_CORRUPT_STREAM;
  const uint8_t* in = static_cast<const uint8_t*>(h_in);
  size_t n = 0;
  falcon_dtype dt;
  falcon_status st = falcon_stream_info(in, in_len, &n, &dt);
  if (st != FALCON_OK) return st;
  const uint64_t payload = rd64(in + 24);
  const uint64_t nc = chunks_of(n);
  if (nc >= 0xFFFFFFF0ull || (in_len - 32) / 4 < nc || payload > in_len - 32 - 4 * nc)
    return FALCON_ERR_CORRUPT_STREAM;
  *n_out = n;
  const size_t es = elem_size(dt);
  if (out_cap_bytes / es < n) return FALCON_ERR_BUFFER_TOO_SMALL;
  if (n == 0) return payload == 0 ? FALCON_OK : FALCON_ERR_CORRUPT_STREAM;
  if (!h_out) return FALCON_ERR_INVALID_ARG;
  // Every batch's payload offset, from the size array in host memory.
  const uint64_t bc = ctx->pipe_batch_chunks;
  const uint64_t nbatch = (nc + bc - 1) / bc;
  const uint8_t* sizes = in + 32;
  const uint32_t lo = dt == FALCON_FLOAT64 ? 11u : 7u, hi = (uint32_t)max_chunk_bytes(dt);
  std::vector<uint64_t> boff(nbatch + 1);
  uint64_t acc = 0;
  for (uint64_t c = 0; c < nc; ++c) {
    if (c % bc == 0) boff[c / bc] = acc;
    const uint32_t v = rd32(sizes + 4 * c);
    if (v < lo || v > hi) return FALCON_ERR_CORRUPT_STREAM;
    acc += v;
  }
  boff[nbatch] = acc;
  if (acc != payload) return FALCON_ERR_CORRUPT_STREAM;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  const bool in_pinned = is_pinned(h_in), out_pinned = is_pinned(h_out);
  if ((st = pipe_ensure(ctx, !(in_pinned && out_pinned))) != FALCON_OK) return st;
  const uint8_t* payload_base = in + 32 + 4 * nc;
  uint8_t* out = static_cast<uint8_t*>(h_out);
  const int ns = (int)ctx->pipe.size();
  uint64_t next = 0, done = 0, launched = 0;
  bool corrupt = false;
  for (auto& p : ctx->pipe) p.state = kIdle;
  while (done < launched || (!corrupt && next < nbatch)) {
    bool moved = false;
    for (int i = 0; i < ns; ++i) {
      PipeLane& p = ctx->pipe[i];
      hipStream_t s = p.lane.stream;
      if (p.state == kIdle) {
        if (corrupt || next >= nbatch) continue;
        const uint64_t b = next++;
        p.c0 = b * bc;
        p.nchunks = nc - p.c0 < bc ? nc - p.c0 : bc;
        const uint64_t v0 = p.c0 * kChunkN;
        p.nvals = n - v0 < p.nchunks * kChunkN ? n - v0 : p.nchunks * kChunkN;
        const uint64_t pb = boff[b + 1] - boff[b];
        const uint64_t slen = 32 + 4 * p.nchunks + pb;
        write_header(p.lane.stage, dt, p.nvals, pb);
        if (in_pinned) {
          if ((st = dev_err(hipMemcpyAsync(p.g_in, p.lane.stage, 32, hipMemcpyHostToDevice, s))) != FALCON_OK ||
              (st = dev_err(hipMemcpyAsync(p.g_in + 32, sizes + 4 * p.c0, 4 * p.nchunks, hipMemcpyHostToDevice,
                                           s))) != FALCON_OK ||
              (st = dev_err(hipMemcpyAsync(p.g_in + 32 + 4 * p.nchunks, payload_base + boff[b], pb,
                                           hipMemcpyHostToDevice, s))) != FALCON_OK)
            goto fail;
        } else {
          memcpy(p.p_in, p.lane.stage, 32);
          memcpy(p.p_in + 32, sizes + 4 * p.c0, 4 * p.nchunks);
          memcpy(p.p_in + 32 + 4 * p.nchunks, payload_base + boff[b], pb);
          if ((st = dev_err(hipMemcpyAsync(p.g_in, p.p_in, slen, hipMemcpyHostToDevice, s))) != FALCON_OK) goto fail;
        }
        if ((st = enqueue_decompress(ctx, p.lane, p.g_in, p.nvals, dt, pb, p.g_out, s, false)) != FALCON_OK ||
            (st = dev_err(hipMemcpyAsync(out_pinned ? out + v0 * es : p.p_out, p.g_out, p.nvals * es,
                                         hipMemcpyDeviceToHost, s))) != FALCON_OK ||
            (st = dev_err(hipEventRecord(p.ev, s))) != FALCON_OK)
          goto fail;
        ++launched;
        p.state = kBusy;
        moved = true;
      } else if (p.state == kBusy) {
        const int r = poll(p);
        if (r < 0) { st = FALCON_ERR_DEVICE; goto fail; }
        if (r == 0) continue;
        if (decompress_failed(p.lane)) corrupt = true;
        else if (!out_pinned) memcpy(out + p.c0 * kChunkN * es, p.p_out, p.nvals * es);
        ++done;
        p.state = kIdle;
        moved = true;
      }
    }
    if (!moved) std::this_thread::yield();
  }
  return corrupt ? FALCON_ERR_CORRUPT_STREAM : FALCON_OK;
fail:
  drain(ctx);
  return st;
}

}  // extern "C"
