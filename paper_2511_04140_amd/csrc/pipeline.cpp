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
  if (ctx->pre_buf) (void)hipHostFree(ctx->pre_buf);
  ctx->pre_buf = nullptr;
  ctx->pre_cap = 0;
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

namespace {

struct CompressJob {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n, nc, bc, nbatch, payload_base;
  falcon_dtype dt;
  size_t es;
  bool in_pinned, out_pinned;
};

// H2D of batch b and its compression into p.g_out on p's stream; with
// m_d2h, the copy of the batch's payload byte count to p.lane.stage + 40.
falcon_status issue_batch(falcon_ctx* ctx, PipeLane& p, const CompressJob& j, uint64_t b, bool m_d2h) {
  hipStream_t s = p.lane.stream;
  p.c0 = b * j.bc;
  p.nchunks = j.nc - p.c0 < j.bc ? j.nc - p.c0 : j.bc;
  const uint64_t v0 = p.c0 * kChunkN;
  p.nvals = j.n - v0 < p.nchunks * kChunkN ? j.n - v0 : p.nchunks * kChunkN;
  const uint8_t* src = j.in + v0 * j.es;
  if (!j.in_pinned) {
    memcpy(p.p_in, src, p.nvals * j.es);
    src = p.p_in;
  }
  falcon_status st;
  if ((st = dev_err(hipMemcpyAsync(p.g_in, src, p.nvals * j.es, hipMemcpyHostToDevice, s))) != FALCON_OK ||
      (st = enqueue_compress(ctx, p.lane, p.g_in, p.nvals, j.dt, p.g_out, s, false)) != FALCON_OK)
    return st;
  if (m_d2h) return dev_err(hipMemcpyAsync(p.lane.stage + 40, p.g_out + 24, 8, hipMemcpyDeviceToHost, s));
  return FALCON_OK;
}

// P-D2H: the batch's sizes and its cs payload bytes to their final place
// (payload at offset), or to the lane's pinned staging for pageable output.
falcon_status issue_placement(PipeLane& p, const CompressJob& j, uint64_t offset) {
  hipStream_t s = p.lane.stream;
  p.dst = offset;
  const uint8_t* sizes = p.g_out + 32;
  falcon_status st;
  if (j.out_pinned) {
    if ((st = dev_err(hipMemcpyAsync(j.out + 32 + 4 * p.c0, sizes, 4 * p.nchunks, hipMemcpyDeviceToHost, s))) !=
        FALCON_OK)
      return st;
    return dev_err(
        hipMemcpyAsync(j.out + j.payload_base + offset, sizes + 4 * p.nchunks, p.cs, hipMemcpyDeviceToHost, s));
  }
  return dev_err(hipMemcpyAsync(p.p_out, sizes, 4 * p.nchunks + p.cs, hipMemcpyDeviceToHost, s));
}

// After the placement copies: the host copies of staged output.
void finish_placement(const PipeLane& p, const CompressJob& j) {
  if (j.out_pinned) return;
  memcpy(j.out + 32 + 4 * p.c0, p.p_out, 4 * p.nchunks);
  memcpy(j.out + j.payload_base + p.dst, p.p_out + 4 * p.nchunks, p.cs);
}

falcon_status read_cs(PipeLane& p, const CompressJob& j) {
  p.cs = rd64(p.lane.stage + 40);
  return p.cs > p.nchunks * max_chunk_bytes(j.dt) ? FALCON_ERR_DEVICE : FALCON_OK;
}

// Alg. 1 (event-driven): lanes cycle Idle -> MPend -> PPend -> Idle; a lane
// in MPend places its payload once its byte count has arrived and every
// batch launched before it has been placed (launch order is kept in a
// queue, which is what Alg. 1's `current` stands for).
falcon_status compress_event_driven(falcon_ctx* ctx, const CompressJob& j, uint64_t* total) {
  const int ns = (int)ctx->pipe.size();
  std::vector<int> order(j.nbatch);
  uint64_t next = 0, placed = 0, done = 0, offset = 0;
  falcon_status st;
  for (auto& p : ctx->pipe) p.state = kIdle;
  while (done < j.nbatch) {
    bool moved = false;
    for (int i = 0; i < ns; ++i) {
      PipeLane& p = ctx->pipe[i];
      if (p.state == kIdle) {
        if (next >= j.nbatch) continue;
        const uint64_t b = next++;
        if ((st = issue_batch(ctx, p, j, b, true)) != FALCON_OK ||
            (st = dev_err(hipEventRecord(p.ev, p.lane.stream))) != FALCON_OK)
          return st;
        order[b] = i;
        p.state = kMPend;
        moved = true;
      } else if (p.state == kMPend) {
        if (order[placed] != i) continue;  // not the current lane yet
        const int r = poll(p);
        if (r < 0) return FALCON_ERR_DEVICE;
        if (r == 0) continue;
        if ((st = read_cs(p, j)) != FALCON_OK || (st = issue_placement(p, j, offset)) != FALCON_OK ||
            (st = dev_err(hipEventRecord(p.ev, p.lane.stream))) != FALCON_OK)
          return st;
        offset += p.cs;
        ++placed;
        p.state = kPPend;
        moved = true;
      } else {  // kPPend
        const int r = poll(p);
        if (r < 0) return FALCON_ERR_DEVICE;
        if (r == 0) continue;
        finish_placement(p, j);
        ++done;
        p.state = kIdle;
        moved = true;
      }
    }
    if (!moved) std::this_thread::yield();
  }
  *total = offset;
  return FALCON_OK;
}

// Sync-Based Scheduler (Sec. 3.1, Fig. 5b): the host waits for each batch's
// byte count before it launches the next batch; only the payload copy of a
// batch overlaps the transfer and compression of the next.
falcon_status compress_sync_based(falcon_ctx* ctx, const CompressJob& j, uint64_t* total) {
  const int ns = (int)ctx->pipe.size();
  uint64_t offset = 0;
  falcon_status st;
  for (auto& p : ctx->pipe) p.state = kIdle;
  for (uint64_t b = 0; b < j.nbatch; ++b) {
    PipeLane& p = ctx->pipe[b % ns];
    if (p.state == kPPend) {
      if (hipEventSynchronize(p.ev) != hipSuccess) return FALCON_ERR_DEVICE;
      finish_placement(p, j);
    }
    if ((st = issue_batch(ctx, p, j, b, true)) != FALCON_OK ||
        (st = dev_err(hipEventRecord(p.ev, p.lane.stream))) != FALCON_OK)
      return st;
    if (hipEventSynchronize(p.ev) != hipSuccess) return FALCON_ERR_DEVICE;  // M-D2H received
    if ((st = read_cs(p, j)) != FALCON_OK || (st = issue_placement(p, j, offset)) != FALCON_OK ||
        (st = dev_err(hipEventRecord(p.ev, p.lane.stream))) != FALCON_OK)
      return st;
    offset += p.cs;
    p.state = kPPend;
  }
  for (auto& p : ctx->pipe) {
    if (p.state != kPPend) continue;
    if (hipEventSynchronize(p.ev) != hipSuccess) return FALCON_ERR_DEVICE;
    finish_placement(p, j);
    p.state = kIdle;
  }
  *total = offset;
  return FALCON_OK;
}

// Pre-Allocation Scheduler (Sec. 3.1, Fig. 5a): every batch copies its whole
// worst-case output region (sizes and bound-sized payload area) into a
// fixed slot of a pinned host buffer, in any order; a merge step then packs
// the slots into the stream.
falcon_status compress_pre_allocation(falcon_ctx* ctx, const CompressJob& j, uint64_t* total) {
  const int ns = (int)ctx->pipe.size();
  const size_t slot = 32 + j.bc * (4 + max_chunk_bytes(j.dt));
  const size_t need = slot * j.nbatch;
  if (need > ctx->pre_cap) {
    if (ctx->pre_buf) (void)hipHostFree(ctx->pre_buf);
    ctx->pre_buf = nullptr;
    ctx->pre_cap = 0;
    if (hipHostMalloc(&ctx->pre_buf, need, hipHostMallocDefault) != hipSuccess) return FALCON_ERR_OUT_OF_MEMORY;
    ctx->pre_cap = need;
  }
  std::vector<uint64_t> batch_of(ns, 0);
  uint64_t next = 0, done = 0;
  falcon_status st;
  for (auto& p : ctx->pipe) p.state = kIdle;
  while (done < j.nbatch) {
    bool moved = false;
    for (int i = 0; i < ns; ++i) {
      PipeLane& p = ctx->pipe[i];
      if (p.state == kIdle) {
        if (next >= j.nbatch) continue;
        const uint64_t b = next++;
        if ((st = issue_batch(ctx, p, j, b, false)) != FALCON_OK) return st;
        const size_t region = 32 + p.nchunks * (4 + max_chunk_bytes(j.dt));
        if (
            (st = dev_err(hipMemcpyAsync(ctx->pre_buf + b * slot, p.g_out, region, hipMemcpyDeviceToHost,
                                         p.lane.stream))) != FALCON_OK ||
            (st = dev_err(hipEventRecord(p.ev, p.lane.stream))) != FALCON_OK)
          return st;
        batch_of[i] = b;
        p.state = kBusy;
        moved = true;
      } else {
        const int r = poll(p);
        if (r < 0) return FALCON_ERR_DEVICE;
        if (r == 0) continue;
        ++done;
        p.state = kIdle;
        moved = true;
      }
    }
    if (!moved) std::this_thread::yield();
  }
  // merge
  uint64_t offset = 0;
  for (uint64_t b = 0; b < j.nbatch; ++b) {
    const uint8_t* sl = ctx->pre_buf + b * slot;
    const uint64_t c0 = b * j.bc, nb = j.nc - c0 < j.bc ? j.nc - c0 : j.bc;
    const uint64_t cs = rd64(sl + 24);
    if (cs > nb * max_chunk_bytes(j.dt)) return FALCON_ERR_DEVICE;
    memcpy(j.out + 32 + 4 * c0, sl + 32, 4 * nb);
    memcpy(j.out + j.payload_base + offset, sl + 32 + 4 * nb, cs);
    offset += cs;
  }
  *total = offset;
  return FALCON_OK;
}

}  // namespace

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
  CompressJob j;
  j.in = static_cast<const uint8_t*>(h_in);
  j.out = out;
  j.n = n;
  j.nc = nc;
  j.bc = ctx->pipe_batch_chunks;
  j.nbatch = (nc + j.bc - 1) / j.bc;
  j.payload_base = 32 + 4 * nc;
  j.dt = dt;
  j.es = es;
  j.in_pinned = is_pinned(h_in);
  j.out_pinned = is_pinned(h_out);
  falcon_status st = pipe_ensure(ctx, !(j.in_pinned && j.out_pinned));
  if (st != FALCON_OK) return st;
  uint64_t total = 0;
  if (ctx->pipe_scheduler == FALCON_SCHED_SYNC_BASED) st = compress_sync_based(ctx, j, &total);
  else if (ctx->pipe_scheduler == FALCON_SCHED_PRE_ALLOCATION) st = compress_pre_allocation(ctx, j, &total);
  else st = compress_event_driven(ctx, j, &total);
  if (st != FALCON_OK) {
    drain(ctx);
    return st;
  }
  write_header(out, dt, n, total);
  *out_len = j.payload_base + total;
  return FALCON_OK;
}

falcon_status falcon_set_pipeline_scheduler(falcon_ctx* ctx, falcon_scheduler kind) {
  if (!ctx || (kind != FALCON_SCHED_EVENT_DRIVEN && kind != FALCON_SCHED_SYNC_BASED &&
               kind != FALCON_SCHED_PRE_ALLOCATION))
    return FALCON_ERR_INVALID_ARG;
  ctx->pipe_scheduler = (int)kind;
  return FALCON_OK;
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
        if ((st = enqueue_decompress(ctx, p.lane, p.g_in, slen, p.nvals, dt, pb, p.g_out, s, false)) != FALCON_OK ||
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
