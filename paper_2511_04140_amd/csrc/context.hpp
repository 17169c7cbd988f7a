// context.hpp -- host-side state of a Falcon context, shared by the C ABI
// translation units (api.cpp, pipeline.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <vector>

#include "../../include/falcon.h"
#include "internal.hpp"

namespace falcon_host {

constexpr uint64_t kChunkN = 1025;
constexpr size_t kF64Chunk = 8211, kF32Chunk = 4107;  // largest chunk payloads
constexpr size_t kStageBytes = 64;                    // pinned bytes per lane

inline size_t elem_size(falcon_dtype dt) { return dt == FALCON_FLOAT64 ? 8 : dt == FALCON_FLOAT32 ? 4 : 0; }
inline size_t max_chunk_bytes(falcon_dtype dt) {
  return dt == FALCON_FLOAT64 ? kF64Chunk : dt == FALCON_FLOAT32 ? kF32Chunk : 0;
}
inline uint64_t chunks_of(uint64_t n) { return (n + kChunkN - 1) / kChunkN; }
inline uint32_t rd32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t rd64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }
inline falcon_status dev_err(hipError_t e) { return e == hipSuccess ? FALCON_OK : FALCON_ERR_DEVICE; }

// Writes the 32-byte stream header (format in falcon.h) to host memory.
void write_header(uint8_t* h, falcon_dtype dt, uint64_t n, uint64_t payload);

// One independent launch queue: a stream and the device scratch that a
// compression or decompression launch needs for itself (chunk offsets,
// scan tile sums, size-pass results, control block).  Launches on
// different lanes may run concurrently.
struct Lane {
  hipStream_t stream = nullptr;
  uint64_t* offsets = nullptr;  // one per chunk: exclusive prefix of the chunk sizes
  size_t offsets_cap = 0;
  uint64_t* tiles = nullptr;    // scan tile sums
  size_t tiles_cap = 0;
  falcon_dev::Ctl* ctl = nullptr;
  uint8_t* stage = nullptr;     // pinned host bytes: [0,32) header, [32,40) copy of the control block's
                                // two error words, [40,48) payload size
  uint32_t epoch = 0;
  falcon_dev::ChunkMeta* meta = nullptr;  // compression size pass results, one per chunk
  size_t meta_cap = 0;
  uint32_t* gsizes = nullptr;             // compression chunk sizes (scan input)
  size_t gsizes_cap = 0;
  // single-pass compression: one status word per chunk (look-back), the
  // 16-bit tag of the last launch's words (the array is cleared whenever the
  // tag wraps or the array is reallocated), and the ticket counters
  // (kQueueGroups x kQueueStride words, cleared before every launch)
  uint64_t* status = nullptr;
  size_t status_cap = 0;
  uint32_t qtag = 0;
  uint64_t* qctr = nullptr;
};

falcon_status lane_init(Lane& l);
void lane_free(Lane& l);

// State of one stream of the host <-> device pipeline (Alg. 1).
struct PipeLane {
  Lane lane;
  uint8_t* g_in = nullptr;   // device batch buffers
  uint8_t* g_out = nullptr;
  uint8_t* p_in = nullptr;   // pinned host staging, used for pageable caller buffers
  uint8_t* p_out = nullptr;
  hipEvent_t ev = nullptr;
  int state = 0;
  uint64_t c0 = 0, nchunks = 0, nvals = 0, cs = 0, dst = 0;
};

// ---- batch launches (batch.cpp) -------------------------------------------
// Launch geometry of a batch: one launch per dtype (split) or one over both,
// wavefronts per compression workgroup, grid as a percentage of the
// co-resident workgroups.
struct BatchGeom {
  int split = 1;
  // 8-wave workgroups by default: the float32 kernels then run 6 waves per
  // SIMD (three workgroups per CU), the float64 ones 4, as with 16
  int nw = falcon_dev::kCompressWaves32;
  int grid_pct = 100;
  int form = 0;  // compression: 0 two passes (static striding), 1 single pass (work queue, look-back)
};

// Where a batch's series sit in launch-chunk space (float64 series first).
struct BatchLayout {
  int op = 0;
  size_t count = 0;
  uint64_t total = 0, t64 = 0;
  bool has64 = false, has32 = false;
  falcon_dev::CompressSeries one_c{};
  falcon_dev::DecompressSeries one_d{};
  size_t desc_bytes = 0;
};

// Device and pinned scratch of batch launches; grows on demand.  Scratch
// that a recorded graph uses must not grow afterwards.
struct BatchScratch {
  void* many = nullptr;          // device descriptors
  size_t many_cap = 0;
  uint8_t* h_desc = nullptr;     // pinned host copy of the descriptors
  size_t h_desc_cap = 0;
  uint64_t* offsets = nullptr;   // chunk offsets (scan of all chunk sizes)
  size_t offsets_cap = 0;
  uint64_t* tiles = nullptr;
  size_t tiles_cap = 0;
  uint32_t* sizes = nullptr;     // decompression: gathered chunk sizes; compression: chunk sizes
  size_t sizes_cap = 0;
  falcon_dev::ChunkMeta* meta = nullptr;  // compression size pass results
  size_t meta_cap = 0;
  falcon_dev::Ctl* ctl = nullptr;
  uint64_t* lens = nullptr;      // device stream lengths (compression)
  size_t lens_cap = 0;
  uint64_t* h_lens = nullptr;    // pinned: lengths, then the error word
  size_t h_lens_cap = 0;
  uint64_t* status = nullptr;    // single-pass compression: ticket counters, then one status word per chunk
  size_t status_cap = 0;
};

}  // namespace falcon_host

struct falcon_ctx {
  int device = 0;
  unsigned opt_flags = 0;   // FALCON_OPT_* of falcon_create
  int compress_form = 0;    // falcon_compress_form of falcon_compress
  falcon_host::Lane main;
  // asynchronous device calls: every call waits (on the device) for the
  // previous one when it uses another stream, and records ev_done after its
  // work; falcon_sync waits for last_stream
  hipEvent_t ev_done = nullptr;
  hipStream_t last_stream = nullptr;
  bool unsynced = false;
  uint32_t sync_epoch = 0;  // main lane's launch epoch at the last falcon_sync
  // stream lengths of compressions that report to host memory: the kernels
  // write them into device words (blocks of kLenBlock, never moved while in
  // use), falcon_sync copies them to pinned memory and on to the caller
  std::vector<uint64_t*> len_blocks;
  uint64_t* len_host = nullptr;  // pinned, len_host_cap words
  size_t len_host_cap = 0;
  struct PendingLen {
    size_t* dst;
    size_t slot;
  };
  std::vector<PendingLen> pending;
  // co-resident workgroups of each kernel: by form (1 = f32, 2 = f64,
  // 3 = mixed) and, for compression, pass (0 single-pass, 1 size, 2 write)
  // and workgroup size (8 or 16 waves)
  int grid_c[4][3][2] = {};
  int grid_d[4] = {};
  // the same for the single-pass compression kernels: [form][8 or 16 waves]
  int grid_q[4][2] = {};
  // the same for the ablation-variant compression kernels: [form][variant][pass]
  int grid_v[3][4][3] = {};
  // events of the last FALCON_TIMED_CALLS timed calls, a ring whose slot
  // ev_slot holds the last call: before the first kernel, after it, after
  // the scan, after the last kernel (decompression: the first two coincide).
  // ev_ok marks a slot whose call enqueued all four.
  hipEvent_t ev[FALCON_TIMED_CALLS][4] = {};
  bool ev_ok[FALCON_TIMED_CALLS] = {};
  int ev_slot = 0;
  // host <-> device pipeline
  // defaults measured on MI355X (4 hardware queues per process): 4 streams
  // of 2048-chunk batches beat the 16 x 4096 setting of Sec. 5.1.4 in both
  // directions
  int pipe_streams = 4;
  uint64_t pipe_batch_chunks = 2048;
  size_t pipe_buf_bytes = 0;     // bytes of each g_in / g_out / p_in / p_out
  bool pipe_staging = false;     // p_in / p_out allocated
  int pipe_scheduler = 0;        // falcon_scheduler of compression
  uint8_t* pre_buf = nullptr;    // pinned per-batch slots of the pre-allocation scheduler
  size_t pre_cap = 0;
  std::vector<falcon_host::PipeLane> pipe;
  // one-shot batch calls
  falcon_host::BatchScratch batch;
  // geometries the plan autotuner chose, by shape class (see batch.cpp)
  std::map<uint64_t, falcon_host::BatchGeom> tuned;
};

namespace falcon_host {

// Enqueues the compression of n values at d_in into the stream buffer d_out
// on lane l (stream s).  Nothing is waited for; the stream's payload byte
// count lands in the stream header at d_out + 24.  With timed, events
// around the kernel feed falcon_last_kernel_ms.  variant != 0 selects an
// ablation variant's kernels (falcon_variant).
falcon_status enqueue_compress(falcon_ctx* ctx, Lane& l, const void* d_in, uint64_t n, falcon_dtype dt, void* d_out,
                               hipStream_t s, bool timed, int variant = 0, int form = 0, uint64_t* d_len = nullptr);
constexpr size_t kLenBlock = 4096;  // stream-length words per device block of a context

// Enqueues the decompression of a stream at d_in of in_len bytes holding n
// values of type dt, into d_out.  With payload = kPayloadFromHeader the
// stream header is read and checked on the device (against n, dt, in_len);
// otherwise the host has checked it and payload is its byte count.  With
// copy_error the error word is then copied into l.stage + 32, and
// decompress_failed() afterwards (once the stream has reached that copy)
// tells whether a chunk failed.
constexpr uint64_t kPayloadFromHeader = ~0ull;
falcon_status enqueue_decompress(falcon_ctx* ctx, Lane& l, const uint8_t* d_in, uint64_t in_len, uint64_t n,
                                 falcon_dtype dt, uint64_t payload, void* d_out, hipStream_t s, bool timed,
                                 bool copy_error = true);
inline bool decompress_failed(const Lane& l) { return rd32(l.stage + 32) == l.epoch; }


inline int max_grid_c(const falcon_ctx* ctx, int form, int pass, int nw);
inline int max_grid_q(const falcon_ctx* ctx, int form, int nw) { return ctx->grid_q[form][nw == 8 ? 0 : 1]; }
inline int max_grid_d(const falcon_ctx* ctx, int form);

// Set-up of falcon_compress_noalloc on `device` (noalloc.hip): the device
// address of its fixed scratch and its launch grids.
falcon_status noalloc_setup(int device);

// Frees the pipeline lanes and their buffers (pipeline.cpp).
void pipe_release(falcon_ctx* ctx);

falcon_status batch_check(int op, const falcon_series& d);
// Lays the series out, writes their descriptors into the pinned copy and
// grows the device scratch to fit (waiting for `s` first if it grows).
falcon_status batch_layout(BatchScratch& b, int op, const falcon_series* s, size_t count, BatchLayout& L,
                           hipStream_t st);
// Enqueues one run: descriptor upload (if upload), clearing fills, the
// launches, and the copy of the lengths or the error word to pinned memory.
falcon_status batch_enqueue(const falcon_ctx* ctx, BatchScratch& b, const BatchLayout& L, const BatchGeom& g,
                            hipStream_t s, bool upload);
// After the run has completed: the error status, and each dst[i].out_len
// (dst may be null; src holds the series the layout was made from).
falcon_status batch_result(const BatchScratch& b, const BatchLayout& L, const falcon_series* src,
                           falcon_series* dst);
void batch_free(BatchScratch& b);

}  // namespace falcon_host

inline int falcon_host::max_grid_c(const falcon_ctx* ctx, int form, int pass, int nw) {
  return ctx->grid_c[form][pass][nw == 8 ? 0 : 1];
}
inline int falcon_host::max_grid_d(const falcon_ctx* ctx, int form) { return ctx->grid_d[form]; }
