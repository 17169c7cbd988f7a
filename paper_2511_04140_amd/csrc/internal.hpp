// internal.hpp -- launch interface between the C ABI (api.cpp) and the
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace falcon_dev {

// Control block of a launch queue: the decompression error word (receives
// the launch epoch when a chunk fails a check), the single-pass compression
// error word (set when a look-back gives up, which a correct run never
// does) and the work-queue ticket counter of single-pass compression.
struct Ctl {
  uint32_t error;
  uint32_t qerror;
  uint64_t pad;
};

// Single-pass compression takes chunks from kQueueGroups ticket counters,
// each in a 128-byte line of its own (a counter is one word every
// kQueueStride): workgroup b draws from counter b mod G and its ticket k
// stands for launch chunk k * G + (b mod G).
constexpr int kQueueGroups = 16;
constexpr int kQueueStride = 16;

// One array to compress.  chunk0 is the global index of its first chunk in
// the launch (prefix of the chunk counts of the series before it).
struct CompressSeries {
  const void* in;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk0;
  uint32_t dtype;    // 1 = f32, 2 = f64
  uint32_t idx;      // position of the series in the caller's list (lens[idx])
};

struct DecompressSeries {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk0;
  uint64_t payload_bytes;  // batch launches: filled on the device from the stream header
  uint64_t in_len;         // stream bytes (batch launches)
  uint32_t dtype;
  uint32_t idx;
};

// What the size pass of compression learns about a chunk and the write pass
// reuses: the row scheme flags (bit p set = plane p is written dense), the
// chunk's byte count, and its header bytes alpha_max, beta_hat_max, w.
struct ChunkMeta {
  uint64_t flags;
  uint32_t S;
  uint8_t A, B, w, pad;
};

struct CompressArgs {
  CompressSeries one;            // the series of a one-series launch (many == null)
  const CompressSeries* many;    // device array, sorted by chunk0, for batch launches
  uint32_t nseries;
  uint32_t total_waves;
  uint64_t total_chunks;  // chunks of this launch: launch chunks t0 .. t0 + total_chunks - 1
  uint64_t t0;
  uint64_t* lens;      // batch launches: stream length of each series (device), else null
  ChunkMeta* meta;     // one per launch chunk, written by the size pass
  uint32_t* gsizes;    // chunk sizes by launch chunk (scan input), written by the size pass
  const uint64_t* offsets;  // exclusive prefix of gsizes, read by the write pass
  uint32_t relative;   // 1: offsets run over all series; a series subtracts its first one
  uint32_t qtag;       // single pass: 16-bit tag of this launch's status words (never 0)
  // single pass (work queue and look-back): qgroups ticket counters at
  // qctr[kQueueStride * g], all 0 at the launch's start; status holds one
  // word per launch chunk
  uint64_t* status;
  uint64_t* qctr;
  Ctl* ctl;
  uint32_t qgroups;
  uint32_t pad2;
};

struct DecompressArgs {
  DecompressSeries one;
  const DecompressSeries* many;
  uint32_t nseries;
  uint32_t total_waves;
  uint64_t total_chunks;
  uint64_t t0;
  const uint64_t* offsets;  // chunk offsets (exclusive prefix of the sizes)
  Ctl* ctl;
  uint32_t epoch;
  uint32_t relative;       // 1: offsets run over all series; a series subtracts its first one
};

constexpr int kCompressWaves = 16;    // default wavefronts per compression workgroup
// The float32 passes run 6 waves per SIMD (their LDS buffer is half the
// float64 one and their registers are held to 80), which workgroups of 8
// waves fill (3 per CU); 16-wave workgroups would fit only one.
constexpr int kCompressWaves32 = 8;
constexpr int compress_waves(int dtype) { return dtype == 1 ? kCompressWaves32 : kCompressWaves; }
constexpr int kDecompressWaves = 4;   // wavefronts per decompression workgroup

// Kernel forms: one instantiation per dtype (1 = f32, 2 = f64) and a mixed
// one (3) that takes either dtype per series.  nw = wavefronts per
// compression workgroup, 8 or 16.
constexpr int kFormMixed = 3;
// pass 1: the size pass of compression (meta, gsizes and the series' size
// arrays); pass 2: the write pass, after a scan of gsizes into offsets.
hipError_t launch_compress(const CompressArgs& a, int form, int pass, int nw, int grid, hipStream_t s);
hipError_t launch_decompress(const DecompressArgs& a, int form, int grid, hipStream_t s);
// Single-pass compression (work queue over chunks, decoupled look-back for
// the offsets): a.status / a.qctr / a.qgroups (<= grid) / a.ctl / a.qtag
// set, the a.qgroups counters cleared beforehand.
hipError_t launch_compress_queue(const CompressArgs& a, int form, int nw, int grid, hipStream_t s);
hipError_t launch_compress_queue_f64(const CompressArgs& a, int nw, int grid, hipStream_t s);
hipError_t launch_compress_queue_f32(const CompressArgs& a, int nw, int grid, hipStream_t s);
hipError_t launch_compress_queue_mixed(const CompressArgs& a, int nw, int grid, hipStream_t s);
const void* compress_queue_kernel_f64(int nw);
const void* compress_queue_kernel_f32(int nw);
const void* compress_queue_kernel_mixed(int nw);
int max_grid_compress_queue(int device, int form, int nw);
// per-form entry points (one translation unit each)
hipError_t launch_compress_f64(const CompressArgs& a, int pass, int nw, int grid, hipStream_t s);
hipError_t launch_compress_f32(const CompressArgs& a, int pass, int nw, int grid, hipStream_t s);
hipError_t launch_compress_mixed(const CompressArgs& a, int pass, int nw, int grid, hipStream_t s);
hipError_t launch_decompress_f64(const DecompressArgs& a, int grid, hipStream_t s);
hipError_t launch_decompress_f32(const DecompressArgs& a, int grid, hipStream_t s);
hipError_t launch_decompress_mixed(const DecompressArgs& a, int grid, hipStream_t s);
const void* compress_kernel_f64(int pass, int nw);
const void* compress_kernel_f32(int pass, int nw);
const void* compress_kernel_mixed(int pass, int nw);
const void* decompress_kernel_f64();
const void* decompress_kernel_f32();
const void* decompress_kernel_mixed();
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s);
// Exclusive prefix of n chunk sizes into offsets; sizes outside [lo, hi] or
// a total other than expect (unless expect is UINT64_MAX) store the epoch in
// ctl->error.  tile_tmp holds
// scan_tiles(n) words.
hipError_t launch_scan_sizes(const uint32_t* sizes, uint64_t n, uint32_t lo, uint32_t hi, uint64_t expect,
                             uint64_t* tile_tmp, uint64_t* offsets, Ctl* ctl, uint32_t epoch, hipStream_t s);
uint64_t scan_tiles(uint64_t n);
// Batch decompression, before the scan: reads every series' stream header
// on the device, checks it against the descriptor (value count, dtype,
// lengths) and stores its payload byte count in the descriptor; then copies
// every series' chunk sizes into one array indexed by launch chunk.
hipError_t launch_batch_dprep(DecompressSeries* many, uint32_t ns, uint64_t total_chunks, uint32_t* sizes_out,
                              Ctl* ctl, uint32_t epoch, hipStream_t s);
// Compression under an ablation variant of Sec. 5.4.2 (variant 1: Elf's
// decimal places, 2: every row sparse, 3: every row dense), one dtype per
// launch (form 1 or 2), kVariantWaves wavefronts per workgroup.
constexpr int kVariantWaves = 8;
hipError_t launch_compress_variant(const CompressArgs& a, int form, int variant, int pass, int grid, hipStream_t s);
const void* compress_variant_kernel_f64(int variant, int pass);
const void* compress_variant_kernel_f32(int variant, int pass);
// Largest number of co-resident workgroups of each kernel on the device.
int max_grid_compress(int device, int form, int pass, int nw);
int max_grid_compress_variant(int device, int form, int variant, int pass);
int max_grid_decompress(int device, int form);

}  // namespace falcon_dev
