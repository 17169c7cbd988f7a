// internal.hpp -- launch interface between the C ABI (api.cpp) and the
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace falcon_dev {

// Control block of one launch: ticket counter handing out chunks in order,
// exit counter (the last wave out resets both, so the next launch finds them
// at zero), and an error word that receives the launch epoch when a chunk
// fails a check.
struct Ctl {
  uint32_t ticket;
  uint32_t exited;
  uint32_t error;
  uint32_t pad;
};

// One array to compress.  chunk0 is the global index of its first chunk in
// the launch (prefix of the chunk counts of the series before it).
struct CompressSeries {
  const void* in;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk0;
  uint64_t group0;   // index of the series' first 64-chunk group status word
  uint32_t dtype;    // 1 = f32, 2 = f64
  uint32_t pad;
};

struct DecompressSeries {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk0;
  uint64_t group0;
  uint64_t payload_bytes;
  uint32_t dtype;
  uint32_t pad;
};

struct CompressArgs {
  CompressSeries one;            // used when nseries == 1
  const CompressSeries* many;    // device array, sorted by chunk0, when nseries > 1
  uint32_t nseries;
  uint32_t total_waves;
  uint64_t total_chunks;
  uint64_t* status;    // one word per chunk of the launch
  uint64_t* gstatus;   // one word per 64-chunk group of each series
  Ctl* ctl;
  uint32_t epoch;
  uint32_t pad;
};

struct DecompressArgs {
  DecompressSeries one;
  const DecompressSeries* many;
  uint32_t nseries;
  uint32_t total_waves;
  uint64_t total_chunks;
  const uint64_t* status;  // chunk offsets (exclusive prefix of the sizes)
  Ctl* ctl;
  uint32_t epoch;
  uint32_t pad;
};

constexpr int kCompressWaves = 16;    // wavefronts per compression workgroup
constexpr int kDecompressWaves = 4;   // wavefronts per decompression workgroup

hipError_t launch_compress(const CompressArgs& a, int dtype, int grid, hipStream_t s);
hipError_t launch_decompress(const DecompressArgs& a, int dtype, int grid, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s);
// Exclusive prefix of n chunk sizes into offsets; sizes outside [lo, hi] or
// a total other than expect store the epoch in ctl->error.  tile_tmp holds
// scan_tiles(n) words.
hipError_t launch_scan_sizes(const uint32_t* sizes, uint64_t n, uint32_t lo, uint32_t hi, uint64_t expect,
                             uint64_t* tile_tmp, uint64_t* offsets, Ctl* ctl, uint32_t epoch, hipStream_t s);
uint64_t scan_tiles(uint64_t n);
// Largest number of co-resident workgroups of each kernel on the device.
int max_grid_compress(int device, int dtype);
int max_grid_decompress(int device, int dtype);

}  // namespace falcon_dev
