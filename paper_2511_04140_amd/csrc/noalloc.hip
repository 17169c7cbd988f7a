// noalloc.hip -- falcon_compress_noalloc: two-pass compression whose scratch
// (control block, scan tile sums, per-chunk metadata, chunk sizes, chunk
// offsets) lives in a fixed device array of this file instead of memory
// allocated by a context, for callers that cannot allocate.
//
// The array is per device: each GPU the library runs on holds its own copy
// at its own address, kept until the process ends.  Host code never passes
// the array's name to a kernel or a copy (in host code it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns,
// taken once per device with that device current and kept in g_state.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "context.hpp"

using namespace falcon_dev;

namespace {

// Largest input, in chunks of 1025 values: 2^19 chunks (537,395,200 values).
constexpr uint64_t kMaxChunks = 1ull << 19;
constexpr size_t kCtlBytes = 256;
constexpr size_t kTileWords = (kMaxChunks + 4095) / 4096 + 1;  // scan tile sums (scan_tiles + 1)
constexpr size_t kTilesBytes = ((kTileWords * 8 + 255) / 256) * 256;
constexpr size_t kMetaBytes = kMaxChunks * sizeof(ChunkMeta);
constexpr size_t kSizesBytes = kMaxChunks * 4;
constexpr size_t kOffsetsBytes = kMaxChunks * 8;
constexpr size_t kScratchBytes = kCtlBytes + kTilesBytes + kMetaBytes + kSizesBytes + kOffsetsBytes;

static_assert(sizeof(ChunkMeta) == 16, "metadata words of 16 bytes");
static_assert(kMetaBytes % 256 == 0 && kSizesBytes % 256 == 0, "sub-arrays stay 256-byte aligned");

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceState {
  bool ready = false;
  uint8_t* ptr = nullptr;  // device address of this device's copy of scratch
  int grid[3][3] = {};     // [form][pass] co-resident workgroups of the compression kernels
};
DeviceState g_state[kMaxDevices];
std::mutex g_lock;

// Set-up on the current device: the scratch's device address and the
// kernels' co-resident grids.  Allocates nothing.
falcon_status setup(int dev, DeviceState** out) {
  if (dev < 0 || dev >= kMaxDevices) return FALCON_ERR_DEVICE;
  std::lock_guard<std::mutex> g(g_lock);
  DeviceState& d = g_state[dev];
  if (!d.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FALCON_ERR_DEVICE;
    d.ptr = static_cast<uint8_t*>(p);
    for (int form = 1; form <= 2; ++form)
      for (int pass = 1; pass <= 2; ++pass)
        d.grid[form][pass] = max_grid_compress(dev, form, pass, compress_waves(form));
    d.ready = true;
  }
  *out = &d;
  return FALCON_OK;
}

int grid_of(int max_grid, uint64_t nchunks, int nw) {
  uint64_t want = (nchunks + nw - 1) / nw;
  if (want < 1) want = 1;
  return (int)(want < (uint64_t)max_grid ? want : (uint64_t)max_grid);
}

}  // namespace

namespace falcon_host {

// Called by falcon_create for its device, so that the set-up does not wait
// for the first falcon_compress_noalloc (which may run under graph capture).
falcon_status noalloc_setup(int device) {
  DeviceState* d;
  return setup(device, &d);
}

}  // namespace falcon_host

extern "C" falcon_status falcon_compress_noalloc(const void* d_in, size_t n, falcon_dtype dt, void* d_out,
                                                 size_t out_cap, size_t* d_out_len, void* stream) {
  using namespace falcon_host;
  if (!d_out || (n && !d_in)) return FALCON_ERR_INVALID_ARG;
  const size_t es = elem_size(dt);
  if (es == 0) return FALCON_ERR_INVALID_ARG;
  if (((uintptr_t)d_in % es) || ((uintptr_t)d_out % 4) || ((uintptr_t)d_out_len % 8)) return FALCON_ERR_INVALID_ARG;
  if (out_cap < falcon_compress_bound(n, dt)) return FALCON_ERR_BUFFER_TOO_SMALL;
  const uint64_t nc = chunks_of(n);
  if (nc > kMaxChunks) return FALCON_ERR_OUT_OF_MEMORY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FALCON_ERR_DEVICE;
  DeviceState* d;
  falcon_status st = setup(dev, &d);
  if (st != FALCON_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* base = d->ptr;
  Ctl* ctl = reinterpret_cast<Ctl*>(base);
  uint64_t* tiles = reinterpret_cast<uint64_t*>(base + kCtlBytes);
  ChunkMeta* meta = reinterpret_cast<ChunkMeta*>(base + kCtlBytes + kTilesBytes);
  uint32_t* sizes = reinterpret_cast<uint32_t*>(base + kCtlBytes + kTilesBytes + kMetaBytes);
  uint64_t* offsets = reinterpret_cast<uint64_t*>(base + kCtlBytes + kTilesBytes + kMetaBytes + kSizesBytes);
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
  a.lens = reinterpret_cast<uint64_t*>(d_out_len);
  a.meta = meta;
  a.gsizes = sizes;
  a.offsets = offsets;
  a.relative = 0;
  // every scratch word is written before it is read: the size pass writes
  // meta and sizes, the scan the tile sums and offsets; the control block
  // takes an error word only for a chunk size outside [0, 2^32), which never
  // happens, so nothing needs clearing between calls
  const int nw = compress_waves((int)dt);
  const int g1 = grid_of(d->grid[dt][1], nc, nw), g2 = grid_of(d->grid[dt][2], nc, nw);
  if (nc) {
    a.total_waves = (uint32_t)(g1 * nw);
    if ((st = dev_err(launch_compress(a, (int)dt, 1, nw, g1, s))) != FALCON_OK) return st;
    if ((st = dev_err(launch_scan_sizes(sizes, nc, 0, ~0u, ~0ull, tiles, offsets, ctl, 1, s))) != FALCON_OK)
      return st;
  }
  a.total_waves = (uint32_t)(g2 * nw);
  if ((st = dev_err(launch_compress(a, (int)dt, 2, nw, g2, s))) != FALCON_OK) return st;
  // an empty input has no chunk to write its length
  if (n == 0 && d_out_len)
    return dev_err(launch_fill_u64(reinterpret_cast<uint64_t*>(d_out_len), 1, 32, s));
  return FALCON_OK;
}
