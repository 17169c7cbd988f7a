// kernels_common.hip -- prefix scan of chunk sizes, batch preparation,
// fill, and the dispatch of launches to the per-form translation units.
#include "codec_kernels.hpp"

namespace falcon_dev {

// ---------------------------------------------------------------------------
// Prefix sum of a chunk size array into chunk offsets (decompression, Sec. 4:
// the size array is scanned into the offset array).  Three small kernels over
// tiles of kScanTile sizes: tile sums, a scan of the tile sums (which also
// checks the total against the payload byte count), and the per-tile scan.
// Sizes outside [lo, hi] set the error word.
// ---------------------------------------------------------------------------
constexpr int kScanTile = 4096;  // 256 threads x 16 sizes

__device__ __forceinline__ uint64_t block_excl_scan256(uint64_t v, uint64_t* tmp, uint64_t& total) {
  // tmp: 4 words of LDS (one per wave)
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t incl = wave_incl_scan64(v, lane);
  if (lane == 63) tmp[wid] = incl;
  __syncthreads();
  uint64_t before = 0;
  for (int i = 0; i < wid; ++i) before += tmp[i];
  total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
  __syncthreads();
  return before + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t* sizes, uint64_t n, uint32_t lo, uint32_t hi,
                                                    uint64_t* tile_sum, Ctl* ctl, uint32_t epoch) {
  __shared__ uint64_t tmp[4];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * 16;
  uint64_t sum = 0;
  bool bad = false;
  for (int k = 0; k < 16; ++k) {
    if (base + k < n) {
      const uint32_t v = sizes[base + k];
      bad |= v < lo || v > hi;
      sum += v;
    }
  }
  if (bad) __hip_atomic_store(&ctl->error, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint64_t total;
  block_excl_scan256(sum, tmp, total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_tile_sums(uint64_t* tile_sum, uint64_t ntiles, uint64_t expect,
                                                        Ctl* ctl, uint32_t epoch) {
  __shared__ uint64_t tmp[4];
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < ntiles; b0 += 256) {
    const uint64_t i = b0 + threadIdx.x;
    const uint64_t v = i < ntiles ? tile_sum[i] : 0;
    uint64_t total;
    const uint64_t ex = block_excl_scan256(v, tmp, total);
    if (i < ntiles) tile_sum[i] = carry + ex;  // becomes the tile's offset
    carry += total;
  }
  if (threadIdx.x == 0 && expect != ~0ull && carry != expect)
    __hip_atomic_store(&ctl->error, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* sizes, uint64_t n, const uint64_t* tile_off,
                                                    uint64_t* offsets) {
  __shared__ uint64_t tmp[4];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * 16;
  uint32_t v[16];
  uint64_t sum = 0;
  for (int k = 0; k < 16; ++k) {
    v[k] = base + k < n ? sizes[base + k] : 0u;
    sum += v[k];
  }
  uint64_t total;
  uint64_t run = tile_off[blockIdx.x] + block_excl_scan256(sum, tmp, total);
  for (int k = 0; k < 16; ++k) {
    if (base + k < n) offsets[base + k] = run;
    run += v[k];
  }
}

__global__ void k_fill_u64(uint64_t* p, size_t n, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Batch decompression preparation.
// ---------------------------------------------------------------------------
// One thread per series: checks the stream header against the descriptor
// and stores the payload byte count.  A failing series gets payload 0, so
// that every one of its chunks fails its bounds check without reading.
__global__ __launch_bounds__(256) void k_batch_headers(DecompressSeries* many, uint32_t ns, Ctl* ctl,
                                                       uint32_t epoch) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  DecompressSeries& sd = many[i];
  const uint64_t nc = (sd.n + kChunk - 1) / kChunk;
  const uint32_t* h = reinterpret_cast<const uint32_t*>(sd.in);
  uint64_t payload = 0;
  bool ok = sd.in_len >= kHdrBytes + 4 * nc;  // also checked on the host
  if (ok) {
    ok = h[0] == 0x4E434C46u && h[1] == (1u | (sd.dtype << 8)) && h[2] == (uint32_t)kChunk && h[3] == 0 &&
         ((uint64_t)h[4] | ((uint64_t)h[5] << 32)) == sd.n;
    payload = (uint64_t)h[6] | ((uint64_t)h[7] << 32);
    ok = ok && payload <= sd.in_len - kHdrBytes - 4 * nc && (sd.n != 0 || payload == 0);
  }
  if (!ok) {
    payload = 0;
    __hip_atomic_store(&ctl->error, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  sd.payload_bytes = payload;
}

// Copies the chunk sizes of all series into one array indexed by launch
// chunk t; each thread handles 16 consecutive chunks.
__global__ __launch_bounds__(256) void k_gather_sizes(const DecompressSeries* many, uint32_t ns, uint64_t total,
                                                      uint32_t* out) {
  const uint64_t t0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (t0 >= total) return;
  uint32_t lo = 0, hi = ns - 1;  // last series with chunk0 <= t0
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (many[mid].chunk0 <= t0) lo = mid;
    else hi = mid - 1;
  }
  uint32_t i = lo;
  for (uint64_t t = t0; t < t0 + 16 && t < total; ++t) {
    while (i + 1 < ns && many[i + 1].chunk0 <= t) ++i;
    out[t] = reinterpret_cast<const uint32_t*>(many[i].in + kHdrBytes)[t - many[i].chunk0];
  }
}

hipError_t launch_batch_dprep(DecompressSeries* many, uint32_t ns, uint64_t total_chunks, uint32_t* sizes_out,
                              Ctl* ctl, uint32_t epoch, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_headers, dim3((ns + 255) / 256), dim3(256), 0, s, many, ns, ctl, epoch);
  if (total_chunks) {
    const uint64_t threads = (total_chunks + 15) / 16;
    hipLaunchKernelGGL(k_gather_sizes, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (const DecompressSeries*)many, ns, total_chunks, sizes_out);
  }
  return hipGetLastError();
}

hipError_t launch_compress(const CompressArgs& a, int form, int pass, int nw, int grid, hipStream_t s) {
  if (form == 2) return launch_compress_f64(a, pass, nw, grid, s);
  if (form == 1) return launch_compress_f32(a, pass, nw, grid, s);
  return launch_compress_mixed(a, pass, nw, grid, s);
}

hipError_t launch_compress_queue(const CompressArgs& a, int form, int nw, int grid, hipStream_t s) {
  if (form == 2) return launch_compress_queue_f64(a, nw, grid, s);
  if (form == 1) return launch_compress_queue_f32(a, nw, grid, s);
  return launch_compress_queue_mixed(a, nw, grid, s);
}

hipError_t launch_compress_variant(const CompressArgs& a, int form, int variant, int pass, int grid, hipStream_t s) {
  const void* fn = form == 2 ? compress_variant_kernel_f64(variant, pass)
                             : form == 1 ? compress_variant_kernel_f32(variant, pass) : nullptr;
  if (!fn) return hipErrorInvalidValue;
  CompressArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(64 * kVariantWaves), args, 0, s);
}

hipError_t launch_decompress(const DecompressArgs& a, int form, int grid, hipStream_t s) {
  if (form == 2) return launch_decompress_f64(a, grid, s);
  if (form == 1) return launch_decompress_f32(a, grid, s);
  return launch_decompress_mixed(a, grid, s);
}

hipError_t launch_scan_sizes(const uint32_t* sizes, uint64_t n, uint32_t lo, uint32_t hi, uint64_t expect,
                             uint64_t* tile_tmp, uint64_t* offsets, Ctl* ctl, uint32_t epoch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, s, sizes, n, lo, hi, tile_tmp, ctl, epoch);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(256), 0, s, tile_tmp, ntiles, expect, ctl, epoch);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(256), 0, s, sizes, n, tile_tmp, offsets);
  return hipGetLastError();
}
uint64_t scan_tiles(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

static int max_grid_of(const void* fn, int device, int block) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 256;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return per_cu * prop.multiProcessorCount;
}

int max_grid_compress(int device, int form, int pass, int nw) {
  const void* fn = form == 2 ? compress_kernel_f64(pass, nw)
                             : form == 1 ? compress_kernel_f32(pass, nw) : compress_kernel_mixed(pass, nw);
  return max_grid_of(fn, device, 64 * nw);
}

int max_grid_compress_queue(int device, int form, int nw) {
  const void* fn = form == 2 ? compress_queue_kernel_f64(nw)
                             : form == 1 ? compress_queue_kernel_f32(nw) : compress_queue_kernel_mixed(nw);
  return max_grid_of(fn, device, 64 * nw);
}

int max_grid_compress_variant(int device, int form, int variant, int pass) {
  const void* fn = form == 2 ? compress_variant_kernel_f64(variant, pass)
                             : form == 1 ? compress_variant_kernel_f32(variant, pass) : nullptr;
  return fn ? max_grid_of(fn, device, 64 * kVariantWaves) : 0;
}

int max_grid_decompress(int device, int form) {
  const void* fn = form == 2 ? decompress_kernel_f64() : form == 1 ? decompress_kernel_f32()
                                                                    : decompress_kernel_mixed();
  return max_grid_of(fn, device, 64 * kWavesD);
}

}  // namespace falcon_dev
