// kernels_mixed.hip -- kernels that take series of both dtypes in one launch
// (the wave branches on the dtype of each chunk's series), and their
// launchers.
#include "codec_kernels.hpp"

namespace falcon_dev {

__global__ __launch_bounds__(64 * kWavesD) __attribute__((amdgpu_waves_per_eu(4))) void k_decompress_mixed(
    DecompressArgs a) {
  __shared__ BlockLdsT<kWavesD> sm;
  load_tables(sm.tab);
  __syncthreads();
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);  // wave-uniform: keeps the chunk loop scalar
  uint8_t* buf = wave_bytes(sm, wid);
  decompress_loop(a, buf, lane, wid,
                  [&](const DecompressSeries& sd, uint64_t c, uint32_t S, uint32_t pad, uint32_t total, bool bad) {
                    if (uniform(sd.dtype) == 2)
                      decompress_chunk<TF64>(sm.tab, buf, sd, c, S, pad, total, bad, a.epoch, lane, a.ctl);
                    else
                      decompress_chunk<TF32>(sm.tab, buf, sd, c, S, pad, total, bad, a.epoch, lane, a.ctl);
                  });
}

template <int NW>
static hipError_t launch_nw(const CompressArgs& a, int pass, int grid, hipStream_t s) {
  if (pass == 1) hipLaunchKernelGGL((k_compress_pass_mixed<NW, 1>), dim3(grid), dim3(64 * NW), 0, s, a);
  else hipLaunchKernelGGL((k_compress_pass_mixed<NW, 2>), dim3(grid), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_compress_mixed(const CompressArgs& a, int pass, int nw, int grid, hipStream_t s) {
  return nw == 8 ? launch_nw<8>(a, pass, grid, s) : launch_nw<16>(a, pass, grid, s);
}

hipError_t launch_decompress_mixed(const DecompressArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_decompress_mixed, dim3(grid), dim3(64 * kWavesD), 0, s, a);
  return hipGetLastError();
}

template <int NW>
static const void* kernel_nw(int pass) {
  if (pass == 1) return reinterpret_cast<const void*>(&k_compress_pass_mixed<NW, 1>);
  return reinterpret_cast<const void*>(&k_compress_pass_mixed<NW, 2>);
}

const void* compress_kernel_mixed(int pass, int nw) { return nw == 8 ? kernel_nw<8>(pass) : kernel_nw<16>(pass); }

const void* decompress_kernel_mixed() { return reinterpret_cast<const void*>(&k_decompress_mixed); }

hipError_t launch_compress_queue_mixed(const CompressArgs& a, int nw, int grid, hipStream_t s) {
  if (nw == 8) hipLaunchKernelGGL((k_compress_queue_mixed<8>), dim3(grid), dim3(64 * 8), 0, s, a);
  else hipLaunchKernelGGL((k_compress_queue_mixed<16>), dim3(grid), dim3(64 * 16), 0, s, a);
  return hipGetLastError();
}

const void* compress_queue_kernel_mixed(int nw) {
  return nw == 8 ? reinterpret_cast<const void*>(&k_compress_queue_mixed<8>)
                 : reinterpret_cast<const void*>(&k_compress_queue_mixed<16>);
}

}  // namespace falcon_dev
