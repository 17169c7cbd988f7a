// kernels_f64.hip -- the f64 instantiations of the compression and
// decompression kernels (codec_kernels.hpp) and their launchers.
#include "codec_kernels.hpp"

namespace falcon_dev {

hipError_t launch_compress_f64(const CompressArgs& a, int nw, int grid, hipStream_t s) {
  if (nw == 8) hipLaunchKernelGGL((k_compress<TF64, 8>), dim3(grid), dim3(64 * 8), 0, s, a);
  else hipLaunchKernelGGL((k_compress<TF64, 16>), dim3(grid), dim3(64 * 16), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decompress_f64(const DecompressArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_decompress<TF64>, dim3(grid), dim3(64 * kWavesD), 0, s, a);
  return hipGetLastError();
}

const void* compress_kernel_f64(int nw) {
  return nw == 8 ? reinterpret_cast<const void*>(&k_compress<TF64, 8>)
                 : reinterpret_cast<const void*>(&k_compress<TF64, 16>);
}

const void* decompress_kernel_f64() { return reinterpret_cast<const void*>(&k_decompress<TF64>); }

}  // namespace falcon_dev
