// kernels_f32.hip -- the f32 instantiations of the compression and
// decompression kernels (codec_kernels.hpp) and their launchers.
#include "codec_kernels.hpp"

namespace falcon_dev {

template <int NW>
static hipError_t launch_nw(const CompressArgs& a, int pass, int grid, hipStream_t s) {
  if (pass == 1) hipLaunchKernelGGL((k_compress_pass<TF32, NW, 1>), dim3(grid), dim3(64 * NW), 0, s, a);
  else hipLaunchKernelGGL((k_compress_pass<TF32, NW, 2>), dim3(grid), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_compress_f32(const CompressArgs& a, int pass, int nw, int grid, hipStream_t s) {
  return nw == 8 ? launch_nw<8>(a, pass, grid, s) : launch_nw<16>(a, pass, grid, s);
}

hipError_t launch_decompress_f32(const DecompressArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_decompress<TF32>, dim3(grid), dim3(64 * kWavesD), 0, s, a);
  return hipGetLastError();
}

template <int NW>
static const void* kernel_nw(int pass) {
  if (pass == 1) return reinterpret_cast<const void*>(&k_compress_pass<TF32, NW, 1>);
  return reinterpret_cast<const void*>(&k_compress_pass<TF32, NW, 2>);
}

const void* compress_kernel_f32(int pass, int nw) { return nw == 8 ? kernel_nw<8>(pass) : kernel_nw<16>(pass); }

template <int V>
static const void* size_pass_variant_f32() {
  return reinterpret_cast<const void*>(&k_compress_pass<TF32, kVariantWaves, 1, V, kVarWaveBlocks>);
}

// The write pass follows the flags the size pass stored, so one write
// kernel serves every variant.
const void* compress_variant_kernel_f32(int variant, int pass) {
  if (pass == 2)
    return reinterpret_cast<const void*>(&k_compress_pass<TF32, kVariantWaves, 2, kVarFalcon, kVarWaveBlocks>);
  if (variant == kVarElf) return size_pass_variant_f32<kVarElf>();
  if (variant == kVarSparse) return size_pass_variant_f32<kVarSparse>();
  if (variant == kVarDense) return size_pass_variant_f32<kVarDense>();
  return nullptr;
}

const void* decompress_kernel_f32() { return reinterpret_cast<const void*>(&k_decompress<TF32>); }

hipError_t launch_compress_queue_f32(const CompressArgs& a, int nw, int grid, hipStream_t s) {
  if (nw == 8) hipLaunchKernelGGL((k_compress_queue<TF32, 8>), dim3(grid), dim3(64 * 8), 0, s, a);
  else hipLaunchKernelGGL((k_compress_queue<TF32, 16>), dim3(grid), dim3(64 * 16), 0, s, a);
  return hipGetLastError();
}

const void* compress_queue_kernel_f32(int nw) {
  return nw == 8 ? reinterpret_cast<const void*>(&k_compress_queue<TF32, 8>)
                 : reinterpret_cast<const void*>(&k_compress_queue<TF32, 16>);
}

}  // namespace falcon_dev
