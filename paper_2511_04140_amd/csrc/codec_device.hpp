// codec_device.hpp -- device-side building blocks of the Falcon codec for
// CDNA4 (gfx950, wave64).
//
// Work decomposition: one wavefront owns one chunk of 1025 values (the paper
// gives one thread a chunk, Sec. 3 / Alg. 3; on CDNA a 64-lane wave keeps the
// chunk in registers and LDS and moves it with coalesced loads).  Inside a
// wave two layouts are used:
//   slot layout        lane L, slot k holds value index 1 + 64k + L
//                      (k = 0..15); value index 0 (v_1) is held by every
//                      lane.  Used for the coalesced load and for the
//                      per-value integer conversion.
//   contiguous layout  lane L holds entries e_{16L..16L+15} of the delta
//                      sequence (entry j = z_{j+2}), i.e. the 16 entries
//                      that make up bytes 2L and 2L+1 of every row of the
//                      transposed bit-plane matrix.  Used for the bit-plane
//                      transpose and the row encoding.
// The switch between the two goes through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace falcon_dev {

constexpr int kChunk = 1025;      // values per chunk (Sec. 5.1.4, n = 64k + 1)
constexpr int kWavesC = 16;       // wavefronts per compression workgroup
constexpr int kWavesD = 4;        // wavefronts per decompression workgroup
constexpr int kGSlots = kChunk + 65;         // skewed slots: one pad every 16
constexpr int kWaveLds = kGSlots * 8;        // 8720 bytes per wave
constexpr int kHdrBytes = 32;

// fl(10^k): binary64 for k = -22..22, binary32 for k = -10..10, each the
// value nearest to the exact power (printed by gen_pow10.py).  For
// 0 <= k <= 22 (binary64) and 0 <= k <= 10 (binary32) the entries are exact
// (Thm. 3: 5^k fits the significand).
__constant__ double c_pow10_f64[45] = {
    0x1.e392010175ee6p-74, 0x1.2e3b40a0e9b4fp-70, 0x1.79ca10c924223p-67, 0x1.d83c94fb6d2acp-64,
    0x1.2725dd1d243acp-60, 0x1.70ef54646d497p-57, 0x1.cd2b297d889bcp-54, 0x1.203af9ee75616p-50,
    0x1.6849b86a12b9bp-47, 0x1.c25c268497682p-44, 0x1.19799812dea11p-40, 0x1.5fd7fe1796495p-37,
    0x1.b7cdfd9d7bdbbp-34, 0x1.12e0be826d695p-30, 0x1.5798ee2308c3ap-27, 0x1.ad7f29abcaf48p-24,
    0x1.0c6f7a0b5ed8dp-20, 0x1.4f8b588e368f1p-17, 0x1.a36e2eb1c432dp-14, 0x1.0624dd2f1a9fcp-10,
    0x1.47ae147ae147bp-7, 0x1.999999999999ap-4, 0x1.0000000000000p+0, 0x1.4000000000000p+3,
    0x1.9000000000000p+6, 0x1.f400000000000p+9, 0x1.3880000000000p+13, 0x1.86a0000000000p+16,
    0x1.e848000000000p+19, 0x1.312d000000000p+23, 0x1.7d78400000000p+26, 0x1.dcd6500000000p+29,
    0x1.2a05f20000000p+33, 0x1.74876e8000000p+36, 0x1.d1a94a2000000p+39, 0x1.2309ce5400000p+43,
    0x1.6bcc41e900000p+46, 0x1.c6bf526340000p+49, 0x1.1c37937e08000p+53, 0x1.6345785d8a000p+56,
    0x1.bc16d674ec800p+59, 0x1.158e460913d00p+63, 0x1.5af1d78b58c40p+66, 0x1.b1ae4d6e2ef50p+69,
    0x1.0f0cf064dd592p+73};
__constant__ float c_pow10_f32[21] = {
    0x1.b7cdfep-34f, 0x1.12e0bep-30f, 0x1.5798eep-27f, 0x1.ad7f2ap-24f, 0x1.0c6f7ap-20f,
    0x1.4f8b58p-17f, 0x1.a36e2ep-14f, 0x1.0624dep-10f, 0x1.47ae14p-7f, 0x1.99999ap-4f,
    0x1.000000p+0f, 0x1.400000p+3f, 0x1.900000p+6f, 0x1.f40000p+9f, 0x1.388000p+13f,
    0x1.86a000p+16f, 0x1.e84800p+19f, 0x1.312d00p+23f, 0x1.7d7840p+26f, 0x1.dcd650p+29f,
    0x1.2a05f2p+33f};

// Shared memory of one workgroup: the power tables (copied once per block so
// that per-lane lookups are LDS reads) and one byte buffer per wavefront.
struct __attribute__((aligned(16))) LdsTables {
  double p64[48];
  float p32[24];
};
template <int NW, int WB = kWaveLds / 16>
struct __attribute__((aligned(16))) BlockLdsT {
  LdsTables tab;
  uint4 wave[NW][WB];
};

// Global-memory views of generic pointers.  An access through a generic
// pointer compiles to a flat instruction, which counts against the LDS
// counter as well as the vector-memory counter, so every wait for an LDS
// access would also wait for outstanding HBM loads (such as the prefetch of
// the next chunk).  Accesses through these views compile to global
// instructions, which count against the vector-memory counter only.
template <class T>
using global_ptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ global_ptr<T> gbl(T* p) {
  return (global_ptr<T>)p;
}
// Constant-address-space views for wave-uniform reads of data no kernel of
// the launch writes (chunk sizes, offsets, per-chunk metadata, series
// descriptors, all produced by earlier launches or the caller): with a
// uniform address they compile to scalar loads, which count against the LDS
// counter instead of the vector-memory counter, so reading them does not
// wait for the wave's outstanding HBM stores.  Read only, never written.
template <class T>
using const_ptr = __attribute__((address_space(4))) const T*;
template <class T>
__device__ __forceinline__ const_ptr<T> cst(const T* p) {
  return (const_ptr<T>)p;
}

// Raw buffer stores: out-of-range lanes are dropped by the hardware, so a
// store with some lanes off needs neither an execution mask nor a branch,
// and every loop iteration issues the same number of memory instructions.
// That lets the compiler wait for a prefetched load with an exact count
// (vmcnt) instead of also waiting for the stores issued after it.
// Descriptor: base, stride 0, num_records bytes, gfx9-family word 3.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t store_window(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
constexpr uint32_t kDropOffset = 0x80000000u;  // beyond any window: the store is dropped
constexpr int kNonTemporal = 2;                 // aux bit: no temporal reuse expected

// 16-byte global load and store (a builtin vector type, which can be read and
// written through an address-space-qualified pointer).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 gload16(const void* p) {
  const u32x4 v = *gbl(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
// The store carries the non-temporal hint: it writes streamed output that
// no later kernel of the same operation reads, and leaves no dirty lines in
// the caches for the next kernel to write back.
__device__ __forceinline__ void gstore16_nt(void* p, const uint4& v) {
  u32x4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  __builtin_nontemporal_store(w, gbl(reinterpret_cast<u32x4*>(p)));
}

__device__ __forceinline__ void load_tables(LdsTables& s) {
  for (int i = threadIdx.x; i < 45; i += blockDim.x) s.p64[i] = c_pow10_f64[i];
  for (int i = threadIdx.x; i < 21; i += blockDim.x) s.p32[i] = c_pow10_f32[i];
}

// ---------------------------------------------------------------------------
// Per-dtype traits.  Constants: alpha <= AMAX keeps 10^alpha exact (Thm. 3),
// beta <= BMAX is the precision guard (Thm. 2, Thm. 4); the binary32 values
// (10, 6) follow from the same arguments with a 24-bit significand.
// ---------------------------------------------------------------------------
struct TF64 {
  using F = double;
  using U = uint64_t;
  using S = int64_t;
  static constexpr int W = 64, ZB = 8, AMAX = 22, BMAX = 15, MANT = 52;
  static constexpr int MARKSTEIN_MAX = 21;  // decoder's division-free quotient up to 5^alpha < 2^51
  static constexpr int EXPMAX = 0x7FF, BIAS = 1023;
  // |v| >= 2^50 > 10^15 means FL10 >= 15 (beta > 15 at alpha = 0);
  // |v| < 2^-74 < fl(10^-22) means FL10 <= -23 (decimal place > 22).
  static constexpr int E2_HI = 50, E2_LO = -75;
  static constexpr int BOUND = 3 + ZB + 8 + 64 * 128;  // 8211
  static constexpr int POFF = 22;
  static __device__ __forceinline__ F f(U b) { return __longlong_as_double((long long)b); }
  static __device__ __forceinline__ U u(F v) { return (U)__double_as_longlong(v); }
  static __device__ __forceinline__ F mu_scale() { return 0x1p-52; }
  static __device__ __forceinline__ F rnd(F x) { return __builtin_rint(x); }
  static __device__ __forceinline__ F abs(F x) { return __builtin_fabs(x); }
  static __device__ __forceinline__ F fma(F a, F b, F c) { return __builtin_fma(a, b, c); }
  static __device__ __forceinline__ F ldexp(F x, int k) { return __builtin_ldexp(x, k); }
  static constexpr U MANT_MASK = (1ull << MANT) - 1;
  static __device__ __forceinline__ int expf(U b) { return (int)((b >> MANT) & EXPMAX); }
  static __device__ __forceinline__ U mag(U b) { return b & 0x7FFFFFFFFFFFFFFFull; }
  // r is an integer with |r| < 2^51: r + 1.5 * 2^52 is exact and its low
  // significand bits are r (two's complement offset).
  static __device__ __forceinline__ S to_int(F r) {
    F t = r + 6755399441055744.0;
    return (S)(u(t) - 0x4338000000000000ull);
  }
  static __device__ __forceinline__ F pow10(const LdsTables& s, int k) { return s.p64[k + POFF]; }
};

struct TF32 {
  using F = float;
  using U = uint32_t;
  using S = int32_t;
  static constexpr int W = 32, ZB = 4, AMAX = 10, BMAX = 6, MANT = 23;
  static constexpr int MARKSTEIN_MAX = 10;  // decoder's division-free quotient (every alpha)
  static constexpr int EXPMAX = 0xFF, BIAS = 127;
  // |v| >= 2^20 > 10^6 means FL10 >= 6; |v| < 2^-34 < fl(10^-10) means
  // FL10 <= -11.
  static constexpr int E2_HI = 20, E2_LO = -35;
  static constexpr int BOUND = 3 + ZB + 4 + 32 * 128;  // 4107
  static constexpr int POFF = 10;
  static __device__ __forceinline__ F f(U b) { return __uint_as_float(b); }
  static __device__ __forceinline__ U u(F v) { return __float_as_uint(v); }
  static __device__ __forceinline__ F mu_scale() { return 0x1p-23f; }
  static __device__ __forceinline__ F rnd(F x) { return __builtin_rintf(x); }
  static __device__ __forceinline__ F abs(F x) { return __builtin_fabsf(x); }
  static __device__ __forceinline__ F fma(F a, F b, F c) { return __builtin_fmaf(a, b, c); }
  static __device__ __forceinline__ F ldexp(F x, int k) { return __builtin_ldexpf(x, k); }
  static constexpr U MANT_MASK = (1u << MANT) - 1;
  static __device__ __forceinline__ int expf(U b) { return (int)((b >> MANT) & EXPMAX); }
  static __device__ __forceinline__ U mag(U b) { return b & 0x7FFFFFFFu; }
  static __device__ __forceinline__ S to_int(F r) {
    F t = r + 12582912.0f;  // 1.5 * 2^23, exact for |r| < 2^22
    return (S)(u(t) - 0x4B400000u);
  }
  static __device__ __forceinline__ F pow10(const LdsTables& s, int k) { return s.p32[k + POFF]; }
};

// Per-wave LDS buffer of a one-dtype decoder, in 16-byte blocks: a chunk's
// values in their skewed slots, which also holds that dtype's largest
// payload at any byte phase (with the clamped row reads past it).  The
// float32 decoder thus takes half the LDS of the float64 one, and its
// registers, not its LDS, set its occupancy.
template <class T>
constexpr int wave_blocks() {
  return (kGSlots * (int)sizeof(typename T::U) + 15) / 16;
}
static_assert(wave_blocks<TF64>() * 16 == kWaveLds, "float64 buffer");
static_assert(wave_blocks<TF32>() * 16 >= 15 + TF32::BOUND + 145, "float32 payloads fit");

// Zigzag of Eq. 4: (x << 1) xor (x >> (W-1)), arithmetic shift.
template <class U>
__device__ __forceinline__ U zigzag(U x) {
  using S = typename std::make_signed<U>::type;
  return (x << 1) ^ (U)((S)x >> (sizeof(U) * 8 - 1));
}
template <class U>
__device__ __forceinline__ U unzigzag(U z) {
  using S = typename std::make_signed<U>::type;
  return (z >> 1) ^ (U)(-(S)(z & 1));
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Cross-lane data movement inside rows of 16 lanes with DPP (a VALU operand
// modifier, no LDS round trip).  Controls (GFX9 encoding): quad_perm
// [1,0,3,2] = 0xB1 and [2,3,0,1] = 0x4E swap lanes at distance 1 and 2;
// row_half_mirror (0x141) and row_mirror (0x140) reverse 8- and 16-lane
// halves; row_shr:k (0x110 + k) shifts right by k inside the row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
// row_shr:K with lanes that have no source reading 0.
template <int K>
__device__ __forceinline__ uint32_t dpp_shr0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + K, 0xF, 0xF, true);
}

// OR over the 16 lanes of each row, delivered to every lane of the row.
__device__ __forceinline__ uint32_t row_or32(uint32_t v) {
  v |= dpp<kDppXor1>(v);
  v |= dpp<kDppXor2>(v);
  v |= dpp<kDppHalfMirror>(v);
  v |= dpp<kDppMirror>(v);
  return v;
}
__device__ __forceinline__ uint32_t rl(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// Wave-wide OR (uniform result).
__device__ __forceinline__ uint32_t wave_or32(uint32_t v) {
  v = row_or32(v);
  return rl(v, 0) | rl(v, 16) | rl(v, 32) | rl(v, 48);
}
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
  return ((uint64_t)wave_or32((uint32_t)(v >> 32)) << 32) | wave_or32((uint32_t)v);
}

// Wave-wide sum (uniform result): the same row steps as the OR above
// combine disjoint lane groups, so they add each lane once.
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppHalfMirror>(v);
  v += dpp<kDppMirror>(v);
  return rl(v, 0) + rl(v, 16) + rl(v, 32) + rl(v, 48);
}

// Wave-wide sum of 64-bit values (uniform result), modulo 2^64.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
  auto step = [&](auto ctrl_tag) {
    constexpr int C = decltype(ctrl_tag)::value;
    v += ((uint64_t)dpp<C>((uint32_t)(v >> 32)) << 32) | dpp<C>((uint32_t)v);
  };
  step(std::integral_constant<int, kDppXor1>{});
  step(std::integral_constant<int, kDppXor2>{});
  step(std::integral_constant<int, kDppHalfMirror>{});
  step(std::integral_constant<int, kDppMirror>{});
  uint64_t m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) m += ((uint64_t)rl((uint32_t)(v >> 32), 16 * r) << 32) | rl((uint32_t)v, 16 * r);
  return m;
}

// Lane L receives v from lane L ^ B: quad permutes for 1 and 2, a row
// rotate by 8 for 8, a swizzle inside 32-lane halves for 4 and 16, a
// backward permute for 32.
constexpr int kDppRor8 = 0x128;
template <int B>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int lane) {
  if constexpr (B == 1) return dpp<kDppXor1>(v);
  else if constexpr (B == 2) return dpp<kDppXor2>(v);
  else if constexpr (B == 8) return dpp<kDppRor8>(v);
  else if constexpr (B == 4 || B == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (B << 10));
  else return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)v);
}

// 64 x 64 bit-matrix transpose across the wave (rows = lanes): afterwards
// bit L of lane p's word is bit p of lane L's word before.  Recursive block
// swaps: lanes L and L ^ B exchange the off-diagonal B x B blocks, B = 32
// (the two dwords), then 16, 8, 4, 2, 1 inside each dword.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  {
    const bool up = lane & 32;
    const uint32_t r = xor_lane<32>(up ? lo : hi, lane);
    if (up) lo = r;
    else hi = r;
  }
  auto stage = [&](auto b_tag, uint32_t m) {  // m: the bits whose index has bit B set
    constexpr int B = decltype(b_tag)::value;
    const bool up = lane & B;
    auto one = [&](uint32_t& v) {
      const uint32_t send = up ? (v & ~m) << B : (v & m) >> B;
      v = (v & (up ? m : ~m)) | xor_lane<B>(send, lane);
    };
    one(lo);
    one(hi);
  };
  stage(std::integral_constant<int, 16>{}, 0xFFFF0000u);
  stage(std::integral_constant<int, 8>{}, 0xFF00FF00u);
  stage(std::integral_constant<int, 4>{}, 0xF0F0F0F0u);
  stage(std::integral_constant<int, 2>{}, 0xCCCCCCCCu);
  stage(std::integral_constant<int, 1>{}, 0xAAAAAAAAu);
  return ((uint64_t)hi << 32) | lo;
}

// Wave-wide unsigned maximum (uniform result).
__device__ __forceinline__ uint64_t wave_max64(uint64_t v) {
  auto step = [&](auto ctrl_tag) {
    constexpr int C = decltype(ctrl_tag)::value;
    const uint64_t o = ((uint64_t)dpp<C>((uint32_t)(v >> 32)) << 32) | dpp<C>((uint32_t)v);
    v = o > v ? o : v;
  };
  step(std::integral_constant<int, kDppXor1>{});
  step(std::integral_constant<int, kDppXor2>{});
  step(std::integral_constant<int, kDppHalfMirror>{});
  step(std::integral_constant<int, kDppMirror>{});
  uint64_t m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint64_t x = ((uint64_t)rl((uint32_t)(v >> 32), 16 * r) << 32) | rl((uint32_t)v, 16 * r);
    m = x > m ? x : m;
  }
  return m;
}
__device__ __forceinline__ int wave_max_i32(int v) {
  auto step = [&](auto ctrl_tag) {
    constexpr int C = decltype(ctrl_tag)::value;
    const int o = (int)dpp<C>((uint32_t)v);
    v = o > v ? o : v;
  };
  step(std::integral_constant<int, kDppXor1>{});
  step(std::integral_constant<int, kDppXor2>{});
  step(std::integral_constant<int, kDppHalfMirror>{});
  step(std::integral_constant<int, kDppMirror>{});
  int m = (int)rl((uint32_t)v, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const int x = (int)rl((uint32_t)v, 16 * r);
    m = x > m ? x : m;
  }
  return m;
}

// Inclusive prefix sum over lanes, modulo 2^64: a scan inside each row of
// 16 lanes (row_shr 1, 2, 4, 8), then the totals of the rows below added
// from scalar registers.
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v, int lane) {
  auto step = [&](auto k_tag) {
    constexpr int K = decltype(k_tag)::value;
    const uint64_t o = ((uint64_t)dpp_shr0<K>((uint32_t)(v >> 32)) << 32) | dpp_shr0<K>((uint32_t)v);
    v += o;
  };
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 4>{});
  step(std::integral_constant<int, 8>{});
  auto row_total = [&](int r) {
    return ((uint64_t)rl((uint32_t)(v >> 32), 16 * r + 15) << 32) | rl((uint32_t)v, 16 * r + 15);
  };
  const uint64_t t0 = row_total(0), t1 = row_total(1), t2 = row_total(2);
  const int row = lane >> 4;
  const uint64_t below = row == 0 ? 0 : row == 1 ? t0 : row == 2 ? t0 + t1 : t0 + t1 + t2;
  return v + below;
}
// Number of set bits of mask in lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Orders this wave's LDS accesses: writes before the barrier are visible to
// reads of other lanes after it.  The fence is restricted to LDS, so it does
// not wait for outstanding global loads or stores.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// ---------------------------------------------------------------------------
// 16 x 16 bit-matrix transpose of four (two) independent 16-bit fields per
// 64-bit (32-bit) word, by recursive block swaps.  Rows are the 16 words of
// one dword column a[0..15]; afterwards bit i of field q of a[j] is bit j of
// field q of the original a[i].  The transpose is its own inverse.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void xpose16(uint32_t (&a)[16]) {
#pragma unroll
  for (int si = 0; si < 4; ++si) {
    const int s = 8 >> si;
    const uint32_t m = si == 0 ? 0x00FF00FFu : si == 1 ? 0x0F0F0F0Fu : si == 2 ? 0x33333333u : 0x55555555u;
    const uint32_t ms = m << s;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i & s) continue;
      const uint32_t x = a[i], y = a[i + s];
      a[i + s] = (y & ~m) | ((x >> s) & m);
      a[i] = (x & ~ms) | ((y << s) & ms);
    }
  }
}

// Byte access into a wave's LDS buffer.
template <int NW, int WB>
__device__ __forceinline__ uint8_t* wave_bytes(BlockLdsT<NW, WB>& s, int wid) {
  return reinterpret_cast<uint8_t*>(&s.wave[wid][0]);
}

}  // namespace falcon_dev
