// codec_kernels.hpp -- Falcon compression and decompression kernels for
// gfx950 (device code; each kernels_*.hip instantiates one form).
//
// Compression runs in two passes (size pass, scan of the sizes, write
// pass) and decompression after a scan of the size array, so no chunk ever
// waits for another: waves take chunks by static striding.
#pragma once

#include <type_traits>

#include "codec_device.hpp"
#include "internal.hpp"

namespace falcon_dev {

// ---------------------------------------------------------------------------
// Alg. 2 building blocks
// ---------------------------------------------------------------------------

// floor(log10 |v|) of a regular value given its magnitude bits, as the
// largest k with fl(10^k) <= |v| (the same k as the exponent of the shortest
// decimal string).  floor(e2 * log10 2) = (e2 * 78913) >> 18 for |e2| < 1700
// gives k0 with fl(10^k0) <= 2^e2 <= |v| < 2^(e2+1) <= fl(10^(k0+2)), so the
// answer is k0 or k0 + 1.
template <class T>
__device__ __forceinline__ int fl10(const LdsTables& sm, typename T::U mag) {
  const int e2 = T::expf(mag) - T::BIAS;
  const int k0 = (e2 * 78913) >> 18;
  return k0 + (mag >= T::u(T::pow10(sm, k0 + 1)) ? 1 : 0);
}

// The stopping test of Alg. 2 (Thm. 4): |x - round(x)| <= |x| * 2^-(p-1)
// with x = v (x) 10^alpha.  Returns the rounded value in r.
template <class T>
__device__ __forceinline__ bool eps_test(typename T::U b, typename T::F P, typename T::F& r) {
  using F = typename T::F;
  const F x = T::f(b) * P;
  r = T::rnd(x);
  return T::abs(x - r) <= T::abs(x) * T::mu_scale();
}

// The trial-and-error stopping test that Sec. 1 attributes to earlier
// codecs (the Fal_Elf ablation of Sec. 5.4.2): v (x) 10^alpha must be an
// exact integer.  Returns the rounded value in r.
template <class T>
__device__ __forceinline__ bool exact_test(typename T::U b, typename T::F P, typename T::F& r) {
  const typename T::F x = T::f(b) * P;
  r = T::rnd(x);
  return x == r;
}

// The recover check of Alg. 2, r / P == v after IEEE division, without the
// division: the quotient rounds to v exactly when the residual r - v * P
// (one fused multiply-add, rounded once, which keeps it on the right side of
// any representable bound) lies inside v's rounding interval scaled by P:
// half an ulp of v away from zero, and toward zero a quarter ulp when |v|
// is a power of two (the binade below is twice as fine).  A residual exactly
// on the bound is a tie and takes the division.  v is a normal number here
// (T1) and P >= 1, so the bound P * ulp(v) / 2 is an exact power-of-two
// scaling of P.
template <class T>
__device__ __forceinline__ bool recovers(typename T::U b, typename T::F r, typename T::F P) {
  using F = typename T::F;
  const F v = T::f(b);
  const F e = T::fma(-v, P, r);
  const F half = T::ldexp(P, T::expf(b) - T::BIAS - T::MANT - 1);
  const bool toward_zero = (e > 0) != (v > 0);
  const F tol = (toward_zero && (b & T::MANT_MASK) == 0) ? half * (F)0.5 : half;
  const F ae = T::abs(e);
  if (ae < tol) return true;
  if (ae > tol) return false;
  return T::u(r / P) == b;
}

// The recover check for an integer r with |r| < 10^BMAX and y = RN(1/P):
// RN(r / P) is RN(q + RN(r - q P) y) with q = RN(r y) up to alpha =
// MARKSTEIN_MAX (see the decoder's inverse of Eq. 3, decompress_chunk), so
// one product and two fused multiply-adds give the quotient to compare
// with v; above that alpha, recovers().  alpha is wave-uniform.
template <class T>
__device__ __forceinline__ bool recovers_int(typename T::U b, typename T::F r, typename T::F P, typename T::F y,
                                             int alpha) {
  using F = typename T::F;
  if (alpha > T::MARKSTEIN_MAX) return recovers<T>(b, r, P);
  const F q = r * y;
  return T::u(T::fma(T::fma(-q, P, r), y, q)) == b;
}

// Stopping test plus the recover check of Alg. 2: round(v (x) 10^a) / 10^a
// must give back v bit for bit.
template <class T>
__device__ __forceinline__ bool full_test(typename T::U b, typename T::F P) {
  typename T::F r;
  const bool ok = eps_test<T>(b, P, r);
  return ok && recovers<T>(b, r, P);
}

// bit k of m |= c.  The shift amount is made opaque so that the compiler
// builds the mask with a shift instead of keeping 1 << k constants in
// registers.
__device__ __forceinline__ void set_bit(uint32_t& m, bool c, int k) {
  int kk = k;
  asm volatile("" : "+s"(kk));
  m |= (c ? 1u : 0u) << kk;
}

// Literal Alg. 2 over the 17 values of this lane, one slot at a time with
// the lanes in lock-step over alpha; with ELF, under the trial-and-error
// stopping test (the Fal_Elf ablation, whose test is not monotone in alpha
// and so admits no bisection).  Returns true if some value is an exception;
// otherwise amax gets the lane's largest decimal place.
template <class T, bool ELF>
__device__ __forceinline__ bool alg2_literal(const LdsTables& sm, const typename T::U (&vb)[17], int& amax) {
  bool exc = false;
  amax = 0;
  for (int k = 0; k < 17; ++k) {
    const typename T::U v = vb[k];
    bool done = v == 0;  // +0.0: alpha = 0
    // loop condition of Alg. 2: beta = alpha + FL10 + 1 <= BMAX
    const int lim = done ? 0 : min(T::AMAX, T::BMAX - 1 - fl10<T>(sm, T::mag(v)));
    for (int a = 0; a <= T::AMAX; ++a) {
      if (ballot(!done) == 0) break;
      if (!done) {
        if (a > lim) {
          exc = true;
          done = true;
        } else {
          const typename T::F P = T::pow10(sm, a);
          typename T::F r;
          if (ELF ? exact_test<T>(v, P, r) : eps_test<T>(v, P, r)) {
            done = true;
            if (!recovers<T>(v, r, P)) exc = true;
            else amax = max(amax, a);
          }
        }
      }
    }
    if (!done) exc = true;
  }
  return exc;
}

// Chunk-level digit transformation decision (Sec. 3.2.3, Alg. 3).  Output:
// header bytes A (alpha_max) and B (beta_hat_max), and whether Case 1 holds.
//
// The paper evaluates Alg. 2 value by value.  Here the wave decides the
// chunk with the same outcome in fewer steps.  The fact used throughout: a
// value that is not an exception passes both the stopping test and the
// recover check at every scale s from its decimal place alpha_i up to its
// limit lim_i = min(AMAX, BMAX-1-FL10(|v|)) (Thm. 2, Thm. 4: v * 10^s is
// then an integer below 10^BMAX, rounded back exactly, and the division
// returns the double nearest v's shortest string), and fails the stopping
// test below alpha_i (Alg. 2 stops at the first pass).
//  1. A value is an exception outright if it is -0.0, subnormal, Inf or NaN
//     or has FL10 >= BMAX or FL10 <= -(AMAX+1); with magnitudes ordered as
//     integers that is |v| < fl(10^-AMAX) or |v| >= fl(10^BMAX) (v != +0).
//  2. Otherwise let L* = min(AMAX, BMAX-1-FL10(v_max)) <= every lim_i, the
//     largest scale at which beta_hat stays within BMAX.  If every value
//     passes the stopping test at L*, alpha_max is the least scale in
//     [0, L*] at which all pass.  A sample gives it in one chunk-wide round
//     when the chunk's places are alike: each lane finds the place of its
//     first value, and if every value passes at the largest of these, that
//     is alpha_max (the recover check is applied in the same round).
//     Otherwise a bisection over the remaining scales finds it, and the
//     recover check is applied there once.  When the wave's previous chunk
//     was settled by the sample, the sample is tried before the test at L*,
//     which a chunk it settles then skips.
//  3. A value failing at L* is an exception if L* is its own limit, or if it
//     fails the full test at its own limit.
//  4. If no failing value is an exception, alpha_max lies in (L*, max lim_i]
//     (so the chunk is Case 2 with a real header): it is the least a at
//     which every value passes the stopping test at min(a, lim_i), found by
//     bisection, and the recover check is applied there once.
// When no value is an exception both bisections are exact and the recover
// checks pass; so a failed recover check means some value is one, and the
// chunk gets the exception header, as Alg. 2 would give it.
template <class T, bool HINT = true>
__device__ __forceinline__ void decide_case(const LdsTables& sm, const typename T::U (&vb)[17], int& A, int& B,
                            bool& case1, bool& hint) {
  using U = typename T::U;
  using F = typename T::F;
  const U mag_lo = T::u(T::pow10(sm, -T::AMAX));
  const U mag_hi = T::u(T::pow10(sm, T::BMAX));
  bool exc = false;
  U vmax = 0;
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const U m = T::mag(vb[k]);
    exc |= (vb[k] != 0) && (m < mag_lo || m >= mag_hi);
    vmax = m > vmax ? m : vmax;
  }
  if (ballot(exc)) {
    A = T::AMAX + 1;
    B = T::BMAX + 1;
    case1 = false;
    return;
  }
  vmax = (U)uniform64((uint64_t)wave_max64((uint64_t)vmax));
  if (vmax == 0) {  // every value is +0.0
    A = 0;
    B = 0;
    case1 = true;
    return;
  }
  const int maxfl = (int)uniform((uint32_t)fl10<T>(sm, vmax));
  const int lstar = min(T::AMAX, T::BMAX - 1 - maxfl);
  // The sample: each lane finds the decimal place of its own first value
  // by bisection over [0, L*] (per-lane bounds, the same number of rounds
  // for all), and the chunk is tested once, stopping test and recover
  // check, at the sample's largest place a_s.  A value that passes both
  // tests at a scale up to its limit is not an exception, and its place is
  // at most that scale; so if every value passes at a_s, no value is an
  // exception and alpha_max = a_s (the sampled value with place a_s fails
  // at a_s - 1).
  int as = 0;
  bool s_bad = false, s_rec_bad = false;
  auto sample = [&]() {
    int slo = 0, shi = lstar;
    for (int k = 0; (1 << k) < lstar + 1; ++k) {
      const int mid = (slo + shi) >> 1;
      F r;
      if (eps_test<T>(vb[0], T::pow10(sm, mid), r)) shi = mid;
      else slo = mid + 1;
    }
    as = (int)uniform((uint32_t)wave_max_i32(shi));
    const F P = T::pow10(sm, as);
    const F y = (F)1 / P;
    bool bad = false, rec_bad = false;
#pragma unroll
    for (int k = 0; k < 17; ++k) {
      F r;
      const bool pass = eps_test<T>(vb[k], P, r);  // |r| < 10^BMAX when it passes (as <= L*)
      bad |= !pass;
      rec_bad |= pass && !recovers_int<T>(vb[k], r, P, y, as);
    }
    s_bad = ballot(bad) != 0;
    s_rec_bad = ballot(rec_bad) != 0;
  };
  // The test at L*: fail gets the values of this lane that fail it.  A
  // failing value whose own limit min(AMAX, BMAX - 1 - FL10(|v|)) equals L*
  // is an exception (step 3); its limit is L* exactly when L* = AMAX or
  // FL10(|v|) = FL10(v_max), i.e. |v| >= fl(10^FL10(v_max)), one compare.
  // The values are tested four slots at a time, and the test stops at the
  // first such exception in the wave (quick): the chunk's header is then
  // the exception header whatever the other values hold.
  uint32_t fail = 0;
  bool quick = false;
  const U thr = T::u(T::pow10(sm, maxfl));
  auto all_pass_at_lstar = [&]() {
    const F P = T::pow10(sm, lstar);
    fail = 0;
    bool qe = false;
#pragma unroll
    for (int k = 0; k < 17; ++k) {
      F r;
      const bool f = !eps_test<T>(vb[k], P, r);
      set_bit(fail, f, k);
      qe |= f && (lstar == T::AMAX || T::mag(vb[k]) >= thr);
      if ((k & 3) == 3 || k == 16) {
        if (ballot(qe)) {
          quick = true;
          return false;
        }
      }
    }
    return ballot(fail != 0) == 0;
  };
  // With the hint set (the wave's previous chunk was settled by the sample)
  // the sample comes first and, when every value passes there, settles the
  // chunk without the test at L*.  Either order gives the same header.
  bool all_pass = (HINT && hint) || all_pass_at_lstar();
  if (all_pass) {
    sample();
    if (!s_bad && !s_rec_bad) {
      A = as;
      B = as + maxfl + 1;
      case1 = true;
      if (HINT) hint = true;
      return;
    }
    if (HINT && hint) {
      hint = false;
      all_pass = all_pass_at_lstar();
    }
  }
  if (all_pass) {
    // alpha_max = max alpha_i lies in [0, L*], at or above a_s.  If every
    // value passes the stopping test at a_s, alpha_max = a_s and the failed
    // recover check there means an exception; otherwise a bisection runs
    // over what the sample leaves.
    if (!s_bad) {
      A = T::AMAX + 1;
      B = T::BMAX + 1;
      case1 = false;
      return;
    }
    int lo = as + 1, hi = lstar;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const F P = T::pow10(sm, mid);
      bool bad = false;
#pragma unroll
      for (int k = 0; k < 17; ++k) {
        F r;
        bad |= !eps_test<T>(vb[k], P, r);
      }
      if (ballot(bad)) lo = mid + 1;
      else hi = mid;
    }
    bool bad = false;
    {
      const F P = T::pow10(sm, hi);
#pragma unroll
      for (int k = 0; k < 17; ++k) bad |= !full_test<T>(vb[k], P);
    }
    if (ballot(bad)) {
      A = T::AMAX + 1;
      B = T::BMAX + 1;
      case1 = false;
      return;
    }
    A = hi;
    B = hi + maxfl + 1;
    case1 = true;
    return;
  }
  {
    // Some value fails at L*.  Unless the test above already met an
    // exception whose limit is L*, every failing value is checked in full
    // at its own limit (above L*: its limit is not L*).
    bool e = false;
    if (!quick) {
#pragma unroll
      for (int k = 0; k < 17; ++k) {
        if ((fail >> k) & 1u) {
          const int f = fl10<T>(sm, T::mag(vb[k]));
          const int lim = min(T::AMAX, T::BMAX - 1 - f);
          if (lim == lstar || !full_test<T>(vb[k], T::pow10(sm, lim))) e = true;
        }
      }
    }
    if (quick || ballot(e)) {
      A = T::AMAX + 1;
      B = T::BMAX + 1;
      case1 = false;
      return;
    }
  }
  // step 4: bisection over (L*, max lim_i] with value k tested at
  // min(a, lim_k); +0.0 passes at every scale
  int lim[17];
  int lmax = lstar;
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    lim[k] = vb[k] == 0 ? T::AMAX : min(T::AMAX, T::BMAX - 1 - fl10<T>(sm, T::mag(vb[k])));
    lmax = max(lmax, lim[k]);
  }
  lmax = (int)uniform((uint32_t)wave_max_i32(lmax));
  int lo = lstar + 1, hi = lmax;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 17; ++k) {
      F r;
      bad |= !eps_test<T>(vb[k], T::pow10(sm, min(mid, lim[k])), r);
    }
    if (ballot(bad)) lo = mid + 1;
    else hi = mid;
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 17; ++k) bad |= !full_test<T>(vb[k], T::pow10(sm, min(hi, lim[k])));
  if (ballot(bad)) {
    A = T::AMAX + 1;
    B = T::BMAX + 1;
    case1 = false;
    return;
  }
  A = hi;
  B = hi + maxfl + 1;
  case1 = B <= T::BMAX;
}

// Ablation variants of Sec. 5.4.2 (Fig. 12b).  Each changes one step and
// keeps the stream layout.
enum : int {
  kVarFalcon = 0,  // the method as described
  kVarElf = 1,     // Alg. 2 with exact_test in place of the bound of Thm. 4
  kVarSparse = 2,  // every bit-plane row sparse
  kVarDense = 3    // every bit-plane row dense
};
// Per-wave LDS buffer of the variant kernels, in 16-byte blocks: an
// all-sparse float64 chunk (11 + 8 + 64 * 144 = 9235 bytes) at any 16-byte
// phase.
constexpr int kVarWaveBlocks = 580;

// decide_case for kVarElf: the same exceptions and header, with every value
// run through Alg. 2 under the trial-and-error stopping test (no shortcut:
// the test is not monotone in alpha, so bisection does not apply).
template <class T>
__device__ __forceinline__ void decide_case_elf(const LdsTables& sm, const typename T::U (&vb)[17], int& A, int& B,
                                                bool& case1) {
  using U = typename T::U;
  const U mag_lo = T::u(T::pow10(sm, -T::AMAX));
  const U mag_hi = T::u(T::pow10(sm, T::BMAX));
  bool exc = false;
  U vmax = 0;
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const U m = T::mag(vb[k]);
    exc |= (vb[k] != 0) && (m < mag_lo || m >= mag_hi);
    vmax = m > vmax ? m : vmax;
  }
  int amax = 0;
  if (!ballot(exc)) exc = alg2_literal<T, true>(sm, vb, amax);
  if (ballot(exc)) {
    A = T::AMAX + 1;
    B = T::BMAX + 1;
    case1 = false;
    return;
  }
  vmax = (U)uniform64((uint64_t)wave_max64((uint64_t)vmax));
  if (vmax == 0) {
    A = 0;
    B = 0;
    case1 = true;
    return;
  }
  const int maxfl = (int)uniform((uint32_t)fl10<T>(sm, vmax));
  A = (int)uniform((uint32_t)wave_max_i32(amax));
  B = A + maxfl + 1;
  case1 = B <= T::BMAX;
}

// Field of bit plane p (16 bits: row bytes 2L, 2L+1) after the transpose.
template <class T, int P>
__device__ __forceinline__ uint32_t plane_field(const uint32_t (&lo)[16], const uint32_t (&hi)[16]) {
  if constexpr (P < 32) return (lo[P & 15] >> (16 * ((P >> 4) & 1))) & 0xFFFFu;
  else return (hi[P & 15] >> (16 * ((P >> 4) & 1))) & 0xFFFFu;
}

template <int P>
__device__ __forceinline__ void plane_put(uint32_t (&lo)[16], uint32_t (&hi)[16], uint32_t fld) {
  if constexpr (P < 32) lo[P & 15] |= fld << (16 * ((P >> 4) & 1));
  else hi[P & 15] |= fld << (16 * ((P >> 4) & 1));
}

// Static loop over planes W-1 .. 0.
template <int P, class Fn>
__device__ __forceinline__ void for_planes_down(Fn&& fn) {
  if constexpr (P >= 0) {
    fn(std::integral_constant<int, P>{});
    for_planes_down<P - 1>(fn);
  }
}

__device__ __forceinline__ void write_stream_header(uint8_t* out, uint32_t dtype, uint64_t n,
                                                    uint64_t payload, int lane) {
  if (lane < 8) {
    uint32_t w;
    switch (lane) {
      case 0: w = 0x4E434C46u; break;       // "FLCN"
      case 1: w = 1u | (dtype << 8); break; // version 1, dtype, u16 0
      case 2: w = (uint32_t)kChunk; break;
      case 3: w = 0; break;
      case 4: w = (uint32_t)n; break;
      case 5: w = (uint32_t)(n >> 32); break;
      case 6: w = (uint32_t)payload; break;
      default: w = (uint32_t)(payload >> 32); break;
    }
    gbl(reinterpret_cast<uint32_t*>(out))[lane] = w;
  }
}

// ---------------------------------------------------------------------------
// Compression of one chunk (Alg. 3 for one chunk, executed by one wave).
// Split in two halves: transform (front) and encode + write (back).
// ---------------------------------------------------------------------------
// a1: coalesced load in the slot layout; positions past the end repeat the
// last value (padding of a partial last chunk).
template <class T>
__device__ __forceinline__ void load_chunk(const CompressSeries& sd, uint64_t c, int lane,
                                           typename T::U (&vb)[17]) {
  using U = typename T::U;
  const global_ptr<const U> in = gbl(reinterpret_cast<const U*>(sd.in));
  const uint64_t base = c * kChunk;
  const uint64_t rem = sd.n - base;
  const uint32_t nv = rem < (uint64_t)kChunk ? (uint32_t)rem : (uint32_t)kChunk;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    uint32_t idx = 1 + 64 * k + lane;
    idx = idx < nv ? idx : nv - 1;
    vb[k] = __builtin_nontemporal_load(in + base + idx);
  }
  vb[16] = in[base];
}

struct ChunkPlanes {
  uint32_t lo[16], hi[16];  // bit planes after the transpose (see plane_field)
  uint64_t or0, or1;        // OR of this lane's elements 0-7 and 8-15 (size pass)
  uint64_t z1;
  int A, B;
  uint32_t w;
};

// a4-a6 once the chunk's case is known (cp.A, cp.B set): Eq. 3, Eq. 4 and
// the bit width.  e receives this lane's entries of the delta sequence in
// the contiguous layout; with ORS, cp.or0 / cp.or1 receive the ORs of each
// row byte's eight elements (which decide whether a row byte is zero).  vb
// is consumed (free for the next chunk's loads when this returns).
template <class T, bool ORS>
__device__ __forceinline__ void transform_front(const LdsTables& sm, uint8_t* buf, const typename T::U (&vb)[17],
                                                int lane_in, bool case1, ChunkPlanes& cp, typename T::U (&e)[16]) {
  using U = typename T::U;
  using F = typename T::F;
  // An opaque copy of the lane index keeps the compiler from hoisting the
  // per-lane address arithmetic out of the chunk loop, where it would stay
  // live (and spill) across every chunk.
  int lane = lane_in;
  asm volatile("" : "+v"(lane));

  // a4: Eq. 3 -> g, written to LDS in skewed natural order.  Element
  // i = 1 + 64k + L goes to slot i + (i >> 4) = s0 + 68k: one base per lane
  // and a constant offset per k (an immediate of the LDS store)
  U* g = reinterpret_cast<U*>(buf);
  {
    const uint32_t s0 = 1u + (uint32_t)lane + ((1u + (uint32_t)lane) >> 4);
    const F P = T::pow10(sm, case1 ? cp.A : 0);
#pragma unroll
    for (int k = 0; k < 17; ++k) {
      U gk;
      if (case1) {
        F r;
        eps_test<T>(vb[k], P, r);
        gk = (U)T::to_int(r);
      } else {
        gk = zigzag<U>(vb[k]);
      }
      if (k < 16) {
        g[s0 + 68u * k] = gk;
      } else if (lane == 0) {
        g[0] = gk;
      }
    }
  }
  wave_lds_sync();

  // a5: Eq. 4 in the contiguous layout: e[q] = z_{16L+q+2}
  {
    const uint32_t b0 = 17u * lane;
    U prev = g[b0];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const U cur = g[b0 + 1 + q + (q == 15 ? 1 : 0)];
      e[q] = zigzag<U>((U)(cur - prev));
      prev = cur;
    }
    cp.z1 = (uint64_t)g[0];
  }
  wave_lds_sync();

  // a6: bit width w = W - min lead over z_2..z_n (lead of 0 is W)
  U orv = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) orv |= e[q];
  if constexpr (sizeof(U) == 8) {
    const uint64_t o = wave_or64((uint64_t)orv);
    cp.w = o ? 64u - (uint32_t)__builtin_clzll(o) : 0u;
  } else {
    const uint32_t o = wave_or32((uint32_t)orv);
    cp.w = o ? 32u - (uint32_t)__builtin_clz(o) : 0u;
  }
  if constexpr (ORS) {
    U o0 = 0, o1 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      o0 |= e[q];
      o1 |= e[8 + q];
    }
    cp.or0 = (uint64_t)o0;
    cp.or1 = (uint64_t)o1;
  }
}

// a7: bit-plane transpose of the entries e (contiguous layout) into cp.lo /
// cp.hi; element q of the lane goes to row q ^ 7 so that the first element
// of each byte lands in its most significant bit.
template <class T>
__device__ __forceinline__ void transform_planes(ChunkPlanes& cp, const typename T::U (&e)[16]) {
  using U = typename T::U;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    cp.lo[i] = (uint32_t)e[i ^ 7];
    cp.hi[i] = sizeof(U) == 8 ? (uint32_t)((uint64_t)e[i ^ 7] >> 32) : 0u;
  }
  xpose16(cp.lo);
  // with w <= 32 every upper half is zero, and so is its transpose
  if constexpr (sizeof(U) == 8)
    if (cp.w > 32) xpose16(cp.hi);
}

// a4-a7: the transform, then the transpose (TRANSPOSE) or, for the size
// pass, only the row-byte ORs.
template <class T, bool TRANSPOSE = true>
__device__ __forceinline__ void compress_transform(const LdsTables& sm, uint8_t* buf,
                                                   const typename T::U (&vb)[17], int lane, bool case1,
                                                   ChunkPlanes& cp) {
  typename T::U e[16];
  transform_front<T, !TRANSPOSE>(sm, buf, vb, lane, case1, cp, e);
  if constexpr (TRANSPOSE) transform_planes<T>(cp, e);
}

// a2-a7: decimal places and case (Alg. 2, Alg. 3), then the transform.
template <class T, bool TRANSPOSE = true, int V = kVarFalcon>
__device__ __forceinline__ void compress_front(const LdsTables& sm, uint8_t* buf, const typename T::U (&vb)[17],
                                               int lane, ChunkPlanes& cp, bool& hint) {
  bool case1;
  if constexpr (V == kVarElf) decide_case_elf<T>(sm, vb, cp.A, cp.B, case1);
  else decide_case<T>(sm, vb, cp.A, cp.B, case1, hint);
  compress_transform<T, TRANSPOSE>(sm, buf, vb, lane, case1, cp);
}

// a8-a9: per-row non-zero byte counts (sparse iff more than 16 of the 128
// bytes are zero; ties dense), scheme flags and the chunk size.
struct ChunkStats {
  uint64_t flags;  // bit p set: plane p is written dense
  uint32_t S;
};

// a8-a9 from the byte ORs of the size pass: byte 2L of row p (elements
// 16L..16L+7, plane p) is non-zero iff bit p of or0 is set; byte 2L+1 the
// same with or1.  A bit-matrix transpose across the wave hands lane p the
// 64 lane bits of plane p, so lane p counts row p's non-zero bytes, decides
// its scheme and its size, and one ballot and one wave sum finish the chunk.
// The kVarSparse / kVarDense ablations fix every row's scheme instead.
template <class T, int V = kVarFalcon>
__device__ __forceinline__ ChunkStats chunk_stats_or(const ChunkPlanes& cp, int lane) {
  const uint32_t w = cp.w;
  uint32_t nnz;  // non-zero bytes of row `lane`
  if constexpr (T::W == 32) {
    // 32 planes: both ORs fit one word, and one transpose hands lane p the
    // bits of or0's plane p and lane 32 + p those of or1's
    const uint64_t t = wave_transpose64(cp.or0 | (cp.or1 << 32), lane);
    const uint32_t c = (uint32_t)__popcll(t);
    nnz = c + xor_lane<32>(c, lane);
  } else {
    const uint64_t t0 = wave_transpose64(cp.or0, lane), t1 = wave_transpose64(cp.or1, lane);
    nnz = (uint32_t)(__popcll(t0) + __popcll(t1));
  }
  const bool row = (uint32_t)lane < w;
  const bool dense = row && (V == kVarDense || (V != kVarSparse && nnz >= 112));
  const uint32_t bytes = !row ? 0u : dense ? 128u : 16u + nnz;
  ChunkStats st;
  st.flags = ballot(dense);
  st.S = 3 + T::ZB + ((w + 7) >> 3) + wave_sum32(bytes);
  return st;
}

// a11 (first half): the chunk payload (header bytes, scheme flags, rows) in
// LDS at buf (any byte offset).
template <class T>
__device__ __forceinline__ void assemble_payload(uint8_t* buf, const ChunkPlanes& cp, uint64_t flags, uint32_t S,
                                                 int lane_in) {
  int lane = lane_in;  // opaque, see compress_transform
  asm volatile("" : "+v"(lane));
  const uint32_t w = cp.w;
  const uint32_t nflag = (w + 7) >> 3;
  const uint32_t hlen = 3 + T::ZB + nflag;
  if (lane < (int)hlen) {
    uint32_t byte;
    if (lane == 0) byte = (uint32_t)cp.A;
    else if (lane == 1) byte = (uint32_t)cp.B;
    else if (lane < 2 + T::ZB) byte = (uint32_t)(cp.z1 >> (8 * (lane - 2))) & 0xFFu;
    else if (lane == 2 + T::ZB) byte = w;
    else byte = (uint32_t)(flags >> (8 * (nflag - 1 - (lane - 3 - T::ZB)))) & 0xFFu;
    buf[lane] = (uint8_t)byte;
  }
  uint32_t cur = hlen;
  for_planes_down<T::W - 1>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    if (p < (int)w) {
      const uint32_t fld = plane_field<T, p>(cp.lo, cp.hi);
      const uint32_t b0 = fld & 0xFFu, b1 = fld >> 8;
      if ((flags >> p) & 1) {
        buf[cur + 2 * lane] = (uint8_t)b0;
        buf[cur + 2 * lane + 1] = (uint8_t)b1;
        cur += 128;
      } else {
        const uint64_t E = ballot(b0 != 0), O = ballot(b1 != 0);
        // bitmap byte q covers row bytes 8q..8q+7, i.e. lanes 4q..4q+3
        uint32_t bits = (((b0 != 0) ? 2u : 0u) | ((b1 != 0) ? 1u : 0u)) << (6 - 2 * (lane & 3));
        bits |= dpp<kDppXor1>(bits);
        bits |= dpp<kDppXor2>(bits);
        if ((lane & 3) == 0) buf[cur + (lane >> 2)] = (uint8_t)bits;
        const uint32_t rank = mbcnt(E) + mbcnt(O);
        if (b0) buf[cur + 16 + rank] = (uint8_t)b0;
        if (b1) buf[cur + 16 + rank + (b0 ? 1 : 0)] = (uint8_t)b1;
        cur += 16u + (uint32_t)(__popcll(E) + __popcll(O));
      }
    }
  });
}

// One piece of a partial block: n = 1, 2, 4 or 8 bytes at an offset that
// is a multiple of n, from LDS to global memory.
__device__ __forceinline__ void copy_piece(const uint8_t* src, uint8_t* dst, uint32_t o, uint32_t n) {
  if (n == 8) *gbl(reinterpret_cast<uint64_t*>(dst + o)) = *reinterpret_cast<const uint64_t*>(src + o);
  else if (n == 4) *gbl(reinterpret_cast<uint32_t*>(dst + o)) = *reinterpret_cast<const uint32_t*>(src + o);
  else if (n == 2) *gbl(reinterpret_cast<uint16_t*>(dst + o)) = *reinterpret_cast<const uint16_t*>(src + o);
  else gbl(dst)[o] = src[o];
}

// a11 (second half): copies a payload assembled in LDS at byte phase ph
// (buf + ph holds its S bytes, ph = the destination's offset inside its
// 16-byte block) to dal + ph, dal being 16-byte aligned: whole blocks with
// one 16-byte LDS read and one non-temporal 16-byte store each (a stream is
// read again, if at all, by a later operation; with ordinary stores its
// last lines stay dirty in the caches and the next kernel, typically a
// decompression, pays for their write-back).  The partial first block
// [ph, 16) and last block [0, end & 15) are each written as at most four
// naturally aligned pieces (1, 2, 4 and 8 bytes); a payload inside a single
// block, byte by byte.
__device__ __forceinline__ void copy_payload(const uint8_t* buf, uint8_t* dal, uint32_t ph, uint32_t S, int lane) {
  const uint32_t end = ph + S;
  const uint32_t nblk = (end + 15) >> 4;
  for (uint32_t k = lane; k < nblk; k += 64) {
    const uint32_t b_lo = 16 * k, b_hi = b_lo + 16;
    if (b_lo >= ph && b_hi <= end) {
      gstore16_nt(dal + b_lo, *reinterpret_cast<const uint4*>(buf + b_lo));
    } else if (b_lo < ph && b_hi <= end) {
      // head: bytes ph .. 15 of the block, pieces in increasing size
      uint32_t o = ph;
      for (uint32_t n = 1; n < 16; n <<= 1)
        if (o & n) {
          copy_piece(buf, dal, o, n);
          o += n;
        }
    } else if (b_lo >= ph) {
      // tail: bytes 0 .. (end & 15) - 1 of the block, pieces in decreasing size
      const uint32_t e = end - b_lo;
      uint32_t o = b_lo;
      for (uint32_t n = 8; n >= 1; n >>= 1)
        if (e & n) {
          copy_piece(buf, dal, o, n);
          o += n;
        }
    } else {
      for (uint32_t b = ph; b < end; ++b) gbl(dal)[b] = buf[b];
    }
  }
}

// ---------------------------------------------------------------------------
// Decompression of one chunk (Sec. 4, executed by one wave)
// ---------------------------------------------------------------------------
// A chunk's payload on its way from HBM to LDS: lane L holds the 16-byte
// blocks L, L + 64, ... of the payload's 16-byte-aligned span (pad = offset
// of the payload's first byte in the first block).  Loading the next chunk
// into these registers while the current one is decoded hides the load
// latency.
// Six blocks per lane cover payload spans up to 6144 bytes and keep the
// kernel within 128 VGPRs (4 waves per SIMD); the blocks beyond (mostly
// dense float64 chunks reach them) are read when the payload is stored
// into LDS.
constexpr int kStageBlocks = 6;

struct Staged {
  uint4 blk[kStageBlocks];
  const uint8_t* sal;  // 16-byte-aligned start of the payload span
  uint64_t avail;      // readable bytes from sal
  uint32_t S, pad, total;
  uint32_t full;       // blocks of the span that lie wholly inside the readable bytes
  bool bad;
};

// Block i of a staged span: whole, or byte by byte where it would pass the
// end of the readable bytes.
__device__ __forceinline__ uint4 load_block(const uint8_t* sal, uint64_t avail, uint32_t i) {
  if (16ull * i + 16 <= avail) return gload16(sal + 16 * i);
  uint32_t wv[4] = {0, 0, 0, 0};
  for (uint32_t b = 0; b < 16 && 16ull * i + b < avail; ++b)
    wv[b >> 2] |= (uint32_t)gbl(sal)[16 * i + b] << (8 * (b & 3));
  return make_uint4(wv[0], wv[1], wv[2], wv[3]);
}

// d1 and the payload loads of launch chunk t of series sd.  The chunk
// offset comes from the prefix scan of the size array (k_scan_*); in a
// batch launch the scan runs over the sizes of all series and a series
// subtracts the offset of its first chunk.  Every size must lie in
// [3 + ZB, BOUND] of the series' dtype and the series' sizes must add up to
// its payload byte count (checked by its last chunk); a chunk that fails
// loads nothing.  The kStageBlocks loads are always issued, through a raw
// buffer window over the span's whole blocks (blocks past it come back as
// zeros without a memory access), so that every iteration of the chunk
// loop issues the same memory instructions and the wait for them is exact.
// A last block that would pass the end of the payload is read byte by byte
// when the payload is stored (stage_store).  With fetch unset (no next
// chunk) the window is empty.
__device__ __forceinline__ Staged stage_issue(const DecompressSeries& sd, uint64_t t, const uint64_t* offsets,
                                              bool relative, int lane_in, bool fetch) {
  int lane = lane_in;
  asm volatile("" : "+v"(lane));
  Staged st;
  const uint64_t c = t - sd.chunk0;
  const uint64_t nc = (sd.n + kChunk - 1) / kChunk;
  const bool f64 = sd.dtype == 2;
  const uint32_t lo = f64 ? (uint32_t)TF64::ZB + 3 : (uint32_t)TF32::ZB + 3;
  const uint32_t hi = f64 ? (uint32_t)TF64::BOUND : (uint32_t)TF32::BOUND;
  const uint8_t* payload = sd.in + kHdrBytes + 4 * nc;
  st.S = uniform(cst(reinterpret_cast<const uint32_t*>(sd.in + kHdrBytes))[c]);
  const uint64_t base = relative ? uniform64(cst(offsets)[sd.chunk0]) : 0;
  const uint64_t off = uniform64(cst(offsets)[t]) - base;
  st.bad = st.S > hi || st.S < lo || off + st.S > sd.payload_bytes ||
           (c == nc - 1 && off + st.S != sd.payload_bytes);
  st.pad = 0;
  st.total = 0;
  st.sal = payload;
  st.avail = 0;
  st.full = 0;
  if (!st.bad) {
    const uint8_t* src = payload + off;
    st.pad = uniform((uint32_t)((uintptr_t)src & 15u));
    st.total = st.pad + st.S;
    st.sal = src - st.pad;
    st.avail = (uint64_t)(payload + sd.payload_bytes - st.sal);
    const uint32_t nblk = (st.total + 15) >> 4;
    st.full = st.avail >= 16ull * nblk ? nblk : (uint32_t)(st.avail >> 4);
  }
  const __amdgpu_buffer_rsrc_t win =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(st.sal), 0, fetch ? (int)(16 * st.full) : 0, 0x00020000);
#pragma unroll
  for (int k = 0; k < kStageBlocks; ++k) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(win, (int)(16u * ((uint32_t)lane + 64u * k)), 0, 0);
    st.blk[k] = make_uint4(v.x, v.y, v.z, v.w);
  }
  return st;
}

// Moves a staged payload into the wave's LDS buffer: the prefetched blocks
// first (their only wait is for the prefetch), then the blocks beyond
// kStageBlocks per lane, then a last block that passes the end of the
// readable bytes (the end of a series' stream only).
__device__ __forceinline__ void stage_store(uint8_t* buf, const Staged& st, int lane) {
  const uint32_t nblk = (st.total + 15) >> 4;
#pragma unroll
  for (int k = 0; k < kStageBlocks; ++k) {
    const uint32_t i = (uint32_t)lane + 64u * k;
    if (i < st.full) *reinterpret_cast<uint4*>(buf + 16 * i) = st.blk[k];
  }
  for (uint32_t i = (uint32_t)lane + 64u * kStageBlocks; i < st.full; i += 64)
    *reinterpret_cast<uint4*>(buf + 16 * i) = gload16(st.sal + 16 * i);
  if (st.full < nblk) {
    const uint32_t i = st.full + (uint32_t)lane;  // nblk - full <= 1
    if (i < nblk) *reinterpret_cast<uint4*>(buf + 16 * i) = load_block(st.sal, st.avail, i);
  }
}

// d2-d5 of one chunk whose payload is in LDS (stage_store done).
template <class T>
__device__ __forceinline__ void decompress_chunk(const LdsTables& sm, uint8_t* buf, const DecompressSeries& sd,
                                                 uint64_t c, uint32_t S, uint32_t pad, uint32_t total, bool bad,
                                                 uint32_t epoch, int lane_in, Ctl* ctl) {
  using U = typename T::U;
  using F = typename T::F;
  using S_ = typename T::S;
  int lane = lane_in;  // opaque, see compress_front
  asm volatile("" : "+v"(lane));
  // the chunk's size, phase and span are wave-uniform; in scalar registers
  // they keep the row cursor below scalar too
  S = uniform(S);
  pad = uniform(pad);
  total = uniform(total);
  bad = uniform((uint32_t)bad) != 0;
  // A chunk that fails a check is decoded all the same (every read below is
  // bounded, so it only produces garbage) and its stores go through an empty
  // window: every chunk issues the same memory instructions (see stage_issue).
  wave_lds_sync();
  // chunk header: alpha_max, beta_hat_max, z_1, w, scheme flags
  const uint32_t hb = (lane < 24 && pad + lane < total) ? buf[pad + lane] : 0u;
  const int A = __builtin_amdgcn_readlane((int)hb, 0);
  const int B = __builtin_amdgcn_readlane((int)hb, 1);
  U z1 = 0;
#pragma unroll
  for (int k = 0; k < T::ZB; ++k) z1 |= (U)(uint32_t)__builtin_amdgcn_readlane((int)hb, 2 + k) << (8 * k);
  const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)hb, 2 + T::ZB);
  if (w > (uint32_t)T::W) bad = true;
  const uint32_t nflag = (w + 7) >> 3;
  if (3 + T::ZB + nflag > S) bad = true;
  // bad, flags and the row cursor below are wave-uniform; saying so keeps
  // the per-row scheme branch and the cursor in scalar registers (a
  // divergent-looking branch would cost exec-mask bookkeeping per row)
  bad = uniform((uint32_t)bad) != 0;
  uint64_t flags = 0;
  if (!bad) {
    for (uint32_t f = 0; f < nflag; ++f)
      flags = (flags << 8) | (uint32_t)__builtin_amdgcn_readlane((int)hb, 3 + T::ZB + (int)f);
  }
  flags = uniform64(flags);
  // a row's scheme bit is tested in one 32-bit half of the flags: one
  // scalar bit test
  const uint32_t flo = (uint32_t)flags, fhi = (uint32_t)(flags >> 32);
  // d2: rows -> bit-plane fields of this lane (row bytes 2L, 2L+1).  The
  // row cursor and the error flag are wave-uniform; reads use clamped
  // addresses so that a corrupt stream never reads outside the buffer (its
  // result is discarded through the flag).
  uint32_t lo[16], hi[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) lo[i] = hi[i] = 0;
  uint32_t cur = uniform(pad + 3 + T::ZB + nflag);
  bool ubad = uniform((uint32_t)bad) != 0;
  constexpr uint32_t kLim = wave_blocks<T>() * 16 - 1;
  static_assert(15 + T::BOUND + 144 <= kLim, "clamped row reads of a valid chunk are never moved");
  const uint32_t sh = 6u - 2u * ((uint32_t)lane & 3u);  // bitmap bit of row byte 2L + 1
  // a dense row's bytes for this lane sit at 2L and 2L + 1 past the cursor;
  // the second offset is opaque so that the compiler cannot merge the two
  // byte reads into one 16-bit read, which is slow at odd addresses
  const uint32_t l2 = 2u * (uint32_t)lane;
  uint32_t l2p = l2 + 1u;
  asm volatile("" : "+v"(l2p));
  for_planes_down<T::W - 1>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    if (p < (int)w) {
      uint32_t fld;
      const bool dense = ((p >= 32 ? fhi : flo) >> (p & 31)) & 1u;
      uint32_t nnz = 0;  // sparse rows: non-zero bytes after the bitmap
      // reads are kept inside the buffer by clamping the (scalar) cursor: in
      // a valid chunk every row ends by total <= 15 + BOUND, below both
      // clamps, so they never move a read; a corrupt chunk is reported by
      // the final cursor check
      if (dense) {
        // two byte reads (see l2p above)
        const uint32_t c0 = min(cur, kLim - 128);
        fld = (uint32_t)buf[c0 + l2] | ((uint32_t)buf[c0 + l2p] << 8);
      } else {
        const uint8_t* q = buf + min(cur, kLim - 145);
        // bitmap byte L/4 covers this lane's row bytes 2L and 2L+1 (MSB first)
        const uint32_t bm = q[(uint32_t)lane >> 2];
        const uint32_t nz0 = (bm >> (sh + 1)) & 1u, nz1 = (bm >> sh) & 1u;
        const uint64_t E = ballot(nz0 != 0), O = ballot(nz1 != 0);
        nnz = (uint32_t)(__popcll(E) + __popcll(O));
        const uint8_t* d = q + 16 + mbcnt(E) + mbcnt(O);  // rank < 128
        const uint32_t r0 = d[0], r1 = d[nz0];
        fld = (nz0 ? r0 : 0u) | ((nz1 ? r1 : 0u) << 8);
      }
      // the row's extent, stepped over after the join so that the cursor
      // stays one scalar value; the cursor only grows, so a row that runs
      // past the payload leaves it above total, which the check after the
      // last row reports
      const uint32_t row = dense ? 128u : 16u + nnz;
      cur += row;
      plane_put<p>(lo, hi, fld);
    }
  });
  const bool err = ubad || cur != total;  // wave-uniform
  // d3: inverse transpose
  xpose16(lo);
  if constexpr (sizeof(U) == 8)
    if (w > 32) xpose16(hi);  // planes 32..63 absent: hi stays zero
  // d4: un-zigzag and prefix sum from g_1 = z_1 (modulo 2^W)
  U gv[16];
  U run = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    U et;
    if constexpr (sizeof(U) == 8) et = ((uint64_t)hi[i ^ 7] << 32) | lo[i ^ 7];
    else et = lo[i ^ 7];
    run += unzigzag<U>(et);
    gv[i] = run;
  }
  const uint64_t incl = wave_incl_scan64((uint64_t)run, lane);
  const U basev = (U)(z1 + (U)(incl - (uint64_t)run));
  // d5: inverse Eq. 3 (a uniform branch on the chunk's case), then
  // coalesced stores of the first nv values.  Store k covers elements
  // 64k - mis .. 64k - mis + 63, where mis aligns it to 128-byte lines, so
  // that only the two lines shared with the neighbouring chunks are written
  // in part.
  const bool case1 = uniform((uint32_t)(A <= T::AMAX && B <= T::BMAX)) != 0;
  wave_lds_sync();
  U* vals = reinterpret_cast<U*>(buf);
  // element 16L + 1 + i sits at slot idx + (idx >> 4) = 17L + 1 + i + ((1 + i) >> 4)
  const uint32_t b17 = 17u * (uint32_t)lane;
  auto slot_of = [](int i) { return (uint32_t)(1 + i + ((1 + i) >> 4)); };
  if (case1) {
    // Inverse Eq. 3: v = g / 10^alpha, correctly rounded.  With y the
    // correctly rounded reciprocal of P = 10^alpha and q = RN(g * y), the
    // residual g - q * P is exact (one fused multiply-add) and
    // RN(q + (g - q * P) * y) is RN(g / P) (Markstein's correction step):
    // q lies within 2 ulps of z = g / P, so q + (g - q P) y = z + (z - q)
    // (P y - 1) is within 2^-52 ulp of z; and z, with |g| < 2^53, lies at
    // least ulp(z) / (2 * 5^alpha) from every midpoint between two floats
    // (never on one), which is more for 5^alpha < 2^51, i.e. alpha <= 21 in
    // binary64 (binary32: checked over every |g| < 10^6 and alpha <= 10).
    // alpha = 22 in binary64 keeps the IEEE division.
    const F P = T::pow10(sm, A);
    const F y = (F)1 / P;
    const bool markstein = A <= T::MARKSTEIN_MAX;  // wave-uniform
    auto quot = [&](F g) {
      if (!markstein) return g / P;
      const F q = g * y;
      return T::fma(T::fma(-q, P, g), y, q);
    };
#pragma unroll
    for (int i = 0; i < 16; ++i) vals[b17 + slot_of(i)] = T::u(quot((F)(S_)(U)(basev + gv[i])));
    if (lane == 0) vals[0] = T::u(quot((F)(S_)z1));
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) vals[b17 + slot_of(i)] = unzigzag<U>((U)(basev + gv[i]));
    if (lane == 0) vals[0] = unzigzag<U>(z1);
  }
  wave_lds_sync();
  const uint64_t base = c * kChunk;
  const uint64_t rem = sd.n - base;
  const int nv = rem < (uint64_t)kChunk ? (int)rem : (int)kChunk;
  U* const out = reinterpret_cast<U*>(sd.out) + base;
  constexpr uint32_t kLine = 128 / sizeof(U);
  const int mis = (int)(((uintptr_t)out / sizeof(U)) % kLine);
  // window from the start of out's line to the chunk's last value: element j
  // sits at byte (j + mis) * sizeof(U); lanes before the chunk (j < 0, only
  // in store 0) get kDropOffset, lanes past its end fall outside the window
  const __amdgpu_buffer_rsrc_t win = store_window(out - mis, err ? 0u : (uint32_t)(mis + nv) * sizeof(U));
  // Store k takes element j = 64k + a0 from slot j + (j >> 4) = 68k + s0.
  // Only stores 0 and 16 can reach past the chunk's slots (j < 0 or
  // j > 1024), so only they clamp; a lane whose j is not below nv reads a
  // slot inside the buffer, and its store falls outside the window.
  const int a0 = lane - mis;
  const int s0 = a0 + (a0 >> 4);
  const int j0 = a0 < 0 ? 0 : a0;
  const int j16 = min(64 * 16 + a0, kChunk - 1);
  const uint32_t vl = (uint32_t)lane * sizeof(U);
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const U v = k == 0 ? vals[j0 + (j0 >> 4)] : k == 16 ? vals[j16 + (j16 >> 4)] : vals[68 * k + s0];
    const uint32_t voff = (k == 0 && a0 < 0) ? kDropOffset : vl + 64u * k * sizeof(U);
    if constexpr (sizeof(U) == 8)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), win, (int)voff, 0, kNonTemporal);
    else
      __builtin_amdgcn_raw_buffer_store_b32(v, win, (int)voff, 0, kNonTemporal);
  }
  if (err && lane == 0) __hip_atomic_store(&ctl->error, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <class Series>
__device__ __forceinline__ Series find_series(const Series& one, const Series* many, uint32_t ns, uint64_t t) {
  if (!many) {  // one-series launch: the descriptor travels in the arguments
    Series s = one;
    // keeps the compiler from merging this copy with the global load below
    // into one load through a generic pointer (a flat access)
    asm volatile("" ::: "memory");
    return s;
  }
  uint32_t lo = 0, hi = ns - 1;  // last series with chunk0 <= t
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (cst(many)[mid].chunk0 <= t) lo = mid;
    else hi = mid - 1;
  }
  // the descriptor as 8-byte scalar loads (a struct copy through an
  // address-space-qualified pointer is not available in C++)
  static_assert(sizeof(Series) % 8 == 0, "descriptor made of 8-byte words");
  uint64_t w[sizeof(Series) / 8];
  const const_ptr<uint64_t> q = cst(reinterpret_cast<const uint64_t*>(many + lo));
#pragma unroll
  for (uint32_t i = 0; i < sizeof(Series) / 8; ++i) w[i] = q[i];
  Series s;
  __builtin_memcpy(&s, w, sizeof(Series));
  return s;
}

// Writes the 32-byte header of every empty series of a batch launch and its
// stream length (no chunk of the launch belongs to them).  Run by the first
// workgroup of a batch launch (one with a descriptor array and a length
// array), one thread per series.
__device__ __forceinline__ void empty_series_headers(const CompressArgs& a) {
  if (!a.lens || !a.many || blockIdx.x != 0) return;
  for (uint32_t i = threadIdx.x; i < a.nseries; i += blockDim.x) {
    const CompressSeries& sd = a.many[i];
    if (sd.n != 0) continue;
    const global_ptr<uint32_t> o = gbl(reinterpret_cast<uint32_t*>(sd.out));
    o[0] = 0x4E434C46u;  // "FLCN"
    o[1] = 1u | (sd.dtype << 8);
    o[2] = (uint32_t)kChunk;
    o[3] = o[4] = o[5] = o[6] = o[7] = 0;
    if (a.lens) a.lens[sd.idx] = kHdrBytes;
  }
}

// ---------------------------------------------------------------------------
// Two-pass compression.  The size pass runs a1-a9 for every chunk and keeps
// what the write pass needs (ChunkMeta); the chunk sizes are then scanned
// into offsets (k_scan_*), and the write pass reloads each chunk, redoes
// a4-a7 with the case already decided, assembles the payload and writes it
// at its offset.  No chunk ever waits for another, so waves take chunks by
// static striding.
// ---------------------------------------------------------------------------
// vb holds the chunk's values when loaded is set (else they are loaded
// here); prefetch() runs as soon as vb is free, so that the next chunk's
// loads overlap the rest of this one.
template <class T, int V, class Prefetch>
__device__ __forceinline__ void size_chunk(const LdsTables& tab, uint8_t* buf, const CompressArgs& a,
                                           const CompressSeries& sd, uint64_t t, int lane,
                                           typename T::U (&vb)[17], bool loaded, bool& hint,
                                           Prefetch&& prefetch) {
  const uint64_t c = t - sd.chunk0;
  if (!loaded) load_chunk<T>(sd, c, lane, vb);
  ChunkPlanes cp;
  compress_front<T, false, V>(tab, buf, vb, lane, cp, hint);
  prefetch();
  const ChunkStats st = chunk_stats_or<T, V>(cp, lane);
  if (lane == 0) {
    ChunkMeta m;
    m.flags = st.flags;
    m.S = st.S;
    m.A = (uint8_t)cp.A;
    m.B = (uint8_t)cp.B;
    m.w = (uint8_t)cp.w;
    m.pad = 0;
    a.meta[t] = m;
    a.gsizes[t] = st.S;
    gbl(reinterpret_cast<uint32_t*>(sd.out + kHdrBytes))[c] = st.S;
  }
  wave_lds_sync();
}

template <class T, class Prefetch>
__device__ __forceinline__ void write_chunk(const LdsTables& tab, uint8_t* buf, const CompressArgs& a,
                                            const CompressSeries& sd, uint64_t t, int lane,
                                            typename T::U (&vb)[17], bool loaded, Prefetch&& prefetch) {
  const uint64_t c = t - sd.chunk0;
  const uint64_t nc = (sd.n + kChunk - 1) / kChunk;
  if (!loaded) load_chunk<T>(sd, c, lane, vb);
  // The chunk's metadata and offset come through scalar loads at a
  // wave-uniform index (readfirstlane): a vector load would count against
  // the vector-memory counter, and waiting for it would also wait for the
  // next chunk's prefetch and this wave's outstanding stores.
  const uint64_t tu = uniform64(t);
  const const_ptr<uint64_t> mp = cst(reinterpret_cast<const uint64_t*>(a.meta + tu));
  const uint64_t flags = uniform64(mp[0]);
  const uint64_t m1 = uniform64(mp[1]);
  const uint64_t base = a.relative ? uniform64(cst(a.offsets)[uniform64(sd.chunk0)]) : 0;
  const uint64_t off = uniform64(cst(a.offsets)[tu]) - base;
  const uint32_t S = (uint32_t)m1;
  ChunkPlanes cp;
  cp.A = (int)((m1 >> 32) & 0xFF);
  cp.B = (int)((m1 >> 40) & 0xFF);
  compress_transform<T>(tab, buf, vb, lane, cp.A <= T::AMAX && cp.B <= T::BMAX, cp);
  prefetch();
  // the payload goes to dst; it is assembled at dst's 16-byte phase so that
  // the copy moves whole aligned blocks
  uint8_t* dst = sd.out + kHdrBytes + 4 * nc + off;
  const uint32_t ph = uniform((uint32_t)((uintptr_t)dst & 15u));
  // the payload's assembly and stores run at a raised wave priority: the
  // SIMD issues this wave's LDS writes and stores ahead of the other waves'
  // arithmetic, so that the payload reaches the memory system sooner
  __builtin_amdgcn_s_setprio(2);
  assemble_payload<T>(buf + ph, cp, flags, S, lane);
  wave_lds_sync();
  copy_payload(buf, dst - ph, ph, S, lane);
  __builtin_amdgcn_s_setprio(0);
  if (c == nc - 1) {
    write_stream_header(sd.out, sd.dtype, sd.n, off + S, lane);
    if (a.lens && lane == 0) a.lens[sd.idx] = kHdrBytes + 4 * nc + off + S;
  }
  wave_lds_sync();
}

template <int NW, int WB>
__device__ __forceinline__ void pass_prologue(BlockLdsT<NW, WB>& sm, const CompressArgs& a, bool headers) {
  load_tables(sm.tab);
  if (headers) empty_series_headers(a);
  __syncthreads();
}

// PASS 1 = size pass, 2 = write pass; one dtype per launch.  V selects an
// ablation variant (size pass only: the write pass follows the flags the
// size pass stored); WB is the per-wave LDS buffer in 16-byte blocks, which
// an all-sparse float64 chunk (up to 9235 bytes) needs larger.  With the
// float32 buffer of wave_blocks, the float32 passes hold their registers to
// 80 and run 6 waves per SIMD; the float64 ones are held to 4 by LDS.
template <class T, int NW, int PASS, int V = kVarFalcon, int WB = wave_blocks<T>()>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu((T::W == 32 && WB == wave_blocks<T>()) ? 6 : 4))) void k_compress_pass(
    CompressArgs a) {
  __shared__ BlockLdsT<NW, WB> sm;
  pass_prologue(sm, a, PASS == 2);
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);  // wave-uniform: keeps the chunk loop scalar
  uint8_t* buf = wave_bytes(sm, wid);
  typename T::U vb[17];
  if (PASS == 2 && a.total_chunks == 0 && !a.many && blockIdx.x == 0 && wid == 0)
    write_stream_header(a.one.out, a.one.dtype, 0, 0, lane);
  uint64_t t = (uint64_t)blockIdx.x * NW + wid;
  if (t >= a.total_chunks) return;
  CompressSeries sd = find_series(a.one, a.many, a.nseries, t + a.t0);
  load_chunk<T>(sd, t + a.t0 - sd.chunk0, lane, vb);
  bool hint = false;  // case-decision order (decide_case), carried across the wave's chunks
  for (;;) {
    const uint64_t tg = t + a.t0;
    const CompressSeries cur = sd;
    const uint64_t tn = t + a.total_waves;
    const bool more = tn < a.total_chunks;
    auto prefetch = [&]() {
      if (more) {
        sd = find_series(a.one, a.many, a.nseries, tn + a.t0);
        load_chunk<T>(sd, tn + a.t0 - sd.chunk0, lane, vb);
      }
    };
    if (PASS == 1) size_chunk<T, V>(sm.tab, buf, a, cur, tg, lane, vb, true, hint, prefetch);
    else write_chunk<T>(sm.tab, buf, a, cur, tg, lane, vb, true, prefetch);
    if (!more) break;
    t = tn;
  }
}

template <int NW, int PASS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_compress_pass_mixed(
    CompressArgs a) {
  __shared__ BlockLdsT<NW> sm;
  pass_prologue(sm, a, PASS == 2);
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);  // wave-uniform: keeps the chunk loop scalar
  uint8_t* buf = wave_bytes(sm, wid);
  bool hint = false;
  for (uint64_t t = (uint64_t)blockIdx.x * NW + wid; t < a.total_chunks; t += a.total_waves) {
    const uint64_t tg = t + a.t0;
    const CompressSeries sd = find_series(a.one, a.many, a.nseries, tg);
    auto none = []() {};
    if (uniform(sd.dtype) == 2) {
      uint64_t vb[17];
      if (PASS == 1) size_chunk<TF64, kVarFalcon>(sm.tab, buf, a, sd, tg, lane, vb, false, hint, none);
      else write_chunk<TF64>(sm.tab, buf, a, sd, tg, lane, vb, false, none);
    } else {
      uint32_t vb[17];
      if (PASS == 1) size_chunk<TF32, kVarFalcon>(sm.tab, buf, a, sd, tg, lane, vb, false, hint, none);
      else write_chunk<TF32>(sm.tab, buf, a, sd, tg, lane, vb, false, none);
    }
  }
}

// ---------------------------------------------------------------------------
// Single-pass compression (Sec. 3.4): one launch computes every chunk and
// writes it at its offset.  Waves take chunks from a work queue (atomic
// ticket counters, see take_ticket), so chunks start close to launch order,
// and each chunk finds its offset with a decoupled look-back over per-chunk
// status words:
//   1. a1-a6 and the row statistics give the chunk's size S, published at
//      once as an aggregate (A, S); a series' first chunk publishes its
//      inclusive prefix (P, S) instead;
//   2. the transpose and the payload assembly (at byte phase 0 in LDS) run
//      while the chunks before it publish their sizes;
//   3. the look-back reads the 64 status words before the chunk, adds the
//      aggregates up to the nearest inclusive prefix and publishes (P, O + S);
//   4. the payload goes to its offset O, shifted to the destination's byte
//      phase on the way out of LDS.
// A chunk waits only for smaller chunks.  The smallest unfinished chunk
// never waits: if a wave holds it, every chunk before it is done; if not,
// every chunk its counter has handed out is smaller and done, so the waves
// of that counter are free to take it.  So the queue always drains, with
// or without other kernels on the device.  The look-back's wait is nevertheless
// bounded: past kSpinLimit rereads (or once another wave has given up) it
// gives up, sets ctl->qerror and the chunk writes nothing; its successors
// then compute offsets that are too small, never too large, and every
// payload write is also checked against the nc chunk bounds the caller's
// buffer holds, so nothing is written out of bounds.
// ---------------------------------------------------------------------------
// Status word: bits 63..62 kind (1 = aggregate, 2 = inclusive prefix),
// bits 61..46 the launch's tag, bits 45..0 the byte count.
constexpr uint64_t kStAgg = 1ull << 62, kStPre = 2ull << 62;
constexpr uint64_t kStValMask = (1ull << 46) - 1;
constexpr uint64_t kStTagMask = 0xFFFFull << 46;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ uint64_t status_word(uint64_t kind, uint32_t tag, uint64_t v) {
  return kind | ((uint64_t)(tag & 0xFFFFu) << 46) | (v & kStValMask);
}

// The next chunk of the calling wave (lane 0 takes the ticket; every lane
// gets the chunk).  Counter g hands out chunks g, g + G, g + 2G, ... in
// increasing order to the waves with (workgroup + wave index) mod G = g;
// one counter would serialise every chunk on one memory location.  Mixing
// the wave index in spreads each counter's waves over all XCDs (workgroups
// are dealt to XCDs round-robin), so that no counter falls behind with a
// slower XCD.
__device__ __forceinline__ uint64_t take_ticket(const CompressArgs& a, int lane) {
  const uint32_t g = (blockIdx.x + uniform(threadIdx.x >> 6)) % a.qgroups;
  uint64_t k = 0;
  if (lane == 0)
    k = __hip_atomic_fetch_add(a.qctr + (size_t)kQueueStride * g, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return uniform64(k) * a.qgroups + g;
}

// Exclusive prefix of the sizes of the chunks tf .. tg - 1 (tf = launch
// index of the series' first chunk, tg > tf): the aggregates of the chunks
// before tg back to the nearest inclusive prefix, plus that prefix.  Lane L
// reads the status word of chunk j - 1 - L; positions before tf act as an
// inclusive prefix of 0.  Sets failed (uniform) after kSpinLimit rereads of
// a window with a word still unpublished.
__device__ __forceinline__ uint64_t look_back(const CompressArgs& a, uint64_t tg, uint64_t tf, int lane,
                                              bool& failed) {
  const uint64_t tag = (uint64_t)(a.qtag & 0xFFFFu) << 46;
  uint64_t acc = 0;
  uint64_t j = tg;
  uint32_t spins = 0;
  for (;;) {
    const bool edge = j < tf + 1 + (uint64_t)lane;  // j - 1 - lane < tf
    uint64_t w = 0;
    if (!edge) w = __hip_atomic_load(a.status + (j - 1 - lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool mine = (w & kStTagMask) == tag;
    const bool pre = edge || (mine && (w >> 62) == 2);
    const bool ready = pre || (mine && (w >> 62) == 1);
    const uint64_t pm = ballot(pre);
    const uint32_t s = pm ? (uint32_t)__builtin_ctzll(pm) : 64u;
    // lanes 0 .. s must all hold a published word
    const uint64_t upto = s >= 63 ? ~0ull : ((2ull << s) - 1);
    if ((ballot(!ready) & upto) == 0) {
      acc += wave_sum64(((uint32_t)lane <= s && !edge) ? (w & kStValMask) : 0ull);
      if (s < 64) return acc;
      j -= 64;
      continue;
    }
    // give up past the limit, or at once when another wave has given up
    // (every 256 rereads the shared error word is checked)
    ++spins;
    if (spins > kSpinLimit ||
        ((spins & 255u) == 0 &&
         __hip_atomic_load(&a.ctl->qerror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
      failed = true;
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// a11 for the single pass: copies a payload assembled at phase 0 (buf holds
// its S bytes) to dst, which may have any byte phase ph = dst & 15.  Whole
// 16-byte destination blocks are built from five aligned LDS dwords shifted
// by the phase (v_alignbyte) and stored with one non-temporal 16-byte store
// each (as in copy_payload); the partial first and last blocks are written
// byte by byte, one byte per lane (lanes 0-15 the first block, 16-31 the
// last).
__device__ __forceinline__ void copy_payload_shifted(const uint8_t* buf, uint8_t* dst, uint32_t S, int lane) {
  const uint32_t ph = uniform((uint32_t)((uintptr_t)dst & 15u));
  uint8_t* const dal = dst - ph;
  const uint32_t end = ph + S;
  const uint32_t nblk = (end + 15) >> 4;
  const uint32_t r = (16u - ph) & 3u;  // byte shift inside a dword (uniform)
  const uint32_t* bw = reinterpret_cast<const uint32_t*>(buf);
  // whole blocks: 16k >= ph and 16k + 16 <= end
  const uint32_t k0 = ph ? 1u : 0u;
  const uint32_t k1 = end >> 4;  // blocks below k1 end at or before `end`
  for (uint32_t k = k0 + (uint32_t)lane; k < k1; k += 64) {
    const uint32_t x = 16u * k - ph;  // first payload byte of the block
    const uint32_t d0 = x >> 2;
    const uint32_t w0 = bw[d0], w1 = bw[d0 + 1], w2 = bw[d0 + 2], w3 = bw[d0 + 3], w4 = bw[d0 + 4];
    uint4 v;
    v.x = __builtin_amdgcn_alignbyte(w1, w0, r);
    v.y = __builtin_amdgcn_alignbyte(w2, w1, r);
    v.z = __builtin_amdgcn_alignbyte(w3, w2, r);
    v.w = __builtin_amdgcn_alignbyte(w4, w3, r);
    gstore16_nt(dal + 16u * k, v);
  }
  // partial blocks: the first if ph > 0 (or the payload ends inside it), the
  // last if end is not block aligned and it is not the first
  const uint32_t j = (uint32_t)lane & 15u;
  if (lane < 16) {
    const bool partial = ph != 0 || end < 16;
    if (partial && j >= ph && j < end) gbl(dal)[j] = buf[j - ph];
  } else if (lane < 32) {
    const uint32_t kl = nblk - 1;
    const uint32_t p = 16u * kl + j;
    if (kl > 0 && (end & 15u) != 0 && p < end) gbl(dal)[p] = buf[p - ph];
  }
}

// One chunk of the single pass, executed by one wave.  vb holds its values;
// next() runs once the chunk's offset is known: it takes the wave's next
// ticket and loads that chunk into vb (so the ticket is drawn when the wave
// is about to start it, and chunks publish their sizes close to ticket
// order), and the loads overlap this chunk's payload copy.
template <class T, class Next>
__device__ __forceinline__ void queue_chunk(const LdsTables& tab, uint8_t* buf, const CompressArgs& a,
                                            const CompressSeries& sd, uint64_t tg, int lane,
                                            typename T::U (&vb)[17], Next&& next) {
  const uint64_t c = tg - sd.chunk0;
  const uint64_t nc = (sd.n + kChunk - 1) / kChunk;
  // a2-a6 and the row statistics (a8-a9)
  ChunkPlanes cp;
  bool case1, no_hint = false;  // the queue's waves take chunks far apart: no order hint
  decide_case<T, false>(tab, vb, cp.A, cp.B, case1, no_hint);
  typename T::U e[16];
  transform_front<T, true>(tab, buf, vb, lane, case1, cp, e);
  const ChunkStats st = chunk_stats_or<T>(cp, lane);
  const uint32_t S = uniform(st.S);
  const uint64_t flags = uniform64(st.flags);
  // step 1: publish the size
  if (lane == 0) {
    __hip_atomic_store(a.status + tg, status_word(c == 0 ? kStPre : kStAgg, a.qtag, S), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    gbl(reinterpret_cast<uint32_t*>(sd.out + kHdrBytes))[c] = S;
  }
  // step 2: a7 and the payload at phase 0
  transform_planes<T>(cp, e);
  assemble_payload<T>(buf, cp, flags, S, lane);
  // step 3: the offset
  bool failed = false;
  const uint64_t off = c == 0 ? 0 : look_back(a, tg, sd.chunk0, lane, failed);
  // a payload always ends within nc chunk bounds of the payload's start
  // (the caller's buffer holds at least that much): a look-back that gave
  // up, or any offset past that, writes nothing
  failed = failed || off + S > nc * (uint64_t)T::BOUND;
  if (c != 0 && lane == 0)
    __hip_atomic_store(a.status + tg, status_word(kStPre, a.qtag, off + S), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  next();
  wave_lds_sync();
  // step 4: the payload at its offset
  if (!failed) copy_payload_shifted(buf, sd.out + kHdrBytes + 4 * nc + off, S, lane);
  else if (lane == 0) __hip_atomic_store(&a.ctl->qerror, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (c == nc - 1) {
    write_stream_header(sd.out, sd.dtype, sd.n, off + S, lane);
    if (a.lens && lane == 0) a.lens[sd.idx] = kHdrBytes + 4 * nc + off + S;
  }
  wave_lds_sync();
}

// One dtype per launch.  Every wave takes chunks until it draws one past
// the last.
template <class T, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_compress_queue(CompressArgs a) {
  __shared__ BlockLdsT<NW> sm;
  pass_prologue(sm, a, true);
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);
  uint8_t* buf = wave_bytes(sm, wid);
  typename T::U vb[17];
  if (a.total_chunks == 0 && !a.many && blockIdx.x == 0 && wid == 0)
    write_stream_header(a.one.out, a.one.dtype, 0, 0, lane);
  uint64_t t = take_ticket(a, lane);
  if (t >= a.total_chunks) return;
  CompressSeries sd = find_series(a.one, a.many, a.nseries, t + a.t0);
  load_chunk<T>(sd, t + a.t0 - sd.chunk0, lane, vb);
  for (;;) {
    const CompressSeries cur = sd;
    uint64_t tn = 0;
    bool more = false;
    auto next = [&]() {
      tn = take_ticket(a, lane);
      more = tn < a.total_chunks;
      if (more) {
        sd = find_series(a.one, a.many, a.nseries, tn + a.t0);
        load_chunk<T>(sd, tn + a.t0 - sd.chunk0, lane, vb);
      }
    };
    queue_chunk<T>(sm.tab, buf, a, cur, t + a.t0, lane, vb, next);
    if (!more) break;
    t = tn;
  }
}

// Both dtypes in one launch: the wave branches on the dtype of each chunk's
// series (no prefetch across chunks).
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_compress_queue_mixed(
    CompressArgs a) {
  __shared__ BlockLdsT<NW> sm;
  pass_prologue(sm, a, true);
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);
  uint8_t* buf = wave_bytes(sm, wid);
  auto none = []() {};
  for (;;) {
    const uint64_t t = take_ticket(a, lane);
    if (t >= a.total_chunks) break;
    const uint64_t tg = t + a.t0;
    const CompressSeries sd = find_series(a.one, a.many, a.nseries, tg);
    if (uniform(sd.dtype) == 2) {
      uint64_t vb[17];
      load_chunk<TF64>(sd, tg - sd.chunk0, lane, vb);
      queue_chunk<TF64>(sm.tab, buf, a, sd, tg, lane, vb, none);
    } else {
      uint32_t vb[17];
      load_chunk<TF32>(sd, tg - sd.chunk0, lane, vb);
      queue_chunk<TF32>(sm.tab, buf, a, sd, tg, lane, vb, none);
    }
  }
}

// A one-series launch whose header the host has not read
// (payload_bytes == kFromHeader): the header is read here and checked
// against the descriptor (magic, version, dtype, chunk length, zero fields,
// value count, payload bytes within in_len).  A header that fails leaves a
// payload of 0, so that every chunk then fails its bounds check, and stores
// the launch epoch in the error word.  Wave-uniform (scalar loads).
constexpr uint64_t kFromHeader = ~0ull;
__device__ __forceinline__ DecompressSeries resolve_header(const DecompressArgs& a, int lane) {
  DecompressSeries sd = a.one;
  asm volatile("" ::: "memory");
  if (a.many || sd.payload_bytes != kFromHeader) return sd;
  const const_ptr<uint32_t> h = cst(reinterpret_cast<const uint32_t*>(sd.in));
  uint32_t w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = h[i];
  const uint64_t nc = (sd.n + kChunk - 1) / kChunk;
  const uint64_t payload = (uint64_t)w[6] | ((uint64_t)w[7] << 32);
  const bool ok = w[0] == 0x4E434C46u && w[1] == (1u | (sd.dtype << 8)) && w[2] == (uint32_t)kChunk && w[3] == 0 &&
                  ((uint64_t)w[4] | ((uint64_t)w[5] << 32)) == sd.n && sd.in_len >= kHdrBytes + 4 * nc &&
                  payload <= sd.in_len - kHdrBytes - 4 * nc;
  sd.payload_bytes = ok ? payload : 0;
  if (!ok && lane == 0) __hip_atomic_store(&a.ctl->error, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return sd;
}

// Decompression has no dependence between chunks once the offsets are
// known, so waves take chunks by static striding and use no counter.  Each
// wave loads the payload of its next chunk into registers while it decodes
// the current one; dispatch(series, c, S, pad, total, bad) decodes the chunk
// just staged into LDS.
template <class Dispatch>
__device__ __forceinline__ void decompress_loop(const DecompressArgs& a, uint8_t* buf, int lane, int wid,
                                                Dispatch&& dispatch) {
  uint64_t t = (uint64_t)blockIdx.x * kWavesD + wid;
  if (t >= a.total_chunks) return;
  const DecompressSeries one = resolve_header(a, lane);
  DecompressSeries sd = find_series(one, a.many, a.nseries, t + a.t0);
  Staged st = stage_issue(sd, t + a.t0, a.offsets, a.relative != 0, lane, true);
  // Seventeen stores with an empty window (dropped, no memory access): the
  // loop is then entered, as it is re-entered, with the value stores of a
  // chunk issued after the prefetch, so the wait for the prefetch in
  // stage_store can leave those stores in flight.
  {
    const __amdgpu_buffer_rsrc_t none = store_window(buf, 0);
#pragma unroll
    for (int k = 0; k < 17; ++k) __builtin_amdgcn_raw_buffer_store_b32(0u, none, 4 * (lane + 64 * k), 0, kNonTemporal);
  }
  for (;;) {
    stage_store(buf, st, lane);
    const DecompressSeries cur = sd;
    const uint64_t c = t + a.t0 - cur.chunk0;
    const uint32_t S = st.S, pad = st.pad, total = st.total;
    const bool bad = st.bad;
    const uint64_t tn = t + a.total_waves;
    const bool more = tn < a.total_chunks;
    // the next chunk's loads; past the last chunk the same instructions run
    // on the current chunk with an empty window (no memory access)
    const uint64_t tq = more ? tn : t;
    sd = find_series(one, a.many, a.nseries, tq + a.t0);
    st = stage_issue(sd, tq + a.t0, a.offsets, a.relative != 0, lane, more);
    dispatch(cur, c, S, pad, total, bad);
    if (!more) break;
    t = tn;
  }
}

// The float32 decoder's LDS buffer (wave_blocks) and registers (at most 80
// with 6 waves per SIMD) let it hold 6 waves per SIMD; the float64 one is
// held to 4 by its LDS buffer.
template <class T>
__global__ __launch_bounds__(64 * kWavesD) __attribute__((amdgpu_waves_per_eu(T::W == 32 ? 6 : 4))) void k_decompress(DecompressArgs a) {
  __shared__ BlockLdsT<kWavesD, wave_blocks<T>()> sm;
  load_tables(sm.tab);
  __syncthreads();
  const int lane = lane_id();
  const int wid = (int)uniform(threadIdx.x >> 6);  // wave-uniform: keeps the chunk loop scalar
  uint8_t* buf = wave_bytes(sm, wid);
  decompress_loop(a, buf, lane, wid,
                  [&](const DecompressSeries& sd, uint64_t c, uint32_t S, uint32_t pad, uint32_t total, bool bad) {
                    decompress_chunk<T>(sm.tab, buf, sd, c, S, pad, total, bad, a.epoch, lane, a.ctl);
                  });
}

}  // namespace falcon_dev
