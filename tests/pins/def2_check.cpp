// def2_check.cpp -- pins the oracle's decimal place / significand search
// (the per-value step of Sec. 3.2.2) against Definition 2 computed from the
// shortest round-trip decimal string of each value (std::to_chars, C++17),
// which is reading R1 of the design notes: DP = digits after the decimal
// point of that string, DS = its significant digits counting integer
// trailing zeros (Eq. 2).  Theorems 2-4 then fix what the search returns:
// (DP, DS) when DS <= B_MAX and DP <= A_MAX, the exception otherwise.
//
// Test infrastructure: it loads the oracle's shared library with dlopen and
// shares nothing with the HIP library.
//
// Modes (each prints a summary line and exits 0 only with no mismatch):
//   f32-all      LIB THREADS              every one of the 2^32 binary32 bit patterns
//   f64-random   LIB THREADS COUNT SEED   COUNT binary64 values from four families
//   f64-decimals LIB THREADS MMAX         +-m * 10^-s, 1 <= m < MMAX, s = 0..24
//   f32-decimals LIB THREADS MMAX         +-m * 10^-s, 1 <= m < MMAX, s = 0..12
#include <dlfcn.h>

#include <atomic>
#include <charconv>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using dpds_many_fn = void (*)(const void*, size_t, int, int*, int*, int*);
static dpds_many_fn dpds_many;

struct Def2 {
  int dp, ds;
};

// DP and DS of the shortest round-trip string of a nonzero finite value.
template <class F>
static Def2 def2(F v) {
  char buf[64];
  auto r = std::to_chars(buf, buf + sizeof buf, std::fabs(v), std::chars_format::scientific);
  *r.ptr = 0;
  const char* e = std::strchr(buf, 'e');
  int k = 0;  // significant digits
  for (const char* p = buf; p < e; ++p)
    if (*p >= '0' && *p <= '9') ++k;
  const int E = std::atoi(e + 1);
  Def2 d;
  d.dp = k - 1 - E > 0 ? k - 1 - E : 0;
  d.ds = d.dp + E + 1;
  return d;
}

struct Expect {
  int a, b, e;
};

template <class F, class U>
static Expect expected(F v, int amax, int bmax) {
  U bits;
  std::memcpy(&bits, &v, sizeof bits);
  constexpr int mant = sizeof(F) == 8 ? 52 : 23;
  constexpr U emask = sizeof(F) == 8 ? 0x7FF : 0xFF;
  if (bits == 0) return {0, 0, 0};
  const U ef = (bits >> mant) & emask;
  if (ef == 0 || ef == emask) return {amax + 1, bmax + 1, 1};  // -0.0, subnormal, Inf, NaN
  const Def2 d = def2(v);
  if (d.ds <= bmax && d.dp <= amax) return {d.dp, d.ds, 0};
  return {amax + 1, bmax + 1, 1};
}

struct Tally {
  std::atomic<uint64_t> checked{0}, bad{0}, regular{0};
  std::atomic<uint64_t> alpha_seen{0};  // bit a: some value got decimal place a
  std::mutex mu;
  std::vector<std::string> first;
};

template <class F, class U>
static void check_block(const F* v, size_t n, int dt, int amax, int bmax, Tally& t) {
  std::vector<int> a(n), b(n), e(n);
  dpds_many(v, n, dt, a.data(), b.data(), e.data());
  uint64_t bad = 0, reg = 0, seen = 0;
  for (size_t i = 0; i < n; ++i) {
    const Expect x = expected<F, U>(v[i], amax, bmax);
    if (!x.e) {
      ++reg;
      seen |= 1ull << x.a;
    }
    if (a[i] != x.a || b[i] != x.b || (e[i] != 0) != (x.e != 0)) {
      ++bad;
      std::lock_guard<std::mutex> g(t.mu);
      if (t.first.size() < 10) {
        char s[200];
        std::snprintf(s, sizeof s, "%.17g: oracle (%d,%d,%d) definition (%d,%d,%d)", (double)v[i], a[i], b[i], e[i],
                      x.a, x.b, x.e);
        t.first.push_back(s);
      }
    }
  }
  t.checked += n;
  t.bad += bad;
  t.regular += reg;
  t.alpha_seen |= seen;
}

// Runs job(block) for block = 0..nblocks-1 on `threads` threads.
template <class Job>
static void parallel(int threads, uint64_t nblocks, Job job) {
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> th;
  for (int i = 0; i < threads; ++i)
    th.emplace_back([&] {
      for (uint64_t k; (k = next++) < nblocks;) job(k);
    });
  for (auto& x : th) x.join();
}

static uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int report(const char* mode, Tally& t) {
  std::printf("%s checked %llu regular %llu mismatches %llu alpha_seen 0x%llx\n", mode,
              (unsigned long long)t.checked.load(), (unsigned long long)t.regular.load(),
              (unsigned long long)t.bad.load(), (unsigned long long)t.alpha_seen.load());
  for (auto& s : t.first) std::printf("  %s\n", s.c_str());
  return t.bad.load() == 0 ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc < 4) {
    std::fprintf(stderr, "usage: %s MODE LIB THREADS ...\n", argv[0]);
    return 2;
  }
  const std::string mode = argv[1];
  void* h = dlopen(argv[2], RTLD_NOW);
  if (!h) {
    std::fprintf(stderr, "dlopen: %s\n", dlerror());
    return 2;
  }
  dpds_many = reinterpret_cast<dpds_many_fn>(dlsym(h, "orc_dpds_many"));
  if (!dpds_many) return 2;
  const int threads = std::atoi(argv[3]);
  Tally t;
  if (mode == "f32-all") {
    constexpr uint64_t kBlock = 1 << 20;
    parallel(threads, (1ull << 32) / kBlock, [&](uint64_t k) {
      std::vector<uint32_t> bits(kBlock);
      for (uint64_t i = 0; i < kBlock; ++i) bits[i] = (uint32_t)(k * kBlock + i);
      check_block<float, uint32_t>(reinterpret_cast<const float*>(bits.data()), kBlock, 1, 10, 6, t);
    });
  } else if (mode == "f64-random" && argc >= 6) {
    const uint64_t count = std::strtoull(argv[4], nullptr, 10);
    const uint64_t seed = std::strtoull(argv[5], nullptr, 10);
    constexpr uint64_t kBlock = 1 << 16;
    parallel(threads, (count + kBlock - 1) / kBlock, [&](uint64_t k) {
      uint64_t s = seed * 0x100000001B3ull + k;
      const uint64_t n = std::min<uint64_t>(kBlock, count - k * kBlock);
      std::vector<double> v(n);
      for (uint64_t i = 0; i < n; ++i) {
        const uint64_t r = splitmix(s);
        double x;
        switch (r & 3) {
          case 0: {  // a random bit pattern
            const uint64_t b = splitmix(s);
            std::memcpy(&x, &b, 8);
            break;
          }
          case 1: {  // a decimal of 1..17 significant digits at place -5..30
            const int digits = 1 + (int)((r >> 2) % 17);
            const uint64_t m = splitmix(s) % (uint64_t)std::pow(10.0, digits);
            const int sc = -5 + (int)((r >> 8) % 36);
            char buf[48];
            std::snprintf(buf, sizeof buf, "%llue%d", (unsigned long long)m, -sc);
            x = std::strtod(buf, nullptr);
            break;
          }
          case 2: {  // a sum of two short decimals (the 0.1 + 0.2 kind)
            const double a = (double)((int64_t)(splitmix(s) % 200001) - 100000) / 100.0;
            const double b = (double)((int64_t)(splitmix(s) % 2000001) - 1000000) / 1000.0;
            x = a + b;
            break;
          }
          default: {  // within a few ulps of a power of ten
            const int e10 = -25 + (int)((r >> 2) % 42);
            char buf[16];
            std::snprintf(buf, sizeof buf, "1e%d", e10);
            const double p = std::strtod(buf, nullptr);
            x = std::nextafter(p, (r >> 10) & 1 ? 1e300 : 0.0);
            for (int j = (int)((r >> 11) % 3); j > 0; --j) x = std::nextafter(x, (r >> 13) & 1 ? 1e300 : 0.0);
            if ((r >> 14) & 1) x = -x;
          }
        }
        v[i] = x;
      }
      check_block<double, uint64_t>(v.data(), n, 2, 22, 15, t);
    });
  } else if ((mode == "f64-decimals" || mode == "f32-decimals") && argc >= 5) {
    const uint64_t mmax = std::strtoull(argv[4], nullptr, 10);
    const bool f64 = mode == "f64-decimals";
    const int smax = f64 ? 24 : 12;
    constexpr uint64_t kBlock = 1 << 16;
    const uint64_t per_s = (mmax + kBlock - 1) / kBlock;
    parallel(threads, per_s * (uint64_t)(smax + 1) * 2, [&](uint64_t k) {
      const int sign = (k & 1) ? -1 : 1;
      const int s = (int)((k >> 1) / per_s);
      const uint64_t m0 = 1 + ((k >> 1) % per_s) * kBlock;
      const uint64_t m1 = std::min<uint64_t>(m0 + kBlock, mmax);
      if (m0 >= m1) return;
      char buf[48];
      if (f64) {
        std::vector<double> v;
        for (uint64_t m = m0; m < m1; ++m) {
          std::snprintf(buf, sizeof buf, "%s%llue-%d", sign < 0 ? "-" : "", (unsigned long long)m, s);
          v.push_back(std::strtod(buf, nullptr));  // the double nearest m * 10^-s
        }
        check_block<double, uint64_t>(v.data(), v.size(), 2, 22, 15, t);
      } else {
        std::vector<float> v;
        for (uint64_t m = m0; m < m1; ++m) {
          std::snprintf(buf, sizeof buf, "%s%llue-%d", sign < 0 ? "-" : "", (unsigned long long)m, s);
          v.push_back(std::strtof(buf, nullptr));  // the binary32 value nearest m * 10^-s
        }
        check_block<float, uint32_t>(v.data(), v.size(), 1, 10, 6, t);
      }
    });
  } else {
    std::fprintf(stderr, "bad mode or arguments\n");
    return 2;
  }
  return report(mode.c_str(), t);
}
