/* Checks the decoder's division-free quotient for Case 1 (inverse Eq. 3):
 * with y = RN(1/P), P = 10^alpha, q = RN(g * y),
 *   RN(q + RN(g - q * P) * y)   (two fused multiply-adds)
 * against the IEEE quotient RN(g / P), bit for bit.
 *   f32                  every |g| < 10^6, alpha = 0..10 (all of Case 1)
 *   f64 N SEED           every |g| <= 2 * 10^6, then N random g with
 *                        |g| < 10^15 (log-uniform magnitude), alpha = 0..21
 * Prints "checked C mismatches M" and exits 1 on any mismatch.  The libm
 * fma/fmaf are correctly rounded. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t s_state;
static uint64_t next64(void) { /* splitmix64 */
  uint64_t z = (s_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static long bad, total;

static void one64(double g, double P, double y) {
  volatile double vp = P;
  const double want = g / vp;
  const double q = g * y;
  const double got = fma(fma(-q, P, g), y, q);
  uint64_t a, b;
  memcpy(&a, &want, 8);
  memcpy(&b, &got, 8);
  if (a != b) {
    if (bad < 5) printf("f64 g=%.17g P=%.17g want %a got %a\n", g, P, want, got);
    ++bad;
  }
  ++total;
}

int main(int argc, char** argv) {
  if (argc >= 2 && strcmp(argv[1], "f32") == 0) {
    for (int a = 0; a <= 10; ++a) {
      float P = 1.0f;
      for (int k = 0; k < a; ++k) P *= 10.0f; /* exact for a <= 10 */
      volatile float one = 1.0f, vp = P;
      const float y = one / vp;
      for (int32_t g = -999999; g <= 999999; ++g) {
        const float x = (float)g;
        const float want = x / vp;
        const float q = x * y;
        const float got = fmaf(fmaf(-q, P, x), y, q);
        uint32_t wa, wb;
        memcpy(&wa, &want, 4);
        memcpy(&wb, &got, 4);
        if (wa != wb) {
          if (bad < 5) printf("f32 g=%d P=%.9g want %a got %a\n", g, (double)P, (double)want, (double)got);
          ++bad;
        }
        ++total;
      }
    }
  } else if (argc >= 4 && strcmp(argv[1], "f64") == 0) {
    const long n = atol(argv[2]);
    s_state = (uint64_t)atoll(argv[3]);
    for (int a = 0; a <= 21; ++a) {
      double P = 1.0;
      for (int k = 0; k < a; ++k) P *= 10.0; /* exact for a <= 22 */
      volatile double one = 1.0, vp = P;
      const double y = one / vp;
      for (int64_t g = -2000000; g <= 2000000; ++g) one64((double)g, P, y);
      for (long i = 0; i < n; ++i) {
        const uint64_t r = next64();
        const int bits = 1 + (int)(r % 50);               /* magnitude 2^0 .. 2^50 */
        int64_t g = (int64_t)(next64() >> (64 - bits));
        if (g >= 1000000000000000ll) g %= 1000000000000000ll;
        one64((double)((r >> 63) ? -g : g), P, y);
      }
    }
  } else {
    fprintf(stderr, "usage: quotient_check f32 | f64 N SEED\n");
    return 2;
  }
  printf("checked %ld mismatches %ld\n", total, bad);
  return bad != 0;
}
