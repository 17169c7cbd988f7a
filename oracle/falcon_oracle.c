/*
 * falcon_oracle.c -- plain, slow CPU oracle of the Falcon lossless float codec
 * (arXiv 2511.04140, "Falcon: GPU-Based Floating-point Adaptive Lossless
 * Compression").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant generator
 * with the HIP library; the two meet only at the byte stream.
 *
 * Arithmetic: IEEE binary64 (binary32 for the float path), round to nearest
 * even, no FMA contraction (built with -ffp-contract=off), no fast-math, no
 * flush-to-zero.  Integer arithmetic is done on unsigned types, i.e. two's
 * complement modulo 2^64 (2^32).
 *
 * Each step cites the passage of the paper it follows.  Where the paper is
 * silent the reading taken is stated next to the code (R-numbers match the
 * list of readings kept with the design notes).
 *
 * Stream layout (all little-endian):
 *   container header, 32 bytes: "FLCN", version u8 = 1, dtype u8 (1 = f32,
 *     2 = f64), u16 0, chunk length u32 = 1025, u32 0, N u64,
 *     payload_bytes u64;
 *   compressed chunk size array, u32 per chunk (Sec. 3.4, Alg. 3);
 *   chunk payloads in chunk order (layout of Fig. 9(c), Sec. 3.3).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_SMALL 2
#define ORC_ERR_CORRUPT 3

#define DT_F32 1
#define DT_F64 2

#define CHUNK_N 1025 /* Sec. 5.1.4: 1025 values per chunk; n = 64k + 1 (Sec. 3.3) */

/* Variants of the ablation study (Sec. 5.4.2, Fig. 12b).  Only the step named
 * changes; every variant writes a stream of the same layout, which the one
 * decoder reads.
 *   V_FALCON  the method as described;
 *   V_ELF     Alg. 2 with the trial-and-error stopping test of Sec. 1 (the
 *             scaled value must be an exact integer) in place of the error
 *             bound of Thm. 4 (reading R22);
 *   V_SPARSE  every bit-plane row written sparse (reading R23);
 *   V_DENSE   every bit-plane row written dense. */
#define V_FALCON 0
#define V_ELF 1
#define V_SPARSE 2
#define V_DENSE 3
#define HDR_BYTES 32

/* ------------------------------------------------------------------------- */
/* Bit helpers                                                               */
/* ------------------------------------------------------------------------- */
static uint64_t bits64(double v) { uint64_t u; memcpy(&u, &v, 8); return u; }
static double from_bits64(uint64_t u) { double v; memcpy(&v, &u, 8); return v; }
static uint32_t bits32(float v) { uint32_t u; memcpy(&u, &v, 4); return u; }
static float from_bits32(uint32_t u) { float v; memcpy(&v, &u, 4); return v; }

/* Zigzag (Eq. 4): (x << 1) xor (x >> 63) with an arithmetic right shift. */
static uint64_t zz64(uint64_t x) { return (x << 1) ^ (0 - (x >> 63)); }
static uint64_t unzz64(uint64_t z) { return (z >> 1) ^ (0 - (z & 1)); }
static uint32_t zz32(uint32_t x) { return (x << 1) ^ (0u - (x >> 31)); }
static uint32_t unzz32(uint32_t z) { return (z >> 1) ^ (0u - (z & 1u)); }

/* ------------------------------------------------------------------------- */
/* Powers of ten and floor(log10)                                            */
/* ------------------------------------------------------------------------- */
/* P[k] = fl(10^k), correctly rounded (strtod / strtof round correctly).
 * For 0 <= k <= 22 (binary64) and 0 <= k <= 10 (binary32) the value is exact
 * (Thm. 3: 5^k fits the significand).  Range k in [-330, 320] (binary64) and
 * [-50, 45] (binary32); the ends round to 0 and to infinity, which serve as
 * sentinels for the search below. */
#define P64_LO (-330)
#define P64_HI 320
#define P32_LO (-50)
#define P32_HI 45
static double P64[P64_HI - P64_LO + 1];
static float P32[P32_HI - P32_LO + 1];
static int tables_ready = 0;

static void init_tables(void) {
  if (tables_ready) return;
  char buf[32];
  for (int k = P64_LO; k <= P64_HI; ++k) {
    snprintf(buf, sizeof buf, "1e%d", k);
    P64[k - P64_LO] = strtod(buf, NULL);
  }
  for (int k = P32_LO; k <= P32_HI; ++k) {
    snprintf(buf, sizeof buf, "1e%d", k);
    P32[k - P32_LO] = strtof(buf, NULL);
  }
  tables_ready = 1;
}
static double pow10_64(int k) { return P64[k - P64_LO]; }
static float pow10_32(int k) { return P32[k - P32_LO]; }

/* FL10(a) for a positive normal value: the largest k with fl(10^k) <= a.
 * Reading R4: the paper writes floor(log10|v|) (Alg. 2, Eq. 2, Sec. 3.2.3)
 * without saying how a machine computes it.  Because rounding is monotone,
 * this k equals the decimal exponent of the shortest round-trip string of a,
 * i.e. floor(log10 DF(a)).  Plain binary search over the table. */
static int fl10_64(double a) {
  int lo = P64_LO, hi = P64_HI; /* invariant: P[lo] <= a < P[hi] */
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    if (pow10_64(mid) <= a) lo = mid; else hi = mid;
  }
  return lo;
}
static int fl10_32(float a) {
  int lo = P32_LO, hi = P32_HI;
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    if (pow10_32(mid) <= a) lo = mid; else hi = mid;
  }
  return lo;
}

/* ------------------------------------------------------------------------- */
/* Decimal place and significand (Def. 2, Sec. 3.2.2)                        */
/* ------------------------------------------------------------------------- */
/* binary64 constants: alpha <= 22 keeps 10^alpha exact (Thm. 3);
 * beta <= 15 is the precision guard of Thm. 2 / Thm. 4. */
#define A_MAX64 22
#define B_MAX64 15
/* binary32 constants, re-derived with the same arguments for a 24-bit
 * significand: 5^10 < 2^24 < 5^11 gives alpha <= 10; 10^-6 * 2^23 > 4.5 >
 * 10^-7 * 2^23 gives beta <= 6 (the "easily extended" remark of Sec. 2.1). */
#define A_MAX32 10
#define B_MAX32 6

/* Decimal place and decimal significand of one value (Def. 2), found the
 * way Sec. 3.2.2 finds them: scale the value by growing powers of ten until
 * the product is an integer within the error bound of Thm. 4, then make sure
 * that integer divides back to the same value.  The result is (alpha, beta,
 * exc); exc = 1 marks a value the digit transformation cannot take, reported
 * as (A_MAX+1, B_MAX+1) whatever made it fail (reading R7). */
typedef struct { int alpha, beta, exc; } dpds_t;

static dpds_t dpds_exception(int a_max, int b_max) {
  dpds_t e = {a_max + 1, b_max + 1, 1};
  return e;
}

/* The largest decimal place the search may reach for a value whose
 * FL10 is fl: beta = alpha + fl + 1 (Eq. 2) must stay within B_MAX, the
 * precision guard of Thm. 2 / Thm. 4, and 10^alpha must be exact, alpha
 * within A_MAX (Thm. 3).  Negative when no place is allowed. */
static int place_limit(int fl, int a_max, int b_max) {
  int lim = b_max - 1 - fl;
  return lim < a_max ? lim : a_max;
}

/* binary64 ------------------------------------------------------------------ */
/* Does the search stop at place alpha?  x = v (x) 10^alpha, one rounded
 * product (the machine multiply of Sec. 1).  Thm. 4: x stands for an
 * integer when it lies within |x| * 2^-52 of its nearest integer (round =
 * rint, reading R5).  Fal_Elf's rule (Sec. 1): only where x is an exact
 * integer.  The nearest integer is handed back in *r. */
static int stops_at_64(double v, int alpha, int elf, double* r) {
  const double x = v * pow10_64(alpha);
  *r = rint(x);
  if (elf) return x == floor(x);
  return fabs(x - *r) <= fabs(x) * 0x1p-52;
}

/* Exactness guard of Alg. 2: the integer, divided by 10^alpha with IEEE
 * division (correctly rounded), must give back v bit for bit. */
static int recovers_64(double v, double r, int alpha) {
  return bits64(r / pow10_64(alpha)) == bits64(v);
}

/* The first place in [0, lim] where the search stops, or -1. */
static int first_stop_64(double v, int lim, int elf, double* r) {
  for (int alpha = 0; alpha <= lim; ++alpha)
    if (stops_at_64(v, alpha, elf, r)) return alpha;
  return -1;
}

static dpds_t dpds_f64(double v, int elf) {
  const uint64_t b = bits64(v);
  /* Alg. 2's special case v = 0 is taken only by +0.0, the all-zero bit
   * pattern of Sec. 2.1 (reading R2); -0.0 keeps its sign through Case 2. */
  if (b == 0) {
    dpds_t z = {0, 0, 0};
    return z;
  }
  const unsigned ef = (unsigned)((b >> 52) & 0x7FF);
  if (ef == 0 || ef == 0x7FF) return dpds_exception(A_MAX64, B_MAX64); /* R3 */
  const int fl = fl10_64(fabs(v));
  double r = 0.0;
  const int alpha = first_stop_64(v, place_limit(fl, A_MAX64, B_MAX64), elf, &r);
  if (alpha < 0 || !recovers_64(v, r, alpha)) return dpds_exception(A_MAX64, B_MAX64);
  dpds_t d = {alpha, alpha + fl + 1, 0}; /* Eq. 2 */
  return d;
}

/* binary32: the same steps in binary32 arithmetic, bound 2^-23 ---------------- */
static int stops_at_32(float v, int alpha, int elf, float* r) {
  const float x = v * pow10_32(alpha);
  *r = rintf(x);
  if (elf) return x == floorf(x);
  return fabsf(x - *r) <= fabsf(x) * 0x1p-23f;
}

static int recovers_32(float v, float r, int alpha) {
  return bits32(r / pow10_32(alpha)) == bits32(v);
}

static int first_stop_32(float v, int lim, int elf, float* r) {
  for (int alpha = 0; alpha <= lim; ++alpha)
    if (stops_at_32(v, alpha, elf, r)) return alpha;
  return -1;
}

static dpds_t dpds_f32(float v, int elf) {
  const uint32_t b = bits32(v);
  if (b == 0) {
    dpds_t z = {0, 0, 0};
    return z;
  }
  const unsigned ef = (b >> 23) & 0xFF;
  if (ef == 0 || ef == 0xFF) return dpds_exception(A_MAX32, B_MAX32);
  const int fl = fl10_32(fabsf(v));
  float r = 0.0f;
  const int alpha = first_stop_32(v, place_limit(fl, A_MAX32, B_MAX32), elf, &r);
  if (alpha < 0 || !recovers_32(v, r, alpha)) return dpds_exception(A_MAX32, B_MAX32);
  dpds_t d = {alpha, alpha + fl + 1, 0};
  return d;
}

/* ------------------------------------------------------------------------- */
/* Digit transformation (Sec. 3.2.3, Eq. 3, Eq. 4, Alg. 3)                   */
/* ------------------------------------------------------------------------- */
/* Computes the chunk header bytes (A, B) and Z = {z_1..z_n} for n values.
 * z is returned as uint64 (for binary32 only the low 32 bits are used). */
static void transform_f64(const double* v, int n, int elf, int* A, int* B, uint64_t* z) {
  int any_exc = 0, amax = 0;
  double vmax = 0.0;
  for (int i = 0; i < n; ++i) {
    dpds_t d = dpds_f64(v[i], elf);
    if (d.exc) any_exc = 1;
    else if (d.alpha > amax) amax = d.alpha;
    if (!d.exc && fabs(v[i]) > vmax) vmax = fabs(v[i]);
  }
  int case1;
  if (any_exc) {             /* reading R7: any exception -> header (23, 16) */
    *A = A_MAX64 + 1; *B = B_MAX64 + 1; case1 = 0;
  } else {                   /* alpha_max and beta_hat_max of Sec. 3.2.3 */
    *A = amax;
    *B = (vmax == 0.0) ? 0 : amax + fl10_64(vmax) + 1;
    case1 = (*A <= A_MAX64 && *B <= B_MAX64);
  }
  uint64_t prev = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t g;
    if (case1) {
      double r = rint(v[i] * pow10_64(*A));   /* Eq. 3, Case 1 */
      g = (uint64_t)(int64_t)r;               /* |r| < 10^15: exact */
    } else {
      g = zz64(bits64(v[i]));                 /* Eq. 3, Case 2: Zigzag(BinLong) */
    }
    z[i] = (i == 0) ? g : zz64(g - prev);     /* Eq. 4 (mod 2^64, reading R19) */
    prev = g;
  }
}

static void transform_f32(const float* v, int n, int elf, int* A, int* B, uint64_t* z) {
  int any_exc = 0, amax = 0;
  float vmax = 0.0f;
  for (int i = 0; i < n; ++i) {
    dpds_t d = dpds_f32(v[i], elf);
    if (d.exc) any_exc = 1;
    else if (d.alpha > amax) amax = d.alpha;
    if (!d.exc && fabsf(v[i]) > vmax) vmax = fabsf(v[i]);
  }
  int case1;
  if (any_exc) {
    *A = A_MAX32 + 1; *B = B_MAX32 + 1; case1 = 0;
  } else {
    *A = amax;
    *B = (vmax == 0.0f) ? 0 : amax + fl10_32(vmax) + 1;
    case1 = (*A <= A_MAX32 && *B <= B_MAX32);
  }
  uint32_t prev = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t g;
    if (case1) {
      float r = rintf(v[i] * pow10_32(*A));
      g = (uint32_t)(int32_t)r;               /* |r| < 10^6: exact */
    } else {
      g = zz32(bits32(v[i]));
    }
    z[i] = (i == 0) ? g : zz32(g - prev);
    prev = g;
  }
}

/* ------------------------------------------------------------------------- */
/* Adaptive bit-plane encoding (Sec. 3.3, Fig. 9)                            */
/* ------------------------------------------------------------------------- */
/* Bit p of z. */
static int zbit(uint64_t z, int p) { return (int)((z >> p) & 1u); }

/* Encodes one chunk whose Z has n = 64k+1 entries.  W = 64 or 32 is the
 * integer width, zb = 8 or 4 the number of bytes of z_1; variant V_SPARSE or
 * V_DENSE fixes every row's scheme.  Returns the byte count written to out
 * (out must hold the worst case). */
static size_t encode_chunk_z(const uint64_t* z, int n, int W, int zb, int A, int B, int variant,
                             uint8_t* out) {
  const int m = n - 1;          /* entries of M: z_2..z_n */
  const int rowb = m / 8;       /* bytes per row of M^T */
  const int bmb = m / 64;       /* bitmap bytes, (n-1)/64 */
  /* bit width w = W - lead_min over z_2..z_n; lead of 0 is W (reading R11) */
  int w = 0;
  for (int j = 0; j < m; ++j) {
    int width = 0;
    for (int p = W - 1; p >= 0; --p) if (zbit(z[j + 1], p)) { width = p + 1; break; }
    if (width > w) w = width;
  }
  size_t o = 0;
  out[o++] = (uint8_t)A;
  out[o++] = (uint8_t)B;
  for (int k = 0; k < zb; ++k) out[o++] = (uint8_t)(z[0] >> (8 * k)); /* z_1 LE (R15) */
  out[o++] = (uint8_t)w;
  const int nflag = (w + 7) / 8;
  size_t flag_pos = o;
  for (int k = 0; k < nflag; ++k) out[o++] = 0;
  uint8_t row[128];
  for (int r = 1; r <= w; ++r) {
    int p = w - r;              /* row 1 holds the most significant plane (R12) */
    /* Row byte b holds plane p of entries 8b..8b+7, first entry in the most
     * significant bit (R13). */
    for (int b = 0; b < rowb; ++b) {
      unsigned byte = 0;
      for (int t = 0; t < 8; ++t) byte |= (unsigned)zbit(z[1 + 8 * b + t], p) << (7 - t);
      row[b] = (uint8_t)byte;
    }
    int lambda = 0;             /* number of zero bytes */
    for (int b = 0; b < rowb; ++b) if (row[b] == 0) lambda++;
    /* Sparse iff lambda > (n-1)/64 (Sec. 3.3); the tie goes to Dense (R9, R10). */
    int dense = !(lambda > bmb);
    if (variant == V_SPARSE) dense = 0;
    if (variant == V_DENSE) dense = 1;
    if (dense) {
      /* Flag bits: big-endian bit string, right-aligned, row r at bit (w - r),
       * '1' = dense (R14). */
      int bitpos = w - r;
      out[flag_pos + (size_t)(nflag - 1 - bitpos / 8)] |= (uint8_t)(1u << (bitpos % 8));
      for (int b = 0; b < rowb; ++b) out[o++] = row[b];
    } else {
      for (int k = 0; k < bmb; ++k) out[o + (size_t)k] = 0;
      for (int b = 0; b < rowb; ++b)
        if (row[b]) out[o + (size_t)(b / 8)] |= (uint8_t)(1u << (7 - b % 8));
      o += (size_t)bmb;
      for (int b = 0; b < rowb; ++b) if (row[b]) out[o++] = row[b];
    }
  }
  return o;
}

/* Decodes one chunk payload of exactly len bytes into z[0..n-1] and (A, B).
 * Returns ORC_OK or ORC_ERR_CORRUPT; never reads outside in[0..len). */
static int decode_chunk_z(const uint8_t* in, size_t len, int n, int W, int zb,
                          int* A, int* B, uint64_t* z) {
  const int m = n - 1, rowb = m / 8, bmb = m / 64;
  size_t o = 0;
  if (len < (size_t)(3 + zb)) return ORC_ERR_CORRUPT;
  *A = in[o++];
  *B = in[o++];
  uint64_t z1 = 0;
  for (int k = 0; k < zb; ++k) z1 |= (uint64_t)in[o++] << (8 * k);
  z[0] = z1;
  int w = in[o++];
  if (w > W) return ORC_ERR_CORRUPT;
  const int nflag = (w + 7) / 8;
  if (o + (size_t)nflag > len) return ORC_ERR_CORRUPT;
  const uint8_t* flags = in + o;
  o += (size_t)nflag;
  for (int j = 0; j < m; ++j) z[1 + j] = 0;
  uint8_t row[128];
  for (int r = 1; r <= w; ++r) {
    int p = w - r, bitpos = w - r;
    int dense = (flags[nflag - 1 - bitpos / 8] >> (bitpos % 8)) & 1;
    if (dense) {
      if (o + (size_t)rowb > len) return ORC_ERR_CORRUPT;
      for (int b = 0; b < rowb; ++b) row[b] = in[o++];
    } else {
      if (o + (size_t)bmb > len) return ORC_ERR_CORRUPT;
      const uint8_t* bm = in + o;
      o += (size_t)bmb;
      for (int b = 0; b < rowb; ++b) {
        if ((bm[b / 8] >> (7 - b % 8)) & 1) {
          if (o + 1 > len) return ORC_ERR_CORRUPT;
          row[b] = in[o++];
        } else {
          row[b] = 0;
        }
      }
    }
    for (int b = 0; b < rowb; ++b)
      for (int t = 0; t < 8; ++t)
        z[1 + 8 * b + t] |= (uint64_t)((row[b] >> (7 - t)) & 1u) << p;
  }
  if (o != len) return ORC_ERR_CORRUPT;
  return ORC_OK;
}

/* Inverse of Eq. 4 and Eq. 3 (Sec. 4). */
static int untransform_f64(const uint64_t* z, int n, int A, int B, double* v) {
  int case1 = (A <= A_MAX64 && B <= B_MAX64);
  uint64_t g = 0;
  for (int i = 0; i < n; ++i) {
    g = (i == 0) ? z[0] : g + unzz64(z[i]);
    if (case1) v[i] = (double)(int64_t)g / pow10_64(A);   /* g / 10^alpha_max */
    else v[i] = from_bits64(unzz64(g));                  /* BinLong^-1(Zigzag^-1) */
  }
  return ORC_OK;
}

static int untransform_f32(const uint64_t* z, int n, int A, int B, float* v) {
  int case1 = (A <= A_MAX32 && B <= B_MAX32);
  uint32_t g = 0;
  for (int i = 0; i < n; ++i) {
    g = (i == 0) ? (uint32_t)z[0] : g + unzz32((uint32_t)z[i]);
    if (case1) v[i] = (float)(int32_t)g / pow10_32(A);
    else v[i] = from_bits32(unzz32(g));
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Public entry points (ctypes)                                              */
/* ------------------------------------------------------------------------- */
static int dtype_bytes(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 0); }
static size_t chunk_bound(int dt) { return dt == DT_F64 ? 11 + 8 + 64 * 128 : 7 + 4 + 32 * 128; }
/* An all-sparse row can take 16 bitmap bytes + 128 data bytes. */
static size_t chunk_bound_v(int dt, int variant) {
  if (variant != V_SPARSE) return chunk_bound(dt);
  return dt == DT_F64 ? 11 + 8 + 64 * 144 : 7 + 4 + 32 * 144;
}

size_t orc_bound_v(size_t n, int dt, int variant) {
  size_t nc = (n + CHUNK_N - 1) / CHUNK_N;
  return HDR_BYTES + nc * (4 + chunk_bound_v(dt, variant));
}
size_t orc_bound(size_t n, int dt) { return orc_bound_v(n, dt, V_FALCON); }

int orc_fl10_f64(double a) { init_tables(); return fl10_64(a); }
int orc_fl10_f32(float a) { init_tables(); return fl10_32(a); }

void orc_dpds_f64(double v, int* alpha, int* beta, int* exc) {
  init_tables();
  dpds_t d = dpds_f64(v, 0);
  *alpha = d.alpha; *beta = d.beta; *exc = d.exc;
}
void orc_dpds_f32(float v, int* alpha, int* beta, int* exc) {
  init_tables();
  dpds_t d = dpds_f32(v, 0);
  *alpha = d.alpha; *beta = d.beta; *exc = d.exc;
}

/* Alg. 2 over an array (batch form of the two functions above, for tests);
 * variant V_ELF uses the trial-and-error stopping test. */
void orc_dpds_many_v(const void* v, size_t n, int dt, int variant, int* alpha, int* beta, int* exc) {
  init_tables();
  const int elf = variant == V_ELF;
  for (size_t i = 0; i < n; ++i) {
    dpds_t d = dt == DT_F64 ? dpds_f64(((const double*)v)[i], elf) : dpds_f32(((const float*)v)[i], elf);
    alpha[i] = d.alpha; beta[i] = d.beta; exc[i] = d.exc;
  }
}
void orc_dpds_many(const void* v, size_t n, int dt, int* alpha, int* beta, int* exc) {
  orc_dpds_many_v(v, n, dt, V_FALCON, alpha, beta, exc);
}
void orc_fl10_many(const void* v, size_t n, int dt, int* out) {
  init_tables();
  for (size_t i = 0; i < n; ++i)
    out[i] = dt == DT_F64 ? fl10_64(((const double*)v)[i]) : fl10_32(((const float*)v)[i]);
}

/* Fills n values of a chunk of length chunk_n: positions at or past nv repeat
 * the bits of the last valid value (reading R17). */
static void pad_f64(const double* v, size_t nv, int chunk_n, double* buf) {
  for (int i = 0; i < chunk_n; ++i) buf[i] = v[(size_t)i < nv ? (size_t)i : nv - 1];
}
static void pad_f32(const float* v, size_t nv, int chunk_n, float* buf) {
  for (int i = 0; i < chunk_n; ++i) buf[i] = v[(size_t)i < nv ? (size_t)i : nv - 1];
}

/* Encodes one chunk of nv (1 <= nv <= chunk_n) values with chunk length
 * chunk_n = 64k+1 (k >= 1).  Used for the full stream and for small-n tests. */
int orc_encode_chunk_v(const void* vals, size_t nv, int dt, int chunk_n, int variant, uint8_t* out,
                       size_t* out_len) {
  init_tables();
  if (chunk_n < 65 || (chunk_n - 1) % 64 != 0 || nv == 0 || nv > (size_t)chunk_n)
    return ORC_ERR_ARG;
  if (variant < V_FALCON || variant > V_DENSE) return ORC_ERR_ARG;
  const int elf = variant == V_ELF;
  uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)chunk_n);
  int A = 0, B = 0;
  if (dt == DT_F64) {
    double* buf = (double*)malloc(sizeof(double) * (size_t)chunk_n);
    pad_f64((const double*)vals, nv, chunk_n, buf);
    transform_f64(buf, chunk_n, elf, &A, &B, z);
    *out_len = encode_chunk_z(z, chunk_n, 64, 8, A, B, variant, out);
    free(buf);
  } else if (dt == DT_F32) {
    float* buf = (float*)malloc(sizeof(float) * (size_t)chunk_n);
    pad_f32((const float*)vals, nv, chunk_n, buf);
    transform_f32(buf, chunk_n, elf, &A, &B, z);
    *out_len = encode_chunk_z(z, chunk_n, 32, 4, A, B, variant, out);
    free(buf);
  } else {
    free(z);
    return ORC_ERR_ARG;
  }
  free(z);
  return ORC_OK;
}
int orc_encode_chunk(const void* vals, size_t nv, int dt, int chunk_n, uint8_t* out, size_t* out_len) {
  return orc_encode_chunk_v(vals, nv, dt, chunk_n, V_FALCON, out, out_len);
}

/* Decodes one chunk payload of len bytes into chunk_n values. */
int orc_decode_chunk(const uint8_t* in, size_t len, int dt, int chunk_n, void* out) {
  init_tables();
  if (chunk_n < 65 || (chunk_n - 1) % 64 != 0) return ORC_ERR_ARG;
  uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)chunk_n);
  int A = 0, B = 0, st;
  if (dt == DT_F64) {
    st = decode_chunk_z(in, len, chunk_n, 64, 8, &A, &B, z);
    if (st == ORC_OK) st = untransform_f64(z, chunk_n, A, B, (double*)out);
  } else if (dt == DT_F32) {
    st = decode_chunk_z(in, len, chunk_n, 32, 4, &A, &B, z);
    if (st == ORC_OK) st = untransform_f32(z, chunk_n, A, B, (float*)out);
  } else {
    st = ORC_ERR_ARG;
  }
  free(z);
  return st;
}

/* Chunk introspection for tests: header bytes, case, bit width and the
 * dense/sparse flag word (bit p = plane p is dense). */
int orc_chunk_info(const void* vals, size_t nv, int dt, int chunk_n, int* A, int* B,
                   int* w, uint64_t* dense_mask) {
  uint8_t* out = (uint8_t*)malloc(chunk_bound(dt) + 64);
  size_t len = 0;
  int st = orc_encode_chunk(vals, nv, dt, chunk_n, out, &len);
  if (st == ORC_OK) {
    int zb = dt == DT_F64 ? 8 : 4;
    *A = out[0];
    *B = out[1];
    *w = out[2 + zb];
    int nflag = (*w + 7) / 8;
    uint64_t f = 0;
    for (int k = 0; k < nflag; ++k) f = (f << 8) | out[3 + zb + k];
    *dense_mask = f;
  }
  free(out);
  return st;
}

static void put_u32(uint8_t* p, uint32_t v) { for (int k = 0; k < 4; ++k) p[k] = (uint8_t)(v >> (8 * k)); }
static void put_u64(uint8_t* p, uint64_t v) { for (int k = 0; k < 8; ++k) p[k] = (uint8_t)(v >> (8 * k)); }
static uint32_t get_u32(const uint8_t* p) { uint32_t v = 0; for (int k = 0; k < 4; ++k) v |= (uint32_t)p[k] << (8 * k); return v; }
static uint64_t get_u64(const uint8_t* p) { uint64_t v = 0; for (int k = 0; k < 8; ++k) v |= (uint64_t)p[k] << (8 * k); return v; }

/* Whole-array compression into the container format.  Chunks are independent
 * (Sec. 3, Alg. 3); their sizes are prefix-summed into offsets (Sec. 3.4)
 * and the payloads written back to back. */
int orc_compress_v(const void* in, size_t n, int dt, int variant, uint8_t* out, size_t cap, size_t* out_len) {
  init_tables();
  int s = dtype_bytes(dt);
  if (s == 0 || variant < V_FALCON || variant > V_DENSE) return ORC_ERR_ARG;
  if (cap < orc_bound_v(n, dt, variant)) { *out_len = orc_bound_v(n, dt, variant); return ORC_ERR_SMALL; }
  size_t nc = (n + CHUNK_N - 1) / CHUNK_N;
  uint8_t* sizes = out + HDR_BYTES;
  uint8_t* pay = sizes + 4 * nc;
  size_t off = 0;
  for (size_t c = 0; c < nc; ++c) {
    size_t nv = n - c * CHUNK_N;
    if (nv > CHUNK_N) nv = CHUNK_N;
    size_t len = 0;
    int st = orc_encode_chunk_v((const uint8_t*)in + c * CHUNK_N * (size_t)s, nv, dt, CHUNK_N, variant,
                                pay + off, &len);
    if (st != ORC_OK) return st;
    put_u32(sizes + 4 * c, (uint32_t)len);
    off += len;
  }
  memcpy(out, "FLCN", 4);
  out[4] = 1;
  out[5] = (uint8_t)dt;
  out[6] = 0;
  out[7] = 0;
  put_u32(out + 8, CHUNK_N);
  put_u32(out + 12, 0);
  put_u64(out + 16, (uint64_t)n);
  put_u64(out + 24, (uint64_t)off);
  *out_len = HDR_BYTES + 4 * nc + off;
  return ORC_OK;
}
int orc_compress(const void* in, size_t n, int dt, uint8_t* out, size_t cap, size_t* out_len) {
  return orc_compress_v(in, n, dt, V_FALCON, out, cap, out_len);
}

/* Parses and checks the container header; fills n, dt, nc, payload bytes. */
static int parse_header(const uint8_t* in, size_t len, size_t* n, int* dt, size_t* nc,
                        size_t* payload) {
  if (len < HDR_BYTES) return ORC_ERR_CORRUPT;
  if (memcmp(in, "FLCN", 4) != 0 || in[4] != 1) return ORC_ERR_CORRUPT;
  if (in[5] != DT_F32 && in[5] != DT_F64) return ORC_ERR_CORRUPT;
  if (in[6] || in[7] || get_u32(in + 8) != CHUNK_N || get_u32(in + 12)) return ORC_ERR_CORRUPT;
  uint64_t nn = get_u64(in + 16), pb = get_u64(in + 24);
  uint64_t ncc = (nn + CHUNK_N - 1) / CHUNK_N;
  if (ncc > (len - HDR_BYTES) / 4) return ORC_ERR_CORRUPT;
  if (pb > len - HDR_BYTES - 4 * ncc) return ORC_ERR_CORRUPT;
  *n = (size_t)nn; *dt = in[5]; *nc = (size_t)ncc; *payload = (size_t)pb;
  return ORC_OK;
}

int orc_stream_info(const uint8_t* in, size_t len, size_t* n, int* dt) {
  size_t nc, pb;
  return parse_header(in, len, n, dt, &nc, &pb);
}

/* Decompression (Sec. 4): scan the size array into offsets, decode each
 * chunk, invert Eq. 4 and Eq. 3, keep the first N values. */
int orc_decompress(const uint8_t* in, size_t len, void* out, size_t cap_bytes, size_t* n_out) {
  init_tables();
  size_t n, nc, pb;
  int dt;
  int st = parse_header(in, len, &n, &dt, &nc, &pb);
  if (st != ORC_OK) return st;
  int s = dtype_bytes(dt);
  *n_out = n;
  if (cap_bytes / (size_t)s < n) return ORC_ERR_SMALL;
  const uint8_t* sizes = in + HDR_BYTES;
  const uint8_t* pay = sizes + 4 * nc;
  size_t off = 0;
  uint8_t* buf = (uint8_t*)malloc((size_t)CHUNK_N * (size_t)s);
  for (size_t c = 0; c < nc; ++c) {
    size_t cs = get_u32(sizes + 4 * c);
    if (cs > pb - off) { free(buf); return ORC_ERR_CORRUPT; }
    st = orc_decode_chunk(pay + off, cs, dt, CHUNK_N, buf);
    if (st != ORC_OK) { free(buf); return st; }
    size_t nv = n - c * CHUNK_N;
    if (nv > CHUNK_N) nv = CHUNK_N;
    memcpy((uint8_t*)out + c * CHUNK_N * (size_t)s, buf, nv * (size_t)s);
    off += cs;
  }
  free(buf);
  if (off != pb) return ORC_ERR_CORRUPT;
  return ORC_OK;
}

/* Stream validator: checks every bound while parsing, then requires each
 * chunk to be canonical, i.e. decoding it and encoding the decoded values
 * again gives the same bytes, and the padding of the last chunk repeats its
 * last value.  Returns ORC_OK or ORC_ERR_CORRUPT; never reads outside
 * in[0..len). */
int orc_validate(const uint8_t* in, size_t len) {
  init_tables();
  size_t n, nc, pb;
  int dt;
  int st = parse_header(in, len, &n, &dt, &nc, &pb);
  if (st != ORC_OK) return st;
  if (HDR_BYTES + 4 * nc + pb != len) return ORC_ERR_CORRUPT;
  int s = dtype_bytes(dt);
  const uint8_t* sizes = in + HDR_BYTES;
  const uint8_t* pay = sizes + 4 * nc;
  uint8_t* vals = (uint8_t*)malloc((size_t)CHUNK_N * (size_t)s);
  uint8_t* re = (uint8_t*)malloc(chunk_bound(dt) + 64);
  size_t off = 0;
  st = ORC_OK;
  for (size_t c = 0; c < nc && st == ORC_OK; ++c) {
    size_t cs = get_u32(sizes + 4 * c);
    if (cs > pb - off || cs > chunk_bound(dt)) { st = ORC_ERR_CORRUPT; break; }
    st = orc_decode_chunk(pay + off, cs, dt, CHUNK_N, vals);
    if (st != ORC_OK) break;
    size_t nv = n - c * CHUNK_N;
    if (nv > CHUNK_N) nv = CHUNK_N;
    for (size_t i = nv; i < CHUNK_N; ++i)
      if (memcmp(vals + i * (size_t)s, vals + (nv - 1) * (size_t)s, (size_t)s) != 0) st = ORC_ERR_CORRUPT;
    if (st != ORC_OK) break;
    size_t rl = 0;
    st = orc_encode_chunk(vals, nv, dt, CHUNK_N, re, &rl);
    if (st != ORC_OK) break;
    if (rl != cs || memcmp(re, pay + off, cs) != 0) st = ORC_ERR_CORRUPT;
    off += cs;
  }
  if (st == ORC_OK && off != pb) st = ORC_ERR_CORRUPT;
  free(vals);
  free(re);
  return st;
}
