/*
 * Plain CPU oracle for TFHE programmable bootstrapping of LIF neurons.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call,
 * link or execute this file; only the tests, the smoke check and the
 * bench's CPU-baseline leg use it.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * Everything is the plain definition, written out with plain loops:
 *   - negacyclic products in Z_{2^32}[X]/(X^N+1) by schoolbook summation
 *     (Sec. 2.1, the ring R_{q,N});
 *   - LWE / RLWE encryption and decryption (Sec. 2.1, LWE and RLWE items);
 *   - RGSW (TGSW) rows and the external product with signed gadget
 *     digits (Sec. 2.1, the RGSW item and its product);
 *   - Initialization, Blind Rotation, Sample Extraction, Key Switching and
 *     their composition into bootstrapping (Sec. 2.1, Theorem 2.1 and the
 *     itemised steps after it);
 *   - WeightSum over ciphertexts (Sec. 4.1, Eq. "noise grows");
 *   - the FHE-Fire / FHE-Reset program functions (Sec. 4.2).
 *
 * Arithmetic: q = 2^32, so every torus value is a uint32_t and wraps.
 * Only k = 1 (one RLWE mask polynomial) is implemented.
 *
 * Readings of points the paper leaves open (the binding list of readings
 * is kept with the design notes):
 *   - encoding Delta*(m mod p) with Delta = 2^32/p (exact, p | 2^32);
 *   - test-polynomial window uses half-window rounding floor((i*p+N)/2N);
 *   - blind rotation is the CGGI CMux form with BSK_i = TGSW_z(s_i),
 *     binary s and z;
 *   - sample extraction uses the negacyclic index reversal;
 *   - key switching is digit decomposition base 2^beta, t digits, with one
 *     fresh encryption per non-zero digit value;
 *   - Reset's fourth branch is forced to the negacyclic image
 *     -leak(r - p/2); the leak factor is (tau-1)/tau rounded half up.
 *
 * Randomness: ChaCha20 (RFC 8439 block function) used as a counter-based
 * generator: key = seed, nonce = (domain, object index), counter = block
 * index of the word.  Gaussian noise by Box-Muller in binary64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439, section 2.3)                     */
/* ------------------------------------------------------------------ */

static uint32_t or_rotl(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

OR_API void or_chacha_quarter(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *d) {
  *a += *b; *d ^= *a; *d = or_rotl(*d, 16);
  *c += *d; *b ^= *c; *b = or_rotl(*b, 12);
  *a += *b; *d ^= *a; *d = or_rotl(*d, 8);
  *c += *d; *b ^= *c; *b = or_rotl(*b, 7);
}

/* state = constants | key[8] | counter | nonce[3]; 20 rounds; add input. */
OR_API void or_chacha20_block(const uint32_t key[8], uint32_t counter,
                              const uint32_t nonce[3], uint32_t out[16]) {
  uint32_t x[16], in[16];
  in[0] = 0x61707865u; in[1] = 0x3320646eu; in[2] = 0x79622d32u; in[3] = 0x6b206574u;
  for (int i = 0; i < 8; i++) in[4 + i] = key[i];
  in[12] = counter;
  in[13] = nonce[0]; in[14] = nonce[1]; in[15] = nonce[2];
  memcpy(x, in, sizeof x);
  for (int r = 0; r < 10; r++) {
    /* column round */
    or_chacha_quarter(&x[0], &x[4], &x[8], &x[12]);
    or_chacha_quarter(&x[1], &x[5], &x[9], &x[13]);
    or_chacha_quarter(&x[2], &x[6], &x[10], &x[14]);
    or_chacha_quarter(&x[3], &x[7], &x[11], &x[15]);
    /* diagonal round */
    or_chacha_quarter(&x[0], &x[5], &x[10], &x[15]);
    or_chacha_quarter(&x[1], &x[6], &x[11], &x[12]);
    or_chacha_quarter(&x[2], &x[7], &x[8], &x[13]);
    or_chacha_quarter(&x[3], &x[4], &x[9], &x[14]);
  }
  for (int i = 0; i < 16; i++) out[i] = x[i] + in[i];
}

/* Word `w` of the stream (seed, domain, obj): key = (seed lo, seed hi, 0..),
 * nonce = (domain, obj lo, obj hi), block counter = w / 16. */
OR_API uint32_t or_stream_word(uint64_t seed, uint32_t domain, uint64_t obj, uint64_t w) {
  uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
  uint32_t nonce[3] = {domain, (uint32_t)obj, (uint32_t)(obj >> 32)};
  uint32_t blk[16];
  or_chacha20_block(key, (uint32_t)(w / 16), nonce, blk);
  return blk[w % 16];
}

/* Fill `count` consecutive words starting at word 0 of a stream. */
static void or_stream_fill(uint64_t seed, uint32_t domain, uint64_t obj,
                           uint32_t *dst, size_t count) {
  uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
  uint32_t nonce[3] = {domain, (uint32_t)obj, (uint32_t)(obj >> 32)};
  uint32_t blk[16];
  for (size_t w = 0; w < count; w++) {
    if (w % 16 == 0) or_chacha20_block(key, (uint32_t)(w / 16), nonce, blk);
    dst[w] = blk[w % 16];
  }
}

/* Stream domains. */
enum { D_S = 1, D_Z = 2, D_BSK_A = 3, D_BSK_E = 4, D_KSK_A = 5, D_KSK_E = 6,
       D_ENC_A = 7, D_ENC_E = 8 };

/* Gaussian torus noise from two stream words (Box-Muller, cosine branch):
 * u = (x+1)/2^32 in (0,1]; g = sqrt(-2 ln u1) cos(2 pi u2);
 * e = round-half-even(sigma * 2^32 * g), reduced mod 2^32. */
OR_API uint32_t or_gauss_from_words(uint32_t x1, uint32_t x2, double sigma) {
  double u1 = ((double)x1 + 1.0) * 0x1p-32;
  double u2 = ((double)x2 + 1.0) * 0x1p-32;
  double r = sqrt(-2.0 * log(u1));
  double g = r * cos(6.283185307179586 * u2);
  double e = nearbyint((sigma * 0x1p32) * g);
  return (uint32_t)(int64_t)e;
}

/* ------------------------------------------------------------------ */
/* Parameters                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
  uint32_t n;           /* LWE dimension                                  */
  uint32_t N;           /* ring degree, power of two                      */
  uint32_t l;           /* gadget levels                                  */
  uint32_t bg_bit;      /* log2 of the gadget base Bg                     */
  uint32_t ks_t;        /* key-switch digits                              */
  uint32_t ks_base_bit; /* log2 of the key-switch base                    */
  uint32_t p;           /* message modulus, power of two                  */
  uint32_t pad;
  double sigma_lwe, sigma_bsk, sigma_ksk;
} or_params;

static uint32_t or_log2(uint32_t v) { uint32_t r = 0; while ((1u << r) < v) r++; return r; }

/* ------------------------------------------------------------------ */
/* Ring R_{q,N} = Z_{2^32}[X]/(X^N+1)  (Sec. 2.1)                       */
/* ------------------------------------------------------------------ */

/* out = a * b in Z_{2^32}[X]/(X^N+1), by schoolbook summation:
 * X^i * X^j = X^{i+j} if i+j < N, else -X^{i+j-N}. */
OR_API void or_negacyclic_mul(uint32_t N, const uint32_t *a, const uint32_t *b, uint32_t *out) {
  for (uint32_t k = 0; k < N; k++) out[k] = 0;
  for (uint32_t i = 0; i < N; i++) {
    uint32_t ai = a[i];
    const uint32_t *bw = b + (N - i);
    for (size_t j = 0; j < N - i; j++) out[i + j] += ai * b[j];
    for (size_t j = 0; j < i; j++) out[j] -= ai * bw[j];
  }
}

/* out += d * b with d a small signed integer polynomial (gadget digits). */
static void or_negacyclic_mac_small(uint32_t N, const int32_t *restrict d,
                                    const uint32_t *restrict b, uint32_t *restrict out) {
  for (uint32_t i = 0; i < N; i++) {
    uint32_t di = (uint32_t)d[i];
    if (di == 0) continue;
    const uint32_t *bw = b + (N - i);  /* terms with i+j >= N wrap with a minus sign */
    for (size_t j = 0; j < N - i; j++) out[i + j] += di * b[j];
    for (size_t j = 0; j < i; j++) out[j] -= di * bw[j];
  }
}

/* out = X^e * a, for e in [0, 2N): coefficient i moves to i+e; passing
 * index N flips the sign (X^N = -1). */
OR_API void or_mul_xpow(uint32_t N, uint32_t e, const uint32_t *a, uint32_t *out) {
  for (uint32_t i = 0; i < N; i++) {
    uint32_t t = i + e; /* < 3N */
    uint32_t v = a[i];
    if (t >= 2 * N) { t -= 2 * N; }
    else if (t >= N) { t -= N; v = 0u - v; }
    out[t] = v;
  }
}

/* ------------------------------------------------------------------ */
/* Keys (Sec. 2.1: LWE secret s, RLWE secret z, evaluation key)         */
/* ------------------------------------------------------------------ */

/* Binary secrets: bit = low bit of the stream word. */
OR_API void or_secret_keys(const or_params *P, uint64_t seed, int32_t *s, int32_t *z) {
  uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (P->N > P->n ? P->N : P->n));
  or_stream_fill(seed, D_S, 0, w, P->n);
  for (uint32_t i = 0; i < P->n; i++) s[i] = (int32_t)(w[i] & 1u);
  or_stream_fill(seed, D_Z, 0, w, P->N);
  for (uint32_t i = 0; i < P->N; i++) z[i] = (int32_t)(w[i] & 1u);
  free(w);
}

/* LWE_key(mu) with explicit mask stream (domain_a, obj) and noise stream
 * (domain_e, obj): a uniform, b = <a,key> + e + mu  (Sec. 2.1, LWE item). */
static void or_lwe_encrypt_raw(uint32_t dim, const int32_t *key, uint32_t mu, double sigma,
                               uint64_t seed, uint32_t dom_a, uint32_t dom_e, uint64_t obj,
                               uint32_t *ct) {
  or_stream_fill(seed, dom_a, obj, ct, dim);
  uint32_t b = 0;
  for (uint32_t i = 0; i < dim; i++) b += ct[i] * (uint32_t)key[i];
  uint32_t e = or_gauss_from_words(or_stream_word(seed, dom_e, obj, 0),
                                   or_stream_word(seed, dom_e, obj, 1), sigma);
  ct[dim] = b + e + mu;
}

/* Bootstrapping key: BSK_i = TGSW_z(s_i), i < n (reading: CGGI form of the
 * Blind Rotation step, with ek_i = RGSW(X^{s_i}) realised as TGSW(s_i)).
 * Layout [n][2l rows][2 polys][N]; row r = c*l + j is TLWE_z(0) =
 * (a_r, a_r*z + e_r), plus s_i * 2^{32-(j+1)bg_bit} added to the constant
 * coefficient of polynomial c (c = 0: mask, c = 1: body). */
OR_API void or_keygen_bsk_range(const or_params *P, uint64_t seed, const int32_t *s,
                                const int32_t *z, uint32_t i0, uint32_t i1, uint32_t *bsk) {
  const uint32_t N = P->N, rows = 2 * P->l;
  uint32_t *zz = (uint32_t *)malloc(sizeof(uint32_t) * N);
  uint32_t *az = (uint32_t *)malloc(sizeof(uint32_t) * N);
  uint32_t *ew = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  for (uint32_t i = 0; i < N; i++) zz[i] = (uint32_t)z[i];
  for (uint32_t i = i0; i < i1 && i < P->n; i++) {
    for (uint32_t r = 0; r < rows; r++) {
      uint64_t obj = (uint64_t)i * rows + r;
      uint32_t *row = bsk + ((size_t)i * rows + r) * 2 * N;
      uint32_t *a = row, *b = row + N;
      or_stream_fill(seed, D_BSK_A, obj, a, N);
      or_negacyclic_mul(N, a, zz, az);
      or_stream_fill(seed, D_BSK_E, obj, ew, 2 * N);
      for (uint32_t m = 0; m < N; m++)
        b[m] = az[m] + or_gauss_from_words(ew[2 * m], ew[2 * m + 1], P->sigma_bsk);
      uint32_t c = r / P->l, j = r % P->l;
      uint32_t g = 1u << (32 - (j + 1) * P->bg_bit);
      row[c * N] += (uint32_t)s[i] * g;
    }
  }
  free(zz); free(az); free(ew);
}

OR_API void or_keygen_bsk(const or_params *P, uint64_t seed, const int32_t *s,
                          const int32_t *z, uint32_t *bsk) {
  or_keygen_bsk_range(P, seed, s, z, 0, P->n, bsk);
}

/* Key-switching key z -> s: KSK[i][j][v-1] = LWE_s(v * z_i * 2^{32-(j+1)beta})
 * for i < N, j < t, v in 1..base-1, each a fresh encryption with sigma_ksk.
 * Layout [N][t][base-1][n+1]. */
OR_API void or_keygen_ksk_range(const or_params *P, uint64_t seed, const int32_t *s,
                                const int32_t *z, uint32_t i0, uint32_t i1, uint32_t *ksk) {
  const uint32_t base = 1u << P->ks_base_bit, dim = P->n;
  for (uint32_t i = i0; i < i1 && i < P->N; i++)
    for (uint32_t j = 0; j < P->ks_t; j++)
      for (uint32_t v = 1; v < base; v++) {
        uint64_t obj = ((uint64_t)i * P->ks_t + j) * (base - 1) + (v - 1);
        uint32_t mu = v * (uint32_t)z[i] * (1u << (32 - (j + 1) * P->ks_base_bit));
        or_lwe_encrypt_raw(dim, s, mu, P->sigma_ksk, seed, D_KSK_A, D_KSK_E, obj,
                           ksk + obj * (dim + 1));
      }
}

OR_API void or_keygen_ksk(const or_params *P, uint64_t seed, const int32_t *s,
                          const int32_t *z, uint32_t *ksk) {
  or_keygen_ksk_range(P, seed, s, z, 0, P->N, ksk);
}

/* ------------------------------------------------------------------ */
/* LWE encryption / decryption of messages in Z_p  (Sec. 2.1)           */
/* ------------------------------------------------------------------ */

/* ct_k = (a, <a,s> + e + Delta*(m_k mod p)), Delta = 2^32/p; the k-th
 * ciphertext draws from stream object first_index + k. */
OR_API void or_encrypt(const or_params *P, const int32_t *s, const int32_t *m, size_t count,
                       uint64_t seed, uint64_t first_index, uint32_t *ct) {
  const uint32_t delta = (uint32_t)(0x100000000ull / P->p);
  for (size_t k = 0; k < count; k++) {
    uint32_t r = (uint32_t)(((int64_t)m[k] % (int64_t)P->p + P->p) % P->p);
    or_lwe_encrypt_raw(P->n, s, r * delta, P->sigma_lwe, seed, D_ENC_A, D_ENC_E,
                       first_index + k, ct + k * (size_t)(P->n + 1));
  }
}

/* Decrypt: phase = b - <a,key>; round to the nearest multiple of Delta;
 * return the centred representative in {-p/2+1, ..., p/2}. */
OR_API void or_decrypt(uint32_t p, const int32_t *key, uint32_t dim, const uint32_t *ct,
                       size_t count, int32_t *m) {
  const uint32_t lp = or_log2(p);
  for (size_t k = 0; k < count; k++) {
    const uint32_t *c = ct + k * (size_t)(dim + 1);
    uint32_t phase = c[dim];
    for (uint32_t i = 0; i < dim; i++) phase -= c[i] * (uint32_t)key[i];
    uint32_t r = (phase + (1u << (31 - lp))) >> (32 - lp);
    m[k] = (r > p / 2) ? (int32_t)r - (int32_t)p : (int32_t)r;
  }
}

/* Raw phase b - <a,key> (for noise measurements). */
OR_API void or_phase(const int32_t *key, uint32_t dim, const uint32_t *ct, size_t count,
                     uint32_t *out) {
  for (size_t k = 0; k < count; k++) {
    const uint32_t *c = ct + k * (size_t)(dim + 1);
    uint32_t phase = c[dim];
    for (uint32_t i = 0; i < dim; i++) phase -= c[i] * (uint32_t)key[i];
    out[k] = phase;
  }
}

/* ------------------------------------------------------------------ */
/* Bootstrapping (Sec. 2.1, Theorem 2.1 and its four steps)            */
/* ------------------------------------------------------------------ */

/* Program function -> test polynomial: v_i = Delta * f(floor((i*p+N)/(2N))
 * mod p), i < N.  f is given by its residues f[0..p-1].  Returns -1 unless
 * f(r + p/2) = -f(r) mod p for every r (the condition of Theorem 2.1). */
OR_API int or_test_poly(uint32_t N, uint32_t p, const int32_t *f, uint32_t *v) {
  for (uint32_t r = 0; r < p; r++) {
    int64_t a = ((int64_t)f[(r + p / 2) % p] % p + p) % p;
    int64_t b = ((-(int64_t)f[r]) % p + p) % p;
    if (a != b) return -1;
  }
  const uint32_t delta = (uint32_t)(0x100000000ull / p);
  for (uint32_t i = 0; i < N; i++) {
    uint64_t idx = ((uint64_t)i * p + N) / (2ull * N);
    int64_t val = ((int64_t)f[idx % p] % p + p) % p;
    v[i] = (uint32_t)val * delta;
  }
  return 0;
}

/* The same with a different output message space (the message-space change
 * of the bootstrapping that Sec. 5.1 borrows from DiNN): inputs encode
 * Z_p_in with Delta_in = 2^32/p_in, f maps Z_p_in to Z_p_out, and
 * v_i = (2^32/p_out) f(floor((i p_in + N)/(2N)) mod p_in).  The rotation
 * by a phase in the upper half negates, so f must satisfy
 * f(r + p_in/2) = -f(r) mod p_out. */
OR_API int or_test_poly_ms(uint32_t N, uint32_t p_in, uint32_t p_out, const int32_t *f,
                           uint32_t *v) {
  const int64_t q = p_out;
  for (uint32_t r = 0; r < p_in; r++) {
    int64_t a = ((int64_t)f[(r + p_in / 2) % p_in] % q + q) % q;
    int64_t b = ((-(int64_t)f[r]) % q + q) % q;
    if (a != b) return -1;
  }
  const uint32_t delta = (uint32_t)(0x100000000ull / p_out);
  for (uint32_t i = 0; i < N; i++) {
    uint64_t idx = ((uint64_t)i * p_in + N) / (2ull * N);
    int64_t val = ((int64_t)f[idx % p_in] % q + q) % q;
    v[i] = (uint32_t)val * delta;
  }
  return 0;
}

/* Switch a torus value to Z_{2N}: round(x * 2N / 2^32), ties up. */
OR_API uint32_t or_mod_switch(uint32_t x, uint32_t N) {
  uint32_t nu = or_log2(2 * N);
  return (uint32_t)(((uint64_t)x + (1ull << (31 - nu))) % 0x100000000ull) >> (32 - nu);
}

/* Signed gadget digits of x: with u = x + sum_{j=1..l} (Bg/2) 2^{32-j*bg}
 * + 2^{31-l*bg}, digit_j = ((u >> (32-(j+1)bg)) & (Bg-1)) - Bg/2, j < l,
 * so that sum_j digit_j 2^{32-(j+1)bg} rounds x to l*bg bits. */
OR_API void or_gadget_digits(uint32_t x, uint32_t l, uint32_t bg_bit, int32_t *dig) {
  uint32_t half = 1u << (bg_bit - 1), mask = (1u << bg_bit) - 1;
  uint32_t off = 1u << (31 - l * bg_bit);
  for (uint32_t j = 1; j <= l; j++) off += half << (32 - j * bg_bit);
  uint32_t u = x + off;
  for (uint32_t j = 0; j < l; j++)
    dig[j] = (int32_t)((u >> (32 - (j + 1) * bg_bit)) & mask) - (int32_t)half;
}

/* External product TGSW_z(mu) [x] (c0, c1): decompose both polynomials of
 * the RLWE input into l signed digit polynomials each and sum the digit
 * polynomials times the matching TGSW rows (Sec. 2.1, RGSW item). */
static void or_external_product(const or_params *P, const uint32_t *tgsw, const uint32_t *in,
                                uint32_t *out, int32_t *digbuf) {
  const uint32_t N = P->N, l = P->l;
  memset(out, 0, sizeof(uint32_t) * 2 * N);
  int32_t dig[16];
  for (uint32_t c = 0; c < 2; c++) {
    /* digbuf[j*N + m] = digit j of coefficient m of polynomial c */
    for (uint32_t m = 0; m < N; m++) {
      or_gadget_digits(in[c * N + m], l, P->bg_bit, dig);
      for (uint32_t j = 0; j < l; j++) digbuf[j * N + m] = dig[j];
    }
    for (uint32_t j = 0; j < l; j++) {
      const uint32_t *row = tgsw + (size_t)(c * l + j) * 2 * N;
      or_negacyclic_mac_small(N, digbuf + j * N, row, out);         /* mask */
      or_negacyclic_mac_small(N, digbuf + j * N, row + N, out + N); /* body */
    }
  }
}

/* Initialization and Blind Rotation.
 * ACC = (0, X^{-b~} v), then for i = 0..n-1:
 *   ACC <- ACC + BSK_i [x] (X^{a~_i} ACC - ACC)      (CMux)
 * with a~, b~ the inputs switched to Z_{2N}.  acc has layout [2][N]. */
/* Switch to the even exponents of Z_{2N}: 2 round(x * N / 2^32), ties up
 * (the phase rounded to Z_N, for test polynomials that interleave two
 * program functions). */
OR_API uint32_t or_mod_switch_even(uint32_t x, uint32_t N) {
  uint32_t nu = or_log2(N);
  uint32_t r = (uint32_t)(((uint64_t)x + (1ull << (31 - nu))) % 0x100000000ull) >> (32 - nu);
  return (2 * r) % (2 * N);
}

/* Blind rotation with the exponents from or_mod_switch (even = 0) or
 * or_mod_switch_even (even = 1). */
OR_API void or_blind_rotate_ms(const or_params *P, const uint32_t *bsk, const uint32_t *v,
                               const uint32_t *ct, int even, uint32_t *acc) {
  const uint32_t N = P->N, n = P->n, rows = 2 * P->l;
  uint32_t *rot = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t *diff = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t *prod = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  int32_t *digbuf = (int32_t *)malloc(sizeof(int32_t) * P->l * N);

  uint32_t bbar = even ? or_mod_switch_even(ct[n], N) : or_mod_switch(ct[n], N);
  memset(acc, 0, sizeof(uint32_t) * N);
  or_mul_xpow(N, (2 * N - bbar) % (2 * N), v, acc + N);

  for (uint32_t i = 0; i < n; i++) {
    uint32_t abar = even ? or_mod_switch_even(ct[i], N) : or_mod_switch(ct[i], N);
    if (abar == 0) continue; /* X^0 ACC - ACC = 0: every digit is 0 */
    for (uint32_t c = 0; c < 2; c++) {
      or_mul_xpow(N, abar, acc + c * N, rot + c * N);
      for (uint32_t m = 0; m < N; m++) diff[c * N + m] = rot[c * N + m] - acc[c * N + m];
    }
    or_external_product(P, bsk + (size_t)i * rows * 2 * N, diff, prod, digbuf);
    for (uint32_t m = 0; m < 2 * N; m++) acc[m] += prod[m];
  }
  free(rot); free(diff); free(prod); free(digbuf);
}

OR_API void or_blind_rotate(const or_params *P, const uint32_t *bsk, const uint32_t *v,
                            const uint32_t *ct, uint32_t *acc) {
  or_blind_rotate_ms(P, bsk, v, ct, 0, acc);
}

/* Sample Extraction of coefficient 0: LWE_z = (a', b0) with a'_0 = a_0 and
 * a'_j = -a_{N-j} (the negacyclic reversal), so that b0 - <a', z> equals the
 * constant coefficient of the RLWE phase b(X) - a(X) z(X). */
OR_API void or_sample_extract(uint32_t N, const uint32_t *acc, uint32_t *out) {
  out[0] = acc[0];
  for (uint32_t j = 1; j < N; j++) out[j] = 0u - acc[N - j];
  out[N] = acc[N];
}

/* Sample Extraction of coefficient k: coefficient k of a(X) z(X) is
 * sum_{j<=k} a_{k-j} z_j - sum_{j>k} a_{N+k-j} z_j, so a'_j = a_{k-j} for
 * j <= k, a'_j = -a_{N+k-j} for j > k, and b' = b_k. */
OR_API void or_sample_extract_at(uint32_t N, const uint32_t *acc, uint32_t k, uint32_t *out) {
  for (uint32_t j = 0; j < N; j++) out[j] = j <= k ? acc[k - j] : 0u - acc[N + k - j];
  out[N] = acc[N + k];
}

/* Test polynomial holding two program functions (f0, f1: Z_p -> Z_p)
 * interleaved: with the phase on even exponents 2u of Z_{2N}, coefficient
 * 2u carries f0 and 2u+1 carries f1 of the message round(u p / N) (ties
 * up): v_{2u+r} = Delta f_r(floor((u p + N/2) / N) mod p), u < N/2.
 * Both functions must be negacyclic (Theorem 2.1's condition). */
OR_API int or_test_poly_two(uint32_t N, uint32_t p, const int32_t *f0, const int32_t *f1,
                            uint32_t *v) {
  const int32_t *f[2] = {f0, f1};
  for (int r = 0; r < 2; r++)
    for (uint32_t m = 0; m < p; m++) {
      int64_t a = ((int64_t)f[r][(m + p / 2) % p] % p + p) % p;
      int64_t b = ((-(int64_t)f[r][m]) % p + p) % p;
      if (a != b) return -1;
    }
  const uint32_t delta = (uint32_t)(0x100000000ull / p);
  for (uint32_t u = 0; u < N / 2; u++) {
    uint64_t idx = ((uint64_t)u * p + N / 2) / N;
    for (int r = 0; r < 2; r++) {
      int64_t val = ((int64_t)f[r][idx % p] % p + p) % p;
      v[2 * u + r] = (uint32_t)val * delta;
    }
  }
  return 0;
}

/* Key Switching z -> s: round each a'_i to t*beta bits, split into t
 * base-2^beta digits (most significant first) and subtract the KSK row of
 * each non-zero digit from (0, ..., 0, b'). */
OR_API void or_keyswitch(const or_params *P, const uint32_t *ksk, const uint32_t *in,
                         uint32_t *out) {
  const uint32_t n = P->n, N = P->N, t = P->ks_t, beta = P->ks_base_bit;
  const uint32_t base = 1u << beta, prec = t * beta;
  memset(out, 0, sizeof(uint32_t) * (n + 1));
  out[n] = in[N];
  for (uint32_t i = 0; i < N; i++) {
    uint32_t abar = (uint32_t)(((uint64_t)in[i] + (1ull << (31 - prec))) % 0x100000000ull) >> (32 - prec);
    for (uint32_t j = 0; j < t; j++) {
      uint32_t d = (abar >> ((t - 1 - j) * beta)) & (base - 1);
      if (d == 0) continue;
      const uint32_t *row = ksk + (((size_t)i * t + j) * (base - 1) + (d - 1)) * (n + 1);
      for (uint32_t w = 0; w <= n; w++) out[w] -= row[w];
    }
  }
}

/* Two bootstrappings from one blind rotation: the even-exponent rotation of
 * a test polynomial from or_test_poly_two, then extraction of coefficients
 * 0 (f0) and 1 (f1), each key-switched when keyswitch != 0. */
OR_API void or_pbs_two(const or_params *P, const uint32_t *bsk, const uint32_t *ksk,
                       const uint32_t *v, const uint32_t *ct, int keyswitch, uint32_t *out0,
                       uint32_t *out1) {
  const uint32_t N = P->N;
  uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
  uint32_t *outs[2] = {out0, out1};
  or_blind_rotate_ms(P, bsk, v, ct, 1, acc);
  for (uint32_t k = 0; k < 2; k++) {
    or_sample_extract_at(N, acc, k, ext);
    if (keyswitch) or_keyswitch(P, ksk, ext, outs[k]);
    else memcpy(outs[k], ext, sizeof(uint32_t) * (N + 1));
  }
  free(acc); free(ext);
}

/* bootstrapping = KeySwitch o Extract o BlindRotate o Initialize.
 * keyswitch = 0 returns the extracted LWE_z (N+1 words) instead. */
OR_API void or_pbs(const or_params *P, const uint32_t *bsk, const uint32_t *ksk,
                   const uint32_t *v, const uint32_t *ct, int keyswitch, uint32_t *out) {
  const uint32_t N = P->N;
  uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
  or_blind_rotate(P, bsk, v, ct, acc);
  or_sample_extract(N, acc, ext);
  if (keyswitch) or_keyswitch(P, ksk, ext, out);
  else memcpy(out, ext, sizeof(uint32_t) * (N + 1));
  free(acc); free(ext);
}

/* ------------------------------------------------------------------ */
/* WeightSum over ciphertexts (Sec. 4.1)                               */
/* ------------------------------------------------------------------ */

/* y[o] = add[o] + sum_i W[o][i] * x[i], word by word mod 2^32 (W is a
 * plaintext integer; add may be NULL). */
OR_API void or_lwe_linear(uint32_t dim1, const int32_t *W, size_t O, size_t I,
                          const uint32_t *x, const uint32_t *add, uint32_t *y) {
  for (size_t o = 0; o < O; o++)
    for (uint32_t w = 0; w < dim1; w++) {
      uint32_t acc = add ? add[o * dim1 + w] : 0u;
      for (size_t i = 0; i < I; i++) acc += (uint32_t)W[o * I + i] * x[i * dim1 + w];
      y[o * dim1 + w] = acc;
    }
}

/* 2-D convolution of ciphertext feature maps: x is [Ci][H][Wd] ciphertexts,
 * W is [Co][Ci][K][K]; output [Co][Ho][Wo] with Ho = (H+2pad-K)/stride+1;
 * taps outside the input contribute nothing (zero padding). */
OR_API void or_lwe_conv2d(uint32_t dim1, const int32_t *W, uint32_t Ci, uint32_t H, uint32_t Wd,
                          uint32_t Co, uint32_t K, uint32_t stride, uint32_t pad,
                          const uint32_t *x, const uint32_t *add, uint32_t *y) {
  const uint32_t Ho = (H + 2 * pad - K) / stride + 1, Wo = (Wd + 2 * pad - K) / stride + 1;
  for (uint32_t co = 0; co < Co; co++)
    for (uint32_t oy = 0; oy < Ho; oy++)
      for (uint32_t ox = 0; ox < Wo; ox++) {
        size_t o = ((size_t)co * Ho + oy) * Wo + ox;
        for (uint32_t w = 0; w < dim1; w++) {
          uint32_t acc = add ? add[o * dim1 + w] : 0u;
          for (uint32_t ci = 0; ci < Ci; ci++)
            for (uint32_t ky = 0; ky < K; ky++)
              for (uint32_t kx = 0; kx < K; kx++) {
                int64_t iy = (int64_t)oy * stride + ky - pad;
                int64_t ix = (int64_t)ox * stride + kx - pad;
                if (iy < 0 || iy >= H || ix < 0 || ix >= Wd) continue;
                uint32_t wt = (uint32_t)W[((co * Ci + ci) * K + ky) * K + kx];
                acc += wt * x[(((size_t)ci * H + iy) * Wd + ix) * dim1 + w];
              }
          y[o * dim1 + w] = acc;
        }
      }
}

/* Add Delta*c to the body of each ciphertext (trivial plaintext add). */
OR_API void or_add_plain(uint32_t p, uint32_t dim, uint32_t *ct, size_t count, int32_t c) {
  const uint32_t delta = (uint32_t)(0x100000000ull / p);
  uint32_t r = (uint32_t)(((int64_t)c % p + p) % p);
  for (size_t k = 0; k < count; k++) ct[k * (size_t)(dim + 1) + dim] += r * delta;
}

/* ------------------------------------------------------------------ */
/* LIF program functions (Sec. 4.2, FHE-Fire and FHE-Reset)            */
/* ------------------------------------------------------------------ */

/* Fire with the threshold V folded in: +1 when (r - V) mod p lies in
 * [0, p/2), else -1; r is a residue in [0, p). */
OR_API void or_lut_fire(uint32_t p, int32_t V, int32_t *f) {
  for (uint32_t r = 0; r < p; r++) {
    int64_t d = (((int64_t)r - V) % p + p) % p;
    f[r] = d < (int64_t)(p / 2) ? 1 : -1;
  }
}

/* leak(h) = (tau-1)/tau * h rounded half up; tau = 0 encodes IF (no leak). */
OR_API int32_t or_leak(int32_t h, uint32_t tau) {
  if (tau == 0) return h;
  int64_t num = 2 * (int64_t)(tau - 1) * h + tau, den = 2 * (int64_t)tau;
  int64_t q = num / den;
  if ((num % den != 0) && ((num < 0) != (den < 0))) q -= 1; /* floor */
  return (int32_t)q;
}

/* Reset: leak(r) on [0, V); 0 on [V, p/2); -leak(r - p/2) on
 * [p/2, p/2 + V); 0 on [p/2 + V, p). */
OR_API void or_lut_reset(uint32_t p, int32_t V, uint32_t tau, int32_t *f) {
  for (uint32_t r = 0; r < p; r++) {
    int32_t h = (int32_t)r;
    if (h < V) f[r] = or_leak(h, tau);
    else if (h < (int32_t)(p / 2)) f[r] = 0;
    else if (h < (int32_t)(p / 2) + V) f[r] = -or_leak(h - (int32_t)(p / 2), tau);
    else f[r] = 0;
  }
}
