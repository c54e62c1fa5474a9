// Client side of the engine: parameter sets, the ChaCha20 counter stream,
// noise sampling, key generation, LWE encryption and decryption, and the
// program-function tables.  Plain host C++ (compiled into libfhesnn).
//
// Sec. 2.1 (LWE, RLWE, RGSW items; the bootstrapping key
// ek = (RGSW(X^{s_1}), ..., RGSW(X^{s_n})) of the Blind Rotation step, here
// in its TGSW_z(s_i) form, and the key-switching key of the Key Switching
// step); Sec. 4.2 (FHE-Fire, FHE-Reset program functions).
#include <cmath>
#include <cstring>
#include <thread>

#include "fs_internal.h"

namespace fs {

// ------------------------------------------------------------------ params

bool params_supported(const fs_params& p, std::string* why) {
  auto no = [&](const char* m) { if (why) *why = m; return false; };
  if (p.version != FS_PARAMS_VERSION) return no("fs_params.version mismatch");
  if (p.k != 1) return no("only k = 1 is implemented");
  if (p.n == 0 || p.n > 4096) return no("n must be in 1..4096");
  if (p.p < 2 || (p.p & (p.p - 1)) != 0 || p.p > 2 * p.N) return no("p must be a power of two <= 2N");
  if (p.ks_base_bit == 0 || p.ks_t == 0 || p.ks_t * p.ks_base_bit > 31) return no("bad key-switch digits");
  bool shape_a = p.N == 1024 && p.l == 3 && p.bg_bit == 7;
  bool shape_b = p.N == 2048 && p.l == 2 && p.bg_bit == 10;
  if (!shape_a && !shape_b) return no("kernels exist for (N,l,bg_bit) = (1024,3,7) and (2048,2,10)");
  return true;
}

// ------------------------------------------------------------------ ChaCha20 (RFC 8439 Sec. 2.3)

static inline uint32_t rotl32(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

#define FS_QR(a, b, c, d)                 \
  a += b; d ^= a; d = rotl32(d, 16);      \
  c += d; b ^= c; b = rotl32(b, 12);      \
  a += b; d ^= a; d = rotl32(d, 8);       \
  c += d; b ^= c; b = rotl32(b, 7);

void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3],
                    uint32_t out[16]) {
  const uint32_t init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                             key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                             counter, nonce[0], nonce[1], nonce[2]};
  uint32_t s0 = init[0], s1 = init[1], s2 = init[2], s3 = init[3], s4 = init[4], s5 = init[5],
           s6 = init[6], s7 = init[7], s8 = init[8], s9 = init[9], s10 = init[10],
           s11 = init[11], s12 = init[12], s13 = init[13], s14 = init[14], s15 = init[15];
  for (int dr = 0; dr < 10; ++dr) {
    FS_QR(s0, s4, s8, s12) FS_QR(s1, s5, s9, s13) FS_QR(s2, s6, s10, s14) FS_QR(s3, s7, s11, s15)
    FS_QR(s0, s5, s10, s15) FS_QR(s1, s6, s11, s12) FS_QR(s2, s7, s8, s13) FS_QR(s3, s4, s9, s14)
  }
  const uint32_t fin[16] = {s0, s1, s2, s3, s4, s5, s6, s7, s8, s9, s10, s11, s12, s13, s14, s15};
  for (int i = 0; i < 16; ++i) out[i] = fin[i] + init[i];
}
#undef FS_QR

ChaChaStream::ChaChaStream(uint64_t seed, uint32_t domain, uint64_t object) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  for (int i = 2; i < 8; ++i) key[i] = 0;
  nonce[0] = domain;
  nonce[1] = (uint32_t)object;
  nonce[2] = (uint32_t)(object >> 32);
}

uint32_t ChaChaStream::word(uint64_t w) {
  uint64_t b = w >> 4;
  if (b != blk_index) {
    chacha20_block(key, (uint32_t)b, nonce, block);
    blk_index = b;
  }
  return block[w & 15];
}

// Box-Muller (cosine branch) on u = (w + 1) 2^-32 in (0, 1]; the torus
// noise is round-half-even(sigma 2^32 g) mod 2^32.
uint32_t torus_gaussian(uint32_t w0, uint32_t w1, double sigma) {
  const double u1 = ((double)w0 + 1.0) * 0x1p-32;
  const double u2 = ((double)w1 + 1.0) * 0x1p-32;
  const double radius = std::sqrt(-2.0 * std::log(u1));
  const double g = radius * std::cos(6.283185307179586 * u2);
  const double scaled = std::nearbyint((sigma * 0x1p32) * g);
  return (uint32_t)(int64_t)scaled;
}

// ------------------------------------------------------------------ keys

namespace {

// TLWE_z(0) body: b(X) = a(X) z(X) + e(X).  z is binary, so the product is
// the signed sum of the rotations X^k a(X) over the k with z_k = 1.
void rlwe_zero_body(uint32_t N, const uint32_t* a, const std::vector<uint32_t>& zidx,
                    uint32_t* b) {
  for (uint32_t m = 0; m < N; ++m) b[m] = 0;
  for (uint32_t k : zidx) {
    // X^k a: coefficient i goes to i + k, negated once it passes N
    for (uint32_t i = 0; i + k < N; ++i) b[i + k] += a[i];
    for (uint32_t i = N - k; i < N; ++i) b[i + k - N] -= a[i];
  }
}

template <class F>
void parallel_for(uint32_t count, F&& f) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 16) nt = 16;
  if (nt > count) nt = count ? count : 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (uint32_t i = t; i < count; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

int keygen(const fs_params& prm, uint64_t seed, Secret** sk_out, EvalKey** evk_out) {
  const uint32_t n = prm.n, N = prm.N, l = prm.l, rows = 2 * l;
  auto* sk = new Secret{prm, std::vector<int32_t>(n), std::vector<int32_t>(N)};
  {
    ChaChaStream cs(seed, kDomS, 0);
    for (uint32_t i = 0; i < n; ++i) sk->s[i] = (int32_t)(cs.word(i) & 1u);
    ChaChaStream cz(seed, kDomZ, 0);
    for (uint32_t i = 0; i < N; ++i) sk->z[i] = (int32_t)(cz.word(i) & 1u);
  }
  std::vector<uint32_t> zidx;
  for (uint32_t i = 0; i < N; ++i)
    if (sk->z[i]) zidx.push_back(i);

  auto* evk = new EvalKey{prm, {}, {}};
  evk->bsk.assign((size_t)n * rows * 2 * N, 0u);
  // BSK_i = TGSW_z(s_i): row r = c*l + j is TLWE_z(0) plus s_i * g_j on
  // the constant coefficient of polynomial c, g_j = 2^{32-(j+1) bg_bit}.
  parallel_for(n, [&](uint32_t i) {
    std::vector<uint32_t> body(N);
    for (uint32_t r = 0; r < rows; ++r) {
      const uint64_t obj = (uint64_t)i * rows + r;
      uint32_t* row = evk->bsk.data() + ((size_t)i * rows + r) * 2 * N;
      ChaChaStream ca(seed, kDomBskA, obj);
      for (uint32_t m = 0; m < N; ++m) row[m] = ca.word(m);
      rlwe_zero_body(N, row, zidx, body.data());
      ChaChaStream ce(seed, kDomBskE, obj);
      for (uint32_t m = 0; m < N; ++m)
        row[N + m] = body[m] + torus_gaussian(ce.word(2 * m), ce.word(2 * m + 1), prm.sigma_bsk);
      const uint32_t c = r / l, j = r % l;
      row[c * N] += (uint32_t)sk->s[i] << (32 - (j + 1) * prm.bg_bit);
    }
  });
  // KSK[i][j][v-1] = LWE_s(v z_i 2^{32-(j+1) beta}), a fresh sample each.
  const uint32_t base = ks_base(prm), t = prm.ks_t, w = n + 1;
  evk->ksk.assign((size_t)N * t * (base - 1) * w, 0u);
  parallel_for(N, [&](uint32_t i) {
    for (uint32_t j = 0; j < t; ++j)
      for (uint32_t v = 1; v < base; ++v) {
        const uint64_t obj = ((uint64_t)i * t + j) * (base - 1) + (v - 1);
        uint32_t* ct = evk->ksk.data() + obj * w;
        ChaChaStream ca(seed, kDomKskA, obj);
        uint32_t dot = 0;
        for (uint32_t k = 0; k < n; ++k) {
          ct[k] = ca.word(k);
          dot += ct[k] * (uint32_t)sk->s[k];
        }
        ChaChaStream ce(seed, kDomKskE, obj);
        const uint32_t e = torus_gaussian(ce.word(0), ce.word(1), prm.sigma_ksk);
        const uint32_t mu = (v * (uint32_t)sk->z[i]) << (32 - (j + 1) * prm.ks_base_bit);
        ct[n] = dot + e + mu;
      }
  });
  *sk_out = sk;
  *evk_out = evk;
  return FS_OK;
}

void encrypt(const Secret& sk, const int32_t* m, size_t count, uint64_t seed, uint64_t first,
             uint32_t* ct, bool under_z) {
  const uint32_t n = under_z ? sk.prm.N : sk.prm.n, p = sk.prm.p, delta = delta_of(p);
  const int32_t* key = under_z ? sk.z.data() : sk.s.data();
  for (size_t k = 0; k < count; ++k) {
    uint32_t* c = ct + k * (size_t)(n + 1);
    ChaChaStream ca(seed, kDomEncA, first + k);
    uint32_t dot = 0;
    for (uint32_t i = 0; i < n; ++i) {
      c[i] = ca.word(i);
      dot += c[i] * (uint32_t)key[i];
    }
    ChaChaStream ce(seed, kDomEncE, first + k);
    const uint32_t e = torus_gaussian(ce.word(0), ce.word(1), sk.prm.sigma_lwe);
    const uint32_t res = (uint32_t)m[k] & (p - 1);  // m mod p (p a power of two)
    c[n] = dot + e + res * delta;
  }
}

int decrypt(const Secret& sk, const uint32_t* ct, size_t count, uint32_t dim, int32_t* m) {
  const uint32_t n = sk.prm.n, N = sk.prm.N, p = sk.prm.p;
  const int32_t* key;
  uint32_t d;
  if (dim == n + 1) { key = sk.s.data(); d = n; }
  else if (dim == N + 1) { key = sk.z.data(); d = N; }
  else return fail(FS_EINVAL, "fs_decrypt: dim must be n+1 or N+1");
  const uint32_t lp = ilog2(p);
  for (size_t k = 0; k < count; ++k) {
    const uint32_t* c = ct + k * (size_t)dim;
    uint32_t ph = c[d];
    for (uint32_t i = 0; i < d; ++i) ph -= c[i] * (uint32_t)key[i];
    const uint32_t r = (ph + (1u << (31 - lp))) >> (32 - lp);
    m[k] = r > p / 2 ? (int32_t)r - (int32_t)p : (int32_t)r;
  }
  return FS_OK;
}

// ------------------------------------------------------------------ program functions

int test_poly(uint32_t N, uint32_t p, const int32_t* f, uint32_t* v) {
  return test_poly_ms(N, p, p, f, v);
}

// Input messages in Z_p_in (phase window of coefficient i: message
// floor((i p_in + N) / 2N), i.e. i p_in / 2N rounded half up), outputs in
// Z_p_out with Delta_out = 2^32 / p_out.  A phase in the upper half of the
// torus rotates the polynomial past X^N = -1, hence the negacyclic
// condition f(r + p_in/2) = -f(r) mod p_out.
int test_poly_ms(uint32_t N, uint32_t p_in, uint32_t p_out, const int32_t* f, uint32_t* v) {
  const uint32_t in_mask = p_in - 1, out_mask = p_out - 1;
  for (uint32_t r = 0; r < p_in; ++r)
    if ((((uint32_t)f[(r + p_in / 2) & in_mask] + (uint32_t)f[r]) & out_mask) != 0)
      return fail(FS_EINVAL, "program function violates f(r + p/2) = -f(r) (Theorem 2.1)");
  const uint32_t delta = delta_of(p_out);
  for (uint32_t i = 0; i < N; ++i) {
    const uint32_t msg = (uint32_t)(((uint64_t)i * p_in + N) / (2ull * N)) & in_mask;
    v[i] = ((uint32_t)f[msg] & out_mask) * delta;
  }
  return FS_OK;
}

// Two functions in one test polynomial, for a rotation by even exponents
// only: coefficient 2u carries f0 and 2u + 1 carries f1 of the message at
// phase 2u / 2N, round(u p / N) with ties up.
int test_poly_two(uint32_t N, uint32_t p, const int32_t* f0, const int32_t* f1, uint32_t* v) {
  const uint32_t mask = p - 1;
  const int32_t* f[2] = {f0, f1};
  for (int k = 0; k < 2; ++k)
    for (uint32_t r = 0; r < p; ++r)
      if ((((uint32_t)f[k][(r + p / 2) & mask] + (uint32_t)f[k][r]) & mask) != 0)
        return fail(FS_EINVAL, "program function violates f(r + p/2) = -f(r) (Theorem 2.1)");
  const uint32_t delta = delta_of(p);
  for (uint32_t u = 0; u < N / 2; ++u) {
    const uint32_t msg = (uint32_t)(((uint64_t)u * p + N / 2) / N) & mask;
    v[2 * u] = ((uint32_t)f0[msg] & mask) * delta;
    v[2 * u + 1] = ((uint32_t)f1[msg] & mask) * delta;
  }
  return FS_OK;
}

static int32_t leak_of(int32_t h, uint32_t tau) {
  if (tau == 0) return h;  // IF: no leak
  // (tau-1)/tau * h rounded half up = floor((2 (tau-1) h + tau) / (2 tau)), h >= 0
  const int64_t num = 2 * (int64_t)(tau - 1) * h + (int64_t)tau;
  const int64_t den = 2 * (int64_t)tau;
  int64_t q = num / den;
  if (num % den != 0 && num < 0) q -= 1;
  return (int32_t)q;
}

void lif_luts(const fs_lif& lif, uint32_t p, int32_t* fire, int32_t* reset) {
  const int32_t half = (int32_t)(p / 2), V = lif.v_th;
  for (int32_t r = 0; r < (int32_t)p; ++r) {
    if (fire) {
      const int32_t d = (int32_t)(((uint32_t)(r - V)) & (p - 1));
      fire[r] = d < half ? 1 : -1;
    }
    if (reset) {
      int32_t out;
      if (r < V) out = leak_of(r, lif.tau);
      else if (r < half) out = 0;
      else if (r < half + V) out = -leak_of(r - half, lif.tau);
      else out = 0;
      reset[r] = out;
    }
  }
}

}  // namespace fs
