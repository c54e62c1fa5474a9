// Internal declarations shared by the host and device translation units of
// libfhesnn.  Not part of the public ABI (include/fhesnn.h is).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "fhesnn.h"

namespace fs {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// ------------------------------------------------------------------ params
bool params_supported(const fs_params& p, std::string* why);
inline uint32_t ilog2(uint32_t v) {
  uint32_t r = 0;
  while ((1u << r) < v) r++;
  return r;
}
inline uint32_t ks_base(const fs_params& p) { return 1u << p.ks_base_bit; }
inline uint32_t delta_of(uint32_t p) { return (uint32_t)(0x100000000ull / p); }

// ------------------------------------------------------------------ host key material
struct Secret {
  fs_params prm;
  std::vector<int32_t> s;  // [n] in {0,1}
  std::vector<int32_t> z;  // [N] in {0,1}
};

struct EvalKey {
  fs_params prm;
  std::vector<uint32_t> bsk;  // [n][2l][2][N] coefficient domain (Torus32)
  std::vector<uint32_t> ksk;  // [N][t][base-1][n+1]
};

// ChaCha20 (RFC 8439 block function) as a counter-addressed generator.
struct ChaChaStream {
  uint32_t key[8];
  uint32_t nonce[3];
  uint32_t block[16];
  uint64_t blk_index = ~0ull;
  ChaChaStream(uint64_t seed, uint32_t domain, uint64_t object);
  uint32_t word(uint64_t w);  // word w of the stream
};
void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3],
                    uint32_t out[16]);
uint32_t torus_gaussian(uint32_t w0, uint32_t w1, double sigma);

enum Domain : uint32_t {
  kDomS = 1, kDomZ = 2, kDomBskA = 3, kDomBskE = 4, kDomKskA = 5, kDomKskE = 6,
  kDomEncA = 7, kDomEncE = 8
};

int keygen(const fs_params& prm, uint64_t seed, Secret** sk, EvalKey** evk);
void encrypt(const Secret& sk, const int32_t* m, size_t count, uint64_t seed, uint64_t first,
             uint32_t* ct, bool under_z = false);
int decrypt(const Secret& sk, const uint32_t* ct, size_t count, uint32_t dim, int32_t* m);
int test_poly(uint32_t N, uint32_t p, const int32_t* f, uint32_t* v);
int test_poly_ms(uint32_t N, uint32_t p_in, uint32_t p_out, const int32_t* f, uint32_t* v);
int test_poly_two(uint32_t N, uint32_t p, const int32_t* f0, const int32_t* f1, uint32_t* v);
void lif_luts(const fs_lif& lif, uint32_t p, int32_t* fire, int32_t* reset);

}  // namespace fs
