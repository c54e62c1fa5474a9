// Host-side client code of libfhesnn (key generation, encryption, decryption,
// program-function tables) exercised under AddressSanitizer and
// UndefinedBehaviorSanitizer; built and run by tests/test_host_sanitizers.py
// with g++ (no GPU code involved).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "fs_internal.h"

namespace fs {
// the error channel lives in the C ABI file, which this sanitizer compilation leaves out
static std::string g_last;
void set_error(const std::string& msg) { g_last = msg; }
int fail(int code, const std::string& msg) {
  g_last = msg;
  return code;
}
}  // namespace fs

static fs_params shape(int b) {
  fs_params p{};
  p.version = FS_PARAMS_VERSION;
  p.n = 630; p.k = 1; p.ks_t = 8; p.ks_base_bit = 2;
  p.sigma_lwe = p.sigma_ksk = 0x1p-15;
  if (b == 0) { p.N = 1024; p.l = 3; p.bg_bit = 7; p.p = 32; p.sigma_bsk = 0x1p-25; }
  else { p.N = 2048; p.l = 2; p.bg_bit = 10; p.p = 64; p.sigma_bsk = 0x1p-31; }
  return p;
}

#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main() {
  for (int b = 0; b < 2; ++b) {
    const fs_params P = shape(b);
    fs::Secret* sk = nullptr;
    fs::EvalKey* evk = nullptr;
    CHECK(fs::keygen(P, 7, &sk, &evk) == FS_OK);
    CHECK(evk->bsk.size() == (size_t)P.n * 2 * P.l * 2 * P.N);
    CHECK(evk->ksk.size() == (size_t)P.N * P.ks_t * 3 * (P.n + 1));
    // every message, encrypted and decrypted, including the centred range ends
    std::vector<int32_t> m(P.p), back(P.p);
    for (uint32_t i = 0; i < P.p; ++i) m[i] = (int32_t)i - (int32_t)P.p / 2 + 1;
    std::vector<uint32_t> ct((size_t)P.p * (P.n + 1));
    fs::encrypt(*sk, m.data(), m.size(), 3, 100, ct.data());
    CHECK(fs::decrypt(*sk, ct.data(), m.size(), P.n + 1, back.data()) == FS_OK);
    CHECK(back == m);
    // program functions: LIF tables (LIF and IF) and their test polynomials
    for (uint32_t tau : {0u, 2u, 3u}) {
      fs_lif lif{4, tau};
      std::vector<int32_t> fire(P.p), reset(P.p);
      fs::lif_luts(lif, P.p, fire.data(), reset.data());
      std::vector<uint32_t> v(P.N);
      CHECK(fs::test_poly(P.N, P.p, fire.data(), v.data()) == FS_OK);
      CHECK(fs::test_poly(P.N, P.p, reset.data(), v.data()) == FS_OK);
    }
    // a table that is not negacyclic is rejected, not read out of range
    std::vector<int32_t> bad(P.p, 1);
    std::vector<uint32_t> v(P.N);
    CHECK(fs::test_poly(P.N, P.p, bad.data(), v.data()) != FS_OK);
    // wrong ciphertext width is an error
    CHECK(fs::decrypt(*sk, ct.data(), 1, 7, back.data()) != FS_OK);
    delete sk;
    delete evk;
  }
  // unsupported parameters are refused with a reason
  fs_params q = shape(0);
  q.N = 512;
  std::string why;
  CHECK(!fs::params_supported(q, &why) && !why.empty());
  std::puts("host sanitizer run: ok");
  return 0;
}
