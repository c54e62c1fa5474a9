/* A C99 client of the library that uses nothing but include/fhesnn.h and the
 * HIP runtime: key generation, encryption, key upload, one LIF activation
 * (fs_pbs_lif) on device buffers, decryption, and the error path.  It
 * checks every decrypted output against the LIF program functions of its
 * message and prints "c-abi: ok" on success (exit status 0). */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fhesnn.h"

#define COUNT 32

static int check(int rc, const char* what) {
  if (rc != FS_OK) fprintf(stderr, "c-abi: %s failed (%d): %s\n", what, rc, fs_last_error());
  return rc != FS_OK;
}

int main(void) {
  fs_params prm;
  fs_secret* sk = NULL;
  fs_evk* evk = NULL;
  fs_ctx* ctx = NULL;
  fs_devkey* dk = NULL;
  if (check(fs_params_default(0, &prm), "fs_params_default")) return 1;
  if (check(fs_keygen(&prm, 1, &sk, &evk), "fs_keygen")) return 1;

  const size_t w = prm.n + 1;
  int32_t m[COUNT], s2[COUNT], v[COUNT], fire[64], reset[64];
  for (int i = 0; i < COUNT; ++i) m[i] = i - (int)prm.p / 2 + 1; /* every message of Z_32 */
  uint32_t* ct = (uint32_t*)malloc(COUNT * w * sizeof(uint32_t));
  uint32_t* out = (uint32_t*)malloc(2 * COUNT * w * sizeof(uint32_t));
  if (!ct || !out) return 1;
  if (check(fs_encrypt(sk, m, COUNT, 2, 0, ct), "fs_encrypt")) return 1;

  if (check(fs_ctx_create(0, &ctx), "fs_ctx_create")) return 1;
  if (check(fs_evk_upload(ctx, evk, &dk), "fs_evk_upload")) return 1;
  void *d_h = NULL, *d_s = NULL, *d_v = NULL;
  const size_t bytes = COUNT * w * sizeof(uint32_t);
  if (hipMalloc(&d_h, bytes) != hipSuccess || hipMalloc(&d_s, bytes) != hipSuccess ||
      hipMalloc(&d_v, bytes) != hipSuccess)
    return 1;
  if (hipMemcpy(d_h, ct, bytes, hipMemcpyHostToDevice) != hipSuccess) return 1;

  const fs_lif lif = {4, 2};
  if (check(fs_pbs_lif(ctx, dk, &lif, (const uint32_t*)d_h, COUNT, (uint32_t*)d_s,
                       (uint32_t*)d_v, NULL),
            "fs_pbs_lif"))
    return 1;
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  if (hipMemcpy(out, d_s, bytes, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(out + COUNT * w, d_v, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return 1;
  if (check(fs_decrypt(sk, out, COUNT, (uint32_t)w, s2), "fs_decrypt") ||
      check(fs_decrypt(sk, out + COUNT * w, COUNT, (uint32_t)w, v), "fs_decrypt") ||
      check(fs_lif_luts(&lif, prm.p, fire, reset), "fs_lif_luts"))
    return 1;
  int bad = 0;
  for (int i = 0; i < COUNT; ++i) {
    const int r = ((m[i] % (int)prm.p) + (int)prm.p) % (int)prm.p;
    int want_s = (fire[r] + 1) % (int)prm.p, want_v = ((reset[r] % (int)prm.p) + (int)prm.p) % (int)prm.p;
    if (want_s > (int)prm.p / 2) want_s -= (int)prm.p;
    if (want_v > (int)prm.p / 2) want_v -= (int)prm.p;
    if (s2[i] != want_s || v[i] != want_v) {
      fprintf(stderr, "c-abi: message %d: 2S %d (want %d), V %d (want %d)\n", m[i], s2[i], want_s,
              v[i], want_v);
      ++bad;
    }
  }
  /* the error path: a null output is reported, not a crash */
  const int rc = fs_pbs_lif(ctx, dk, &lif, (const uint32_t*)d_h, COUNT, NULL, (uint32_t*)d_v, NULL);
  if (rc != FS_EINVAL) {
    fprintf(stderr, "c-abi: null output returned %d\n", rc);
    ++bad;
  }
  (void)hipFree(d_h);
  (void)hipFree(d_s);
  (void)hipFree(d_v);
  fs_devkey_free(dk);
  fs_ctx_destroy(ctx);
  fs_evk_free(evk);
  fs_secret_free(sk);
  free(ct);
  free(out);
  if (bad) return 1;
  printf("c-abi: ok (%d messages through Fire and Reset)\n", COUNT);
  return 0;
}
