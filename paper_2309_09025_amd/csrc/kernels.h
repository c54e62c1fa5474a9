// Kernel argument blocks and launchers (internal to libfhesnn).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "ntt_fp64.h"

namespace fs {

// A contiguous range of ciphertexts bootstrapped in a multi-key launch: its
// input and output rows and the NTT-domain key of the client it belongs
// to.  Ranges are listed in job order; `first` is the index of the range's
// first ciphertext among all ciphertexts of the launch.
struct JobRange {
  const uint32_t* in;
  uint32_t* out0;
  uint32_t* out1;
  const double* bsk;
  uint64_t first;
};

// index of the range holding ciphertext g (ranges sorted by `first`)
__device__ __forceinline__ uint32_t find_range(const JobRange* r, uint32_t nr, uint64_t g) {
  uint32_t lo = 0, hi = nr;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (r[mid].first <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct BrArgs {
  const uint32_t* in;     // [B][n+1] input samples under s
  const uint32_t* tpoly0; // [N] test polynomial of program function 0
  const uint32_t* tpoly1; // [N] test polynomial of program function 1
  uint32_t nlut;          // job j bootstraps sample j / nlut with function j % nlut
  uint32_t n;
  const double* bsk;      // NTT-domain bootstrapping key
  const double* fwd_tw;   // [N] psi^{brv(k)}
  const double* inv_tw;   // [N/2] omega^{-e}
  const double* post;     // [N] psi^{-j} N^{-1}
  uint32_t* ext;          // [jobs][N+1] extracted samples under z
  // routed extraction (single-key launches): when out0 is set, job j's
  // sample goes to row j / nlut of out0 (function 0) or out1 (function 1)
  // with plain_b[j % nlut] added to its body, instead of to ext
  uint32_t* out0;
  uint32_t* out1;
  uint32_t plain_b[2];
  // two functions from one rotation: exponents rounded to even values, the
  // test polynomial interleaves function 0 (even coefficients) and 1 (odd);
  // coefficients 0 and 1 are extracted, to ext rows 2 job and 2 job + 1
  // (or routed as functions 0 and 1).  nlut must be 1.
  uint32_t even;
  UniTw uni;              // roots shared by all threads (scalar operands)
  // multi-key launch: per-range inputs and keys (in and bsk unused)
  const JobRange* ranges;
  uint32_t nranges;
  uint64_t jobs;          // jobs in the launch (set by launch_blind_rotate)
  // 16-bit key limbs of the NTT-domain key: 2 at N = 2048 for exactness
  // with every key, 1 for the one-limb key form (and always at N = 1024)
  uint32_t limbs;
};

struct KsArgs {
  const uint32_t* in;  // [jobs][N+1]
  const uint32_t* ksk; // [N][t][base-1][n+1]
  // the same key as signed byte planes in matrix-core operand order (t = 8,
  // base 4; see launch_ksk_to_planes), or null
  const int8_t* kskp;
  uint32_t* out0;      // program function 0 outputs, [jobs/nlut][n+1]
  uint32_t* out1;      // program function 1 outputs (nlut == 2)
  uint32_t plain_add[2];  // Delta * c added to b per program function
  uint32_t nlut, n, N, t, beta;
  // multi-key launch: outputs per range; sample m is job job0 + m
  const JobRange* ranges;
  uint32_t nranges;
  uint64_t job0;
};

int launch_bsk_to_ntt(uint32_t N, uint32_t n, uint32_t l, uint32_t limbs,
                      const uint32_t* bsk_coef, double* out, const double* tw, hipStream_t st);
int blind_rotate_variants(uint32_t N);
// Thread groups per job: 1 (large batches; `variant` picks the tuned
// instance), 2 (one group per input polynomial), 3 (two such jobs per
// workgroup, N = 1024) or 0 = one group per digit row (smallest batches,
// latency; at N = 1024 one wave per digit-row half, at N = 2048 with the
// two-limb key only).
enum BrGroups { kBrOne = 1, kBrTwo = 2, kBrRows = 0, kBrTwoPaired = 3 };
int launch_blind_rotate(uint32_t N, const BrArgs& a, size_t jobs, int variant, int groups,
                        hipStream_t st);
int launch_keyswitch(const KsArgs& a, size_t count, hipStream_t st);
// words per KSK row n+1 rounded up to the 32-word tiles of the matrix-core
// key switch, and the byte size of its plane layout
uint32_t ks_word_tiles(uint32_t n);
size_t ksk_planes_bytes(uint32_t N, uint32_t n);
int launch_ksk_to_planes(uint32_t N, uint32_t n, const uint32_t* ksk, int8_t* planes,
                         hipStream_t st);
int launch_polymul(uint32_t N, const int32_t* d, const uint32_t* b, uint32_t R, uint32_t* out,
                   const double* tw, const double* itw, const double* post, const UniTw& uni,
                   hipStream_t st);

// Static scratch of fs_pbs_lif_noalloc (noalloc.hip): two test polynomials
// of up to 2048 words, then extracted samples for up to 4096 neurons at
// N = 1024 (2 x 4096 x 1025 words; 2048 neurons at N = 2048).  33.6 MB
// per device, held until the process ends.
constexpr size_t kNoallocTpWords = 2 * 2048;
constexpr size_t kNoallocExtWords = 2 * 4096 * 1025;
constexpr uint32_t kTpPairMaxP = 256;
struct TpPair {
  uint32_t f[2][kTpPairMaxP];  // residues of functions 0 and 1 (first p used)
  uint32_t N, p, delta;
};
int noalloc_setup(int device);
uint32_t* noalloc_scratch(int device);
int launch_tpoly_pair(const TpPair& a, uint32_t* dst, hipStream_t st);

int launch_lwe_linear(const int32_t* W, size_t O, size_t I, uint32_t dim, const uint32_t* x,
                      const uint32_t* add, uint32_t* y, hipStream_t st);
int launch_lwe_conv2d(const int32_t* W, uint32_t Ci, uint32_t H, uint32_t Wd, uint32_t Co,
                      uint32_t K, uint32_t stride, uint32_t pad, uint32_t dim,
                      const uint32_t* x, const uint32_t* add, uint32_t* y, hipStream_t st);
int launch_lwe_add(const uint32_t* a, const uint32_t* b, size_t words, uint32_t* y,
                   hipStream_t st);
int launch_lwe_add_plain(const uint32_t* x, const int32_t* c, uint32_t delta, size_t count,
                         uint32_t dim, uint32_t* y, hipStream_t st);

}  // namespace fs
