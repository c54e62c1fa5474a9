// extern "C" boundary of libfhesnn (declared in include/fhesnn.h): argument
// checking, error reporting, device-resident keys, NTT tables, the test
// polynomial cache and scratch management around the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fs_internal.h"
#include "kernels.h"

// ------------------------------------------------------------------ handles

struct fs_secret : fs::Secret {};
struct fs_evk : fs::EvalKey {};

struct fs_devkey {
  fs_params prm{};
  int device = 0;
  double* bsk = nullptr;    // NTT domain, see launch_bsk_to_ntt
  // the KSK: byte planes for the matrix-core key switch (t = 8, base 4),
  // else [N][t][base-1][n+1] words for the generic kernel; the other is null
  uint32_t* ksk = nullptr;
  int8_t* kskp = nullptr;
  double* fwd_tw = nullptr;
  double* inv_tw = nullptr;
  double* post = nullptr;
  fs::UniTw uni{};  // roots shared by all threads of a transform
  size_t bytes = 0;
  uint32_t limbs = 1;  // 16-bit key limbs of the NTT-domain BSK (2: N = 2048, exact form)
};

// Batch-size thresholds of the thread-group forms for one ring degree (see
// br_groups): up to `rows` jobs one group per digit row, then up to `paired`
// two-group jobs in pairs (N = 1024 only), then up to `split` two groups per
// job, then one group.
struct GroupLimits {
  size_t rows = 0, paired = 0, split = 0;
};

struct fs_ctx {
  int device = 0;
  int cus = 0;  // compute units of the device
  std::mutex mu;
  uint32_t* ext = nullptr;  // extracted samples between blind rotation and key switch
  size_t ext_words = 0;
  // Scratch buffers replaced by larger ones.  They stay allocated until
  // fs_ctx_destroy: work captured into a graph before the growth holds
  // their addresses in its kernel arguments and still runs on them.
  std::vector<void*> retired;
  size_t retired_bytes = 0;
  // test polynomials on the device, keyed by (N, p, residue table)
  std::map<std::vector<int32_t>, uint32_t*> tpoly;
  // NTT tables per ring degree for fs_ntt_polymul
  std::map<uint32_t, double*> tables;
  std::map<uint32_t, fs::UniTw> table_uni;
  // blind-rotation kernel variant per ring degree (chosen by the tuner)
  std::map<uint32_t, int> br_variant;
  // thread-group thresholds per ring degree (defaults: default_limits)
  std::map<uint32_t, GroupLimits> limits;
  // device copy of the range table of the last multi-key launch
  fs::JobRange* ranges = nullptr;
  size_t ranges_cap = 0;
  std::vector<fs::JobRange> ranges_host;
  // admission of a serving loop's requests: bytes admitted and their budget
  // (0 = no budget), guarded by mu
  size_t budget = 0, admitted = 0;
};

namespace fs {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(FS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define FS_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int launch_rc(int rc, const char* what) {
  if (rc == 0) return FS_OK;
  if (rc == -2) return fail(FS_EINVAL, std::string(what) + ": no such kernel variant");
  if (rc < 0) return fail(FS_ENOTSUP, std::string(what) + ": unsupported ring degree");
  return fail(FS_EDEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)rc));
}

// ---- NTT tables (exact integer arithmetic on the host)

using u128 = unsigned __int128;
constexpr uint64_t kPr = 0x6000000100001ull;  // same prime as the device transform

uint64_t mulm(uint64_t a, uint64_t b) { return (uint64_t)((u128)a * b % kPr); }
uint64_t powm(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mulm(r, a);
    a = mulm(a, a);
    e >>= 1;
  }
  return r;
}
double centred(uint64_t v) { return v > kPr / 2 ? -(double)(kPr - v) : (double)v; }
uint32_t bitrev(uint32_t k, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((k >> i) & 1u) << (bits - 1 - i);
  return r;
}

// host tables: fwd [N] psi^{brv(k)}, inv [N/2] omega^{-e}, post [N] psi^{-j} N^{-1}
void ntt_tables(uint32_t N, std::vector<double>& fwd, std::vector<double>& inv,
                std::vector<double>& post) {
  const uint32_t logn = ilog2(N);
  uint64_t psi = 0;
  for (uint64_t x = 2;; ++x) {  // smallest x whose (P-1)/2N power has order 2N
    psi = powm(x, (kPr - 1) / (2ull * N));
    if (powm(psi, N) == kPr - 1) break;
  }
  const uint64_t psi_inv = powm(psi, kPr - 2);
  const uint64_t omega_inv = mulm(psi_inv, psi_inv);
  const uint64_t n_inv = powm(N, kPr - 2);
  fwd.assign(N, 0.0);
  for (uint32_t k = 1; k < N; ++k) fwd[k] = centred(powm(psi, bitrev(k, logn)));
  inv.assign(N / 2, 0.0);
  for (uint32_t e = 0; e < N / 2; ++e) inv[e] = centred(powm(omega_inv, e));
  post.assign(N, 0.0);
  for (uint32_t j = 0; j < N; ++j) post[j] = centred(mulm(powm(psi_inv, j), n_inv));
}

int upload_tables(uint32_t N, double** d_fwd, double** d_inv, double** d_post,
                  UniTw* uni = nullptr) {
  std::vector<double> f, i, p;
  ntt_tables(N, f, i, p);
  if (uni) {
    for (int k = 0; k < 16; ++k) uni->fwd[k] = f[k];                 // psi^{brv(k)}
    for (int m = 0; m < 8; ++m) uni->inv[m] = i[(size_t)m * N / 16];  // omega^{-m N/16}
  }
  double* buf = nullptr;
  const size_t total = f.size() + i.size() + p.size();
  FS_HIP(hipMalloc(&buf, total * sizeof(double)));
  hipError_t e = hipMemcpy(buf, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(buf + f.size(), i.data(), i.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(buf + f.size() + i.size(), p.data(), p.size() * sizeof(double),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return hip_fail(e, "upload NTT tables");
  }
  *d_fwd = buf;
  *d_inv = buf + f.size();
  *d_post = buf + f.size() + i.size();
  return FS_OK;
}

int check_params(const fs_params* p) {
  if (!p) return fail(FS_EINVAL, "null fs_params");
  std::string why;
  if (!params_supported(*p, &why)) return fail(FS_ENOTSUP, why);
  return FS_OK;
}

// Grow the extracted-sample scratch to at least `words`.  The old buffer is
// retired, not freed (a captured graph may still use it), and the new one
// is half as large again as the old at least, so the retired buffers of a
// context never add up to more than twice its live scratch.
int ensure_ext(fs_ctx* ctx, size_t words) {
  if (ctx->ext_words >= words) return FS_OK;
  const size_t grown = std::max(words, ctx->ext_words + ctx->ext_words / 2);
  uint32_t* fresh = nullptr;
  hipError_t e = hipMalloc(&fresh, grown * sizeof(uint32_t));
  if (e != hipSuccess) {
    e = hipMalloc(&fresh, words * sizeof(uint32_t));
    if (e != hipSuccess) return fail(FS_ENOMEM, "scratch allocation failed");
  } else {
    words = grown;
  }
  if (ctx->ext) {
    ctx->retired.push_back(ctx->ext);
    ctx->retired_bytes += ctx->ext_words * sizeof(uint32_t);
  }
  ctx->ext = fresh;
  ctx->ext_words = words;
  return FS_OK;
}

// Thresholds of the thread-group forms for ring degree N on this context:
// the tuned ones if set, else the measured defaults.  N = 1024: one job per
// CU on the row kernel, then two-group jobs in pairs up to 2 x CUs, then
// two groups up to 3 x CUs, then one group.  N = 2048: the row kernel holds
// one job per CU (148 KiB of LDS), there is no paired form and two groups
// measured no faster than one beyond the row kernel's range.
GroupLimits limits_for(const fs_ctx* ctx, uint32_t N) {
  auto it = ctx->limits.find(N);
  if (it != ctx->limits.end()) return it->second;
  GroupLimits g;
  g.rows = (size_t)ctx->cus;
  if (N == 1024) {
    g.paired = 2 * (size_t)ctx->cus;
    g.split = 3 * (size_t)ctx->cus;
  }
  return g;
}

// A stream that is being captured into a graph.
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// device test polynomial of a residue table f: Z_p -> Z_p_out (p_out = 0:
// the same space), cached per context
int get_tpoly(fs_ctx* ctx, uint32_t N, uint32_t p, const int32_t* f, uint32_t** out,
              uint32_t p_out = 0) {
  if (p_out == 0) p_out = p;
  std::vector<int32_t> key(f, f + p);
  key.push_back((int32_t)N);
  key.push_back((int32_t)p);
  key.push_back((int32_t)p_out);
  auto it = ctx->tpoly.find(key);
  if (it != ctx->tpoly.end()) {
    *out = it->second;
    return FS_OK;
  }
  std::vector<uint32_t> v(N);
  int rc = test_poly_ms(N, p, p_out, f, v.data());
  if (rc) return rc;
  uint32_t* d = nullptr;
  FS_HIP(hipMalloc(&d, N * sizeof(uint32_t)));
  hipError_t e = hipMemcpy(d, v.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "upload test polynomial");
  }
  ctx->tpoly.emplace(std::move(key), d);
  *out = d;
  return FS_OK;
}

// device test polynomial holding two interleaved residue tables (cached)
int get_tpoly_two(fs_ctx* ctx, uint32_t N, uint32_t p, const int32_t* f0, const int32_t* f1,
                  uint32_t** out) {
  std::vector<int32_t> key(f0, f0 + p);
  key.insert(key.end(), f1, f1 + p);
  key.push_back((int32_t)N);
  key.push_back((int32_t)p);
  key.push_back(-2);  // marks the interleaved form
  auto it = ctx->tpoly.find(key);
  if (it != ctx->tpoly.end()) {
    *out = it->second;
    return FS_OK;
  }
  std::vector<uint32_t> v(N);
  int rc = test_poly_two(N, p, f0, f1, v.data());
  if (rc) return rc;
  uint32_t* d = nullptr;
  FS_HIP(hipMalloc(&d, N * sizeof(uint32_t)));
  hipError_t e = hipMemcpy(d, v.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "upload test polynomial");
  }
  ctx->tpoly.emplace(std::move(key), d);
  *out = d;
  return FS_OK;
}

// thread groups per job for a batch of this size (see launch_blind_rotate),
// from the context's thresholds for ring degree N, checked in order; the
// one-limb N = 2048 key has no row form and takes two groups there
int br_groups(const fs_ctx* ctx, uint32_t N, size_t jobs, uint32_t limbs) {
  const GroupLimits g = limits_for(ctx, N);
  if (jobs <= g.rows) return N == 2048 && limbs == 1 ? kBrTwo : kBrRows;
  if (N == 1024 && jobs <= g.paired) return kBrTwoPaired;
  return jobs <= g.split ? kBrTwo : kBrOne;
}

// blind rotation of jobs = B * nlut, then key switch (or not)
// (into `fixed_ext` instead of the context's scratch when it is set)
int run_pbs(fs_ctx* ctx, const fs_devkey* dk, uint32_t* const tp[2], uint32_t nlut,
            const uint32_t* in, size_t B, uint32_t* out0, uint32_t* out1,
            const uint32_t plain_add[2], int keyswitch, hipStream_t st,
            uint32_t* fixed_ext = nullptr) {
  const fs_params& P = dk->prm;
  const size_t jobs = B * nlut;
  auto vit = ctx->br_variant.find(P.N);
  const int variant = vit == ctx->br_variant.end() ? 0 : vit->second;
  BrArgs br{};
  br.in = in;
  br.tpoly0 = tp[0];
  br.tpoly1 = nlut == 2 ? tp[1] : tp[0];
  br.nlut = nlut;
  br.n = P.n;
  br.bsk = dk->bsk;
  br.fwd_tw = dk->fwd_tw;
  br.inv_tw = dk->inv_tw;
  br.post = dk->post;
  br.uni = dk->uni;
  br.limbs = dk->limbs;
  if (keyswitch && fixed_ext) {
    br.ext = fixed_ext;
  } else if (keyswitch) {
    int rc = ensure_ext(ctx, jobs * (size_t)(P.N + 1));
    if (rc) return rc;
    br.ext = ctx->ext;
  } else {
    br.ext = out0;
  }
  int rc = launch_rc(launch_blind_rotate(P.N, br, jobs, variant,
                                         br_groups(ctx, P.N, jobs, br.limbs), st),
                     "blind rotation");
  if (rc || !keyswitch) return rc;
  KsArgs ks{};
  ks.in = br.ext;
  ks.ksk = dk->ksk;
  ks.kskp = dk->kskp;
  ks.out0 = out0;
  ks.out1 = out1;
  ks.plain_add[0] = plain_add[0];
  ks.plain_add[1] = plain_add[1];
  ks.nlut = nlut;
  ks.n = P.n;
  ks.N = P.N;
  ks.t = P.ks_t;
  ks.beta = P.ks_base_bit;
  return launch_rc(launch_keyswitch(ks, jobs, st), "key switch");
}

// fs_pbs_lif_ranges and its one-rotation form: the blind rotation writes two
// extracted samples per neuron (rows 2 g and 2 g + 1: Fire, Reset) either
// from two jobs per neuron or, `many`, from one even-exponent rotation of
// the interleaved test polynomial; the key switches are the same.
int pbs_lif_ranges(fs_ctx* ctx, const fs_lif* lif, const fs_lif_range* ranges, size_t nranges,
                   void* stream, bool many) {
  if (!ctx || !lif || (nranges && !ranges)) return fail(FS_EINVAL, "fs_pbs_lif_ranges: null argument");
  // order: ranges of one key adjacent (stable), empty ranges dropped
  std::vector<size_t> order;
  for (size_t k = 0; k < nranges; ++k) {
    const fs_lif_range& r = ranges[k];
    if (r.count == 0) continue;
    if (!r.key || !r.h || !r.spike2_out || !r.v_out)
      return fail(FS_EINVAL, "fs_pbs_lif_ranges: null pointer in a range");
    order.push_back(k);
  }
  if (order.empty()) return FS_OK;
  const fs_params& P = ranges[order[0]].key->prm;
  for (size_t k : order) {
    const fs_params& Q = ranges[k].key->prm;
    if (Q.n != P.n || Q.N != P.N || Q.l != P.l || Q.bg_bit != P.bg_bit || Q.p != P.p ||
        Q.ks_t != P.ks_t || Q.ks_base_bit != P.ks_base_bit)
      return fail(FS_EPARAM, "fs_pbs_lif_ranges: keys of different parameter sets");
    if (ranges[k].key->device != ctx->device)
      return fail(FS_EPARAM, "fs_pbs_lif_ranges: a key lives on another device");
    if (ranges[k].key->limbs != ranges[order[0]].key->limbs)
      return fail(FS_EPARAM, "fs_pbs_lif_ranges: keys of different key forms");
  }
  if (P.ks_t != 8 || P.ks_base_bit != 2)
    return fail(FS_ENOTSUP, "fs_pbs_lif_ranges: needs the t = 8, base 4 key switch");
  if (many && P.p > P.N) return fail(FS_ENOTSUP, "fs_pbs_lif_ranges: one rotation needs p <= N");
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    return (uintptr_t)ranges[x].key < (uintptr_t)ranges[y].key;
  });
  std::vector<int32_t> fire(P.p), reset(P.p);
  int rc = fs_lif_luts(lif, P.p, fire.data(), reset.data());
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  // the range table is copied from host memory that the next call rewrites:
  // a graph replaying that copy would read another call's ranges
  if (capturing(st))
    return fail(FS_ENOTSUP, "fs_pbs_lif_ranges: cannot be captured into a graph");
  uint32_t* tp[2] = {nullptr, nullptr};
  if (many) {
    rc = get_tpoly_two(ctx, P.N, P.p, fire.data(), reset.data(), &tp[0]);
    tp[1] = tp[0];
  } else {
    rc = get_tpoly(ctx, P.N, P.p, fire.data(), &tp[0]);
    if (!rc) rc = get_tpoly(ctx, P.N, P.p, reset.data(), &tp[1]);
  }
  if (rc) return rc;
  auto& host = ctx->ranges_host;
  host.clear();
  uint64_t total = 0;
  for (size_t k : order) {
    const fs_lif_range& r = ranges[k];
    host.push_back(JobRange{r.h, r.spike2_out, r.v_out, r.key->bsk, total});
    total += r.count;
  }
  if (total > 0x3FFFFFFFull) return fail(FS_EINVAL, "fs_pbs_lif_ranges: batch too large");
  if (ctx->ranges_cap < host.size()) {
    const size_t cap = std::max(host.size(), 2 * ctx->ranges_cap);
    JobRange* fresh = nullptr;
    FS_HIP(hipMalloc(&fresh, cap * sizeof(JobRange)));
    if (ctx->ranges) {  // retired like the sample scratch
      ctx->retired.push_back(ctx->ranges);
      ctx->retired_bytes += ctx->ranges_cap * sizeof(JobRange);
    }
    ctx->ranges = fresh;
    ctx->ranges_cap = cap;
  }
  FS_HIP(hipMemcpyAsync(ctx->ranges, host.data(), host.size() * sizeof(JobRange),
                        hipMemcpyHostToDevice, st));
  const size_t jobs = many ? total : 2 * total;
  rc = ensure_ext(ctx, 2 * total * (size_t)(P.N + 1));
  if (rc) return rc;
  auto vit = ctx->br_variant.find(P.N);
  const int variant = vit == ctx->br_variant.end() ? 0 : vit->second;
  BrArgs br{};
  br.tpoly0 = tp[0];
  br.tpoly1 = tp[1];
  br.nlut = many ? 1 : 2;
  br.even = many ? 1u : 0u;
  br.n = P.n;
  br.fwd_tw = ranges[order[0]].key->fwd_tw;  // tables depend on N only
  br.inv_tw = ranges[order[0]].key->inv_tw;
  br.post = ranges[order[0]].key->post;
  br.uni = ranges[order[0]].key->uni;
  br.limbs = ranges[order[0]].key->limbs;
  br.ext = ctx->ext;
  br.ranges = ctx->ranges;
  br.nranges = (uint32_t)host.size();
  rc = launch_rc(launch_blind_rotate(P.N, br, jobs, variant,
                                     br_groups(ctx, P.N, jobs, br.limbs), st),
                 "blind rotation");
  if (rc) return rc;
  // one batched key switch per key over its adjacent ranges
  size_t a = 0;
  while (a < order.size()) {
    size_t b = a;
    const fs_devkey* key = ranges[order[a]].key;
    while (b < order.size() && ranges[order[b]].key == key) ++b;
    const uint64_t first = host[a].first;
    const uint64_t last = b < order.size() ? host[b].first : total;
    KsArgs ks{};
    ks.in = ctx->ext + (size_t)(2 * first) * (P.N + 1);
    ks.ksk = key->ksk;
    ks.kskp = key->kskp;
    ks.plain_add[0] = delta_of(P.p);  // 2S = bootstrap_Fire + 1
    ks.plain_add[1] = 0u;
    ks.nlut = 2;
    ks.n = P.n;
    ks.N = P.N;
    ks.t = P.ks_t;
    ks.beta = P.ks_base_bit;
    ks.ranges = ctx->ranges;
    ks.nranges = (uint32_t)host.size();
    ks.job0 = 2 * first;
    rc = launch_rc(launch_keyswitch(ks, (size_t)(2 * (last - first)), st), "key switch");
    if (rc) return rc;
    a = b;
  }
  return FS_OK;
}

}  // namespace
}  // namespace fs

using namespace fs;

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* fs_last_error(void) { return g_err.c_str(); }

int fs_params_default(int shape, fs_params* out) {
  if (!out) return fail(FS_EINVAL, "null output");
  fs_params p{};
  p.n = 630;
  p.k = 1;
  p.ks_t = 8;
  p.ks_base_bit = 2;
  p.sigma_lwe = 0x1p-15;
  p.sigma_ksk = 0x1p-15;
  p.version = FS_PARAMS_VERSION;
  if (shape == 0) {
    p.N = 1024; p.l = 3; p.bg_bit = 7; p.p = 32; p.sigma_bsk = 0x1p-25;
  } else if (shape == 1) {
    p.N = 2048; p.l = 2; p.bg_bit = 10; p.p = 64; p.sigma_bsk = 0x1p-31;
  } else {
    return fail(FS_EINVAL, "shape must be 0 or 1");
  }
  *out = p;
  return FS_OK;
}

int fs_keygen(const fs_params* params, uint64_t seed, fs_secret** sk, fs_evk** evk) {
  if (!sk || !evk) return fail(FS_EINVAL, "null output handle");
  int rc = check_params(params);
  if (rc) return rc;
  try {
    Secret* s = nullptr;
    EvalKey* e = nullptr;
    rc = keygen(*params, seed, &s, &e);
    if (rc) return rc;
    auto* so = new fs_secret;
    static_cast<Secret&>(*so) = std::move(*s);
    auto* eo = new fs_evk;
    static_cast<EvalKey&>(*eo) = std::move(*e);
    delete s;
    delete e;
    *sk = so;
    *evk = eo;
    return FS_OK;
  } catch (const std::bad_alloc&) {
    return fail(FS_ENOMEM, "fs_keygen: out of host memory");
  }
}

int fs_encrypt(const fs_secret* sk, const int32_t* m, size_t count, uint64_t seed,
               uint64_t first_index, uint32_t* ct_out) {
  if (!sk || (count && (!m || !ct_out))) return fail(FS_EINVAL, "fs_encrypt: null argument");
  encrypt(*sk, m, count, seed, first_index, ct_out);
  return FS_OK;
}

int fs_encrypt_z(const fs_secret* sk, const int32_t* m, size_t count, uint64_t seed,
                 uint64_t first_index, uint32_t* ct_out) {
  if (!sk || (count && (!m || !ct_out))) return fail(FS_EINVAL, "fs_encrypt_z: null argument");
  encrypt(*sk, m, count, seed, first_index, ct_out, true);
  return FS_OK;
}

int fs_decrypt(const fs_secret* sk, const uint32_t* ct, size_t count, uint32_t dim,
               int32_t* m_out) {
  if (!sk || (count && (!ct || !m_out))) return fail(FS_EINVAL, "fs_decrypt: null argument");
  return decrypt(*sk, ct, count, dim, m_out);
}

int fs_secret_export(const fs_secret* sk, int32_t* s, int32_t* z) {
  if (!sk) return fail(FS_EINVAL, "null secret");
  if (s) std::memcpy(s, sk->s.data(), sk->s.size() * sizeof(int32_t));
  if (z) std::memcpy(z, sk->z.data(), sk->z.size() * sizeof(int32_t));
  return FS_OK;
}

int fs_evk_export(const fs_evk* evk, uint32_t* bsk, uint32_t* ksk) {
  if (!evk) return fail(FS_EINVAL, "null evaluation key");
  if (bsk) std::memcpy(bsk, evk->bsk.data(), evk->bsk.size() * sizeof(uint32_t));
  if (ksk) std::memcpy(ksk, evk->ksk.data(), evk->ksk.size() * sizeof(uint32_t));
  return FS_OK;
}

int fs_evk_params(const fs_evk* evk, fs_params* out) {
  if (!evk || !out) return fail(FS_EINVAL, "null argument");
  *out = evk->prm;
  return FS_OK;
}

void fs_secret_free(fs_secret* sk) { delete sk; }
void fs_evk_free(fs_evk* evk) { delete evk; }

int fs_test_poly(uint32_t N, uint32_t p, const int32_t* f, uint32_t* v_out) {
  if (!f || !v_out) return fail(FS_EINVAL, "fs_test_poly: null argument");
  if (N < 2 || (N & (N - 1)) || p < 2 || (p & (p - 1)) || p > 2 * N)
    return fail(FS_EINVAL, "fs_test_poly: N and p must be powers of two with p <= 2N");
  return test_poly(N, p, f, v_out);
}

static bool pow2_in(uint64_t x, uint64_t lo, uint64_t hi) {
  return x >= lo && x <= hi && (x & (x - 1)) == 0;
}

int fs_test_poly_mspace(uint32_t N, uint32_t p_in, uint32_t p_out, const int32_t* f,
                        uint32_t* v_out) {
  if (!f || !v_out) return fail(FS_EINVAL, "fs_test_poly_mspace: null argument");
  if (!pow2_in(N, 2, 1u << 20) || !pow2_in(p_in, 2, 2ull * N) || !pow2_in(p_out, 2, 1u << 31))
    return fail(FS_EINVAL,
                "fs_test_poly_mspace: N, p_in, p_out must be powers of two, p_in <= 2N, "
                "p_out <= 2^31");
  return test_poly_ms(N, p_in, p_out, f, v_out);
}

int fs_test_poly_two(uint32_t N, uint32_t p, const int32_t* f0, const int32_t* f1,
                     uint32_t* v_out) {
  if (!f0 || !f1 || !v_out) return fail(FS_EINVAL, "fs_test_poly_two: null argument");
  if (!pow2_in(N, 4, 1u << 20) || !pow2_in(p, 2, N))
    return fail(FS_EINVAL, "fs_test_poly_two: N and p must be powers of two with p <= N");
  return test_poly_two(N, p, f0, f1, v_out);
}

int fs_lif_luts(const fs_lif* lif, uint32_t p, int32_t* fire, int32_t* reset) {
  if (!lif) return fail(FS_EINVAL, "null fs_lif");
  if (p < 4 || (p & (p - 1))) return fail(FS_EINVAL, "p must be a power of two >= 4");
  if (lif->v_th <= 0 || lif->v_th > (int32_t)(p / 2))
    return fail(FS_EINVAL, "v_th must be in 1..p/2");
  if (lif->tau == 1) return fail(FS_EINVAL, "tau must be 0 (IF) or >= 2");
  lif_luts(*lif, p, fire, reset);
  return FS_OK;
}

int fs_lif_range_check(const fs_lif* lif, uint32_t p, const int32_t* W, size_t O, size_t I,
                       int32_t x_lo, int32_t x_hi, int64_t* m_out) {
  if (!lif || !W || !m_out) return fail(FS_EINVAL, "fs_lif_range_check: null argument");
  const int64_t xa = std::max<int64_t>(x_lo < 0 ? -(int64_t)x_lo : x_lo,
                                       x_hi < 0 ? -(int64_t)x_hi : x_hi);
  int64_t worst = 0;
  for (size_t o = 0; o < O; ++o) {
    int64_t s = 0;
    for (size_t i = 0; i < I; ++i) s += (W[o * I + i] < 0 ? -(int64_t)W[o * I + i] : W[o * I + i]);
    worst = std::max(worst, s * xa);
  }
  *m_out = (int64_t)lif->v_th + worst;
  return *m_out <= (int64_t)(p / 2) ? FS_OK : 1;
}

int fs_ctx_create(int device, fs_ctx** ctx) {
  if (!ctx) return fail(FS_EINVAL, "null output handle");
  int count = 0;
  FS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(FS_EINVAL, "no such HIP device");
  int cus = 0;
  FS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  {
    // this device's address of the static scratch of fs_pbs_lif_noalloc
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const int rc = noalloc_setup(device);
    if (rc) return fail(FS_EDEVICE, std::string("static scratch lookup: ") +
                                        hipGetErrorString((hipError_t)rc));
  }
  auto* c = new fs_ctx;
  c->device = device;
  c->cus = cus;  // the thread-group thresholds default to multiples of it
  *ctx = c;
  return FS_OK;
}

int fs_ctx_destroy(fs_ctx* ctx) {
  if (!ctx) return FS_OK;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->ext) (void)hipFree(ctx->ext);
  if (ctx->ranges) (void)hipFree(ctx->ranges);
  for (void* p : ctx->retired) (void)hipFree(p);
  for (auto& kv : ctx->tpoly) (void)hipFree(kv.second);
  for (auto& kv : ctx->tables) (void)hipFree(kv.second);
  delete ctx;
  return FS_OK;
}

int fs_ctx_reserve(fs_ctx* ctx, uint32_t N, size_t max_jobs) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  return ensure_ext(ctx, max_jobs * (size_t)(N + 1));
}

int fs_ctx_scratch_bytes(const fs_ctx* ctx, size_t* live, size_t* retired) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  if (live) *live = ctx->ext_words * sizeof(uint32_t) + ctx->ranges_cap * sizeof(JobRange);
  if (retired) *retired = ctx->retired_bytes;
  return FS_OK;
}

int fs_ctx_set_budget(fs_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->budget = bytes;
  return FS_OK;
}

int fs_ctx_admit(fs_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->budget && (ctx->admitted > ctx->budget || bytes > ctx->budget - ctx->admitted))
    return fail(FS_EBUDGET, "fs_ctx_admit: " + std::to_string(bytes) + " bytes do not fit the budget (" +
                                std::to_string(ctx->admitted) + " of " + std::to_string(ctx->budget) +
                                " admitted)");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  size_t free_b = 0, total_b = 0;
  FS_HIP(hipMemGetInfo(&free_b, &total_b));
  if (bytes > free_b)
    return fail(FS_EBUDGET, "fs_ctx_admit: " + std::to_string(bytes) + " bytes exceed the " +
                                std::to_string(free_b) + " free on the device");
  ctx->admitted += bytes;
  return FS_OK;
}

int fs_ctx_release(fs_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (bytes > ctx->admitted) return fail(FS_EINVAL, "fs_ctx_release: more bytes than admitted");
  ctx->admitted -= bytes;
  return FS_OK;
}

int fs_ctx_admission(fs_ctx* ctx, size_t* budget, size_t* admitted) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (budget) *budget = ctx->budget;
  if (admitted) *admitted = ctx->admitted;
  return FS_OK;
}

int fs_br_variants(uint32_t N) { return blind_rotate_variants(N); }

// one threshold of ring degree N: which = 0 rows, 1 paired, 2 split
static int set_limit(fs_ctx* ctx, uint32_t N, int which, size_t max_jobs, size_t* previous) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  if (N != 1024 && N != 2048) return fail(FS_ENOTSUP, "ring degree without kernels");
  std::lock_guard<std::mutex> lk(ctx->mu);
  GroupLimits g = limits_for(ctx, N);
  size_t& v = which == 0 ? g.rows : which == 1 ? g.paired : g.split;
  if (previous) *previous = v;
  v = max_jobs;
  ctx->limits[N] = g;
  return FS_OK;
}

int fs_ctx_set_rows(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous) {
  return set_limit(ctx, N, 0, max_jobs, previous);
}

int fs_ctx_set_paired(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous) {
  return set_limit(ctx, N, 1, max_jobs, previous);
}

int fs_ctx_set_split(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous) {
  return set_limit(ctx, N, 2, max_jobs, previous);
}

int fs_ctx_set_br_variant(fs_ctx* ctx, uint32_t N, int variant) {
  if (!ctx) return fail(FS_EINVAL, "null context");
  if (N != 1024 && N != 2048) return fail(FS_ENOTSUP, "ring degree without kernels");
  if (variant < 0 || variant >= blind_rotate_variants(N))
    return fail(FS_EINVAL, "no such kernel variant");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->br_variant[N] = variant;
  return FS_OK;
}

int fs_evk_upload(fs_ctx* ctx, const fs_evk* evk, fs_devkey** dk_out) {
  return fs_evk_upload_form(ctx, evk, FS_KEY_EXACT, dk_out);
}

int fs_evk_upload_form(fs_ctx* ctx, const fs_evk* evk, int form, fs_devkey** dk_out) {
  if (!ctx || !evk || !dk_out) return fail(FS_EINVAL, "fs_evk_upload: null argument");
  if (form != FS_KEY_EXACT && form != FS_KEY_ONE_LIMB)
    return fail(FS_EINVAL, "fs_evk_upload: unknown key form");
  int rc = check_params(&evk->prm);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const fs_params& P = evk->prm;
  const uint32_t limbs = P.N == 2048 && form == FS_KEY_EXACT ? 2 : 1;
  auto* dk = new fs_devkey;
  dk->prm = P;
  dk->device = ctx->device;
  dk->limbs = limbs;
  // The matrix-core key switch (t = 8 digits of base 4) reads the KSK only
  // as byte planes, built on the device from a staging copy that is then
  // freed; other digit shapes keep the uint32 key for the generic kernel.
  const bool planes_form = P.ks_t == 8 && P.ks_base_bit == 2;
  uint32_t* coef = nullptr;
  uint32_t* kstage = nullptr;
  auto cleanup = [&](int code) {
    if (coef) (void)hipFree(coef);
    if (kstage) (void)hipFree(kstage);
    fs_devkey_free(dk);
    return code;
  };
  const size_t bsk_words = evk->bsk.size();
  const size_t bsk_ntt = bsk_words * limbs;  // doubles
  const size_t ksk_bytes = evk->ksk.size() * sizeof(uint32_t);
  hipError_t e = hipMalloc(&dk->bsk, bsk_ntt * sizeof(double));
  if (e != hipSuccess) return cleanup(fail(FS_ENOMEM, "fs_evk_upload: BSK allocation failed"));
  uint32_t** ksk_dst = planes_form ? &kstage : &dk->ksk;
  e = hipMalloc(ksk_dst, ksk_bytes);
  if (e != hipSuccess) return cleanup(fail(FS_ENOMEM, "fs_evk_upload: KSK allocation failed"));
  const size_t planes = planes_form ? fs::ksk_planes_bytes(P.N, P.n) : 0;
  if (planes_form) {
    e = hipMalloc(&dk->kskp, planes);
    if (e != hipSuccess)
      return cleanup(fail(FS_ENOMEM, "fs_evk_upload: KSK plane allocation failed"));
  }
  e = hipMalloc(&coef, bsk_words * sizeof(uint32_t));
  if (e != hipSuccess) return cleanup(fail(FS_ENOMEM, "fs_evk_upload: staging allocation failed"));
  rc = upload_tables(P.N, &dk->fwd_tw, &dk->inv_tw, &dk->post, &dk->uni);
  if (rc) return cleanup(rc);
  e = hipMemcpy(coef, evk->bsk.data(), bsk_words * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(*ksk_dst, evk->ksk.data(), ksk_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(hip_fail(e, "fs_evk_upload: copy"));
  rc = launch_rc(launch_bsk_to_ntt(P.N, P.n, P.l, limbs, coef, dk->bsk, dk->fwd_tw, nullptr),
                 "BSK conversion");
  if (rc) return cleanup(rc);
  if (planes_form) {
    rc = launch_rc(launch_ksk_to_planes(P.N, P.n, kstage, dk->kskp, nullptr), "KSK conversion");
    if (rc) return cleanup(rc);
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return cleanup(hip_fail(e, "fs_evk_upload: conversion"));
  (void)hipFree(coef);
  coef = nullptr;
  if (kstage) (void)hipFree(kstage);
  kstage = nullptr;
  dk->bytes = bsk_ntt * sizeof(double) + (planes_form ? planes : ksk_bytes) +
              (size_t)(5 * P.N / 2) * sizeof(double);
  *dk_out = dk;
  return FS_OK;
}

int fs_devkey_form(const fs_devkey* dk) {
  if (!dk) return fail(FS_EINVAL, "null device key");
  return dk->prm.N == 2048 && dk->limbs == 1 ? FS_KEY_ONE_LIMB : FS_KEY_EXACT;
}

int fs_devkey_params(const fs_devkey* dk, fs_params* out) {
  if (!dk || !out) return fail(FS_EINVAL, "null argument");
  *out = dk->prm;
  return FS_OK;
}

size_t fs_devkey_bytes(const fs_devkey* dk) { return dk ? dk->bytes : 0; }

void fs_devkey_free(fs_devkey* dk) {
  if (!dk) return;
  DeviceGuard g(dk->device);
  if (dk->bsk) (void)hipFree(dk->bsk);
  if (dk->ksk) (void)hipFree(dk->ksk);
  if (dk->kskp) (void)hipFree(dk->kskp);
  if (dk->fwd_tw) (void)hipFree(dk->fwd_tw);  // one allocation holds all three tables
  delete dk;
}

int fs_lwe_linear(fs_ctx* ctx, const int32_t* W, size_t O, size_t I, uint32_t dim,
                  const uint32_t* x, const uint32_t* add, uint32_t* y, void* stream) {
  if (!ctx || (O && (!W || !y)) || (O && I && !x) || dim == 0)
    return fail(FS_EINVAL, "fs_lwe_linear: null argument or zero width");
  if (O > 0xFFFFFFFFu || I > 0xFFFFFFFFu) return fail(FS_EINVAL, "fs_lwe_linear: shape too large");
  DeviceGuard g(ctx->device);
  return launch_rc(launch_lwe_linear(W, O, I, dim, x, add, y, as_stream(stream)), "lwe_linear");
}

int fs_lwe_conv2d(fs_ctx* ctx, const int32_t* W, uint32_t Ci, uint32_t H, uint32_t Wd,
                  uint32_t Co, uint32_t K, uint32_t stride, uint32_t pad, uint32_t dim,
                  const uint32_t* x, const uint32_t* add, uint32_t* y, void* stream) {
  if (!ctx || !W || !x || !y || dim == 0) return fail(FS_EINVAL, "fs_lwe_conv2d: null argument");
  if (Ci == 0 || Co == 0 || K == 0 || stride == 0 || H + 2 * pad < K || Wd + 2 * pad < K)
    return fail(FS_EINVAL, "fs_lwe_conv2d: bad geometry");
  const uint64_t Ho = (H + 2 * pad - K) / stride + 1, Wo = (Wd + 2 * pad - K) / stride + 1;
  if ((uint64_t)Co * Ho * Wo > 0x7FFFFFFFull) return fail(FS_EINVAL, "fs_lwe_conv2d: too many outputs");
  DeviceGuard g(ctx->device);
  return launch_rc(launch_lwe_conv2d(W, Ci, H, Wd, Co, K, stride, pad, dim, x, add, y,
                                     as_stream(stream)), "lwe_conv2d");
}

int fs_lwe_add(fs_ctx* ctx, const uint32_t* a, const uint32_t* b, size_t words, uint32_t* y,
               void* stream) {
  if (!ctx || (words && (!a || !b || !y))) return fail(FS_EINVAL, "fs_lwe_add: null argument");
  if (words / 256 >= 0x7FFFFFFFull) return fail(FS_EINVAL, "fs_lwe_add: too many words");
  DeviceGuard g(ctx->device);
  return launch_rc(launch_lwe_add(a, b, words, y, as_stream(stream)), "lwe_add");
}

int fs_lwe_add_plain(fs_ctx* ctx, uint32_t p, const uint32_t* x, const int32_t* c, size_t count,
                     uint32_t dim, uint32_t* y, void* stream) {
  if (!ctx || (count && (!x || !c || !y))) return fail(FS_EINVAL, "fs_lwe_add_plain: null argument");
  if (p < 2 || (p & (p - 1)) != 0) return fail(FS_EINVAL, "fs_lwe_add_plain: p must be a power of two");
  if (dim == 0 || (count * dim) / 256 >= 0x7FFFFFFFull)
    return fail(FS_EINVAL, "fs_lwe_add_plain: bad shape");
  DeviceGuard g(ctx->device);
  return launch_rc(launch_lwe_add_plain(x, c, delta_of(p), count, dim, y, as_stream(stream)),
                   "lwe_add_plain");
}

int fs_pbs(fs_ctx* ctx, const fs_devkey* dk, const int32_t* lut, const uint32_t* in, size_t B,
           uint32_t* out, int keyswitch, void* stream) {
  if (!ctx || !dk || !lut || (B && (!in || !out))) return fail(FS_EINVAL, "fs_pbs: null argument");
  if (dk->device != ctx->device) return fail(FS_EPARAM, "fs_pbs: key lives on another device");
  if (B > 0x7FFFFFFFull) return fail(FS_EINVAL, "fs_pbs: batch too large");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  uint32_t* tp[2] = {nullptr, nullptr};
  int rc = get_tpoly(ctx, dk->prm.N, dk->prm.p, lut, &tp[0]);
  if (rc) return rc;
  const uint32_t zero[2] = {0u, 0u};
  return run_pbs(ctx, dk, tp, 1, in, B, out, nullptr, zero, keyswitch, as_stream(stream));
}

int fs_pbs_mspace(fs_ctx* ctx, const fs_devkey* dk, const int32_t* lut, uint32_t p_in,
                  uint32_t p_out, const uint32_t* in, size_t B, uint32_t* out, int keyswitch,
                  void* stream) {
  if (!ctx || !dk || !lut || (B && (!in || !out)))
    return fail(FS_EINVAL, "fs_pbs_mspace: null argument");
  if (dk->device != ctx->device) return fail(FS_EPARAM, "fs_pbs_mspace: key lives on another device");
  if (B > 0x7FFFFFFFull) return fail(FS_EINVAL, "fs_pbs_mspace: batch too large");
  if (!pow2_in(p_in, 2, 2ull * dk->prm.N) || !pow2_in(p_out, 2, 1u << 31))
    return fail(FS_EINVAL, "fs_pbs_mspace: p_in, p_out must be powers of two, p_in <= 2N, "
                           "p_out <= 2^31");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  uint32_t* tp[2] = {nullptr, nullptr};
  int rc = get_tpoly(ctx, dk->prm.N, p_in, lut, &tp[0], p_out);
  if (rc) return rc;
  const uint32_t zero[2] = {0u, 0u};
  return run_pbs(ctx, dk, tp, 1, in, B, out, nullptr, zero, keyswitch, as_stream(stream));
}

int fs_pbs_lif(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif, const uint32_t* h, size_t B,
               uint32_t* spike2_out, uint32_t* v_out, void* stream) {
  if (!ctx || !dk || !lif || (B && (!h || !spike2_out || !v_out)))
    return fail(FS_EINVAL, "fs_pbs_lif: null argument");
  if (dk->device != ctx->device) return fail(FS_EPARAM, "fs_pbs_lif: key lives on another device");
  if (B > 0x3FFFFFFFull) return fail(FS_EINVAL, "fs_pbs_lif: batch too large");
  const uint32_t p = dk->prm.p;
  std::vector<int32_t> fire(p), reset(p);
  int rc = fs_lif_luts(lif, p, fire.data(), reset.data());
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  uint32_t* tp[2] = {nullptr, nullptr};
  rc = get_tpoly(ctx, dk->prm.N, p, fire.data(), &tp[0]);
  if (rc) return rc;
  rc = get_tpoly(ctx, dk->prm.N, p, reset.data(), &tp[1]);
  if (rc) return rc;
  const uint32_t add[2] = {delta_of(p), 0u};  // 2S = bootstrap_Fire + 1
  return run_pbs(ctx, dk, tp, 2, h, B, spike2_out, v_out, add, 1, as_stream(stream));
}

int fs_pbs_lif_noalloc(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif, const uint32_t* h,
                       size_t B, uint32_t* spike2_out, uint32_t* v_out, void* stream) {
  if (!ctx || !dk || !lif || (B && (!h || !spike2_out || !v_out)))
    return fail(FS_EINVAL, "fs_pbs_lif_noalloc: null argument");
  if (dk->device != ctx->device)
    return fail(FS_EPARAM, "fs_pbs_lif_noalloc: key lives on another device");
  const fs_params& P = dk->prm;
  if (P.p > kTpPairMaxP) return fail(FS_ENOTSUP, "fs_pbs_lif_noalloc: needs p <= 256");
  if (B > kNoallocExtWords / (2 * (size_t)(P.N + 1)))
    return fail(FS_EINVAL, "fs_pbs_lif_noalloc: batch exceeds the static scratch (" +
                               std::to_string(kNoallocExtWords / (2 * (size_t)(P.N + 1))) +
                               " neurons at N = " + std::to_string(P.N) + ")");
  // residue tables on the stack: nothing on this path allocates
  int32_t fire[kTpPairMaxP], reset[kTpPairMaxP];
  int rc = fs_lif_luts(lif, P.p, fire, reset);
  if (rc) return rc;
  TpPair tp{};
  tp.N = P.N;
  tp.p = P.p;
  tp.delta = delta_of(P.p);
  for (uint32_t r = 0; r < P.p; ++r) {
    tp.f[0][r] = (uint32_t)fire[r];
    tp.f[1][r] = (uint32_t)reset[r];
  }
  for (int k = 0; k < 2; ++k)  // Theorem 2.1: f(r + p/2) = -f(r) mod p
    for (uint32_t r = 0; r < P.p; ++r)
      if (((tp.f[k][(r + P.p / 2) & (P.p - 1)] + tp.f[k][r]) & (P.p - 1)) != 0)
        return fail(FS_EINVAL, "fs_pbs_lif_noalloc: program function is not negacyclic");
  if (B == 0) return FS_OK;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  uint32_t* base = noalloc_scratch(ctx->device);
  if (!base) return fail(FS_EDEVICE, "fs_pbs_lif_noalloc: static scratch not set up");
  hipStream_t st = as_stream(stream);
  rc = launch_rc(launch_tpoly_pair(tp, base, st), "test polynomials");
  if (rc) return rc;
  uint32_t* const tps[2] = {base, base + P.N};
  const uint32_t add[2] = {delta_of(P.p), 0u};  // 2S = bootstrap_Fire + 1
  return run_pbs(ctx, dk, tps, 2, h, B, spike2_out, v_out, add, 1, st, base + kNoallocTpWords);
}

int fs_pbs_lif_many_lut(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif, const uint32_t* h,
                        size_t B, uint32_t* spike2_out, uint32_t* v_out, void* stream) {
  if (!ctx || !dk || !lif || (B && (!h || !spike2_out || !v_out)))
    return fail(FS_EINVAL, "fs_pbs_lif_many_lut: null argument");
  if (dk->device != ctx->device)
    return fail(FS_EPARAM, "fs_pbs_lif_many_lut: key lives on another device");
  if (B > 0x3FFFFFFFull) return fail(FS_EINVAL, "fs_pbs_lif_many_lut: batch too large");
  const fs_params& P = dk->prm;
  if (P.p > P.N) return fail(FS_ENOTSUP, "fs_pbs_lif_many_lut: needs p <= N");
  std::vector<int32_t> fire(P.p), reset(P.p);
  int rc = fs_lif_luts(lif, P.p, fire.data(), reset.data());
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  uint32_t* tp = nullptr;
  rc = get_tpoly_two(ctx, P.N, P.p, fire.data(), reset.data(), &tp);
  if (rc) return rc;
  if (B == 0) return FS_OK;
  hipStream_t st = as_stream(stream);
  // one rotation per neuron; coefficients 0 (Fire) and 1 (Reset) extracted
  // into rows 2 g and 2 g + 1, then key-switched like a two-function batch
  rc = ensure_ext(ctx, 2 * B * (size_t)(P.N + 1));
  if (rc) return rc;
  auto vit = ctx->br_variant.find(P.N);
  const int variant = vit == ctx->br_variant.end() ? 0 : vit->second;
  BrArgs br{};
  br.in = h;
  br.tpoly0 = tp;
  br.tpoly1 = tp;
  br.nlut = 1;
  br.even = 1;
  br.n = P.n;
  br.bsk = dk->bsk;
  br.fwd_tw = dk->fwd_tw;
  br.inv_tw = dk->inv_tw;
  br.post = dk->post;
  br.uni = dk->uni;
  br.limbs = dk->limbs;
  br.ext = ctx->ext;
  rc = launch_rc(launch_blind_rotate(P.N, br, B, variant, br_groups(ctx, P.N, B, br.limbs), st),
                 "blind rotation");
  if (rc) return rc;
  KsArgs ks{};
  ks.in = ctx->ext;
  ks.ksk = dk->ksk;
  ks.kskp = dk->kskp;
  ks.out0 = spike2_out;
  ks.out1 = v_out;
  ks.plain_add[0] = delta_of(P.p);  // 2S = bootstrap_Fire + 1
  ks.plain_add[1] = 0u;
  ks.nlut = 2;
  ks.n = P.n;
  ks.N = P.N;
  ks.t = P.ks_t;
  ks.beta = P.ks_base_bit;
  return launch_rc(launch_keyswitch(ks, 2 * B, st), "key switch");
}

int fs_pbs_lif_ks_first(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif, const uint32_t* h,
                        size_t B, uint32_t* spike2_out, uint32_t* v_out, void* stream) {
  if (!ctx || !dk || !lif || (B && (!h || !spike2_out || !v_out)))
    return fail(FS_EINVAL, "fs_pbs_lif_ks_first: null argument");
  if (dk->device != ctx->device)
    return fail(FS_EPARAM, "fs_pbs_lif_ks_first: key lives on another device");
  if (B > 0x3FFFFFFFull) return fail(FS_EINVAL, "fs_pbs_lif_ks_first: batch too large");
  if (B && spike2_out == v_out) return fail(FS_EINVAL, "fs_pbs_lif_ks_first: the two outputs alias");
  const fs_params& P = dk->prm;
  std::vector<int32_t> fire(P.p), reset(P.p);
  int rc = fs_lif_luts(lif, P.p, fire.data(), reset.data());
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  uint32_t* tp[2] = {nullptr, nullptr};
  rc = get_tpoly(ctx, P.N, P.p, fire.data(), &tp[0]);
  if (rc) return rc;
  rc = get_tpoly(ctx, P.N, P.p, reset.data(), &tp[1]);
  if (rc) return rc;
  if (B == 0) return FS_OK;
  hipStream_t st = as_stream(stream);
  // LWE_z(H) -> LWE_s(H), once per neuron: both functions bootstrap it
  rc = ensure_ext(ctx, B * (size_t)(P.n + 1));
  if (rc) return rc;
  KsArgs ks{};
  ks.in = h;
  ks.ksk = dk->ksk;
  ks.kskp = dk->kskp;
  ks.out0 = ctx->ext;
  ks.nlut = 1;
  ks.n = P.n;
  ks.N = P.N;
  ks.t = P.ks_t;
  ks.beta = P.ks_base_bit;
  rc = launch_rc(launch_keyswitch(ks, B, st), "key switch");
  if (rc) return rc;
  // Fire and Reset blind rotations, extracted straight into the outputs
  const size_t jobs = 2 * B;
  auto vit = ctx->br_variant.find(P.N);
  const int variant = vit == ctx->br_variant.end() ? 0 : vit->second;
  BrArgs br{};
  br.in = ctx->ext;
  br.tpoly0 = tp[0];
  br.tpoly1 = tp[1];
  br.nlut = 2;
  br.n = P.n;
  br.bsk = dk->bsk;
  br.fwd_tw = dk->fwd_tw;
  br.inv_tw = dk->inv_tw;
  br.post = dk->post;
  br.uni = dk->uni;
  br.limbs = dk->limbs;
  br.out0 = spike2_out;
  br.out1 = v_out;
  br.plain_b[0] = delta_of(P.p);  // 2S = bootstrap_Fire + 1
  br.plain_b[1] = 0u;
  return launch_rc(
      launch_blind_rotate(P.N, br, jobs, variant, br_groups(ctx, P.N, jobs, br.limbs), st),
      "blind rotation");
}

int fs_pbs_lif_ranges(fs_ctx* ctx, const fs_lif* lif, const fs_lif_range* ranges,
                      size_t nranges, void* stream) {
  return pbs_lif_ranges(ctx, lif, ranges, nranges, stream, false);
}

int fs_pbs_lif_ranges_many_lut(fs_ctx* ctx, const fs_lif* lif, const fs_lif_range* ranges,
                               size_t nranges, void* stream) {
  return pbs_lif_ranges(ctx, lif, ranges, nranges, stream, true);
}

int fs_keyswitch(fs_ctx* ctx, const fs_devkey* dk, const uint32_t* in, size_t B, uint32_t* out,
                 void* stream) {
  if (!ctx || !dk || (B && (!in || !out))) return fail(FS_EINVAL, "fs_keyswitch: null argument");
  if (dk->device != ctx->device) return fail(FS_EPARAM, "fs_keyswitch: key lives on another device");
  if (B > 0x7FFFFFFFull) return fail(FS_EINVAL, "fs_keyswitch: batch too large");
  DeviceGuard g(ctx->device);
  const fs_params& P = dk->prm;
  KsArgs ks{};
  ks.in = in;
  ks.ksk = dk->ksk;
  ks.kskp = dk->kskp;
  ks.out0 = out;
  ks.out1 = nullptr;
  ks.nlut = 1;
  ks.n = P.n;
  ks.N = P.N;
  ks.t = P.ks_t;
  ks.beta = P.ks_base_bit;
  return launch_rc(launch_keyswitch(ks, B, as_stream(stream)), "key switch");
}

int fs_ntt_polymul(fs_ctx* ctx, uint32_t N, uint32_t R, int32_t dmax, const int32_t* d,
                   const uint32_t* b, uint32_t* out, void* stream) {
  if (!ctx || !d || !b || !out || R == 0 || dmax <= 0)
    return fail(FS_EINVAL, "fs_ntt_polymul: null argument or empty product");
  if (N != 1024 && N != 2048) return fail(FS_ENOTSUP, "fs_ntt_polymul: N must be 1024 or 2048");
  const double coef = N == 2048 ? 32768.0 : 2147483648.0;  // 2^15 per half, or 2^31
  if ((double)R * N * dmax * coef >= 844424930656256.0)
    return fail(FS_EINVAL, "fs_ntt_polymul: R*N*dmax exceeds the exactness bound of the transform");
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  auto it = ctx->tables.find(N);
  double *f = nullptr, *iv = nullptr, *po = nullptr;
  if (it == ctx->tables.end()) {
    UniTw uni{};
    int rc = upload_tables(N, &f, &iv, &po, &uni);
    if (rc) return rc;
    ctx->tables[N] = f;
    ctx->table_uni[N] = uni;
  } else {
    f = it->second;
  }
  iv = f + N;
  po = f + N + N / 2;
  return launch_rc(launch_polymul(N, d, b, R, out, f, iv, po, ctx->table_uni[N], as_stream(stream)),
                   "polymul");
}

}  // extern "C"
