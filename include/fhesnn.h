/*
 * fhesnn.h -- C ABI of the MI355X encrypted-LIF engine (TFHE programmable
 * bootstrapping of LWE ciphertexts, plus the integer WeightSum layers that
 * feed it), after "Efficient Privacy-Preserving Convolutional Spiking Neural
 * Networks with FHE" (FHE-DiCSNN).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Torus32: q = 2^32; every ciphertext word is a uint32_t and all
 *    arithmetic on it wraps mod 2^32 (Sec. 2.1, LWE item, with q = 2^32).
 *  - An LWE ciphertext of dimension d is d+1 words (a_0 .. a_{d-1}, b), b
 *    last.  Batches are row-major [count][d+1].  Under the LWE key s the
 *    width is n+1; an extracted, not yet key-switched ciphertext (key z) is
 *    N+1 words.
 *  - Messages are int32 residues of Z_p; decryption returns the centred
 *    representative in {-p/2+1, ..., p/2} (Sec. 2.1, definition of Z_p).
 *    Encoding is Delta*(m mod p), Delta = 2^32/p.
 *  - Pointers marked "dev" are device (HBM) pointers owned by the caller;
 *    "host" pointers are host memory owned by the caller.  The library
 *    never frees or retains caller pointers beyond the call; device work is
 *    enqueued on the given stream (a hipStream_t passed as void*; NULL = the
 *    default stream) and the caller keeps buffers alive until it has
 *    synchronised that stream.
 *  - Every function returns FS_OK (0) or a negative FS_E* code; the reason
 *    is then available from fs_last_error() (thread-local).  Nothing aborts
 *    and no C++ exception crosses this boundary.
 *  - Handles (fs_secret, fs_evk, fs_ctx, fs_devkey) are created by the
 *    library and released by the matching fs_*_free / fs_ctx_destroy.
 *  - A context (fs_ctx) owns the scratch that its bootstrapping and key
 *    switching calls write between their kernels (extracted samples, range
 *    tables).  Calls on one context are safe from any host thread (a mutex
 *    guards its host state) and are ordered when they share a stream; work
 *    of one context enqueued on two streams at once races on that scratch.
 *    Use one context per concurrent stream; device keys may be shared.
 *    Growing the scratch retires the old buffer instead of freeing it: it
 *    stays allocated until fs_ctx_destroy, so work already enqueued, or
 *    captured into a graph before the growth, still runs on valid memory
 *    (and keeps using the old buffer when replayed).  fs_ctx_reserve before
 *    a capture avoids growth altogether.
 *  - Only k = 1 (one mask polynomial per RLWE sample) is supported.
 */
#ifndef FHESNN_H
#define FHESNN_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define FS_API __attribute__((visibility("default")))
#else
#define FS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define FS_OK 0
#define FS_EINVAL (-1)   /* bad argument: null, shape, non-negacyclic LUT, p not a power of 2 */
#define FS_ENOMEM (-2)   /* host or device allocation failed                                  */
#define FS_EDEVICE (-3)  /* a HIP runtime call or kernel launch failed                        */
#define FS_EPARAM (-4)   /* key / parameter set mismatch                                      */
#define FS_EBUDGET (-5)  /* request does not fit the memory budget (fs_ctx_admit)             */
#define FS_ENOTSUP (-6)  /* parameter set outside what the kernels implement                  */

#define FS_PARAMS_VERSION 1u

/* TFHE parameter set.
 *   n           LWE dimension (key s).
 *   N, k        RLWE ring degree (power of two) and mask size; k must be 1.
 *   l, bg_bit   gadget levels and log2 of the gadget base Bg (TGSW rows).
 *   ks_t, ks_base_bit   key-switch digits and log2 of their base.
 *   p           message modulus, a power of two with p <= 2N.
 *   sigma_*     Gaussian noise standard deviations on the unit torus.
 * Kernels exist for (N, l, bg_bit) = (1024, 3, 7) and (2048, 2, 10). */
typedef struct fs_params {
  uint32_t n, N, k, l, bg_bit, ks_t, ks_base_bit, p;
  double sigma_lwe, sigma_bsk, sigma_ksk;
  uint32_t version; /* FS_PARAMS_VERSION */
} fs_params;

/* LIF neuron: integer threshold V_th (0 < v_th <= p/2) and leak time
 * constant tau (tau >= 2; 0 means the IF neuron, tau = infinity), as in
 * Theorem 3.1 (Eq. DiscretEquation). */
typedef struct fs_lif {
  int32_t v_th;
  uint32_t tau;
} fs_lif;

typedef struct fs_secret fs_secret; /* client: binary s (n) and z (N)                          */
typedef struct fs_evk fs_evk;       /* client-built evaluation key: BSK + KSK, host memory     */
typedef struct fs_ctx fs_ctx;       /* server: device binding, LUT cache, scratch              */
typedef struct fs_devkey fs_devkey; /* server: HBM-resident BSK (NTT domain) + KSK             */

/* Thread-local text of the last error (never NULL). */
FS_API const char* fs_last_error(void);

/* Fill *out with a built-in parameter set: shape 0 = n 630, N 1024, l 3,
 * Bg 2^7, KS base 2^2 t 8, p 32, sigma_lwe = sigma_ksk = 2^-15,
 * sigma_bsk = 2^-25; shape 1 = the same with N 2048, l 2, Bg 2^10, p 64,
 * sigma_bsk = 2^-31. */
FS_API int fs_params_default(int shape, fs_params* out);

/* ---------------------------------------------------------------- client */

/* Key generation (Sec. 2.1: LWE key s, RLWE key z, bootstrapping key
 * ek = (RGSW(X^{s_1}) .. RGSW(X^{s_n})) realised as BSK_i = TGSW_z(s_i),
 * and the key-switching key z -> s).  All randomness is drawn from a
 * ChaCha20 counter stream keyed by `seed` (RFC 8439 block function), so the
 * keys are a deterministic function of (params, seed).  Host memory only. */
FS_API int fs_keygen(const fs_params* params, uint64_t seed, fs_secret** sk, fs_evk** evk);

/* LWE encryption of count messages (Sec. 2.1, LWE item):
 * ct_k = (a, <a,s> + e + Delta*(m_k mod p)).  Ciphertext k draws its mask
 * and noise from stream object first_index + k of `seed`.
 * ct_out: host [count][n+1]. */
FS_API int fs_encrypt(const fs_secret* sk, const int32_t* m, size_t count, uint64_t seed,
               uint64_t first_index, uint32_t* ct_out);

/* The same encryption under the extracted key z (Sec. 2.1, LWE item, with
 * the RLWE secret's coefficients as the LWE key): ct_out: host [count][N+1].
 * Input for the key-switch-first ordering (fs_pbs_lif_ks_first), where the
 * ciphertexts between bootstrappings live under z.  Stream objects are
 * shared with fs_encrypt: use distinct first_index ranges for the two. */
FS_API int fs_encrypt_z(const fs_secret* sk, const int32_t* m, size_t count, uint64_t seed,
                        uint64_t first_index, uint32_t* ct_out);

/* Decryption (Sec. 2.1): m = round((b - <a,key>) p / 2^32) mod p, centred.
 * dim = n+1 decrypts under s; dim = N+1 under z (extracted samples).
 * ct: host [count][dim]; m_out: host [count]. */
FS_API int fs_decrypt(const fs_secret* sk, const uint32_t* ct, size_t count, uint32_t dim,
               int32_t* m_out);

/* Copies of the key material for inspection (tests):
 * s: host [n], z: host [N]; bsk: host [n][2l][2][N] (coefficient domain);
 * ksk: host [N][t][base-1][n+1].  Any output pointer may be NULL. */
FS_API int fs_secret_export(const fs_secret* sk, int32_t* s, int32_t* z);
FS_API int fs_evk_export(const fs_evk* evk, uint32_t* bsk, uint32_t* ksk);
FS_API int fs_evk_params(const fs_evk* evk, fs_params* out);

FS_API void fs_secret_free(fs_secret* sk);
FS_API void fs_evk_free(fs_evk* evk);

/* Program function -> test polynomial (the Initialization step after
 * Theorem 2.1): v_i = Delta * f(floor((i p + N) / (2N)) mod p), i < N.
 * f: host [p] residues.  Returns FS_EINVAL unless f(r + p/2) = -f(r) mod p
 * for all r (the condition of Theorem 2.1).  v_out: host [N]. */
FS_API int fs_test_poly(uint32_t N, uint32_t p, const int32_t* f, uint32_t* v_out);

/* Test polynomial that also changes the message space (the dynamic message
 * space of DiNN that Sec. 5.1 notes applies here): inputs encode Z_p_in
 * (Delta_in = 2^32/p_in), outputs Z_p_out (Delta_out = 2^32/p_out):
 * v_i = Delta_out * f(floor((i p_in + N) / (2N)) mod p_in).  f: host [p_in]
 * values taken mod p_out; FS_EINVAL unless f(r + p_in/2) = -f(r) mod p_out
 * for all r.  N, p_in, p_out powers of two, p_in <= 2N, p_out <= 2^31. */
FS_API int fs_test_poly_mspace(uint32_t N, uint32_t p_in, uint32_t p_out, const int32_t* f,
                               uint32_t* v_out);

/* Test polynomial holding two program functions for a rotation by even
 * exponents only (fs_pbs_lif_many_lut): coefficient 2u carries f0 and
 * 2u + 1 carries f1 of the message round(u p / N) (ties up):
 * v_{2u+r} = Delta f_r(floor((u p + N/2) / N) mod p), u < N/2.  Both f0
 * and f1 must satisfy f(r + p/2) = -f(r) mod p.  p <= N. */
FS_API int fs_test_poly_two(uint32_t N, uint32_t p, const int32_t* f0, const int32_t* f1,
                            uint32_t* v_out);

/* FHE-Fire and FHE-Reset program functions (Sec. 4.2) as residue tables:
 * fire[r] = +1 if (r - V_th) mod p < p/2 else -1;
 * reset[r] = leak(r) on [0, V_th), 0 on [V_th, p/2), -leak(r - p/2) on
 * [p/2, p/2 + V_th), 0 on [p/2 + V_th, p), with leak(h) = (tau-1)/tau * h
 * rounded half up (leak = identity for IF).  Either output may be NULL. */
FS_API int fs_lif_luts(const fs_lif* lif, uint32_t p, int32_t* fire, int32_t* reset);

/* Range condition of Theorem 4.1: M = V_th + max |I|, with
 * max |I| = max_o sum_i |W[o][i]| * max(|x_lo|, |x_hi|) over inputs in
 * [x_lo, x_hi].  Writes M to *m_out; returns FS_OK when M <= p/2 and 1 when
 * the condition is violated (the layer then wraps mod p).  W: host [O][I]. */
FS_API int fs_lif_range_check(const fs_lif* lif, uint32_t p, const int32_t* W, size_t O, size_t I,
                       int32_t x_lo, int32_t x_hi, int64_t* m_out);

/* ---------------------------------------------------------------- server */

/* Bind to HIP device `device`. */
FS_API int fs_ctx_create(int device, fs_ctx** ctx);
FS_API int fs_ctx_destroy(fs_ctx* ctx);

/* Pre-size the context's scratch for up to max_jobs bootstrappings per
 * call at ring degree N, so later calls allocate nothing (needed before
 * stream capture into a graph). */
FS_API int fs_ctx_reserve(fs_ctx* ctx, uint32_t N, size_t max_jobs);

/* Device bytes of the context's scratch: *live = the buffers in use now,
 * *retired = buffers replaced by larger ones, held until fs_ctx_destroy
 * (see the conventions above).  Either pointer may be NULL. */
FS_API int fs_ctx_scratch_bytes(const fs_ctx* ctx, size_t* live, size_t* retired);

/* Admission of a serving loop's requests by device memory (the cloud side
 * of Sec. 5.3 accepts encrypted requests while memory allows).  A context
 * carries a budget of device bytes for admitted requests (0 = no budget,
 * the initial state).  fs_ctx_admit(ctx, bytes) admits a request whose
 * buffers take `bytes`: FS_EBUDGET, with nothing admitted, when the bytes
 * already admitted plus `bytes` exceed the budget or when the device
 * reports fewer than `bytes` free; fs_ctx_release gives them back when the
 * request leaves (FS_EINVAL if more than admitted).  The context's own
 * scratch is not counted (fs_ctx_reserve sizes it), so a call on an
 * admitted request never fails for the budget.  fs_ctx_admission reports
 * the budget and the admitted bytes (either pointer may be NULL).  Safe
 * from any host thread. */
FS_API int fs_ctx_set_budget(fs_ctx* ctx, size_t bytes);
FS_API int fs_ctx_admit(fs_ctx* ctx, size_t bytes);
FS_API int fs_ctx_release(fs_ctx* ctx, size_t bytes);
FS_API int fs_ctx_admission(fs_ctx* ctx, size_t* budget, size_t* admitted);

/* Tuning of the blind-rotation kernel.  Every variant computes the same
 * bits; they differ in when the key slice of a digit row is requested
 * (before or after its forward transform), in the register budget the
 * compiler was held to (waves per SIMD), in how many jobs share a workgroup
 * in lockstep, and in which transform roots stay in registers for the whole
 * job.  fs_br_variants(N) returns the
 * number of variants for ring degree N (0 if N is not supported);
 * fs_ctx_set_br_variant selects one for N on this context (default 0).
 * The autotuner times them and picks. */
FS_API int fs_br_variants(uint32_t N);
FS_API int fs_ctx_set_br_variant(fs_ctx* ctx, uint32_t N, int variant);

/* Thread-group form of the blind rotation by batch size, per ring degree N
 * (1024 or 2048; else FS_ENOTSUP).  A launch of B jobs (ciphertexts x
 * program functions) takes the first form whose threshold it does not
 * exceed, in this order; every form computes the same bits:
 *  - rows (fs_ctx_set_rows): one thread group per digit row of the external
 *    product (Sec. 2.1, RGSW product), so a CMux step's critical path is
 *    one forward and one inverse transform: the lowest latency for one
 *    bootstrapping or a few.  At N = 1024 each row is split further into
 *    its two transform halves (2l x 2 waves per job, and the inverse
 *    transforms on four waves); at N = 2048, 2l groups of N/16 threads.
 *    Default: the device's compute units.
 *  - paired (fs_ctx_set_paired, N = 1024 only): the two-group form below
 *    with two jobs per workgroup, so that every SIMD of a CU holds one
 *    wave.  Default: 2 x the compute units at N = 1024, 0 at N = 2048.
 *  - split (fs_ctx_set_split): two groups of N/16 threads per job that split
 *    the accumulator's two polynomials and exchange partial products once
 *    per CMux step.  Default: 3 x the compute units at N = 1024, 0 at
 *    N = 2048.
 *  - otherwise one group per job (full batches).
 * 0 disables a form.  The thresholds of one ring degree leave the other's
 * unchanged.  The previous threshold is stored in *previous unless it is
 * NULL.  The autotuner derives them from timings of every form. */
FS_API int fs_ctx_set_rows(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous);
FS_API int fs_ctx_set_paired(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous);
FS_API int fs_ctx_set_split(fs_ctx* ctx, uint32_t N, size_t max_jobs, size_t* previous);

/* Upload an evaluation key to HBM: the BSK is moved to the NTT domain of
 * the exact negacyclic transform on the device; the KSK is kept as signed
 * byte planes for the matrix-core key switch when its digits are t = 8 of
 * base 4 (the word form is then freed after the conversion), else copied
 * as is.  fs_devkey_bytes reports what stays resident.  Synchronous.  The
 * device key is immutable afterwards and may be shared by calls on any
 * stream of the context's device. */
FS_API int fs_evk_upload(fs_ctx* ctx, const fs_evk* evk, fs_devkey** dk);

/* Key forms of the NTT-domain BSK (fs_evk_upload_form).  The external
 * product of a CMux step (Sec. 2.1, RGSW product) sums (k+1) l N products of
 * digits and key coefficients; the transform returns that integer exactly
 * while it stays below (p_ntt - 1)/2, p_ntt ~ 2^50.6.
 *  FS_KEY_EXACT (fs_evk_upload): exact for every key.  At N = 2048,
 *    Bg = 2^10 the worst case is 2^53, so the 32-bit key coefficients are
 *    split into two 16-bit limbs: twice the pointwise products and the
 *    inverse transforms, twice the key bytes (165 MB).
 *  FS_KEY_ONE_LIMB: the coefficients stay whole (83 MB at N = 2048; the
 *    same as FS_KEY_EXACT at N = 1024).  For a key generated as fs_keygen
 *    does, a step's key rows are uniform words independent of that step's
 *    digits, so every sum is sub-Gaussian with standard deviation at most
 *    2^45.7 (2^44.9 for the uniform digits of a typical step) and passes
 *    (p_ntt - 1)/2, 14.7 of those deviations, with probability below
 *    2^-150 per coefficient (2^-128 per bootstrapping); the outputs are
 *    then the same bits as FS_KEY_EXACT.  (Rows of the body column are
 *    uniform when z is invertible mod 2; otherwise the bound grows by the
 *    index 2^v of the image of multiplication by z.)  A key crafted
 *    against this bound can only corrupt its own results.  Opt-in. */
#define FS_KEY_EXACT 0
#define FS_KEY_ONE_LIMB 1
FS_API int fs_evk_upload_form(fs_ctx* ctx, const fs_evk* evk, int form, fs_devkey** dk);
/* FS_KEY_EXACT or FS_KEY_ONE_LIMB (N = 1024 keys report FS_KEY_EXACT), or
 * a negative error code. */
FS_API int fs_devkey_form(const fs_devkey* dk);
FS_API int fs_devkey_params(const fs_devkey* dk, fs_params* out);
FS_API size_t fs_devkey_bytes(const fs_devkey* dk);
FS_API void fs_devkey_free(fs_devkey* dk);

/* WeightSum on ciphertexts (Sec. 4.1, Eq. "noise grows"):
 * y[o] = add[o] + sum_i W[o][i] * x[i], word by word mod 2^32.
 * W: dev int32 [O][I]; x: dev [I][dim]; add: dev [O][dim] or NULL;
 * y: dev [O][dim]; y == add is allowed (in-place accumulate); otherwise y
 * must not overlap add, and never x.  dim = ciphertext width: n+1 under s, or N+1 for the
 * ciphertexts under z that the key-switch-first order keeps between
 * bootstrappings (fs_pbs_lif_ks_first), hence an argument. */
FS_API int fs_lwe_linear(fs_ctx* ctx, const int32_t* W, size_t O, size_t I, uint32_t dim,
                  const uint32_t* x, const uint32_t* add, uint32_t* y, void* stream);

/* WeightSum of a 2-D convolution over ciphertext feature maps (Sec. 4.1):
 * x: dev [Ci][H][Wd][dim]; W: dev int32 [Co][Ci][K][K];
 * y: dev [Co][Ho][Wo][dim], Ho = (H + 2 pad - K)/stride + 1 (same for Wo);
 * taps falling in the zero padding contribute nothing.  add and dim as
 * above. */
FS_API int fs_lwe_conv2d(fs_ctx* ctx, const int32_t* W, uint32_t Ci, uint32_t H, uint32_t Wd,
                  uint32_t Co, uint32_t K, uint32_t stride, uint32_t pad, uint32_t dim,
                  const uint32_t* x, const uint32_t* add, uint32_t* y, void* stream);

/* Word-wise ciphertext sum y = a + b mod 2^32 (homomorphic addition).
 * a, b, y: dev [words]; y may alias a or b. */
FS_API int fs_lwe_add(fs_ctx* ctx, const uint32_t* a, const uint32_t* b, size_t words, uint32_t* y,
               void* stream);

/* Plaintext addition y = x + Delta c mod 2^32 on the body word of each
 * ciphertext (a trivial encryption of c has zero mask, Sec. 4.1), Delta =
 * 2^32 / p, p a power of two.  x, y: dev [count][dim] (y may alias x);
 * c: dev int32 [count], one plaintext per row. */
FS_API int fs_lwe_add_plain(fs_ctx* ctx, uint32_t p, const uint32_t* x, const int32_t* c,
                            size_t count, uint32_t dim, uint32_t* y, void* stream);

/* Programmable bootstrapping (Sec. 2.1: KeySwitch o Extract o BlindRotate
 * o Initialize) of B ciphertexts with one program function.
 * lut: host [p] residues, negacyclic (else FS_EINVAL).
 * in: dev [B][n+1]; out: dev [B][n+1] when keyswitch != 0, else the
 * extracted LWE_z samples, dev [B][N+1]. */
FS_API int fs_pbs(fs_ctx* ctx, const fs_devkey* dk, const int32_t* lut, const uint32_t* in, size_t B,
           uint32_t* out, int keyswitch, void* stream);

/* One LIF activation of B neurons (Sec. 4.2, Eq. FHE-Fire and
 * Eq. FHE-Reset): both outputs bootstrap the same input LWE(H):
 * spike2_out = bootstrap_Fire(LWE(H)) + 1 = LWE(2S), 2S in {0, 2};
 * v_out = bootstrap_Reset(LWE(H)) = LWE(V').  The threshold is folded into
 * the Fire function.  h, spike2_out, v_out: dev [B][n+1]; v_out may alias h. */
FS_API int fs_pbs_lif(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif, const uint32_t* h, size_t B,
               uint32_t* spike2_out, uint32_t* v_out, void* stream);

/* fs_pbs_lif for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs and bits as fs_pbs_lif, but it calls no hipMalloc,
 * hipFree or allocating library routine: the test polynomials and the
 * extracted samples between the blind rotation and the key switch live in
 * one static device array of the library (33.6 MB per GPU, reserved when the
 * library's code is loaded on that GPU and held until the process ends),
 * whose address fs_ctx_create looks up once per device.
 * Limits: B <= 4096 neurons at N = 1024 and B <= 2048 at N = 2048
 * (2 B (N+1) words of samples must fit 2 x 4096 x 1025), p <= 256; larger
 * batches return FS_EINVAL before any work is enqueued.
 * Every call on one GPU shares that GPU's array, whatever its context, and
 * the array keeps the last call's contents: calls that overlap on one GPU
 * (on two streams, or from two contexts) race and give wrong results.
 * Order them on one stream or synchronise between them. */
FS_API int fs_pbs_lif_noalloc(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif,
                              const uint32_t* h, size_t B, uint32_t* spike2_out,
                              uint32_t* v_out, void* stream);

/* fs_pbs with a change of message space (test polynomial of
 * fs_test_poly_mspace): inputs carry messages of Z_p_in, outputs
 * LWE(f(m)) with Delta_out = 2^32/p_out, e.g. a larger p_out so that the
 * next WeightSum does not wrap, or a smaller one to widen the decryption
 * margin.  Layout, keyswitch and errors as fs_pbs. */
FS_API int fs_pbs_mspace(fs_ctx* ctx, const fs_devkey* dk, const int32_t* lut, uint32_t p_in,
                         uint32_t p_out, const uint32_t* in, size_t B, uint32_t* out,
                         int keyswitch, void* stream);

/* The LIF activation with FHE-Fire and FHE-Reset (Sec. 4.2) read from ONE
 * blind rotation instead of two: the test polynomial interleaves the two
 * tables (fs_test_poly_two), the phase is rounded to even exponents of
 * X (i.e. to Z_N instead of Z_2N), and coefficients 0 and 1 of the
 * rotated accumulator are extracted and key-switched.  Half the blind
 * rotations of fs_pbs_lif, but the modulus-switching error doubles, so
 * decryption margins shrink (at N = 1024, p = 32 the input window is
 * 3.1 standard deviations of that error instead of 6.2).  A different
 * computation from fs_pbs_lif: the outputs are not the same ciphertexts.
 * Needs p <= N.  h, spike2_out, v_out: dev [B][n+1]; v_out may alias h. */
FS_API int fs_pbs_lif_many_lut(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif,
                               const uint32_t* h, size_t B, uint32_t* spike2_out,
                               uint32_t* v_out, void* stream);

/* The LIF activation in the key-switch-first order (the bootstrapping of
 * Sec. 2.1 with its Key Switching step moved in front of the Blind
 * Rotation): LWE_z(H) is key-switched to LWE_s(H) once, then blind-rotated
 * with the Fire and Reset functions and extracted, so the outputs stay
 * under z and carry the blind-rotation noise only (no key-switch noise),
 * and one key switch serves both functions.
 * h, spike2_out, v_out: dev [B][N+1] under z; spike2_out = LWE(2S),
 * v_out = LWE(V') as in fs_pbs_lif.  Either output may alias h; the two
 * outputs may not alias each other.  Uses the context's scratch. */
FS_API int fs_pbs_lif_ks_first(fs_ctx* ctx, const fs_devkey* dk, const fs_lif* lif,
                               const uint32_t* h, size_t B, uint32_t* spike2_out,
                               uint32_t* v_out, void* stream);

/* One contiguous range of LIF neurons of one client for fs_pbs_lif_ranges:
 * its evaluation key and its h / spike2_out / v_out rows (as in
 * fs_pbs_lif), count neurons. */
typedef struct fs_lif_range {
  const fs_devkey* key;
  const uint32_t* h;
  uint32_t* spike2_out;
  uint32_t* v_out;
  size_t count;
} fs_lif_range;

/* fs_pbs_lif over many ranges in one blind-rotation launch (continuous
 * batching across requests and clients): every neuron of every range is
 * bootstrapped with its own range's key; results are bit-identical to one
 * fs_pbs_lif call per range.  All keys must share one parameter set and
 * device; ranges of one key are key-switched together.  ranges: host
 * [nranges].  The context's scratch and range table are reused by the next
 * call: calls on one context must not overlap (use one context per
 * stream).  The range table is copied from host memory at the call, so the
 * call cannot be captured into a graph: on a capturing stream it returns
 * FS_ENOTSUP. */
FS_API int fs_pbs_lif_ranges(fs_ctx* ctx, const fs_lif* lif, const fs_lif_range* ranges,
                             size_t nranges, void* stream);

/* fs_pbs_lif_ranges with the one-rotation activation of fs_pbs_lif_many_lut
 * (Fire and Reset read from one even-exponent blind rotation per neuron;
 * its doubled rounding error applies).  Same ranges, keys and outputs. */
FS_API int fs_pbs_lif_ranges_many_lut(fs_ctx* ctx, const fs_lif* lif, const fs_lif_range* ranges,
                                      size_t nranges, void* stream);

/* Key switching z -> s alone (Sec. 2.1, Key Switching step).
 * in: dev [B][N+1] under z; out: dev [B][n+1] under s; the key must live
 * on the context's device (else FS_EPARAM). */
FS_API int fs_keyswitch(fs_ctx* ctx, const fs_devkey* dk, const uint32_t* in, size_t B, uint32_t* out,
                 void* stream);

/* Negacyclic product through the device's exact NTT (the transform used by
 * blind rotation; exposed to check it against schoolbook products):
 * out = sum_{r<R} d_r(X) b_r(X) in Z_{2^32}[X]/(X^N+1).
 * d: dev int32 [R][N] with |d| <= dmax; b: dev uint32 [R][N]; out: dev [N].
 * N in {1024, 2048}; FS_EINVAL unless R*N*dmax*2^31 < p_ntt/2 (the
 * exactness bound of the transform; for N = 2048 the b_r are split in two
 * 16-bit halves internally, as the blind rotation does). */
FS_API int fs_ntt_polymul(fs_ctx* ctx, uint32_t N, uint32_t R, int32_t dmax, const int32_t* d,
                   const uint32_t* b, uint32_t* out, void* stream);

/* ---------------------------------------------------------- measurement */

/* Issue-rate ceiling of the binary64 vector ALU, which bounds the blind
 * rotation (its exact modular arithmetic; Sec. 2.1, RGSW product).  Runs
 * one register-only kernel on `device` with exactly waves_per_simd (1..8)
 * waves on every SIMD and stores the lane-instructions per second it
 * issued (and the kernel time in *ms unless NULL).  kind 0: butterflies of
 * the modular product (8 instructions each, the transforms' inner step);
 * 1: modular multiply-accumulate (7, the pointwise products, plus one add
 * that keeps its operand loop-carried); 2: bare fused multiply-add (1).  Allocates and frees its own small buffer;
 * synchronous; the caller's current device is restored. */
FS_API int fs_probe_valu(int device, uint32_t waves_per_simd, uint32_t kind,
                         double* lane_instr_per_s, double* ms);

/* HBM streaming ceiling: a device copy of bytes/2 into bytes/2 (bytes
 * >= 1 MiB), timed over five launches; stores bytes moved per second (read
 * plus written) and the time per copy in *ms unless NULL.  Allocates and
 * frees its buffers; synchronous. */
FS_API int fs_probe_hbm(int device, size_t bytes, double* bytes_per_s, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* FHESNN_H */
