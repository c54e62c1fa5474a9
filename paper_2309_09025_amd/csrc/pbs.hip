// Programmable bootstrapping on gfx950: BSK conversion to the NTT domain,
// blind rotation with fused initialisation and sample extraction, key
// switching with the LIF epilogue, and an NTT polynomial-product check.
//
// Sec. 2.1, Theorem 2.1 and the four steps after it (Initialization, Blind
// Rotation, Sample Extraction, Key Switching); Sec. 4.2 (FHE-Fire adds 1
// after bootstrapping).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "ntt_fp64.h"

namespace fs {

// ---------------------------------------------------------------------------
// BSK: coefficient domain [n][rows][2][N] (Torus32) -> NTT domain, layout
// [n][rows][16][TP][2 * limbs] doubles, so that in the blind rotation thread
// t of the polynomial reads, for register r, one contiguous group of
// 2*limbs values (mask and body product of digit row `row`).
// limbs = 1: the centred 32-bit coefficient; limbs = 2: its low and high
// signed 16-bit halves (coefficient = lo + 2^16 hi).
template <int LOGN, int LIMBS>
__global__ void __launch_bounds__(NttShape<LOGN>::TP)
bsk_to_ntt_kernel(const uint32_t* __restrict__ bsk, double* __restrict__ out, uint32_t rows,
                  const double* __restrict__ tw) {
  using S = NttShape<LOGN>;
  __shared__ double lds[S::LDS_DOUBLES];
  const int t = threadIdx.x;
  const uint32_t poly = blockIdx.x;       // (i*rows + row)*2 + o
  const uint32_t limb = blockIdx.y;       // < LIMBS
  const uint32_t o = poly & 1, irow = poly >> 1;
  const uint32_t* src = bsk + (size_t)poly * S::N;
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int32_t c = (int32_t)src[t + S::TP * r];
    if (LIMBS == 1) {
      x[r] = (double)c;
    } else {
      const int32_t lo = (int32_t)(int16_t)(uint16_t)(uint32_t)c;
      const int32_t hi = (c - lo) >> 16;
      x[r] = (double)(limb == 0 ? lo : hi);
    }
  }
  ntt_fwd<LOGN>(x, lds, tw, t);
  double* dst = out + (size_t)irow * 16 * S::TP * 2 * LIMBS;
#pragma unroll
  for (int r = 0; r < 16; ++r) dst[((size_t)r * S::TP + t) * 2 * LIMBS + o * LIMBS + limb] = x[r];
}

// The first two forward stages of a digit row by table (small digit ranges).
// Stage LOGN-1 pairs registers r and r + 8 with the root i = psi^{brv(1)},
// stage LOGN-2 pairs r and r + 4 with w = psi^{brv(2)} (r < 8) or
// psi^{brv(3)} = i psi^{brv(2)} (r >= 8).  For the digits d0..d3 of
// registers r, r + 4, r + 8, r + 12 (r < 4) the first stage gives
// d0 +- i d2 and d1 +- i d3, and the second stage's products are
//   (d1 + i d3) w2 = d1 w2 + d3 w3,   (d1 - i d3) w3 = d1 w3 + d3 w2,
// so a row needs three tables of d * root over the 2 HALF field values
// f = d + HALF, stored reduced: tab = [d i | d w2 | d w3].  Outputs are
// congruent to the arithmetic stages' and bounded by 1.5 P + 64.
template <uint32_t HALF>
__device__ __forceinline__ void fill_stage_tables(double* tab, const UniTw& u, int tid, int nt) {
  constexpr int TW = 2 * HALF;
  for (int f = tid; f < 3 * TW; f += nt)
    tab[f] = redc(mulmod((double)(f % TW - (int)HALF), u.fwd[1 + f / TW]));
}

template <int BG>
__device__ __forceinline__ void digit_row_two_stages(const uint32_t d[16], uint32_t sh,
                                                     const double* tab, double xd[16]) {
  constexpr uint32_t HALF = 1u << (BG - 1);
  constexpr int TW = 2 * HALF;
  // All twelve lookups of the row are requested before any is used (the
  // scheduling barrier keeps the compiler from interleaving them with the
  // sums, which it otherwise does into one set of registers, waiting for
  // each group of three in turn).
  double m1[4], a1[4], b1[4], a3[4], b3[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t f1 = __builtin_amdgcn_ubfe(d[r + 4], sh, BG);
    const uint32_t f2 = __builtin_amdgcn_ubfe(d[r + 8], sh, BG);
    const uint32_t f3 = __builtin_amdgcn_ubfe(d[r + 12], sh, BG);
    m1[r] = tab[f2];
    a1[r] = tab[TW + f1];
    b1[r] = tab[2 * TW + f1];
    a3[r] = tab[TW + f3];
    b3[r] = tab[2 * TW + f3];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double d0 = (double)((int32_t)__builtin_amdgcn_ubfe(d[r], sh, BG) - (int32_t)HALF);
    const double lo = d0 + m1[r], hi = d0 - m1[r];
    const double ma = a1[r] + b3[r];
    const double mb = b1[r] + a3[r];
    xd[r] = lo + ma;
    xd[r + 4] = lo - ma;
    xd[r + 8] = hi + mb;
    xd[r + 12] = hi - mb;
  }
}

// ---------------------------------------------------------------------------
// Blind rotation.  One workgroup of TP threads per job (ciphertext, test
// polynomial); the accumulator lives in LDS in natural order for all n
// CMux steps.  Step i (a~ = a~_i != 0):
//   D_c = X^{a~} ACC_c - ACC_c (c = 0 mask, 1 body)
//   for each gadget level j: digit polynomial -> forward NTT -> multiply by
//       the two NTT-domain TGSW_i row entries and accumulate
//   inverse NTT of the two accumulators -> exact integers -> ACC_c +=
// Initialization ACC = (0, X^{-b~} v) and sample extraction of
// coefficient 0 are fused at both ends; the key switch of the batch follows
// in keyswitch_mfma_kernel.
//
// Latency: the key slice of a digit row (16 registers x 2*limbs values per
// thread) is requested at a point set by PF and consumed after the row's
// forward transform: PF = 0 after the transform, in two halves; 1 first half
// before the transform, second after it; 2 the whole slice before; 3 after
// the transform in quarters (fewest live registers: the N = 2048 job fits
// two waves per SIMD only this way).  The roots shared by all threads come
// from the kernel-argument segment and the per-thread ones are requested one
// round ahead.  WPE is the number of waves per SIMD the register allocation
// must allow.
//
// W = 2 splits one job over two polynomial groups of TP threads (two waves
// at N = 1024), for batches too small to fill the device: group c
// decomposes and transforms the digits of D_c only, accumulating partial
// products for both outputs; once per step the groups swap the partial sums
// of the other's output through LDS, and group c inverse-transforms and
// updates ACC_c.  Each group reads only its own ACC_c, so the only
// cross-group synchronisation is the swap.
//
// JPW = 2 puts two such jobs in one workgroup (four waves at N = 1024), so
// that a batch of up to 2 x CUs jobs occupies every SIMD once: two separate
// two-wave workgroups on one CU may share two of its SIMDs.  Both jobs then
// pass the same workgroup barriers, so neither skips a step (a step with
// a~_i = 0 adds zero, so the bits are the same); the last workgroup of a
// batch that JPW does not divide repeats the last job without writing.
//
// JPW > 1 with W = 1 (lockstep form): the jobs a CU holds at once share one
// workgroup and a barrier at the end of every CMux step, so they read the
// same key rows within a short window and all but the first find them in
// the CU's L1 (one step's slice is 96 KiB at N = 1024, a digit row 16 KiB),
// where separate workgroups drift apart and each streams the key from L2.
template <int LOGN, int L, int BG, int LIMBS, int PF, int WPE, int W, int JPW = 1,
          bool HELD = false, int HELDI = 0>
__global__ void __launch_bounds__(JPW * W * NttShape<LOGN>::TP, WPE)
blind_rotate_kernel(BrArgs a) {
  using S = NttShape<LOGN>;
  constexpr int N = S::N, TP = S::TP, ROWS = 2 * L;
  constexpr uint32_t HALF = 1u << (BG - 1);
  constexpr uint32_t NU = LOGN + 1;  // log2(2N)
  constexpr int G = 2 * LIMBS;       // key values per slot and digit row
  static_assert(W == 1 || W == 2, "one or two polynomial groups per job");
  static_assert(JPW == 1 || W == 1 || (JPW == 2 && W == 2), "paired jobs use two groups each");
  static_assert(16 * TP <= S::LDS_DOUBLES, "a partial sum fits an exchange buffer");
  __shared__ double lds_all[JPW * W][S::LDS_DOUBLES];
  __shared__ uint32_t acc_all[JPW][2][N];
  // one-group jobs of several waves use the lean exchange schedule (see
  // exchange): one workgroup barrier per cross-wave exchange and one on
  // entry to a transform instead of two per exchange.  The split form keeps
  // the default, its partial-sum swap reuses the exchange buffers.
  constexpr bool LEAN = W == 1;
  // first two forward stages by table (digit_row_two_stages): their
  // operands are raw digits, so the products take only 2 HALF values per
  // root.  Used for small digit ranges (Bg = 2^7: 3 x 128 entries, which
  // still lets 8 jobs share a CU's LDS); at Bg = 2^10 a one-stage table of
  // 1,024 entries measured no gain.
  constexpr bool TAB1 = 2 * HALF <= 256;
  __shared__ double stage1[TAB1 ? 6 * HALF : 1];

  // job of the workgroup (uniform per wave, so kept in a scalar register)
  const int js = JPW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x / (W * TP));
  const int ltid = (int)threadIdx.x - js * W * TP;             // thread within the job
  const int grp = W == 1 ? 0 : ltid / TP;                      // polynomial group
  const int t = ltid - grp * TP;
  double* lds = lds_all[js * W + grp];
  uint32_t(*acc)[N] = acc_all[js];
  size_t job = (size_t)blockIdx.x * JPW + js;
  const bool writes = JPW == 1 || job < a.jobs;
  if (!writes) job = a.jobs - 1;
  const uint32_t n = a.n;
  // ciphertext and program function of this job (nlut is 1 or 2: shifts,
  // which stay on the scalar unit, unlike a 64-bit division)
  const uint64_t g = a.nlut == 2 ? job >> 1 : job;
  const uint32_t lut = a.nlut == 2 ? (uint32_t)(job & 1u) : 0u;
  const uint32_t* ct;
  const double* bsk;
  if (a.ranges) {  // multi-key launch: the range of g gives input and key
    const JobRange& rg = a.ranges[find_range(a.ranges, a.nranges, g)];
    ct = rg.in + (g - rg.first) * (size_t)(n + 1);
    bsk = rg.bsk;
  } else {
    ct = a.in + g * (size_t)(n + 1);
    bsk = a.bsk;
  }
  // both depend on the workgroup only: pin them to scalar registers, so the
  // key's buffer descriptor is provably uniform (a descriptor the compiler
  // sees in vector registers costs a waterfall loop around every load)
  ct = uniform_ptr(ct);
  bsk = uniform_ptr(bsk);
  const Tab key(bsk), fwd_tw(a.fwd_tw), inv_tw(a.inv_tw), post(a.post);
  const uint32_t* v = lut == 0 ? a.tpoly0 : a.tpoly1;
  // the accumulator polynomials this group decomposes and updates
  constexpr int NC = W == 1 ? 2 : 1;
  const int c0 = W == 1 ? 0 : grp;

  // gadget rounding offset: sum_{j=1..L} (Bg/2) 2^{32 - j BG} + 2^{31 - L BG}
  uint32_t off = 1u << (31 - L * BG);
#pragma unroll
  for (int j = 1; j <= L; ++j) off += HALF << (32 - j * BG);

  // modulus switch: round to Z_2N, or to its even elements (Z_N doubled)
  const uint32_t even = __builtin_amdgcn_readfirstlane(a.even);
  const uint32_t msh = 32 - NU + even, mhalf = 1u << (msh - 1);
  auto mod_switch = [=](uint32_t x) { return ((x + mhalf) >> msh) << even; };

  if constexpr (TAB1) {
    fill_stage_tables<HALF>(stage1, a.uni, threadIdx.x, JPW * W * TP);
    if constexpr (JPW * W * TP > 64) __syncthreads();  // every wave reads the whole table
  }

  // HELD: the forward transforms' per-thread roots, loaded once for the job
  // (they depend on the thread only) instead of once per transform
  double held[HELD ? RegTw<LOGN>::FWD : 1];
  if constexpr (HELD) load_fwd_roots<LOGN>(held, fwd_tw, t);
  // HELDI: likewise the inverse transforms' roots of round B' (1) or of
  // rounds B' and A' (2)
  double heldi[HELDI ? RegTw<LOGN>::IB + (HELDI == 2 ? RegTw<LOGN>::IA : 0) : 1];
  if constexpr (HELDI) load_inv_roots<LOGN, HELDI>(heldi, inv_tw, t);

  // Initialization: ACC = (0, X^{-b~} v), b~ = round(b 2N / 2^32)
  {
    const uint32_t bbar = mod_switch(ct[n]);
    const uint32_t e = (2 * N - bbar) & (2 * N - 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = t + TP * r;
      // (X^e v)_j = v_{j-e} with sign (-1)^{number of wraps past N}
      int src = j - (int)e;
      uint32_t val;
      if (src >= 0) val = v[src];
      else if (src + N >= 0) val = 0u - v[src + N];
      else val = v[src + 2 * N];
      if (c0 == 0) acc[0][j] = 0u;
      if (c0 + NC == 2) acc[1][j] = val;
    }
  }
  poly_sync<TP>();

  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t abar = mod_switch(ct[i]);
    // X^0 ACC - ACC = 0: every digit is zero (paired jobs keep in step)
    if (JPW == 1 && abar == 0) continue;
    double p0[LIMBS][16], p1[LIMBS][16], xd[16];
#pragma unroll
    for (int lb = 0; lb < LIMBS; ++lb)
#pragma unroll
      for (int r = 0; r < 16; ++r) { p0[lb][r] = 0.0; p1[lb][r] = 0.0; }

    // byte offset of step i's key slice (< 2^31: n * 2l * 16 * TP * G * 8)
    const uint32_t key_i = i * (uint32_t)(ROWS * 16 * TP * G * 8);
#pragma unroll 1
    for (int c = c0; c < c0 + NC; ++c) {
      // D_c = X^{a~} ACC_c - ACC_c plus the gadget offset.  Coefficient j of
      // X^{a~} ACC is ACC[k mod N] with k = j - a~ in (-2N, N), negated when
      // k mod 2N >= N (one wrap past X^N = -1).
      uint32_t d[16];
      const uint32_t* ac = acc[c];
      // The rotated indices and signs are the same for both polynomials; the
      // empty asm makes the compiler form them again for each one instead of
      // keeping 3 x 16 registers alive across the step, which cost the N =
      // 2048 job its second wave per SIMD (and the N = 1024 key-first
      // variant its spill-free allocation).
      int kb = t - (int)abar;
      asm volatile("" : "+v"(kb));
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = kb + TP * r;
        const uint32_t v = ac[k & (N - 1)];
        const uint32_t neg = 0u - (((uint32_t)k >> LOGN) & 1u);
        d[r] = ((v ^ neg) - neg) - ac[t + TP * r] + off;
      }
#pragma unroll 1
      for (int lv = 0; lv < L; ++lv) {
        const uint32_t row = key_i + (uint32_t)((c * L + lv) * 16 * TP * G * 8);
        double g[16][G];
        constexpr int KCH = PF == 3 ? 4 : 8;  // registers per key request
        auto load_part = [&](int h) __attribute__((always_inline)) {
#pragma unroll
          for (int r = KCH * h; r < KCH * h + KCH; ++r)
#pragma unroll
            for (int q = 0; q < G; q += 2)
              key.at2((uint32_t)t * (G * 8), row + (uint32_t)((r * TP * G + q) * 8), g[r][q],
                      g[r][q + 1]);
        };
        auto mac_part = [&](int h) __attribute__((always_inline)) {
#pragma unroll
          for (int r = KCH * h; r < KCH * h + KCH; ++r)
#pragma unroll
            for (int lb = 0; lb < LIMBS; ++lb) {
              p0[lb][r] += mulmod(xd[r], g[r][lb]);
              p1[lb][r] += mulmod(xd[r], g[r][LIMBS + lb]);
            }
        };
        if constexpr (PF == 1 || PF == 2) load_part(0);
        if constexpr (PF == 2) load_part(1);
        const uint32_t sh = 32 - (lv + 1) * BG;
        if constexpr (TAB1) {
          digit_row_two_stages<BG>(d, sh, stage1, xd);
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r)
            xd[r] = (double)((int32_t)__builtin_amdgcn_ubfe(d[r], sh, BG) - (int32_t)HALF);
        }
        // entry barrier of the exchange buffer: not before a step's first
        // transform (the previous step ended with one)
        ntt_fwd_reg<LOGN, TAB1 ? 2 : 0, LEAN, HELD>(xd, lds, a.uni, fwd_tw, t,
                                                    c != c0 || lv != 0, held);
        if constexpr (PF == 0 || PF == 3) {
#pragma unroll
          for (int h = 0; h < 16 / KCH; ++h) {
            load_part(h);
            mac_part(h);
          }
        } else if constexpr (PF == 1) {
          load_part(1);
          mac_part(0);
          mac_part(1);
        } else {
          mac_part(0);
          mac_part(1);
        }
      }
    }
    if constexpr (W == 2) {
      // swap partial sums: group c keeps the sums for output c and adds the
      // other group's (both in the same round-C register mapping)
#pragma unroll
      for (int lb = 0; lb < LIMBS; ++lb) {
        const double* mine_other = grp == 0 ? p1[lb] : p0[lb];
        double* mine = grp == 0 ? p0[lb] : p1[lb];
        if (lb > 0) __syncthreads();  // the other group has read the previous limb
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[r * TP + t] = mine_other[r];
        __syncthreads();
        const double* theirs = lds_all[js * W + 1 - grp];
#pragma unroll
        for (int r = 0; r < 16; ++r) mine[r] += theirs[r * TP + t];
      }
      __syncthreads();  // both swaps read before the buffers are reused
    }
    // inverse transforms; p* hold sums of 2L products of transformed digits
    // (|x| < 2 P, not reduced) with reduced key values: < 5 P
#pragma unroll
    for (int c = c0; c < c0 + NC; ++c) {
      uint32_t upd[16];
#pragma unroll
      for (int lb = 0; lb < LIMBS; ++lb) {
        double* y = c == 0 ? p0[lb] : p1[lb];
        // the first inverse follows a forward transform's round-C reads of
        // this wave's own half: no entry barrier
        ntt_inv_reg<LOGN, LEAN, HELDI>(y, lds, a.uni, inv_tw, post, t, c != c0 || lb != 0,
                                       heldi);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t part = low32_magic(y[r]);
          upd[r] = lb == 0 ? part : upd[r] + (part << 16);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][t + TP * r] += upd[r];
    }
    // one-group jobs sharing a workgroup stay in step (lockstep form): the
    // key rows the first of them loads are still in the CU's L1 when the
    // others read them
    if constexpr (W == 1 && JPW > 1) __syncthreads();
    else poly_sync<TP>();
  }
  if constexpr (W == 2) __syncthreads();  // the extraction reads both accumulators

  // Sample Extraction of coefficient k (negacyclic reversal of the mask):
  // a'_j = a_{k-j} for j <= k, -a_{N+k-j} otherwise; b' = b_k.  Coefficient
  // 0 always, coefficient 1 too when two functions share the rotation.
  const int tid = ltid;
  if (!writes) return;
#pragma unroll
  for (uint32_t k = 0; k < 2; ++k) {
    if (k > even) break;
    const uint32_t fn = even ? k : lut;  // program function of this output
    uint32_t* out;
    uint32_t plain = 0u;
    if (a.out0) {
      out = (fn == 0 ? a.out0 : a.out1) + g * (size_t)(N + 1);
      plain = a.plain_b[fn];
    } else {
      out = a.ext + (even ? 2 * job + k : job) * (size_t)(N + 1);
    }
    out = uniform_ptr(out);
#pragma unroll
    for (int r = 0; r < 16 / W; ++r) {
      const int j = tid + W * TP * r;
      out[j] = j <= (int)k ? acc[0][k - j] : 0u - acc[0][N + k - j];
    }
    if (tid == 0) out[N] = acc[1][k] + plain;
  }
}

// ---------------------------------------------------------------------------
// Blind rotation for latency (small batches): one thread group of TP threads
// per digit row, 2l groups per job.  Group g = c l + lv rotates ACC_c,
// extracts digit level lv, transforms it and multiplies it with its key row
// for both outputs (and both key limbs at N = 2048); the products of all
// rows are summed in LDS with exact binary64 atomic adds (integers below
// 5 P < 2^53, so the order of the additions cannot change the sum).  Then
// 2 x limbs groups inverse-transform one (output, limb) sum each and add
// its low 32 bits (shifted by 16 per limb) into ACC with 32-bit atomics
// (wrapping mod 2^32, again order-free).  A step's critical path is one
// forward and one inverse transform.  Same bits as blind_rotate_kernel.
// Launched at N = 2048; at N = 1024 blind_rotate_halfrow_kernel (below)
// spreads the same work over all four SIMDs.
template <int LOGN, int L, int BG, int LIMBS>
__global__ void __launch_bounds__(2 * L * NttShape<LOGN>::TP)
blind_rotate_rows_kernel(BrArgs a) {
  using S = NttShape<LOGN>;
  constexpr int N = S::N, TP = S::TP, ROWS = 2 * L, NT = ROWS * TP;
  constexpr int NINV = 2 * LIMBS;  // inverse transforms per step
  constexpr uint32_t HALF = 1u << (BG - 1);
  constexpr uint32_t NU = LOGN + 1;
  constexpr int G = 2 * LIMBS;  // key values per slot: outputs x limbs
  constexpr bool TAB1 = 2 * HALF <= 256;
  static_assert(NINV <= ROWS, "an inverse transform per (output, limb) group");
  // groups of several wavefronts synchronise their exchanges with workgroup
  // barriers, so then every group must run the same transforms
  static_assert(TP == 64 || NINV == ROWS, "uniform barrier sequence");
  __shared__ double lds_all[ROWS][S::LDS_DOUBLES];
  __shared__ double sums[2][LIMBS][16 * TP];  // [output][limb][r][t]
  __shared__ uint32_t acc[2][N];
  __shared__ double stage1[TAB1 ? 6 * HALF : 1];

  const int grp = (int)threadIdx.x / TP;
  const int t = (int)threadIdx.x - grp * TP;
  const int c = grp / L, lv = grp % L;
  double* lds = lds_all[grp];
  const size_t job = blockIdx.x;
  const uint32_t n = a.n;
  const uint64_t g = a.nlut == 2 ? job >> 1 : job;
  const uint32_t lut = a.nlut == 2 ? (uint32_t)(job & 1u) : 0u;
  const uint32_t* ct;
  const double* bsk;
  if (a.ranges) {
    const JobRange& rg = a.ranges[find_range(a.ranges, a.nranges, g)];
    ct = rg.in + (g - rg.first) * (size_t)(n + 1);
    bsk = rg.bsk;
  } else {
    ct = a.in + g * (size_t)(n + 1);
    bsk = a.bsk;
  }
  ct = uniform_ptr(ct);
  bsk = uniform_ptr(bsk);
  const Tab key(bsk), fwd_tw(a.fwd_tw), inv_tw(a.inv_tw), post(a.post);
  const uint32_t* v = lut == 0 ? a.tpoly0 : a.tpoly1;

  uint32_t off = 1u << (31 - L * BG);
#pragma unroll
  for (int j = 1; j <= L; ++j) off += HALF << (32 - j * BG);
  const uint32_t even = __builtin_amdgcn_readfirstlane(a.even);
  const uint32_t msh = 32 - NU + even, mhalf = 1u << (msh - 1);
  auto mod_switch = [=](uint32_t x) { return ((x + mhalf) >> msh) << even; };

  const int tid = threadIdx.x;
  if constexpr (TAB1) fill_stage_tables<HALF>(stage1, a.uni, tid, NT);
  for (int j = tid; j < 2 * LIMBS * 16 * TP; j += NT) (&sums[0][0][0])[j] = 0.0;
  {
    const uint32_t bbar = mod_switch(ct[n]);
    const uint32_t e = (2 * N - bbar) & (2 * N - 1);
    for (int j = tid; j < N; j += NT) {
      const int src = j - (int)e;
      uint32_t val;
      if (src >= 0) val = v[src];
      else if (src + N >= 0) val = 0u - v[src + N];
      else val = v[src + 2 * N];
      acc[0][j] = 0u;
      acc[1][j] = val;
    }
  }
  __syncthreads();

  const uint32_t sh = 32 - (lv + 1) * BG;
  // key slice of this group's row: registers [r0, r0 + RN) of the 16
  double kv[16][G];
  auto load_key = [&](uint32_t row, int r0, int rn) __attribute__((always_inline)) {
#pragma unroll
    for (int r = r0; r < r0 + rn; ++r)
#pragma unroll
      for (int q = 0; q < G; q += 2)
        key.at2((uint32_t)t * (G * 8), row + (uint32_t)((r * TP * G + q) * 8), kv[r][q],
                kv[r][q + 1]);
  };
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t abar = mod_switch(ct[i]);
    if (abar == 0) continue;
    const uint32_t row = i * (uint32_t)(ROWS * 16 * TP * G * 8) +
                         (uint32_t)(grp * 16 * TP * G * 8);
    // the key row is requested before the transform (half of it when it is
    // two limbs wide, to bound the registers held across the transform)
    constexpr int PRE = G == 2 ? 16 : 8;
    load_key(row, 0, PRE);
    // digit level lv of D_c = X^{a~} ACC_c - ACC_c (plus the rounding offset)
    double xd[16];
    {
      uint32_t d[16];
      const uint32_t* ac = acc[c];
      const int kb = t - (int)abar;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = kb + TP * r;
        const uint32_t val = ac[k & (N - 1)];
        const uint32_t neg = 0u - (((uint32_t)k >> LOGN) & 1u);
        d[r] = ((val ^ neg) - neg) - ac[t + TP * r] + off;
      }
      if constexpr (TAB1) {
        digit_row_two_stages<BG>(d, sh, stage1, xd);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          xd[r] = (double)((int32_t)__builtin_amdgcn_ubfe(d[r], sh, BG) - (int32_t)HALF);
      }
    }
    ntt_fwd_reg<LOGN, TAB1 ? 2 : 0>(xd, lds, a.uni, fwd_tw, t);
    if constexpr (PRE < 16) load_key(row, PRE, 16 - PRE);
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int q = 0; q < G; ++q)  // q = output * LIMBS + limb
        atomicAdd(&sums[q / LIMBS][q % LIMBS][r * TP + t], mulmod(xd[r], kv[r][q]));
    __syncthreads();  // every row's products are in; every rotation has read ACC
    if (grp < NINV) {
      const int co = grp / LIMBS, lb = grp % LIMBS;
      double y[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        y[r] = sums[co][lb][r * TP + t];
        sums[co][lb][r * TP + t] = 0.0;  // cleared for the next step
      }
      ntt_inv_reg<LOGN>(y, lds, a.uni, inv_tw, post, t);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t part = low32_magic(y[r]) << (16 * lb);
        if constexpr (LIMBS == 1) acc[co][t + TP * r] += part;
        else atomicAdd(&acc[co][t + TP * r], part);
      }
    }
    __syncthreads();  // ACC updated and the sums cleared before the next step
  }

#pragma unroll
  for (uint32_t k = 0; k < 2; ++k) {
    if (k > even) break;
    const uint32_t fn = even ? k : lut;
    uint32_t* out;
    uint32_t plain = 0u;
    if (a.out0) {
      out = (fn == 0 ? a.out0 : a.out1) + g * (size_t)(N + 1);
      plain = a.plain_b[fn];
    } else {
      out = a.ext + (even ? 2 * job + k : job) * (size_t)(N + 1);
    }
    out = uniform_ptr(out);
    for (int j = tid; j < N; j += NT) out[j] = j <= (int)k ? acc[0][k - j] : 0u - acc[0][N + k - j];
    if (tid == 0) out[N] = acc[1][k] + plain;
  }
}

// ---------------------------------------------------------------------------
// Blind rotation for latency at N = 1024 in half rows.  After the first
// forward stage (pairs j, j + N/2) the two halves of a digit row's
// transform are independent: the remaining stages act within each half with
// the roots of the full transform.  Likewise the inverse's stages 0 .. 8 act
// within the halves of the bit-reversed order, and only its last stage
// pairs i with i + N/2.  So a job runs as 2l x 2 = 12 waves, one per (digit
// row, half), 8 values per thread, three per SIMD in the forward phase (one
// wave per row would put two rows on two of the four SIMDs), and the
// 2 x 2 (output, half) inverse transforms run on four waves, one per SIMD.
// The stages, roots, reduction points and products are those of the other
// kernels, so the bits are the same.
//
// A half of 512 values is held by 64 threads, 8 values each; exponent bits
// [LO, LO + 3) of its index live in the register number:
//     j'(t, r) = (t & (2^LO - 1)) | (r << LO) | ((t >> LO) << (LO + 3)),
// with forward rounds at LO = 6 (stages 7, 6), 3 (5, 4, 3) and 0 (2, 1, 0)
// and the inverse walking them back (stages 0-2, 3-5, 6-8).
template <int LO>
__device__ __forceinline__ int hmap(int t, int r) {
  return (t & ((1 << LO) - 1)) | (r << LO) | ((t >> LO) << (LO + 3));
}

// Exchange of one wave's half between register mappings through its own LDS
// buffer (in-order within the wave: compiler fences only).  The padded slot
// of j'(t, r) splits into a thread part and a register part as in exchange.
template <int FROM, int TO>
__device__ __forceinline__ void hexchange(double x[8], double* lds, int t) {
  double* wp = lds + lds_slot(hmap<FROM>(t, 0));
  const double* rp = lds + lds_slot(hmap<TO>(t, 0));
#pragma unroll
  for (int r = 0; r < 8; ++r) wp[lds_slot(r << FROM)] = x[r];
  wave_sync();
#pragma unroll
  for (int r = 0; r < 8; ++r) x[r] = rp[lds_slot(r << TO)];
  wave_sync();
}

__device__ __forceinline__ void reduce8(double x[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) x[r] = redc(x[r]);
}

// One forward stage in a round (the butterfly of fwd_stages_reg): pairs
// registers r and r | 2^b, root w[r >> (b+1)].
template <int B, int NW>
__device__ __forceinline__ void hfwd_stage(double x[8], const double* w) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << B)) continue;
    const int r2 = r | (1 << B);
    const double m = mulmod(x[r2], w[(r >> (B + 1)) % NW]);
    x[r2] = x[r] - m;
    x[r] = x[r] + m;
  }
}

// Inverse stage in a round: pairs r and r | 2^b, root w[r & (2^b - 1)].
template <int B>
__device__ __forceinline__ void hinv_stage(double x[8], const double* w) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << B)) continue;
    const int r2 = r | (1 << B);
    const double m = mulmod(x[r2], w[r & ((1 << B) - 1)]);
    x[r2] = x[r] - m;
    x[r] = x[r] + m;
  }
}

// Per-thread roots of half h, loaded once per job.  Forward (index k of
// psi^{brv(k)}, stage s: k = N/2^{s+1} + j/2^{s+1}, j = 512 h + j'):
//   round B: stage 5: 16 + 8h + t/8; 4: 32 + 16h + 2(t/8) + e; 3: 64 + 32h + 4(t/8) + e
//   round C: stage 2: 128 + 64h + t; 1: 256 + 128h + 2t + e; 0: 512 + 256h + 4t + e
// Inverse (index e of omega^-e, stage s: e = (i mod 2^s) N/2^{s+1}; the
// halves share stages 0-8):
//   round B': stage 3: 64 (t&7); 4: 32 ((t&7) | 8e); 5: 16 ((t&7) | 8e)
//   round A': stage 6: 8t; 7: 4 (t | 64e); 8: 2 (t | 64e)
//   stage 9: i' = t | 64 r; twist psi^-j N^-1 at j = 512 h + t + 64 r.
struct HalfRoots {
  double f5, f4[2], f3[4], f2, f1[2], f0[4];
};
// inverse roots of a thread, by stage: offsets into HalfInvRoots::w
enum HalfInv { kI3 = 0, kI4 = 1, kI5 = 3, kI6 = 7, kI7 = 8, kI8 = 10, kI9 = 14, kTw = 22,
               kHalfInvRoots = 30 };
struct HalfInvRoots {
  double w[kHalfInvRoots];
};
__device__ __forceinline__ void load_half_roots(HalfRoots& w, const Tab& tw, int t, uint32_t h) {
  const uint32_t tb = (uint32_t)t >> 3;
  w.f5 = tw.at(tb * 8u, (16u + 8u * h) * 8u);
#pragma unroll
  for (int e = 0; e < 2; ++e) w.f4[e] = tw.at(2u * tb * 8u, (32u + 16u * h + e) * 8u);
#pragma unroll
  for (int e = 0; e < 4; ++e) w.f3[e] = tw.at(4u * tb * 8u, (64u + 32u * h + e) * 8u);
  w.f2 = tw.at((uint32_t)t * 8u, (128u + 64u * h) * 8u);
#pragma unroll
  for (int e = 0; e < 2; ++e) w.f1[e] = tw.at(2u * t * 8u, (256u + 128u * h + e) * 8u);
#pragma unroll
  for (int e = 0; e < 4; ++e) w.f0[e] = tw.at(4u * t * 8u, (512u + 256u * h + e) * 8u);
}
__device__ __forceinline__ void load_half_inv_roots(HalfInvRoots& w, const Tab& itw,
                                                    const Tab& post, int t, uint32_t h) {
  const uint32_t t7 = (uint32_t)t & 7u, tt = (uint32_t)t;
  w.w[kI3] = itw.at(64u * t7 * 8u, 0);
#pragma unroll
  for (int e = 0; e < 2; ++e) w.w[kI4 + e] = itw.at(32u * t7 * 8u, 32u * 8u * e * 8u);
#pragma unroll
  for (int e = 0; e < 4; ++e) w.w[kI5 + e] = itw.at(16u * t7 * 8u, 16u * 8u * e * 8u);
  w.w[kI6] = itw.at(8u * tt * 8u, 0);
#pragma unroll
  for (int e = 0; e < 2; ++e) w.w[kI7 + e] = itw.at(4u * tt * 8u, 4u * 64u * e * 8u);
#pragma unroll
  for (int e = 0; e < 4; ++e) w.w[kI8 + e] = itw.at(2u * tt * 8u, 2u * 64u * e * 8u);
#pragma unroll
  for (int r = 0; r < 8; ++r) w.w[kI9 + r] = itw.at(tt * 8u, 64u * r * 8u);
#pragma unroll
  for (int r = 0; r < 8; ++r) w.w[kTw + r] = post.at(tt * 8u, (512u * h + 64u * r) * 8u);
}

// Digits of half h after the first two forward stages by table: the quads
// of digit_row_two_stages (registers q, q + 4, q + 8, q + 12 of d hold
// positions j, j + 256, j + 512, j + 768, j = t + 64 q); half 0 keeps
// positions j and j + 256 (d0 + i d2 +- (d1 w2 + d3 w3)), half 1 keeps
// j + 512 and j + 768 (d0 - i d2 +- (d1 w3 + d3 w2)).  Output in the
// round-A mapping of the half: x[q] at j' = t + 64 q, x[q + 4] at + 256.
template <int BG>
__device__ __forceinline__ void digit_half_two_stages(const uint32_t d[16], uint32_t sh,
                                                      const double* tab, uint32_t h,
                                                      double x[8]) {
  constexpr uint32_t HALF = 1u << (BG - 1);
  constexpr uint32_t TW = 2 * HALF;
  const uint32_t oa = h ? 2 * TW : TW, ob = h ? TW : 2 * TW;
  double m1[4], ma[4], mb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    m1[q] = tab[__builtin_amdgcn_ubfe(d[q + 8], sh, BG)];
    ma[q] = tab[oa + __builtin_amdgcn_ubfe(d[q + 4], sh, BG)];
    mb[q] = tab[ob + __builtin_amdgcn_ubfe(d[q + 12], sh, BG)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double d0 = (double)((int32_t)__builtin_amdgcn_ubfe(d[q], sh, BG) - (int32_t)HALF);
    const double base = h ? d0 - m1[q] : d0 + m1[q];
    const double m = ma[q] + mb[q];
    x[q] = base + m;
    x[q + 4] = base - m;
  }
}

// Forward stages 7 .. 0 of half h (stages 9 and 8 done by table): the
// reduction points of ntt_fwd_reg (after stage 5 and after stage 1).  Out:
// round-C mapping, x[r] at bit-reversed position 512 h + 8 t + r, |x| < 1.14 P.
__device__ __forceinline__ void ntt_fwd_half(double x[8], double* lds, const UniTw& u,
                                             const HalfRoots& w, uint32_t h, int t) {
  // round A (uniform roots): stage 7, k = 4 + 2h + r/4; stage 6, k = 8 + 4h + r/2
  double a7[2], a6[4];
#pragma unroll
  for (int e = 0; e < 2; ++e) a7[e] = h ? u.fwd[6 + e] : u.fwd[4 + e];
#pragma unroll
  for (int e = 0; e < 4; ++e) a6[e] = h ? u.fwd[12 + e] : u.fwd[8 + e];
  hfwd_stage<1, 2>(x, a7);
  hfwd_stage<0, 4>(x, a6);
  hexchange<6, 3>(x, lds, t);
  hfwd_stage<2, 1>(x, &w.f5);
  reduce8(x);
  hfwd_stage<1, 2>(x, w.f4);
  hfwd_stage<0, 4>(x, w.f3);
  hexchange<3, 0>(x, lds, t);
  hfwd_stage<2, 1>(x, &w.f2);
  hfwd_stage<1, 2>(x, w.f1);
  reduce8(x);
  hfwd_stage<0, 4>(x, w.f0);
}

// Inverse stages 0 .. 8 of one half (input |x| < 5 P in the round-C
// mapping): reductions before stages 0, 3 and 7 as in ntt_inv_reg.  Out:
// round-A mapping, x[r] at i' = t + 64 r.
__device__ __forceinline__ void ntt_inv_half(double x[8], double* lds, const UniTw& u,
                                             const HalfInvRoots& w, int t) {
  reduce8(x);
#pragma unroll
  for (int s = 0; s <= 2; ++s) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r & (1 << s)) continue;
      const int r2 = r | (1 << s);
      const int m8 = (r & ((1 << s) - 1)) << (3 - s);  // e = m8 N / 16
      const double m = m8 == 0 ? x[r2] : mulmod(x[r2], u.inv[m8]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
  reduce8(x);
  hexchange<0, 3>(x, lds, t);
  hinv_stage<0>(x, w.w + kI3);
  hinv_stage<1>(x, w.w + kI4);
  hinv_stage<2>(x, w.w + kI5);
  hexchange<3, 6>(x, lds, t);
  hinv_stage<0>(x, w.w + kI6);
  reduce8(x);
  hinv_stage<1>(x, w.w + kI7);
  hinv_stage<2>(x, w.w + kI8);
}

template <int L, int BG>
__global__ void __launch_bounds__(4 * L * 64)
blind_rotate_halfrow_kernel(BrArgs a) {
  constexpr int LOGN = 10, N = 1024, TP = 64, ROWS = 2 * L, NW = 2 * ROWS, G = 2;
  constexpr uint32_t HALF = 1u << (BG - 1);
  constexpr uint32_t NU = LOGN + 1;
  static_assert(NW >= 4, "four waves run the inverse transforms");
  static_assert(2 * HALF <= 256, "the first two stages come from the digit tables");
  __shared__ double lds_all[NW][512 + 32];
  __shared__ double sums[2][2][8][TP];  // [output][half][r][t]
  __shared__ uint32_t acc[2][N];
  __shared__ double stage1[6 * HALF];
  // the inverse transforms' per-thread roots of each half, [half][root][t]:
  // loaded once, read for every transform (the key stream evicts them from
  // the L1 cache between steps, and held in registers they would cost the
  // forward phase its spill-free allocation)
  __shared__ double iroots[2][kHalfInvRoots][TP];

  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TP);
  const int t = (int)threadIdx.x - wv * TP;
  const int rowi = wv >> 1;  // digit row c l + lv
  const uint32_t h = (uint32_t)wv & 1u;
  const int c = rowi / L, lv = rowi % L;
  double* lds = lds_all[wv];
  const size_t job = blockIdx.x;
  const uint32_t n = a.n;
  const uint64_t g = a.nlut == 2 ? job >> 1 : job;
  const uint32_t lut = a.nlut == 2 ? (uint32_t)(job & 1u) : 0u;
  const uint32_t* ct;
  const double* bsk;
  if (a.ranges) {
    const JobRange& rg = a.ranges[find_range(a.ranges, a.nranges, g)];
    ct = rg.in + (g - rg.first) * (size_t)(n + 1);
    bsk = rg.bsk;
  } else {
    ct = a.in + g * (size_t)(n + 1);
    bsk = a.bsk;
  }
  ct = uniform_ptr(ct);
  bsk = uniform_ptr(bsk);
  const Tab key(bsk), fwd_tw(a.fwd_tw), inv_tw(a.inv_tw), post(a.post);
  const uint32_t* v = lut == 0 ? a.tpoly0 : a.tpoly1;

  uint32_t off = 1u << (31 - L * BG);
#pragma unroll
  for (int j = 1; j <= L; ++j) off += HALF << (32 - j * BG);
  const uint32_t even = __builtin_amdgcn_readfirstlane(a.even);
  const uint32_t msh = 32 - NU + even, mhalf = 1u << (msh - 1);
  auto mod_switch = [=](uint32_t x) { return ((x + mhalf) >> msh) << even; };

  const int tid = threadIdx.x;
  constexpr int NT = NW * TP;
  fill_stage_tables<HALF>(stage1, a.uni, tid, NT);
  for (int j = tid; j < 2 * 2 * 8 * TP; j += NT) (&sums[0][0][0][0])[j] = 0.0;
  {
    const uint32_t bbar = mod_switch(ct[n]);
    const uint32_t e = (2 * N - bbar) & (2 * N - 1);
    for (int j = tid; j < N; j += NT) {
      const int src = j - (int)e;
      uint32_t val;
      if (src >= 0) val = v[src];
      else if (src + N >= 0) val = 0u - v[src + N];
      else val = v[src + 2 * N];
      acc[0][j] = 0u;
      acc[1][j] = val;
    }
  }
  HalfRoots fw;
  load_half_roots(fw, fwd_tw, t, h);
  // the four inverse waves: (output wv >> 1, half wv & 1)
  const bool inv = wv < 4;
  const int co = wv >> 1;
  if (wv < 2) {
    HalfInvRoots iw;
    load_half_inv_roots(iw, inv_tw, post, t, h);
#pragma unroll
    for (int k = 0; k < kHalfInvRoots; ++k) iroots[h][k][t] = iw.w[k];
  }
  __syncthreads();

  const uint32_t sh = 32 - (lv + 1) * BG;
  // key of position 512 h + 8 t + r: slot (r16, t16) = (8 (t & 1) + r, 32 h + t / 2)
  // of the row, G doubles each
  const uint32_t kv_lane = (((uint32_t)t & 1u) * 512u + ((uint32_t)t >> 1)) * (G * 8);
  const uint32_t kv_half = 32u * h * (G * 8);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t abar = mod_switch(ct[i]);
    if (abar == 0) continue;
    const uint32_t row = i * (uint32_t)(ROWS * 16 * TP * G * 8) +
                         (uint32_t)(rowi * 16 * TP * G * 8) + kv_half;
    double kv[8][G];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      key.at2(kv_lane, row + (uint32_t)(r * TP * G * 8), kv[r][0], kv[r][1]);
    double x[8];
    {
      uint32_t d[16];
      const uint32_t* ac = acc[c];
      const int kb = t - (int)abar;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = kb + TP * r;
        const uint32_t val = ac[k & (N - 1)];
        const uint32_t neg = 0u - (((uint32_t)k >> LOGN) & 1u);
        d[r] = ((val ^ neg) - neg) - ac[t + TP * r] + off;
      }
      digit_half_two_stages<BG>(d, sh, stage1, h, x);
    }
    ntt_fwd_half(x, lds, a.uni, fw, h, t);
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int q = 0; q < G; ++q) atomicAdd(&sums[q][h][r][t], mulmod(x[r], kv[r][q]));
    __syncthreads();  // every product is in; every rotation has read ACC
    double y[8];
    HalfInvRoots iw;
    if (inv) {
#pragma unroll
      for (int k = 0; k < kHalfInvRoots; ++k) iw.w[k] = iroots[h][k][t];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        y[r] = sums[co][h][r][t];
        sums[co][h][r][t] = 0.0;  // cleared for the next step
      }
      ntt_inv_half(y, lds, a.uni, iw, t);
      // the last inverse stage pairs i' and 512 + i' across the two halves
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[r * TP + t] = y[r];
    }
    __syncthreads();  // both halves of each output are in LDS
    if (inv) {
      const double* other = lds_all[wv ^ 1];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const double o = other[r * TP + t];
        double z;
        if (h == 0) z = y[r] + mulmod(o, iw.w[kI9 + r]);
        else z = o - mulmod(y[r], iw.w[kI9 + r]);
        const uint32_t part = low32_magic(redc(mulmod(z, iw.w[kTw + r])));
        acc[co][512 * h + t + TP * r] += part;
      }
    }
    __syncthreads();  // ACC updated and the half buffers read before the next step
  }

#pragma unroll
  for (uint32_t k = 0; k < 2; ++k) {
    if (k > even) break;
    const uint32_t fn = even ? k : lut;
    uint32_t* out;
    uint32_t plain = 0u;
    if (a.out0) {
      out = (fn == 0 ? a.out0 : a.out1) + g * (size_t)(N + 1);
      plain = a.plain_b[fn];
    } else {
      out = a.ext + (even ? 2 * job + k : job) * (size_t)(N + 1);
    }
    out = uniform_ptr(out);
    for (int j = tid; j < N; j += NT) out[j] = j <= (int)k ? acc[0][k - j] : 0u - acc[0][N + k - j];
    if (tid == 0) out[N] = acc[1][k] + plain;
  }
}

// ---------------------------------------------------------------------------
// Key switching z -> s with the bootstrapping epilogue.  Thread w owns
// output word w of one sample.  out = (0, b') - sum over coefficients i and
// digits j of KSK[i][j][d_ij - 1] (d_ij != 0), where a'_i is rounded to
// t*beta bits and split into base-2^beta digits, most significant first.
// Sample m is job job0 + m (ciphertext (job0 + m) / nlut, program function
// (job0 + m) % nlut); its result goes to that function's output at the
// ciphertext's row (or its range's row in a multi-key launch), and the
// function's plain_add is added to b (FHE-Fire adds Delta * 1 after
// bootstrapping).
// program function and output row of key-switch sample m (nlut is 1 or 2)
__device__ __forceinline__ uint32_t ks_lut(const KsArgs& a, size_t m) {
  return a.nlut == 2 ? (uint32_t)((a.job0 + m) & 1u) : 0u;
}
__device__ __forceinline__ uint32_t* ks_output_row(const KsArgs& a, size_t m) {
  const uint64_t job = a.job0 + m;
  const uint64_t g = a.nlut == 2 ? job >> 1 : job;
  const uint32_t lut = a.nlut == 2 ? (uint32_t)(job & 1u) : 0u;
  const size_t w1 = a.n + 1;
  if (a.ranges) {
    const JobRange& rg = a.ranges[find_range(a.ranges, a.nranges, g)];
    return (lut == 0 ? rg.out0 : rg.out1) + (g - rg.first) * w1;
  }
  return (lut == 0 ? a.out0 : a.out1) + g * w1;
}

__global__ void __launch_bounds__(256)
keyswitch_kernel(KsArgs a) {
  const uint32_t w = blockIdx.y * 256 + threadIdx.x;
  const size_t m = blockIdx.x;
  const uint32_t n = a.n, N = a.N, t = a.t, beta = a.beta, base1 = (1u << beta) - 1;
  const uint32_t prec = t * beta;
  if (w > n) return;
  const uint32_t* in = a.in + m * (size_t)(N + 1);
  const uint32_t lut = ks_lut(a, m);
  uint32_t r = w == n ? in[N] + a.plain_add[lut] : 0u;
  const size_t stride = (size_t)(n + 1);
  const uint32_t* ksk = a.ksk + w;
  for (uint32_t i = 0; i < N; ++i) {
    const uint32_t abar = (in[i] + (1u << (31 - prec))) >> (32 - prec);
    const uint32_t* rows = ksk + (size_t)i * t * base1 * stride;
    for (uint32_t j = 0; j < t; ++j) {
      const uint32_t dg = (abar >> ((t - 1 - j) * beta)) & base1;
      if (dg) r -= rows[((size_t)j * base1 + (dg - 1)) * stride];
    }
  }
  ks_output_row(a, m)[w] = r;
}

// ---------------------------------------------------------------------------
// Key switching of a batch on the matrix cores (t = 8 digits of base 4).
//
// For sample s the key switch subtracts, for every coefficient i and digit
// position j, the KSK row selected by the digit d_{s,i,j}.  Writing the
// selection as a one-hot vector over the four digit values (value 0 selects
// an all-zero row), the batch is the product
//     out[s][w] = [w = n] b'_s - sum_k A[s][k] K[k][w],  k = (i, j, v),
//     A[s][k] = [d_{s,i,j} = v],  K[(i,j,v)][w] = KSK[i][j][v-1][w] (0 if v = 0)
// over the integers mod 2^32.  K is split into four signed bytes,
// K = sum_b 256^b K_b with K_b in [-128, 128), so each A K_b is an exact
// int8 x int8 -> int32 product (a sum of 8N terms of magnitude <= 128) on
// v_mfma_i32_32x32x32_i8, and out = [w = n] b' - sum_b 256^b (A K_b) mod 2^32.
//
// Operand order of v_mfma_i32_32x32x32_i8 (32 x 32 x 32 tile): lane l holds
// A[l % 32][16 (l / 32) + x] and B[16 (l / 32) + x][l % 32] in byte x of its
// four registers; result C[i][j] sits in lane j + 32 ((i / 4) % 2), register
// (i % 4) + 4 (i / 8).  The 32 k of a tile are one coefficient i: k = 4 j + v.
// So lane l builds, for its sample, one word per digit position
// j = 4 (l / 32) + q: the byte of value d set, 1 << 8 d.
//
// Plane layout (built once per key by ksk_to_planes_kernel): for coefficient
// i, word tile wt and byte plane b, the 64 lanes' 16-byte B registers are
// stored contiguously, [i][wt][b][lane][16].
//
// A wave computes MA fragments of 32 samples times one 32-word tile times
// the four planes (4 MA accumulator tiles); every B register it loads is
// used by MA products.
typedef int fs_v4i __attribute__((ext_vector_type(4)));
typedef int fs_v16i __attribute__((ext_vector_type(16)));

uint32_t ks_word_tiles(uint32_t n) { return (n + 1 + 31) / 32; }
size_t ksk_planes_bytes(uint32_t N, uint32_t n) {
  return (size_t)N * ks_word_tiles(n) * 4 * 64 * 16;
}

__device__ __forceinline__ int8_t signed_byte_plane(uint32_t u, int b) {
  // u = sum_b 256^b s_b (mod 2^32) with s_b in [-128, 128)
  int8_t sb = 0;
#pragma unroll
  for (int q = 0; q <= 3; ++q) {
    sb = (int8_t)(u & 0xFFu);
    if (q == b) break;
    u = (u - (uint32_t)(int32_t)sb) >> 8;
  }
  return sb;
}

__global__ void __launch_bounds__(64)
ksk_to_planes_kernel(const uint32_t* __restrict__ ksk, int8_t* __restrict__ planes, uint32_t n,
                     uint32_t wtiles) {
  const uint32_t l = threadIdx.x, i = blockIdx.x, wt = blockIdx.y;
  const uint32_t w1 = n + 1, w = 32 * wt + (l & 31);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int8_t bytes[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const uint32_t k = 16 * (l >> 5) + x, j = k >> 2, v = k & 3;
      bytes[x] = (v == 0 || w >= w1)
                     ? (int8_t)0
                     : signed_byte_plane(ksk[(((size_t)i * 8 + j) * 3 + (v - 1)) * w1 + w], b);
    }
    int8_t* dst = planes + ((((size_t)i * wtiles + wt) * 4 + b) * 64 + l) * 16;
#pragma unroll
    for (int x = 0; x < 16; ++x) dst[x] = bytes[x];
  }
}

// (0, b' + plain_add) in every output row of the batch; the matrix-core
// kernels then subtract their partial sums atomically (integer addition
// mod 2^32 is exact in any order).
__global__ void __launch_bounds__(256)
ks_body_kernel(KsArgs a, uint32_t count) {
  const uint32_t m = blockIdx.x, w = blockIdx.y * 256 + threadIdx.x, n = a.n;
  if (m >= count || w > n) return;
  const uint32_t body =
      w == n ? a.in[(size_t)m * (a.N + 1) + a.N] + a.plain_add[ks_lut(a, m)] : 0u;
  ks_output_row(a, m)[w] = body;
}

// Grid: (sample groups of 32 MA, word tiles, K splits).  Split z covers
// coefficients [z N / gridDim.z, (z + 1) N / gridDim.z).
template <int N, int MA>
__global__ void __launch_bounds__(64, 2)
keyswitch_mfma_kernel(KsArgs a, uint32_t count) {
  constexpr int PREC = 16;  // 8 digits of 2 bits
  const uint32_t l = threadIdx.x, h = l >> 5, c32 = l & 31;
  const uint32_t s0 = blockIdx.x * (32 * MA);
  const uint32_t wt = blockIdx.y, wtiles = gridDim.y;
  const uint32_t ibeg = blockIdx.z * (N / gridDim.z), iend = ibeg + N / gridDim.z;
  const uint32_t n = a.n, w1 = n + 1;

  fs_v16i acc[MA][4];
#pragma unroll
  for (int f = 0; f < MA; ++f)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[f][b] = fs_v16i{};

  // the sample each lane builds A rows for (padding samples read sample 0
  // and are given digit 0, which selects the zero rows)
  const uint32_t* row[MA];
  bool live[MA];
#pragma unroll
  for (int f = 0; f < MA; ++f) {
    const uint32_t s = s0 + 32 * f + c32;
    live[f] = s < count;
    row[f] = a.in + (size_t)(live[f] ? s : 0) * (N + 1);
  }
  const fs_v4i* __restrict__ bk =
      reinterpret_cast<const fs_v4i*>(a.kskp) + (size_t)wt * 4 * 64 + l;
  const size_t bstep = (size_t)wtiles * 4 * 64;  // fs_v4i per coefficient
  const uint32_t shift = 8 - 8 * h;  // digits 4h .. 4h+3 of the rounded coefficient

#pragma unroll 2
  for (uint32_t i = ibeg; i < iend; ++i) {
    const fs_v4i* bi = bk + (size_t)i * bstep;
    fs_v4i bq[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) bq[b] = bi[b * 64];
#pragma unroll
    for (int f = 0; f < MA; ++f) {
      const uint32_t ai = live[f] ? row[f][i] : 0u;
      const uint32_t abar = (ai + (1u << (31 - PREC))) >> (32 - PREC);
      const uint32_t nib = (abar >> shift) & 0xFFu;
      fs_v4i A;
      A[0] = (int)(1u << (((nib >> 6) & 3u) << 3));
      A[1] = (int)(1u << (((nib >> 4) & 3u) << 3));
      A[2] = (int)(1u << (((nib >> 2) & 3u) << 3));
      A[3] = (int)(1u << ((nib & 3u) << 3));
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[f][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, bq[b], acc[f][b], 0, 0, 0);
    }
  }

  // epilogue: combine the planes and subtract the partial sum
  const uint32_t w = 32 * wt + c32;
  if (w >= w1) return;
#pragma unroll
  for (int f = 0; f < MA; ++f)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t m = s0 + 32 * f + 8 * (r >> 2) + 4 * h + (r & 3);
      if (m >= count) continue;
      const uint32_t sum = (uint32_t)acc[f][0][r] + ((uint32_t)acc[f][1][r] << 8) +
                           ((uint32_t)acc[f][2][r] << 16) + ((uint32_t)acc[f][3][r] << 24);
      atomicSub(ks_output_row(a, m) + w, sum);
    }
}

// ---------------------------------------------------------------------------
// Negacyclic product check: out = sum_r d_r b_r through the transforms the
// blind rotation uses (register-root forward transform of the digit side,
// table forward transform of the key side, register-root inverse).
template <int LOGN, int LIMBS>
__global__ void __launch_bounds__(NttShape<LOGN>::TP)
polymul_kernel(const int32_t* __restrict__ d, const uint32_t* __restrict__ b, uint32_t R,
               uint32_t* __restrict__ out, const double* __restrict__ tw,
               const double* __restrict__ itw, const double* __restrict__ post, UniTw uni) {
  using S = NttShape<LOGN>;
  __shared__ double lds[S::LDS_DOUBLES];
  const int t = threadIdx.x;
  double accv[LIMBS][16];
#pragma unroll
  for (int lb = 0; lb < LIMBS; ++lb)
#pragma unroll
    for (int r = 0; r < 16; ++r) accv[lb][r] = 0.0;
  for (uint32_t q = 0; q < R; ++q) {
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (double)d[(size_t)q * S::N + t + S::TP * r];
    ntt_fwd_reg<LOGN>(x, lds, uni, Tab(tw), t);
#pragma unroll
    for (int lb = 0; lb < LIMBS; ++lb) {
      double y[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int32_t c = (int32_t)b[(size_t)q * S::N + t + S::TP * r];
        if (LIMBS == 1) y[r] = (double)c;
        else {
          const int32_t lo = (int32_t)(int16_t)(uint16_t)(uint32_t)c;
          y[r] = (double)(lb == 0 ? lo : (c - lo) >> 16);
        }
      }
      ntt_fwd<LOGN>(y, lds, tw, t);
      // y is in round-C mapping like x: pointwise products line up
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // as in the blind rotation: up to 2l products summed unreduced
        const double s = accv[lb][r] + mulmod(x[r], y[r]);
        accv[lb][r] = (q % 6 == 5) ? redc(s) : s;
      }
    }
  }
  uint32_t res[16];
#pragma unroll
  for (int lb = 0; lb < LIMBS; ++lb) {
    ntt_inv_reg<LOGN>(accv[lb], lds, uni, Tab(itw), Tab(post), t);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t part = low32_magic(accv[lb][r]);
      res[r] = lb == 0 ? part : res[r] + (part << 16);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) out[t + S::TP * r] = res[r];
}

// ---------------------------------------------------------------------------
// launchers

#define FS_LAUNCH_CHECK()                                     \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return (int)e_;                     \
  } while (0)

int launch_bsk_to_ntt(uint32_t N, uint32_t n, uint32_t l, uint32_t limbs,
                      const uint32_t* bsk_coef, double* out, const double* tw, hipStream_t st) {
  const uint32_t rows = 2 * l;
  if (N == 1024 && limbs == 1) {
    dim3 g(n * rows * 2, 1);
    bsk_to_ntt_kernel<10, 1><<<g, 64, 0, st>>>(bsk_coef, out, rows, tw);
  } else if (N == 2048 && limbs == 2) {
    dim3 g(n * rows * 2, 2);
    bsk_to_ntt_kernel<11, 2><<<g, 128, 0, st>>>(bsk_coef, out, rows, tw);
  } else if (N == 2048 && limbs == 1) {
    dim3 g(n * rows * 2, 1);
    bsk_to_ntt_kernel<11, 1><<<g, 128, 0, st>>>(bsk_coef, out, rows, tw);
  } else {
    return -1;
  }
  FS_LAUNCH_CHECK();
  return 0;
}

// Kernel variants the tuner chooses from: (PF key-slice prefetch point,
// minimum waves per SIMD the register allocation must allow[, jobs per
// workgroup of the lockstep form]), by index:
// N = 1024: (2, 2), (1, 2), (0, 2), (2, 1), (2, 1, 8), (0, 2, 8), (2, 1, 4),
// and (0, 2), (3, 2), (1, 2) with the forward roots held in registers, and
// (0, 2) with the forward and the inverse transforms' roots held;
// N = 2048, two key limbs: (3, 2), (0, 1), (0, 2), (1, 1), (3, 2, 4),
// (3, 2, 2), (0, 2, 2), (1, 1, 2), (0, 1, 2); N = 2048, one limb: (2, 2),
// (1, 2), (0, 2), (0, 2, 2) with held forward and round-B' inverse roots,
// (1, 2, 4), (1, 2, 2), (3, 2) and (0, 2) with held forward and round-B'
// inverse roots, and (1, 2) with held forward roots.  Split launches (two
// polynomial groups per job) use (1, 2) with held forward roots at N = 1024,
// (0, 1) at N = 2048 with two limbs and (1, 2) with one; the paired launch
// (N = 1024) uses (1, 1) with the forward and inverse roots held.  The
// one-limb N = 2048 key has no row form (two of its four groups would run
// no inverse transform, so the groups' barrier sequences would differ).
int blind_rotate_variants(uint32_t N) { return N == 1024 ? 11 : N == 2048 ? 9 : 0; }

int launch_blind_rotate(uint32_t N, const BrArgs& args, size_t jobs, int variant, int groups,
                        hipStream_t st) {
  if (jobs == 0) return 0;
  BrArgs a = args;
  a.jobs = jobs;
  const dim3 g((uint32_t)jobs);
  const bool split = groups == kBrTwo || (groups == kBrTwoPaired && N != 1024);
  if (groups == kBrTwoPaired && N == 1024) {
    // two jobs of two groups per workgroup: every SIMD of a CU holds one
    // wave, so the allocation may take a SIMD's whole register file and
    // hold the forward and inverse transforms' roots for the job
    blind_rotate_kernel<10, 3, 7, 1, 1, 1, 2, 2, true, 2>
        <<<dim3((uint32_t)((jobs + 1) / 2)), 256, 0, st>>>(a);
  } else if (groups == kBrRows && !(N == 2048 && a.limbs == 1)) {
    if (N == 1024) blind_rotate_halfrow_kernel<3, 7><<<g, 12 * 64, 0, st>>>(a);
    else if (N == 2048) blind_rotate_rows_kernel<11, 2, 10, 2><<<g, 4 * 128, 0, st>>>(a);
    else return -1;
  } else if (N == 1024) {
    if (split) {
      blind_rotate_kernel<10, 3, 7, 1, 1, 2, 2, 1, true><<<g, 128, 0, st>>>(a);
    } else {
      const dim3 g8((uint32_t)((jobs + 7) / 8)), g4((uint32_t)((jobs + 3) / 4));
      switch (variant) {
        case 0: blind_rotate_kernel<10, 3, 7, 1, 2, 2, 1><<<g, 64, 0, st>>>(a); break;
        case 1: blind_rotate_kernel<10, 3, 7, 1, 1, 2, 1><<<g, 64, 0, st>>>(a); break;
        case 2: blind_rotate_kernel<10, 3, 7, 1, 0, 2, 1><<<g, 64, 0, st>>>(a); break;
        case 3: blind_rotate_kernel<10, 3, 7, 1, 2, 1, 1><<<g, 64, 0, st>>>(a); break;
        case 4: blind_rotate_kernel<10, 3, 7, 1, 2, 1, 1, 8><<<g8, 512, 0, st>>>(a); break;
        case 5: blind_rotate_kernel<10, 3, 7, 1, 0, 2, 1, 8><<<g8, 512, 0, st>>>(a); break;
        case 6: blind_rotate_kernel<10, 3, 7, 1, 2, 1, 1, 4><<<g4, 256, 0, st>>>(a); break;
        case 7: blind_rotate_kernel<10, 3, 7, 1, 0, 2, 1, 1, true><<<g, 64, 0, st>>>(a); break;
        case 8: blind_rotate_kernel<10, 3, 7, 1, 3, 2, 1, 1, true><<<g, 64, 0, st>>>(a); break;
        case 9: blind_rotate_kernel<10, 3, 7, 1, 1, 2, 1, 1, true><<<g, 64, 0, st>>>(a); break;
        case 10: blind_rotate_kernel<10, 3, 7, 1, 0, 2, 1, 1, true, 2><<<g, 64, 0, st>>>(a); break;
        default: return -2;
      }
    }
  } else if (N == 2048 && a.limbs == 1) {
    if (groups == kBrRows) return -2;
    if (split) {
      blind_rotate_kernel<11, 2, 10, 1, 1, 2, 2><<<g, 256, 0, st>>>(a);
    } else {
      const dim3 g4((uint32_t)((jobs + 3) / 4)), g2((uint32_t)((jobs + 1) / 2));
      switch (variant) {
        case 0: blind_rotate_kernel<11, 2, 10, 1, 2, 2, 1><<<g, 128, 0, st>>>(a); break;
        case 1: blind_rotate_kernel<11, 2, 10, 1, 1, 2, 1><<<g, 128, 0, st>>>(a); break;
        case 2: blind_rotate_kernel<11, 2, 10, 1, 0, 2, 1><<<g, 128, 0, st>>>(a); break;
        case 3: blind_rotate_kernel<11, 2, 10, 1, 0, 2, 1, 2, true, 1><<<g2, 256, 0, st>>>(a); break;
        case 4: blind_rotate_kernel<11, 2, 10, 1, 1, 2, 1, 4><<<g4, 512, 0, st>>>(a); break;
        case 5: blind_rotate_kernel<11, 2, 10, 1, 1, 2, 1, 2><<<g2, 256, 0, st>>>(a); break;
        case 6: blind_rotate_kernel<11, 2, 10, 1, 3, 2, 1, 1, true, 1><<<g, 128, 0, st>>>(a); break;
        case 7: blind_rotate_kernel<11, 2, 10, 1, 0, 2, 1, 1, true, 1><<<g, 128, 0, st>>>(a); break;
        case 8: blind_rotate_kernel<11, 2, 10, 1, 1, 2, 1, 1, true><<<g, 128, 0, st>>>(a); break;
        default: return -2;
      }
    }
  } else if (N == 2048) {
    if (split) {
      blind_rotate_kernel<11, 2, 10, 2, 0, 1, 2><<<g, 256, 0, st>>>(a);
    } else {
      const dim3 g4((uint32_t)((jobs + 3) / 4)), g2((uint32_t)((jobs + 1) / 2));
      switch (variant) {
        case 0: blind_rotate_kernel<11, 2, 10, 2, 3, 2, 1><<<g, 128, 0, st>>>(a); break;
        case 1: blind_rotate_kernel<11, 2, 10, 2, 0, 1, 1><<<g, 128, 0, st>>>(a); break;
        case 2: blind_rotate_kernel<11, 2, 10, 2, 0, 2, 1><<<g, 128, 0, st>>>(a); break;
        case 3: blind_rotate_kernel<11, 2, 10, 2, 1, 1, 1><<<g, 128, 0, st>>>(a); break;
        case 4: blind_rotate_kernel<11, 2, 10, 2, 3, 2, 1, 4><<<g4, 512, 0, st>>>(a); break;
        case 5: blind_rotate_kernel<11, 2, 10, 2, 3, 2, 1, 2><<<g2, 256, 0, st>>>(a); break;
        case 6: blind_rotate_kernel<11, 2, 10, 2, 0, 2, 1, 2><<<g2, 256, 0, st>>>(a); break;
        case 7: blind_rotate_kernel<11, 2, 10, 2, 1, 1, 1, 2><<<g2, 256, 0, st>>>(a); break;
        case 8: blind_rotate_kernel<11, 2, 10, 2, 0, 1, 1, 2><<<g2, 256, 0, st>>>(a); break;
        default: return -2;
      }
    }
  } else {
    return -1;
  }
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_keyswitch(const KsArgs& a, size_t count, hipStream_t st) {
  if (count == 0) return 0;
  const bool mfma = a.kskp && a.t == 8 && a.beta == 2 && (a.N == 1024 || a.N == 2048);
  if (mfma) {
    constexpr int MA = 2, SPLIT = 4;
    ks_body_kernel<<<dim3((uint32_t)count, (a.n + 1 + 255) / 256), 256, 0, st>>>(a, (uint32_t)count);
    FS_LAUNCH_CHECK();
    dim3 g((uint32_t)((count + 32 * MA - 1) / (32 * MA)), ks_word_tiles(a.n), SPLIT);
    if (a.N == 1024) keyswitch_mfma_kernel<1024, MA><<<g, 64, 0, st>>>(a, (uint32_t)count);
    else keyswitch_mfma_kernel<2048, MA><<<g, 64, 0, st>>>(a, (uint32_t)count);
  } else {
    dim3 g((uint32_t)count, (a.n + 1 + 255) / 256);
    keyswitch_kernel<<<g, 256, 0, st>>>(a);
  }
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_ksk_to_planes(uint32_t N, uint32_t n, const uint32_t* ksk, int8_t* planes,
                         hipStream_t st) {
  const uint32_t wtiles = ks_word_tiles(n);
  ksk_to_planes_kernel<<<dim3(N, wtiles), 64, 0, st>>>(ksk, planes, n, wtiles);
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_polymul(uint32_t N, const int32_t* d, const uint32_t* b, uint32_t R, uint32_t* out,
                   const double* tw, const double* itw, const double* post, const UniTw& uni,
                   hipStream_t st) {
  if (N == 1024) polymul_kernel<10, 1><<<1, 64, 0, st>>>(d, b, R, out, tw, itw, post, uni);
  else if (N == 2048) polymul_kernel<11, 2><<<1, 128, 0, st>>>(d, b, R, out, tw, itw, post, uni);
  else return -1;
  FS_LAUNCH_CHECK();
  return 0;
}

}  // namespace fs
