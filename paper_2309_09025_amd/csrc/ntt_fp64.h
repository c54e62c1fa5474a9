// Exact negacyclic number-theoretic transform over Z_P[X]/(X^N+1) for the
// external products of blind rotation (Sec. 2.1, RGSW item: the products
// RLWE (x) RGSW that the Blind Rotation step chains).
//
// Arithmetic.  P = 3*2^49 + 2^20 + 1 is prime, P - 1 = 2^20 * odd, so
// primitive 2N-th roots exist for every N <= 2^19.  Residues are held as
// integer-valued binary64 numbers of magnitude < 2^53, where every sum,
// difference and fused multiply-add of integers is exact.  A modular
// product a*w is formed exactly as
//     h = fl(a w), l = fma(a, w, -h)          (a w = h + l exactly)
//     q = rint(fl(h / P)), r = fma(-q, P, h)  (exact: |r| < 2^53)
//     a w = r + l (mod P)
// which returns a representative of magnitude <= 0.5 P + 1.5 2^-52 |a w|.
// Butterflies are lazy: values grow additively between explicit
// reductions x - rint(x/P) P, and the reduction points below keep every
// intermediate under 4.4 P < 2^53 (with P ~ 2^50.585, 2^53 = 5.33 P).
//
// Exactness of the external product.  With N = 1024, (k+1) l = 6 digit
// polynomials of |digit| <= 64 and key coefficients centred in
// [-2^31, 2^31), every coefficient of the integer product sum is bounded
// by 6 * 1024 * 64 * 2^31 = 3 * 2^48 < (P-1)/2, so the centred residue is
// the integer itself and its low 32 bits are the torus result.  For
// N = 2048 (4 digit polynomials, |digit| <= 512) the bound for 32-bit key
// coefficients is 2^53, so the exact key form splits them into two 16-bit
// halves, each product sum then being below 2^37.  The one-limb key form
// keeps them whole: a step's key rows are fresh uniform words independent of
// that step's digits, so each coefficient sum is sub-Gaussian with variance
// at most 8192 * 512^2 * 2^62 / 3 ((P-1)/2 is 14.7 standard deviations
// away, 25 for the uniform digits of a typical step) and passes the limit
// with probability below 2^-150; exact for every key only in the two-limb
// form.
//
// Data layout.  A polynomial of N = 16 * TP coefficients is held by TP
// threads, 16 values per thread; exponent bits [lo, lo+4) of an index live
// in the register number and the others in the thread number:
//     j(t, r) = (t & (2^lo - 1)) | (r << lo) | ((t >> lo) << (lo + 4)).
// The forward transform (merged negacyclic Cooley-Tukey, natural order in,
// bit-reversed order out) runs its stages in three register rounds with
// lo = log2N-4, log2N-8 and 0, exchanging data through LDS between rounds;
// the inverse (decimation in time on the bit-reversed order with roots
// omega^-1 = psi^-2, then the twist psi^-j N^-1) walks the rounds back.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fs {

// Pointer into global memory.  Pointers read from memory are generic to the
// compiler, which then addresses through the flat aperture; a global one
// lets it use a scalar base with 32-bit per-lane offsets.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}
// Element i (i * sizeof(T) < 2^32) of a global array: the byte offset is
// formed in 32 bits so the load takes the base from scalar registers and
// one 32-bit offset register per lane.
template <class T>
__device__ __forceinline__ T ldg(const T* base, uint32_t i) {
  using gchar = const __attribute__((address_space(1))) char*;
  return *(gptr<T>)((gchar)as_global(base) + i * (uint32_t)sizeof(T));
}

// A pointer that is the same in every lane, moved into scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

// A read-only table of doubles addressed through a raw buffer descriptor:
// the descriptor lives in scalar registers and a load takes a per-lane
// 32-bit byte offset plus a uniform one, so a group of loads whose offsets
// differ by constants shares one vector register however far apart the
// constants are.  (Word 3 = 0x00020000 is the gfx9 raw-buffer format: 32-bit
// data, no swizzle; the range is left open, every offset used is < 2^31.)
struct Tab {
  __amdgpu_buffer_rsrc_t r;
  __device__ explicit Tab(const double* p)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, 0x7fffffff, 0x00020000)) {}
  // element at byte offset vbytes + sbytes
  __device__ double at(uint32_t vbytes, uint32_t sbytes) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vbytes, sbytes, 0));
  }
  // two adjacent elements in one 16-byte load
  __device__ void at2(uint32_t vbytes, uint32_t sbytes, double& lo, double& hi) const {
    struct D2 {
      double lo, hi;
    };
    const D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, vbytes, sbytes, 0));
    lo = v.lo;
    hi = v.hi;
  }
};

constexpr uint64_t kNttPrime = 0x6000000100001ull;  // 3*2^49 + 2^20 + 1
constexpr double kP = 1688849861312513.0;
constexpr double kPinv = 1.0 / 1688849861312513.0;
// bound on |integer product sum| that keeps the centred lift exact
constexpr double kExactBound = 844424930656256.0;  // (P - 1) / 2

__device__ __forceinline__ double mulmod(double a, double w) {
  const double h = a * w;
  const double l = __builtin_fma(a, w, -h);
  const double q = __builtin_rint(h * kPinv);
  const double r = __builtin_fma(-q, kP, h);
  return r + l;
}

__device__ __forceinline__ double redc(double x) {
  const double q = __builtin_rint(x * kPinv);
  return __builtin_fma(-q, kP, x);
}

template <int LOGN, int LO>
__device__ __forceinline__ int jmap(int t, int r) {
  return (t & ((1 << LO) - 1)) | (r << LO) | ((t >> LO) << (LO + 4));
}

// LDS slot of coefficient index j (one padding word per 16 keeps the three
// register mappings free of bank conflicts beyond the minimum two passes).
__device__ __forceinline__ int lds_slot(int j) { return j + (j >> 4); }

// The slot of j(t, r) splits as slot(j(t, 0)) + slot(j(0, r)): the thread and
// register parts of the index occupy disjoint bits, and their bits below 4
// (thread bits under LO, register bits from LO up) never carry into bit 4.
// So an exchange addresses LDS from one per-thread base with compile-time
// offsets for the sixteen registers.
template <int LOGN, int LO>
__device__ __forceinline__ int slot_base(int t) {
  return lds_slot(jmap<LOGN, LO>(t, 0));
}
template <int LO>
__host__ __device__ constexpr int slot_reg(int r) {
  return (r << LO) + ((r << LO) >> 4);
}

template <int LOGN>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int TP = N / 16;           // threads per polynomial
  static constexpr int LOA = LOGN - 4;        // round A: top four bits
  static constexpr int LOB = LOGN - 8;        // round B: middle bits
  static constexpr int LDS_DOUBLES = N + N / 16;
};

// Ordering of the LDS accesses of one polynomial's threads.  When the TP
// threads form a single wavefront, its LDS instructions execute in issue
// order, so a wavefront-scope fence (which only stops the compiler from
// moving accesses across it) is enough and no barrier or wait is spent;
// polynomials spread over several waves need a workgroup barrier.
template <int TP>
__device__ __forceinline__ void poly_sync() {
  if constexpr (TP <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Orders one wavefront's own LDS accesses (compiler fence only).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange between two register mappings through LDS.  Default: barriers
// before and after the reads.  LEAN (polynomials of several waves, for the
// blind rotation's one-group job, whose callers place the remaining
// barriers): with TP = 128 the thread bit 6 is exponent bit 10 in the
// mappings of rounds B and C, so there each wave owns the LDS half of the
// coefficients with that bit equal to its wave number and the B <-> C
// exchanges stay inside the wave (compiler fences only); an A <-> B
// exchange crosses waves and keeps the barrier between its writes and
// reads, but not the one after the reads: the next access of another wave
// to the slots read here comes after the next transform's entry barrier.
// PAIR: the next stage's first butterflies pair registers r and r + PAIR;
// the reads are requested in the order r, r + 1, r + PAIR, r + PAIR + 1, ...
// (the compiler merges each two adjacent registers into one paired read), so
// that the first butterflies wait for two paired reads instead of five.
template <int LOGN, int LO_FROM, int LO_TO, bool LEAN = false, int PAIR = 8>
__device__ __forceinline__ void exchange(double x[16], double* lds, int t) {
  static_assert(PAIR >= 2 && PAIR <= 8 && (PAIR & (PAIR - 1)) == 0, "pairs of registers");
  constexpr int TP = (1 << LOGN) / 16;
  static_assert(!LEAN || TP <= 64 || (TP == 128 && LOGN == 11), "lean schedule derived for TP = 128");
  constexpr bool CROSS = LO_FROM == LOGN - 4 || LO_TO == LOGN - 4;  // into or out of round A
  double* wp = lds + slot_base<LOGN, LO_FROM>(t);
  const double* rp = lds + slot_base<LOGN, LO_TO>(t);
#pragma unroll
  for (int r = 0; r < 16; ++r) wp[slot_reg<LO_FROM>(r)] = x[r];
  if constexpr (LEAN && !CROSS) wave_sync();
  else poly_sync<TP>();
#pragma unroll
  for (int g = 0; g < 16; g += 2) {
    if (g & PAIR) continue;
    x[g] = rp[slot_reg<LO_TO>(g)];
    x[g + 1] = rp[slot_reg<LO_TO>(g + 1)];
    x[g + PAIR] = rp[slot_reg<LO_TO>(g + PAIR)];
    x[g + PAIR + 1] = rp[slot_reg<LO_TO>(g + PAIR + 1)];
  }
  if constexpr (LEAN && TP > 64) wave_sync();
  else poly_sync<TP>();
}

template <int N>
__device__ __forceinline__ void reduce16(double x[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = redc(x[r]);
}

// Forward stages SHI down to SLO, in the mapping with register bits at LO.
// Stage s pairs j and j + 2^s; its root is psi^{brv(k)} with
// k = N/2^{s+1} + j/2^{s+1} (tw holds psi^{brv(k)} at index k).
template <int LOGN, int LO, int SHI, int SLO>
__device__ __forceinline__ void fwd_stages(double x[16], const double* __restrict__ tw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SHI; s >= SLO; --s) {
    const int b = s - LO;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << b)) continue;
      const int r2 = r | (1 << b);
      const int j = jmap<LOGN, LO>(t, r);
      const double w = ldg(tw, (N >> (s + 1)) + (j >> (s + 1)));
      const double m = mulmod(x[r2], w);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

// Forward negacyclic NTT.  In: coefficients in round-A mapping, each of
// magnitude < 2^40.  Out: evaluations in bit-reversed order, round-C mapping
// (thread t holds positions 16t .. 16t+15), reduced to |x| <= P/2 + 1.
template <int LOGN>
__device__ __forceinline__ void ntt_fwd(double x[16], double* lds, const double* __restrict__ tw,
                                        int t) {
  using S = NttShape<LOGN>;
  fwd_stages<LOGN, S::LOA, LOGN - 1, LOGN - 4>(x, tw, t);  // |x| < 3.1 P
  reduce16<S::N>(x);
  exchange<LOGN, S::LOA, S::LOB>(x, lds, t);
  fwd_stages<LOGN, S::LOB, LOGN - 5, 4>(x, tw, t);  // 2 or 3 stages: < 3.1 P
  reduce16<S::N>(x);
  exchange<LOGN, S::LOB, 0>(x, lds, t);
  fwd_stages<LOGN, 0, 3, 0>(x, tw, t);  // < 4.4 P
  reduce16<S::N>(x);
}

// ---------------------------------------------------------------------------
// Register-twiddle forms used by the blind rotation (and the product
// check).  The forward transform is that of ntt_fwd; every root comes from
// registers instead of a table load inside a stage:
//  - forward round A and inverse round C' use roots that are the same for
//    all threads (they depend on register bits only); they are passed in the
//    kernel-argument segment and read as scalars;
//  - in the other rounds, stage s with register bits at LO has a root that
//    depends on the thread and on r >> (b+1) (forward) or r & (2^b - 1)
//    (inverse), b = s - LO: 16 >> (b+1) resp. 2^b values per thread, loaded
//    once per use site into a small register array.

// forward: number of per-thread roots of stages SHI..SLO, and the offset of
// stage S inside that block
template <int LO, int SHI, int SLO>
__host__ __device__ constexpr int fwd_lane_count() {
  int c = 0;
  for (int s = SHI; s >= SLO; --s) c += 16 >> (s - LO + 1);
  return c;
}
__host__ __device__ constexpr int fwd_lane_off(int LO, int SHI, int S) {
  int c = 0;
  for (int s = SHI; s > S; --s) c += 16 >> (s - LO + 1);
  return c;
}
// inverse: 2^b roots per stage
template <int LO, int SLO, int SHI>
__host__ __device__ constexpr int inv_lane_count() {
  int c = 0;
  for (int s = SLO; s <= SHI; ++s) c += 1 << (s - LO);
  return c;
}
__host__ __device__ constexpr int inv_lane_off(int LO, int SLO, int S) {
  int c = 0;
  for (int s = SLO; s < S; ++s) c += 1 << (s - LO);
  return c;
}

template <int LOGN>
struct RegTw {
  using S = NttShape<LOGN>;
  // forward rounds B (stages LOGN-5..4, LO = LOB) and C (stages 3..0, LO = 0)
  static constexpr int FB = fwd_lane_count<S::LOB, LOGN - 5, 4>();
  static constexpr int FC = fwd_lane_count<0, 3, 0>();
  static constexpr int FWD = FB + FC;
  // inverse rounds B' (stages 4..LOGN-5) and A' (LOGN-4..LOGN-1), plus the twist
  static constexpr int IB = inv_lane_count<S::LOB, 4, LOGN - 5>();
  static constexpr int IA = inv_lane_count<S::LOA, LOGN - 4, LOGN - 1>();
  static constexpr int INV = IB + IA + 16;
};

// Uniform roots: forward round A uses psi^{brv(k)}, k = 1..15; inverse round
// C' uses omega^{-m N/16}, m = 0..7.
struct UniTw {
  double fwd[16];
  double inv[8];
};

template <int LOGN, int LO, int SHI, int SLO>
__device__ __forceinline__ void load_fwd_lane(double* w, const Tab& tw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SHI; s >= SLO; --s) {
    const int b = s - LO;
    // j(t, q 2^{b+1}) = j(t, 0) + q 2^{s+1}, so the root index is affine in q
    const uint32_t base = (uint32_t)jmap<LOGN, LO>(t, 0) >> (s + 1);
#pragma unroll
    for (int q = 0; q < (16 >> (b + 1)); ++q)
      w[fwd_lane_off(LO, SHI, s) + q] = tw.at(base * 8u, ((N >> (s + 1)) + q) * 8u);
  }
}

// Forward stages SHI down to SLO of the round whose top stage is RHI.
template <int LOGN, int LO, int RHI, int SHI, int SLO>
__device__ __forceinline__ void fwd_stages_reg(double x[16], const double* w) {
#pragma unroll
  for (int s = SHI; s >= SLO; --s) {
    const int b = s - LO;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << b)) continue;
      const int r2 = r | (1 << b);
      const double m = mulmod(x[r2], w[fwd_lane_off(LO, RHI, s) + (r >> (b + 1))]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

// Stages SHI down to LOGN-4 of round A (SHI = LOGN-2 when the caller has
// done the first stage itself).
template <int LOGN, int SHI = LOGN - 1>
__device__ __forceinline__ void fwd_roundA_uni(double x[16], const UniTw& u) {
  using S = NttShape<LOGN>;
#pragma unroll
  for (int s = SHI; s >= LOGN - 4; --s) {
    const int b = s - S::LOA;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << b)) continue;
      const int r2 = r | (1 << b);
      // k = N/2^{s+1} + j/2^{s+1} with j = t + TP r: the thread part drops out
      const double m = mulmod(x[r2], u.fwd[(1 << (LOGN - 1 - s)) + (r >> (b + 1))]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

// Forward transform with register roots: the transform of ntt_fwd with a
// shorter reduction schedule for digit inputs (|x| <= 512): five stages,
// reduce, four stages, reduce, the remaining one or two stages.  The output
// is NOT reduced: |x| < 1.14 P (N = 1024) or 1.97 P (N = 2048), which keeps
// a sum of 2l products with reduced key values below 5 P < 2^53 (the bound
// check of this schedule is in tests/test_ntt_bounds.py).  DONE = number of
// leading stages the caller has already applied (by table, |x| <= 1.5 P
// after two).  The per-thread roots of rounds B and C are requested one
// round ahead.
//
// LEAN: the exchange schedule of `exchange` for one-group blind-rotation
// jobs; `entry` then places a workgroup barrier before the first LDS write
// (needed unless the caller's last access to the buffer was a transform's
// round-B/C half of its own wave, see exchange).
//
// HELD: the per-thread roots of rounds B and C come from `held` (R::FB then
// R::FC values, loaded once per thread with load_fwd_roots: they depend on
// the thread only) instead of being requested for every transform.
template <int LOGN, int DONE = 0, bool LEAN = false, bool HELD = false>
__device__ __forceinline__ void ntt_fwd_reg(double x[16], double* lds, const UniTw& u,
                                            const Tab& tw, int t, bool entry = true,
                                            const double* held = nullptr) {
  using S = NttShape<LOGN>;
  using R = RegTw<LOGN>;
  constexpr int BHI = LOGN - 5;  // round B: stages BHI..4, round C: 3..0
  static_assert(DONE >= 0 && DONE <= 2, "at most two stages by table");
  double wb_own[HELD ? 1 : R::FB];
  const double* wb = wb_own;
  if constexpr (HELD) wb = held;
  else load_fwd_lane<LOGN, S::LOB, BHI, 4>(wb_own, tw, t);
  fwd_roundA_uni<LOGN, LOGN - 1 - DONE>(x, u);
  if constexpr (LEAN && S::TP > 64) {
    if (entry) __syncthreads();
  }
  exchange<LOGN, S::LOA, S::LOB, LEAN>(x, lds, t);
  double wc_own[HELD ? 1 : R::FC];
  const double* wc = wc_own;
  if constexpr (HELD) wc = held + R::FB;
  else load_fwd_lane<LOGN, 0, 3, 0>(wc_own, tw, t);
  fwd_stages_reg<LOGN, S::LOB, BHI, BHI, BHI>(x, wb);  // fifth stage
  reduce16<S::N>(x);
  fwd_stages_reg<LOGN, S::LOB, BHI, BHI - 1, 4>(x, wb);
  exchange<LOGN, S::LOB, 0, LEAN>(x, lds, t);
  // stages 3 .. LOGN-9 complete the second segment of four
  fwd_stages_reg<LOGN, 0, 3, 3, LOGN - 9>(x, wc);
  reduce16<S::N>(x);
  fwd_stages_reg<LOGN, 0, 3, LOGN - 10, 0>(x, wc);
}

// Every per-thread root of a forward transform's rounds B and C (see
// ntt_fwd_reg's HELD form): RegTw<LOGN>::FWD values.
template <int LOGN>
__device__ __forceinline__ void load_fwd_roots(double* w, const Tab& tw, int t) {
  using S = NttShape<LOGN>;
  load_fwd_lane<LOGN, S::LOB, LOGN - 5, 4>(w, tw, t);
  load_fwd_lane<LOGN, 0, 3, 0>(w + RegTw<LOGN>::FB, tw, t);
}

template <int LOGN, int LO, int SLO, int SHI>
__device__ __forceinline__ void load_inv_lane(double* w, const Tab& itw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SLO; s <= SHI; ++s) {
    const int b = s - LO;
    // i(t, q) mod 2^s = (i(t, 0) mod 2^s) + q 2^LO for q < 2^b: affine in q
    const uint32_t m = (uint32_t)N >> (s + 1);
    const uint32_t base = ((uint32_t)jmap<LOGN, LO>(t, 0) & ((1u << s) - 1)) * m;
#pragma unroll
    for (int q = 0; q < (1 << b); ++q)
      w[inv_lane_off(LO, SLO, s) + q] = itw.at(base * 8u, ((uint32_t)q << LO) * m * 8u);
  }
}

// Inverse stages SLO up to SHI of the round whose first stage is RLO.
template <int LOGN, int LO, int RLO, int SLO, int SHI>
__device__ __forceinline__ void inv_stages_reg(double x[16], const double* w) {
#pragma unroll
  for (int s = SLO; s <= SHI; ++s) {
    const int b = s - LO;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << b)) continue;
      const int r2 = r | (1 << b);
      const double m = mulmod(x[r2], w[inv_lane_off(LO, RLO, s) + (r & ((1 << b) - 1))]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

template <int LOGN>
__device__ __forceinline__ void inv_roundC_uni(double x[16], const UniTw& u, int slo, int shi) {
#pragma unroll
  for (int s = 0; s <= 3; ++s) {
    if (s < slo || s > shi) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << s)) continue;
      const int r2 = r | (1 << s);
      const int m8 = (r & ((1 << s) - 1)) << (3 - s);  // e = m8 * N / 16
      const double m = m8 == 0 ? x[r2] : mulmod(x[r2], u.inv[m8]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

// Inverse negacyclic transform with register roots.  In: round-C mapping
// (bit-reversed positions), |x| < 5 P.  Decimation in time on the
// bit-reversed order with roots omega^-1 = psi^-2: stage s pairs positions
// i and i + 2^s (bit s of i clear) with root omega^{-e}, e = (i mod 2^s)
// N / 2^{s+1}.  Reductions before stages 0, 3 and 7 only (stages 0..2 contain
// butterflies whose root is 1 and double the bound); ends with the twist
// psi^-j N^-1 and a reduction, giving the exact centred residue in round-A
// mapping (thread t, register r: coefficient t + TP r).  The per-thread roots
// of each round are requested one round ahead.
// LEAN and `entry` as for ntt_fwd_reg.  HELD: the per-thread roots of rounds
// B' (HELD >= 1) and A' (HELD = 2) come from `held` (R::IB then R::IA values,
// loaded once with load_inv_roots) instead of being requested for every
// transform.
template <int LOGN, bool LEAN = false, int HELD = 0>
__device__ __forceinline__ void ntt_inv_reg(double x[16], double* lds, const UniTw& u,
                                            const Tab& itw, const Tab& post, int t,
                                            bool entry = true, const double* held = nullptr) {
  using S = NttShape<LOGN>;
  using R = RegTw<LOGN>;
  constexpr int BHI = LOGN - 5;  // round B': stages 4..BHI, round A': BHI+1..LOGN-1
  double wb_own[HELD >= 1 ? 1 : R::IB];
  const double* wb = wb_own;
  if constexpr (HELD >= 1) wb = held;
  else load_inv_lane<LOGN, S::LOB, 4, BHI>(wb_own, itw, t);
  reduce16<S::N>(x);
  inv_roundC_uni<LOGN>(x, u, 0, 2);
  reduce16<S::N>(x);
  inv_roundC_uni<LOGN>(x, u, 3, 3);
  if constexpr (LEAN && S::TP > 64) {
    if (entry) __syncthreads();
  }
  // round B' starts with stage 4, which pairs registers r and r + 2^(4 - LOB)
  exchange<LOGN, 0, S::LOB, LEAN, (1 << (4 - S::LOB))>(x, lds, t);
  double wa_own[HELD == 2 ? 1 : R::IA];
  const double* wa = wa_own;
  if constexpr (HELD == 2) wa = held + R::IB;
  else load_inv_lane<LOGN, S::LOA, LOGN - 4, LOGN - 1>(wa_own, itw, t);
  inv_stages_reg<LOGN, S::LOB, 4, 4, BHI>(x, wb);
  exchange<LOGN, S::LOB, S::LOA, LEAN>(x, lds, t);
  double wp[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) wp[r] = post.at((uint32_t)t * 8u, (uint32_t)(S::TP * r) * 8u);
  if constexpr (LOGN - 4 <= 6) {  // N = 1024: stage 6 is the first of round A'
    inv_stages_reg<LOGN, S::LOA, LOGN - 4, LOGN - 4, 6>(x, wa);
    reduce16<S::N>(x);
    inv_stages_reg<LOGN, S::LOA, LOGN - 4, 7, LOGN - 1>(x, wa);
  } else {  // N = 2048: stages 3..6 end round B'
    reduce16<S::N>(x);
    inv_stages_reg<LOGN, S::LOA, LOGN - 4, LOGN - 4, LOGN - 1>(x, wa);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = redc(mulmod(x[r], wp[r]));
}

// The per-thread roots of an inverse transform's rounds B' and A' (see
// ntt_inv_reg's HELD form): RegTw<LOGN>::IB + IA values (round B' only when
// ROUNDS = 1).
template <int LOGN, int ROUNDS = 2>
__device__ __forceinline__ void load_inv_roots(double* w, const Tab& itw, int t) {
  using S = NttShape<LOGN>;
  load_inv_lane<LOGN, S::LOB, 4, LOGN - 5>(w, itw, t);
  if constexpr (ROUNDS == 2) load_inv_lane<LOGN, S::LOA, LOGN - 4, LOGN - 1>(w + RegTw<LOGN>::IB, itw, t);
}

// Low 32 bits of an integer-valued double e with |e| < 2^51: e + 1.5 * 2^52
// lies in [2^52, 2^53), where the unit in the last place is 1, so the low
// word of its encoding is (e + 2^51) mod 2^32 = e mod 2^32.
__device__ __forceinline__ uint32_t low32_magic(double e) {
  const double y = e + 6755399441055744.0;  // 1.5 * 2^52
  return (uint32_t)__double_as_longlong(y);
}

}  // namespace fs
