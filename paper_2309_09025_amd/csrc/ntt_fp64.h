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
// N = 2048 (4 digit polynomials, |digit| <= 512) the key is split into two
// 16-bit halves, each product sum then being below 2^37.
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

template <int LOGN, int LO_FROM, int LO_TO>
__device__ __forceinline__ void exchange(double x[16], double* lds, int t) {
  constexpr int TP = (1 << LOGN) / 16;
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[lds_slot(jmap<LOGN, LO_FROM>(t, r))] = x[r];
  poly_sync<TP>();
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = lds[lds_slot(jmap<LOGN, LO_TO>(t, r))];
  poly_sync<TP>();
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
      const double w = tw[(N >> (s + 1)) + (j >> (s + 1))];
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

// Inverse stages SLO up to SHI (decimation in time), register bits at LO.
// Stage s pairs positions i and i + 2^s (i with bit s clear); the root is
// omega^{-e}, e = (i mod 2^s) * N / 2^{s+1}; itw holds omega^{-e} at e.
template <int LOGN, int LO, int SLO, int SHI>
__device__ __forceinline__ void inv_stages(double x[16], const double* __restrict__ itw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SLO; s <= SHI; ++s) {
    const int b = s - LO;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & (1 << b)) continue;
      const int r2 = r | (1 << b);
      const int i = jmap<LOGN, LO>(t, r);
      const int e = (i & ((1 << s) - 1)) * (N >> (s + 1));
      double m;
      if (LO == 0 && (r & ((1 << s) - 1)) == 0) m = x[r2];  // omega^0 = 1
      else m = mulmod(x[r2], itw[e]);
      x[r2] = x[r] - m;
      x[r] = x[r] + m;
    }
  }
}

// Inverse negacyclic NTT.  In: round-C mapping (bit-reversed positions),
// |x| < 5 P.  Out: round-A mapping (thread t, register r holds coefficient
// t + TP r), the exact centred residue of the coefficient.
template <int LOGN>
__device__ __forceinline__ void ntt_inv(double x[16], double* lds, const double* __restrict__ itw,
                                        const double* __restrict__ post, int t) {
  using S = NttShape<LOGN>;
  reduce16<S::N>(x);
  inv_stages<LOGN, 0, 0, 1>(x, itw, t);  // trivial roots double the bound: < 2.1 P
  reduce16<S::N>(x);
  inv_stages<LOGN, 0, 2, 3>(x, itw, t);  // < 2.3 P
  reduce16<S::N>(x);
  exchange<LOGN, 0, S::LOB>(x, lds, t);
  inv_stages<LOGN, S::LOB, 4, LOGN - 5>(x, itw, t);  // < 3.1 P
  reduce16<S::N>(x);
  exchange<LOGN, S::LOB, S::LOA>(x, lds, t);
  inv_stages<LOGN, S::LOA, LOGN - 4, LOGN - 1>(x, itw, t);  // < 4.4 P
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = redc(mulmod(x[r], post[t + S::TP * r]));
}

// ---------------------------------------------------------------------------
// Register-twiddle forms used by the blind rotation.  The same transforms as
// ntt_fwd / ntt_inv, but every root comes from registers instead of a table
// load inside the loop:
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
__device__ __forceinline__ void load_fwd_lane(double* w, const double* __restrict__ tw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SHI; s >= SLO; --s) {
    const int b = s - LO;
#pragma unroll
    for (int q = 0; q < (16 >> (b + 1)); ++q) {
      const int j = jmap<LOGN, LO>(t, q << (b + 1));
      w[fwd_lane_off(LO, SHI, s) + q] =
          tw[(N >> (s + 1)) + (j >> (s + 1))];
    }
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

template <int LOGN>
__device__ __forceinline__ void fwd_roundA_uni(double x[16], const UniTw& u) {
  using S = NttShape<LOGN>;
#pragma unroll
  for (int s = LOGN - 1; s >= LOGN - 4; --s) {
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
// check of this schedule is in tests/test_ntt_bounds.py).  The per-thread
// roots of rounds B and C are requested one round ahead.
template <int LOGN>
__device__ __forceinline__ void ntt_fwd_reg(double x[16], double* lds, const UniTw& u,
                                            const double* __restrict__ tw, int t) {
  using S = NttShape<LOGN>;
  using R = RegTw<LOGN>;
  constexpr int BHI = LOGN - 5;  // round B: stages BHI..4, round C: 3..0
  double wb[R::FB];
  load_fwd_lane<LOGN, S::LOB, BHI, 4>(wb, tw, t);
  fwd_roundA_uni<LOGN>(x, u);
  exchange<LOGN, S::LOA, S::LOB>(x, lds, t);
  double wc[R::FC];
  load_fwd_lane<LOGN, 0, 3, 0>(wc, tw, t);
  fwd_stages_reg<LOGN, S::LOB, BHI, BHI, BHI>(x, wb);  // fifth stage
  reduce16<S::N>(x);
  fwd_stages_reg<LOGN, S::LOB, BHI, BHI - 1, 4>(x, wb);
  exchange<LOGN, S::LOB, 0>(x, lds, t);
  // stages 3 .. LOGN-9 complete the second segment of four
  fwd_stages_reg<LOGN, 0, 3, 3, LOGN - 9>(x, wc);
  reduce16<S::N>(x);
  fwd_stages_reg<LOGN, 0, 3, LOGN - 10, 0>(x, wc);
}

template <int LOGN>
__device__ __forceinline__ void load_fwd_tw(double* wf, const double* __restrict__ tw, int t) {
  using S = NttShape<LOGN>;
  load_fwd_lane<LOGN, S::LOB, LOGN - 5, 4>(wf, tw, t);
  load_fwd_lane<LOGN, 0, 3, 0>(wf + RegTw<LOGN>::FB, tw, t);
}

template <int LOGN, int LO, int SLO, int SHI>
__device__ __forceinline__ void load_inv_lane(double* w, const double* __restrict__ itw, int t) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int s = SLO; s <= SHI; ++s) {
    const int b = s - LO;
#pragma unroll
    for (int q = 0; q < (1 << b); ++q) {
      const int i = jmap<LOGN, LO>(t, q);
      w[inv_lane_off(LO, SLO, s) + q] = itw[(i & ((1 << s) - 1)) * (N >> (s + 1))];
    }
  }
}

template <int LOGN>
__device__ __forceinline__ void load_inv_tw(double* wi, const double* __restrict__ itw,
                                            const double* __restrict__ post, int t) {
  using S = NttShape<LOGN>;
  using R = RegTw<LOGN>;
  load_inv_lane<LOGN, S::LOB, 4, LOGN - 5>(wi, itw, t);
  load_inv_lane<LOGN, S::LOA, LOGN - 4, LOGN - 1>(wi + R::IB, itw, t);
#pragma unroll
  for (int r = 0; r < 16; ++r) wi[R::IB + R::IA + r] = post[t + S::TP * r];
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

// Inverse transform with register roots: the transform of ntt_inv with
// reductions before stages 0, 3 and 7 only (stages 0..2 contain butterflies
// whose root is 1 and double the bound); ends with the twist psi^-j N^-1 and
// a reduction, giving the exact centred residue.  The per-thread roots of
// each round are requested one round ahead.
template <int LOGN>
__device__ __forceinline__ void ntt_inv_reg(double x[16], double* lds, const UniTw& u,
                                            const double* __restrict__ itw,
                                            const double* __restrict__ post, int t) {
  using S = NttShape<LOGN>;
  using R = RegTw<LOGN>;
  constexpr int BHI = LOGN - 5;  // round B': stages 4..BHI, round A': BHI+1..LOGN-1
  double wb[R::IB];
  load_inv_lane<LOGN, S::LOB, 4, BHI>(wb, itw, t);
  reduce16<S::N>(x);
  inv_roundC_uni<LOGN>(x, u, 0, 2);
  reduce16<S::N>(x);
  inv_roundC_uni<LOGN>(x, u, 3, 3);
  exchange<LOGN, 0, S::LOB>(x, lds, t);
  double wa[R::IA];
  load_inv_lane<LOGN, S::LOA, LOGN - 4, LOGN - 1>(wa, itw, t);
  inv_stages_reg<LOGN, S::LOB, 4, 4, BHI>(x, wb);
  exchange<LOGN, S::LOB, S::LOA>(x, lds, t);
  double wp[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) wp[r] = post[t + S::TP * r];
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

// Low 32 bits of an integer-valued double e with |e| < 2^51: e + 1.5 * 2^52
// lies in [2^52, 2^53), where the unit in the last place is 1, so the low
// word of its encoding is (e + 2^51) mod 2^32 = e mod 2^32.
__device__ __forceinline__ uint32_t low32_magic(double e) {
  const double y = e + 6755399441055744.0;  // 1.5 * 2^52
  return (uint32_t)__double_as_longlong(y);
}

// Low 32 bits of an integer-valued double of magnitude < 2^52.
__device__ __forceinline__ uint32_t low32(double e) {
  const double hi = __builtin_floor(e * 0x1p-32);
  const double lo = __builtin_fma(-hi, 0x1p32, e);  // in [0, 2^32)
  return (uint32_t)lo;
}

}  // namespace fs
