// WeightSum on LWE ciphertexts (Sec. 4.1, Eq. "noise grows"): plaintext
// integer weights times ciphertexts, summed word by word mod 2^32, for
// fully connected and convolutional layers, plus the homomorphic addition
// that forms H = V + I (Theorem 3.1, Eq. DiscretEquation).
//
// These layers are integer contractions with tiny weights (|w| <= 15 in
// the workloads) and move far fewer operations than the bootstrappings
// they feed; they run on the vector ALUs with coalesced ciphertext rows.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fs {

// y[o][w] = add[o][w] + sum_i W[o][i] x[i][w].  Block: 256 words w of OT
// consecutive outputs o; each x word loaded once feeds OT products.  W
// reads are uniform across the block (scalar loads).
template <int OT>
__global__ void __launch_bounds__(256)
lwe_linear_kernel(const int32_t* __restrict__ W, uint32_t O, uint32_t I, uint32_t dim,
                  const uint32_t* __restrict__ x, const uint32_t* add, uint32_t* y) {
  const uint32_t w = blockIdx.x * 256 + threadIdx.x;
  const uint32_t o0 = blockIdx.y * OT;
  uint32_t acc[OT];
#pragma unroll
  for (int k = 0; k < OT; ++k) acc[k] = 0u;
  const bool live = w < dim;
  const uint32_t wc = live ? w : 0;
  for (uint32_t i = 0; i < I; ++i) {
    const uint32_t xv = x[(size_t)i * dim + wc];
#pragma unroll
    for (int k = 0; k < OT; ++k) {
      const uint32_t o = o0 + k < O ? o0 + k : O - 1;
      acc[k] += (uint32_t)W[(size_t)o * I + i] * xv;
    }
  }
  if (!live) return;
#pragma unroll
  for (int k = 0; k < OT; ++k) {
    const uint32_t o = o0 + k;
    if (o < O) {
      const size_t idx = (size_t)o * dim + w;
      y[idx] = acc[k] + (add ? add[idx] : 0u);
    }
  }
}

// Split form for layers too small to fill the device: blockIdx.z takes
// inputs [z KC, (z + 1) KC) and adds its partial sums into y with 32-bit
// atomics (sums mod 2^32 do not depend on the order); y already holds the
// add rows or zeros (lwe_fill_kernel).
template <int OT>
__global__ void __launch_bounds__(256)
lwe_linear_split_kernel(const int32_t* __restrict__ W, uint32_t O, uint32_t I, uint32_t KC,
                        uint32_t dim, const uint32_t* __restrict__ x, uint32_t* y) {
  const uint32_t w = blockIdx.x * 256 + threadIdx.x;
  const uint32_t o0 = blockIdx.y * OT;
  const uint32_t i0 = blockIdx.z * KC;
  const uint32_t i1 = i0 + KC < I ? i0 + KC : I;
  uint32_t acc[OT];
#pragma unroll
  for (int k = 0; k < OT; ++k) acc[k] = 0u;
  const bool live = w < dim;
  const uint32_t wc = live ? w : 0;
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t xv = x[(size_t)i * dim + wc];
#pragma unroll
    for (int k = 0; k < OT; ++k) {
      const uint32_t o = o0 + k < O ? o0 + k : O - 1;
      acc[k] += (uint32_t)W[(size_t)o * I + i] * xv;
    }
  }
  if (!live) return;
#pragma unroll
  for (int k = 0; k < OT; ++k) {
    const uint32_t o = o0 + k;
    if (o < O) atomicAdd(&y[(size_t)o * dim + w], acc[k]);
  }
}

// y = src (or zeros when src is null), `words` words.
__global__ void __launch_bounds__(256)
lwe_fill_kernel(const uint32_t* src, size_t words, uint32_t* y) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < words) y[i] = src ? src[i] : 0u;
}

// Convolution: block = 256 words of one output position (co, oy, ox).
__global__ void __launch_bounds__(256)
lwe_conv2d_kernel(const int32_t* __restrict__ W, uint32_t Ci, uint32_t H, uint32_t Wd,
                  uint32_t K, uint32_t stride, uint32_t pad, uint32_t Ho, uint32_t Wo,
                  uint32_t dim, const uint32_t* __restrict__ x, const uint32_t* add,
                  uint32_t* y) {
  const uint32_t w = blockIdx.y * 256 + threadIdx.x;
  const uint32_t o = blockIdx.x;  // (co*Ho + oy)*Wo + ox
  if (w >= dim) return;
  const uint32_t ox = o % Wo, oy = (o / Wo) % Ho, co = o / (Wo * Ho);
  uint32_t acc = 0u;
  for (uint32_t ci = 0; ci < Ci; ++ci)
    for (uint32_t ky = 0; ky < K; ++ky) {
      const int iy = (int)(oy * stride + ky) - (int)pad;
      if (iy < 0 || iy >= (int)H) continue;
      for (uint32_t kx = 0; kx < K; ++kx) {
        const int ix = (int)(ox * stride + kx) - (int)pad;
        if (ix < 0 || ix >= (int)Wd) continue;
        const uint32_t wt = (uint32_t)W[((co * Ci + ci) * K + ky) * K + kx];
        acc += wt * x[(((size_t)ci * H + iy) * Wd + ix) * dim + w];
      }
    }
  const size_t idx = (size_t)o * dim + w;
  y[idx] = acc + (add ? add[idx] : 0u);
}

__global__ void __launch_bounds__(256)
lwe_add_kernel(const uint32_t* a, const uint32_t* b, size_t words, uint32_t* y) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < words) y[i] = a[i] + b[i];
}

// y = x + (0, ..., 0, delta * c[row]): a plaintext added to each ciphertext
// (its trivial encryption has zero mask), row by row.
__global__ void __launch_bounds__(256)
lwe_add_plain_kernel(const uint32_t* x, const int32_t* c, uint32_t delta, size_t count,
                     uint32_t dim, uint32_t* y) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count * dim) return;
  const size_t row = i / dim;
  const uint32_t w = (uint32_t)(i - row * dim);
  y[i] = x[i] + (w == dim - 1 ? delta * (uint32_t)c[row] : 0u);
}

#define FS_LAUNCH_CHECK()                 \
  do {                                    \
    hipError_t e_ = hipGetLastError();    \
    if (e_ != hipSuccess) return (int)e_; \
  } while (0)

// A layer whose output tiles give fewer than kLinearBlocks workgroups has
// its inputs split into up to 16 chunks, so that the device holds enough
// waves to hide the load latency of its long reduction.
constexpr uint32_t kLinearBlocks = 2048;

int launch_lwe_linear(const int32_t* W, size_t O, size_t I, uint32_t dim, const uint32_t* x,
                      const uint32_t* add, uint32_t* y, hipStream_t st) {
  if (O == 0) return 0;
  constexpr int OT = 8;
  const uint32_t bx = (dim + 255) / 256, by = (uint32_t)((O + OT - 1) / OT);
  uint32_t split = kLinearBlocks / (bx * by);
  if (split > 16) split = 16;
  if (split > I / 64) split = (uint32_t)(I / 64);  // chunks of at least 64 inputs
  if (split <= 1) {
    lwe_linear_kernel<OT><<<dim3(bx, by), 256, 0, st>>>(W, (uint32_t)O, (uint32_t)I, dim, x, add, y);
    FS_LAUNCH_CHECK();
    return 0;
  }
  const uint32_t kc = (uint32_t)((I + split - 1) / split);
  split = (uint32_t)((I + kc - 1) / kc);
  if (add != y) {  // y = add (or 0); with y == add it already holds the rows
    const size_t words = O * (size_t)dim;
    lwe_fill_kernel<<<dim3((uint32_t)((words + 255) / 256)), 256, 0, st>>>(add, words, y);
    FS_LAUNCH_CHECK();
  }
  lwe_linear_split_kernel<OT><<<dim3(bx, by, split), 256, 0, st>>>(W, (uint32_t)O, (uint32_t)I, kc,
                                                                   dim, x, y);
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_lwe_conv2d(const int32_t* W, uint32_t Ci, uint32_t H, uint32_t Wd, uint32_t Co,
                      uint32_t K, uint32_t stride, uint32_t pad, uint32_t dim,
                      const uint32_t* x, const uint32_t* add, uint32_t* y, hipStream_t st) {
  const uint32_t Ho = (H + 2 * pad - K) / stride + 1, Wo = (Wd + 2 * pad - K) / stride + 1;
  dim3 g(Co * Ho * Wo, (dim + 255) / 256);
  lwe_conv2d_kernel<<<g, 256, 0, st>>>(W, Ci, H, Wd, K, stride, pad, Ho, Wo, dim, x, add, y);
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_lwe_add(const uint32_t* a, const uint32_t* b, size_t words, uint32_t* y,
                   hipStream_t st) {
  if (words == 0) return 0;
  lwe_add_kernel<<<dim3((uint32_t)((words + 255) / 256)), 256, 0, st>>>(a, b, words, y);
  FS_LAUNCH_CHECK();
  return 0;
}

int launch_lwe_add_plain(const uint32_t* x, const int32_t* c, uint32_t delta, size_t count,
                         uint32_t dim, uint32_t* y, hipStream_t st) {
  const size_t words = count * dim;
  if (words == 0) return 0;
  lwe_add_plain_kernel<<<dim3((uint32_t)((words + 255) / 256)), 256, 0, st>>>(x, c, delta, count,
                                                                               dim, y);
  FS_LAUNCH_CHECK();
  return 0;
}

}  // namespace fs
