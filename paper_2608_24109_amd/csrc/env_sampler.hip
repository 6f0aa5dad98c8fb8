// Importance-sampling distribution over environment texels, proportional to the map's
// brightness times the texel's spherical area (Direct Illumination):
//   w_ij = (0.2126 R + 0.7152 G + 0.0722 B) * Omega_i,
//   Omega_i = (2 pi / We) (cos(i pi / He) - cos((i+1) pi / He))        (exact solid angle)
//   q_ij = max(1, floor(w_ij / max w * 2^20))                          (integer weights)
//   cdf_col = inclusive prefix inside a row, cdf_row = inclusive prefix of row totals,
//   pdf_ij = q_ij / (Q Omega_i).
// Two derived tables speed up sampling without changing any pick: the cutpoint tables over
// cdf_row and each row of cdf_col, with compact copies (cdf_col in 32 and 16 bits, column entries
// in 16) for maps narrower than 4096 texels (their layout is described with env_guide_len), and a packed
// record per texel (E_ij, 1/pdf_ij) so that a pick reads one 16-byte record.
// Weights are computed in FP64 without FMA contraction so that the integer tables are the
// exact function of the map. No workspace: intermediate values live in the output buffers
// (cdf_col holds the FP64 weights, cdf_row the row maxima, pdf the row totals) until the
// kernel that owns the final value overwrites them; the kernels run in stream order.
#include <hip/hip_runtime.h>

#include "exm_device.h"
#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ double texel_omega(int32_t i, int32_t He, int32_t We) {
#pragma clang fp contract(off)
  return 2.0 * kPiD / (double)We * (cos((double)i * kPiD / (double)He) - cos((double)(i + 1) * kPiD / (double)He));
}

// one block per row: weights into cdf_col (as double bits), row max into cdf_row[i]
__global__ __launch_bounds__(kThreads) void k_weights(const float* __restrict__ env, int32_t He, int32_t We,
                                                      uint64_t* __restrict__ cdf_row, uint64_t* __restrict__ cdf_col) {
#pragma clang fp contract(off)
  const int32_t i = blockIdx.x;
  const double om = texel_omega(i, He, We);
  double mx = 0.0;
  for (int32_t j = threadIdx.x; j < We; j += kThreads) {
    const float* e = env + 3 * ((int64_t)i * We + j);
    const double lum = (0.2126 * (double)e[0] + 0.7152 * (double)e[1]) + 0.0722 * (double)e[2];
    const double w = lum * om;
    cdf_col[(int64_t)i * We + j] = __double_as_longlong(w);
    mx = fmax(mx, w);
  }
  __shared__ double red[kThreads];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) cdf_row[i] = __double_as_longlong(red[0]);
}

// inclusive block scan of u64 values (one value per thread)
__device__ __forceinline__ uint64_t block_scan(uint64_t v, uint64_t* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    uint64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0ull;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  return sh[threadIdx.x];
}

// one block per row: global max from the row maxima, quantise, in-row inclusive scan;
// the row total goes to the pdf buffer (as u64) until k_row_scan consumes it
__global__ __launch_bounds__(kThreads) void k_quantise(int32_t He, int32_t We, const uint64_t* __restrict__ cdf_row,
                                                       uint64_t* __restrict__ cdf_col, uint64_t* __restrict__ row_tot) {
#pragma clang fp contract(off)
  __shared__ double red[kThreads];
  __shared__ uint64_t sh[kThreads];
  double mx = 0.0;
  for (int32_t r = threadIdx.x; r < He; r += kThreads) mx = fmax(mx, __longlong_as_double(cdf_row[r]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double wmax = red[0];
  const int32_t i = blockIdx.x;
  uint64_t carry = 0;
  for (int32_t j0 = 0; j0 < We; j0 += kThreads) {
    const int32_t j = j0 + threadIdx.x;
    uint64_t q = 0;
    if (j < We) {
      const double w = __longlong_as_double(cdf_col[(int64_t)i * We + j]);
      const double s = wmax > 0.0 ? floor(w / wmax * 1048576.0) : 0.0;
      q = s < 1.0 ? 1ull : (uint64_t)s;
    }
    const uint64_t inc = block_scan(q, sh);
    if (j < We) cdf_col[(int64_t)i * We + j] = carry + inc;
    carry += sh[kThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) row_tot[i] = carry;
}

// single block: inclusive scan of the row totals into cdf_row
__global__ __launch_bounds__(kThreads) void k_row_scan(int32_t He, const uint64_t* __restrict__ row_tot,
                                                       uint64_t* __restrict__ cdf_row) {
  __shared__ uint64_t sh[kThreads];
  uint64_t carry = 0;
  for (int32_t i0 = 0; i0 < He; i0 += kThreads) {
    const int32_t i = i0 + threadIdx.x;
    const uint64_t v = i < He ? row_tot[i] : 0ull;
    const uint64_t inc = block_scan(v, sh);
    if (i < He) cdf_row[i] = carry + inc;
    carry += sh[kThreads - 1];
    __syncthreads();
  }
}

// one block per row: pdf = q / (Q Omega), and the texel's sampling record
__global__ __launch_bounds__(kThreads) void k_pdf(const float* __restrict__ env, int32_t He, int32_t We,
                                                  const uint64_t* __restrict__ cdf_row,
                                                  const uint64_t* __restrict__ cdf_col, float* __restrict__ pdf,
                                                  float4* __restrict__ rec) {
#pragma clang fp contract(off)
  const int32_t i = blockIdx.x;
  const double Q = (double)cdf_row[He - 1];
  const double om = texel_omega(i, He, We);
  for (int32_t j = threadIdx.x; j < We; j += kThreads) {
    const int64_t t = (int64_t)i * We + j;
    const uint64_t q = cdf_col[t] - (j > 0 ? cdf_col[t - 1] : 0ull);
    const float pd = (float)((double)q / (Q * om));
    pdf[t] = pd;
    rec[t] = make_float4(env[3 * t], env[3 * t + 1], env[3 * t + 2], __builtin_amdgcn_rcpf(pd));
  }
}

// smallest s with (T - 1) >> s < n: cuts [0, T) into at most n buckets of 2^s keys
__device__ __forceinline__ uint32_t cut_shift(uint64_t T, int32_t n) {
  uint32_t s = 0;
  if (T == 0) return 0;
  while (s < 63 && ((T - 1) >> s) > (uint64_t)(n - 1)) ++s;
  return s;
}

// single block: row shift, row entries and the column shift of every row
__global__ __launch_bounds__(kThreads) void k_guide_rows(int32_t He, int32_t We, const uint64_t* __restrict__ cdf_row,
                                                         const uint64_t* __restrict__ cdf_col,
                                                         uint32_t* __restrict__ guide) {
  const uint32_t s = cut_shift(cdf_row[He - 1], He);
  if (threadIdx.x == 0) guide[0] = s;
  for (int32_t g = threadIdx.x; g <= He; g += kThreads) {
    const uint64_t key = (uint64_t)g << s;
    guide[1 + g] = (uint32_t)min(upper_bound_u64(cdf_row, He, key), He - 1);
  }
  for (int32_t i = threadIdx.x; i < He; i += kThreads)
    guide[He + 2 + i] = cut_shift(cdf_col[(int64_t)i * We + We - 1], We);
}

// column entries: one thread per (row, g), g in [0, We]
__global__ __launch_bounds__(kThreads) void k_guide_cols(int32_t He, int32_t We, const uint64_t* __restrict__ cdf_col,
                                                         uint32_t* __restrict__ guide) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= (int64_t)He * (We + 1)) return;
  const int32_t i = (int32_t)(k / (We + 1)), g = (int32_t)(k - (int64_t)i * (We + 1));
  const uint64_t* row = cdf_col + (int64_t)i * We;
  const uint32_t s = cut_shift(row[We - 1], We);
  const uint32_t entry = (uint32_t)min(upper_bound_u64(row, We, (uint64_t)g << s), We - 1);
  guide[2 * (int64_t)He + 2 + k] = entry;
  if (We < kCdf32MaxW) {  // compact copies: the column CDF in 32 bits (row totals < 2^32), entries in 16
    reinterpret_cast<uint16_t*>(guide + env_col16_offset(He, We))[k] = (uint16_t)entry;
    if (g < We) {
      const int64_t t = (int64_t)i * We + g;
      guide[env_cdf32_offset(He, We) + t] = (uint32_t)row[g];
      reinterpret_cast<uint16_t*>(guide + env_cdf16_offset(He, We))[t] = (uint16_t)(row[g] - 1u);
    }
  }
}

}  // namespace

hipError_t launch_env_sampler(const float* env, int32_t He, int32_t We, uint64_t* cdf_row, uint64_t* cdf_col,
                              float* pdf, uint32_t* guide, float* rec, hipStream_t s) {
  // the pdf buffer (He*We floats) holds the He u64 row totals between k_quantise and k_row_scan
  uint64_t* row_tot = reinterpret_cast<uint64_t*>(pdf);
  {
    EXM_TIMED("env_weights", s);
    k_weights<<<He, kThreads, 0, s>>>(env, He, We, cdf_row, cdf_col);
  }
  {
    EXM_TIMED("env_quantise", s);
    k_quantise<<<He, kThreads, 0, s>>>(He, We, cdf_row, cdf_col, row_tot);
  }
  {
    EXM_TIMED("env_row_scan", s);
    k_row_scan<<<1, kThreads, 0, s>>>(He, row_tot, cdf_row);
  }
  {
    EXM_TIMED("env_pdf", s);
    k_pdf<<<He, kThreads, 0, s>>>(env, He, We, cdf_row, cdf_col, pdf, reinterpret_cast<float4*>(rec));
  }
  {
    EXM_TIMED("env_guide_rows", s);
    k_guide_rows<<<1, kThreads, 0, s>>>(He, We, cdf_row, cdf_col, guide);
  }
  const int64_t nc = (int64_t)He * (We + 1);
  {
    EXM_TIMED("env_guide_cols", s);
    k_guide_cols<<<(unsigned)((nc + kThreads - 1) / kThreads), kThreads, 0, s>>>(He, We, cdf_col, guide);
  }
  return hipGetLastError();
}

}  // namespace exm
