// The paper's two-layer network (Section 2, eq. NN): a quartic form in n
// variables written as ||B Z A x||^2, with A (m x n), the augmentation
// Z(x) A x = (x_1 A x, ..., x_n A x) and B (k x n m).  Output l is the
// quadratic form f_l(x) = sum_{a,c} P[l, a, c] x_a x_c with
// P[l, a, c] = sum_b B[l, a m + b] A[b, c].
//
// Forms of degree 4 in n variables are the polynomials of degree <= 4 in
// the first n - 1 variables (set x_n = 1; the paper notes the equivalence,
// Section 1.1), so f_l has coefficients over the degree-<=2 basis of a plan
// (n - 1, 2): the row of x_a x_c (a <= c) gets P[l, a, c] + P[l, c, a]
// (a < c) or P[l, a, a].  That is the factor W (N x k) of the one-layer
// method, W = net(A, B), and the loss, its gradient dL/dW and the
// certificate come from the plan's path unchanged.  The chain rule back to
// the weights is three small GEMMs.
//
// Layout of the trainable weights (this library's choice): At = A^T (n x m)
// and Bt = B^T (n m x k), both row-major FP32, so that for every variable a
//   P_a  = At Bt_a                   (n x k)   P_a[c, l] = P[l, a, c]
//   dBt_a = A dP_a = At^T dP_a        (m x k)
//   dAt  = sum_a dP_a Bt_a^T          (n x m)
// with Bt_a the rows a m .. a m + m - 1 of Bt and P, dP stored a-major
// (n x n x k).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace net {

// C[z] (+)= A[z] B[z] with element strides; with reduce_z the
// batches are summed into one C inside each block (fixed order).  Operands
// are read in their own type and multiplied in AccT (double for FP64 plans:
// the products of FP32 weights are then exact).
template <class TA, class TB, class TC>
struct GemmArgs {
  const TA* A;
  const TB* B;
  TC* C;
  int M, N, K, Z, reduce_z, accumulate;
  int64_t sAm, sAk, sBk, sBn, sCm, sCn;
  int64_t zA, zB, zC;
};

constexpr int TM = 64, TN = 64, TK = 16;

// 64 x 64 output tile per 256 threads (4 x 4 per thread), K in chunks of 16
// through LDS.  Plain FMA: these contractions are small (a few 1e10 flop).
template <class TA, class TB, class TC, class AccT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs<TA, TB, TC> g) {
  __shared__ AccT As[TK][TM + 4], Bs[TK][TN + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  AccT acc[4][4] = {};
  const int z0 = g.reduce_z ? 0 : blockIdx.z, z1 = g.reduce_z ? g.Z : blockIdx.z + 1;
  for (int z = z0; z < z1; ++z) {
    const TA* A = g.A + z * g.zA;
    const TB* B = g.B + z * g.zB;
    for (int k0 = 0; k0 < g.K; k0 += TK) {
      for (int e = threadIdx.x; e < TK * TM; e += 256) {
        const int kk = e / TM, ii = e % TM;
        const int i = i0 + ii, k = k0 + kk;
        As[kk][ii] = (i < g.M && k < g.K) ? (AccT)A[i * g.sAm + k * g.sAk] : AccT(0);
        const int j = j0 + ii;
        Bs[kk][ii] = (j < g.N && k < g.K) ? (AccT)B[k * g.sBk + j * g.sBn] : AccT(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TK; ++kk) {
        AccT av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = As[kk][ty + 16 * u];
          bv[u] = Bs[kk][tx + 16 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][w] = fma(av[u], bv[w], acc[u][w]);
      }
      __syncthreads();
    }
  }
  TC* C = g.C + (g.reduce_z ? 0 : blockIdx.z * g.zC);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * w;
      if (i < g.M && j < g.N) {
        TC* c = C + i * g.sCm + j * g.sCn;
        *c = g.accumulate ? (TC)((AccT)*c + acc[u][w]) : (TC)acc[u][w];
      }
    }
}

// W[row, l] from P (a-major): rowpair[row] = a n + c with a <= c.
template <class T>
__global__ void k_net_scatter(const T* __restrict__ P, const int32_t* __restrict__ rowpair, int n, int N, int k,
                              T* __restrict__ W) {
  const int64_t total = (int64_t)N * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / k), l = (int)(e % k);
    const int ac = rowpair[row], a = ac / n, c = ac % n;
    T w = P[(int64_t)(a * n + c) * k + l];
    if (a != c) w += P[(int64_t)(c * n + a) * k + l];
    W[e] = w;
  }
}

// dP[(a, c), l] = dW[row(a, c), l] for every ordered (a, c): rowmap[a n + c].
template <class T>
__global__ void k_net_gather(const T* __restrict__ dW, const int32_t* __restrict__ rowmap, int n, int k,
                             T* __restrict__ dP) {
  const int64_t total = (int64_t)n * n * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int ac = (int)(e / k), l = (int)(e % k);
    dP[e] = dW[(int64_t)rowmap[ac] * k + l];
  }
}

template <class AccT, class TA, class TB, class TC>
static hipError_t gemm(const GemmArgs<TA, TB, TC>& g, hipStream_t s) {
  dim3 grid((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TM - 1) / TM), (unsigned)(g.reduce_z ? 1 : g.Z));
  k_gemm<TA, TB, TC, AccT><<<grid, 256, 0, s>>>(g);
  return hipGetLastError();
}

// out[i] = sum over z of part[z * len + i], in z order
template <class T>
__global__ void k_sum_z(const T* __restrict__ part, int Z, int64_t len, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    T acc = part[i];
    for (int z = 1; z < Z; ++z) acc += part[z * len + i];
    out[i] = (float)acc;
  }
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace net

// P = At Bt_a for every a (P a-major, n x n x k); then W from P.  T is the
// plan's W type (float, or double for FP64 plans).
template <class T>
static hipError_t net_forward(int n, int m, int k, int N, const float* At, const float* Bt, T* P,
                              const int32_t* rowpair, T* W, hipStream_t s) {
  net::GemmArgs<float, float, T> g = {};
  g.A = At; g.sAm = m; g.sAk = 1; g.zA = 0;
  g.B = Bt; g.sBk = k; g.sBn = 1; g.zB = (int64_t)m * k;
  g.C = P; g.sCm = k; g.sCn = 1; g.zC = (int64_t)n * k;
  g.M = n; g.N = k; g.K = m; g.Z = n;
  hipError_t e = net::gemm<T>(g, s);
  if (e != hipSuccess) return e;
  net::k_net_scatter<T><<<net::grid_for((int64_t)N * k), 256, 0, s>>>(P, rowpair, n, N, k, W);
  return hipGetLastError();
}

// dP from dW; dBt_a = At^T dP_a; dAt = sum_a dP_a Bt_a^T (FP32 results,
// accumulated in T; the n products dP_a Bt_a^T go to dAz, n x n x m of T,
// and are summed in a order).  dP may alias P.
template <class T>
static hipError_t net_backward(int n, int m, int k, const float* At, const float* Bt, const T* dW,
                               const int32_t* rowmap, T* dP, float* dAt, float* dBt, T* dAz, bool want_dAt,
                               hipStream_t s) {
  net::k_net_gather<T><<<net::grid_for((int64_t)n * n * k), 256, 0, s>>>(dW, rowmap, n, k, dP);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  net::GemmArgs<float, T, float> g = {};
  g.A = At; g.sAm = 1; g.sAk = m; g.zA = 0;                       // At^T: element (b, c) = At[c, b]
  g.B = dP; g.sBk = k; g.sBn = 1; g.zB = (int64_t)n * k;
  g.C = dBt; g.sCm = k; g.sCn = 1; g.zC = (int64_t)m * k;
  g.M = m; g.N = k; g.K = n; g.Z = n;
  e = net::gemm<T>(g, s);
  if (e != hipSuccess || !want_dAt) return e;
  net::GemmArgs<T, float, T> h = {};
  h.A = dP; h.sAm = k; h.sAk = 1; h.zA = (int64_t)n * k;          // dP_a: (c, l)
  h.B = Bt; h.sBk = 1; h.sBn = k; h.zB = (int64_t)m * k;          // Bt_a^T: element (l, b) = Bt[a m + b, l]
  h.C = dAz; h.sCm = m; h.sCn = 1; h.zC = (int64_t)n * m;
  h.M = n; h.N = m; h.K = k; h.Z = n;
  e = net::gemm<T>(h, s);
  if (e != hipSuccess) return e;
  net::k_sum_z<T><<<net::grid_for((int64_t)n * m), 256, 0, s>>>(dAz, n, (int64_t)n * m, dAt);
  return hipGetLastError();
}

hipError_t launch_net_forward(bool fp64, int n, int m, int k, int N, const float* At, const float* Bt, void* P,
                              const int32_t* rowpair, void* W, hipStream_t s) {
  return fp64 ? net_forward<double>(n, m, k, N, At, Bt, (double*)P, rowpair, (double*)W, s)
              : net_forward<float>(n, m, k, N, At, Bt, (float*)P, rowpair, (float*)W, s);
}

hipError_t launch_net_backward(bool fp64, int n, int m, int k, const float* At, const float* Bt, const void* dW,
                               const int32_t* rowmap, void* dP, float* dAt, float* dBt, void* dAz, bool want_dAt,
                               hipStream_t s) {
  return fp64 ? net_backward<double>(n, m, k, At, Bt, (const double*)dW, rowmap, (double*)dP, dAt, dBt,
                                     (double*)dAz, want_dAt, s)
              : net_backward<float>(n, m, k, At, Bt, (const float*)dW, rowmap, (float*)dP, dAt, dBt, (float*)dAz,
                                    want_dAt, s);
}

}  // namespace sos
