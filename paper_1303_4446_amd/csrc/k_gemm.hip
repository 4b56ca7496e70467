// Batched FP64 / complex-FP64 GEMM over uneven DLU blocks:
//   C_b = alpha op(A_b) op(B_b) + beta C_b,  op in {N, H}, square n_b x n_b.
// One launch covers every block of the batch (blockIdx.z = block); tiles that
// fall outside a smaller block exit at once.  LDS-tiled 64 x 64 x 16 with a
// 4 x 4 register micro-tile per thread.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

template <class T>
__global__ void __launch_bounds__(256)
k_gemm(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA, int opA, int bufB, int opB, int bufC,
       T alpha, T beta) {
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int m0 = blockIdx.y * GB_M, n0 = blockIdx.x * GB_N;
  if (m0 >= n || n0 >= n) return;
  const T* A = bufp<T>(ws, d, bufA);
  const T* B = bufp<T>(ws, d, bufB);
  T* C = bufp<T>(ws, d, bufC);

  __shared__ T As[GB_K][GB_M + 1];
  __shared__ T Bs[GB_K][GB_N + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = tzero<T>();

  for (int k0 = 0; k0 < n; k0 += GB_K) {
    for (int l = threadIdx.x; l < GB_M * GB_K; l += 256) {
      int r, kk;
      T v = tzero<T>();
      if (opA == 0) {
        r = l / GB_K; kk = l % GB_K;
        int gr = m0 + r, gk = k0 + kk;
        if (gr < n && gk < n) v = A[(long long)gr * n + gk];
      } else {
        kk = l / GB_M; r = l % GB_M;
        int gr = m0 + r, gk = k0 + kk;
        if (gr < n && gk < n) v = conjg(A[(long long)gk * n + gr]);
      }
      As[kk][r] = v;
    }
    for (int l = threadIdx.x; l < GB_K * GB_N; l += 256) {
      int c, kk;
      T v = tzero<T>();
      if (opB == 0) {
        kk = l / GB_N; c = l % GB_N;
        int gk = k0 + kk, gc = n0 + c;
        if (gk < n && gc < n) v = B[(long long)gk * n + gc];
      } else {
        c = l / GB_K; kk = l % GB_K;
        int gk = k0 + kk, gc = n0 + c;
        if (gk < n && gc < n) v = conjg(B[(long long)gc * n + gk]);
      }
      Bs[kk][c] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GB_K; ++kk) {
      T a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mad(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  const bool use_beta = (re(beta) != 0.0 || im(beta) != 0.0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r = m0 + ty + 16 * i;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int c = n0 + tx + 16 * j;
      if (c >= n) continue;
      long long idx = (long long)r * n + c;
      T v = alpha * acc[i][j];
      if (use_beta) v = mad(beta, C[idx], v);
      C[idx] = v;
    }
  }
}


template <class T>
void launch_gemm(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                 int bufA, int opA, int bufB, int opB, int bufC, T alpha, T beta) {
  int t = (maxdim + GB_M - 1) / GB_M;
  hipLaunchKernelGGL(k_gemm<T>, dim3(t, t, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA, opA, bufB, opB, bufC,
                     alpha, beta);
}

template void launch_gemm<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int,
                                  int, double, double);
template void launch_gemm<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int,
                                int, cplx, cplx);

}  // namespace x2c
