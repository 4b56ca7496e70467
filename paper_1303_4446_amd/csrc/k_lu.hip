// X from the positive-energy subspace (Appendix, Eq. defxmat: X = C_S C_L^-1).
// With Y = [Y_L; Y_S] (m x n) spanning that subspace in the Cholesky-reduced
// basis, X~ = Y_S Y_L^-1 is solved with an LU factorisation (partial
// pivoting) of Y_L; X = sqrt2 c L_T^-H X~ L_S^H follows by two products.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// In-place LU with partial pivoting of Y_L (first n rows of C_Y, n x n);
// pivots in V_PIV.  A zero pivot sets info 3.  One work-group per block.
template <class T>
__global__ void __launch_bounds__(1024) k_getrf(const BlockDesc* D, char* ws, int* info) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = d.n;
  T* A = bufp<T>(ws, d, C_Y);
  int* piv = bufp<int>(ws, d, V_PIV);
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ int s_p;
  __shared__ int s_fail;
  __shared__ T s_inv;
  if (threadIdx.x == 0) s_fail = 0;
  for (int k = 0; k < n; ++k) {
    // pivot search in column k
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
      double v = abs1(A[(long long)i * n + k]);
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { rv[threadIdx.x >> 6] = best; ri[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bb = -1.0;
      int p = k;
      for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w)
        if (rv[w] > bb || (rv[w] == bb && ri[w] < p)) { bb = rv[w]; p = ri[w]; }
      s_p = p;
      piv[k] = p;
      if (!(bb > 0.0)) s_fail = 1;
    }
    __syncthreads();
    if (s_fail) break;
    const int p = s_p;
    if (p != k)
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        T t = A[(long long)k * n + j];
        A[(long long)k * n + j] = A[(long long)p * n + j];
        A[(long long)p * n + j] = t;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      T dk = A[(long long)k * n + k];
      if constexpr (sizeof(T) == sizeof(double)) s_inv = treal<T>(1.0 / re(dk));
      else s_inv = crecip(*reinterpret_cast<cplx*>(&dk));
    }
    __syncthreads();
    const T inv = s_inv;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[(long long)i * n + k] = A[(long long)i * n + k] * inv;
    __syncthreads();
    const int len = n - k - 1;
    const long long tot = (long long)len * len;
    for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
      int i = k + 1 + (int)(t / len), j = k + 1 + (int)(t % len);
      A[(long long)i * n + j] = A[(long long)i * n + j] - A[(long long)i * n + k] * A[(long long)k * n + j];
    }
    __syncthreads();
  }
  if (s_fail && threadIdx.x == 0) info[b] = 3;
}

// dst[j][i] = src[row0 + i][j] for an n x n slab (src rows row0..row0+n of a
// matrix with n columns).
template <class T>
__global__ void k_transpose(const BlockDesc* D, char* ws, const int* info, int src, int row0sel, int dst) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n = d.n;
  const int row0 = row0sel ? n : 0;
  const T* s = bufp<T>(ws, d, src) + (long long)row0 * n;
  T* o = bufp<T>(ws, d, dst);
  __shared__ T tile[32][33];
  const int tiles = (n + 31) / 32;
  for (int t = blockIdx.x; t < tiles * tiles; t += gridDim.x) {
    int ti = t / tiles, tj = t % tiles;
    int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
    for (int r = ly; r < 32; r += 8) {
      int i = ti * 32 + r, j = tj * 32 + lx;
      if (i < n && j < n) tile[r][lx] = s[(long long)i * n + j];
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {
      int i = tj * 32 + r, j = ti * 32 + lx;
      if (i < n && j < n) o[(long long)i * n + j] = tile[lx][r];
    }
    __syncthreads();
  }
}

// Rows of X~ = Y_S Y_L^-1 with Y_L = P L U (LU in C_Y, pivots V_PIV).
// Input Z = Y_S^T in C_TMP2 (column r of Z = row r of Y_S), solved in place:
// z U = y, then z L = z, then the column interchanges.  Thread per row r.
template <class T>
__global__ void __launch_bounds__(256) k_rsolve(const BlockDesc* D, char* ws, const int* info) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = d.n;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const T* LU = bufp<T>(ws, d, C_Y);
  const int* piv = bufp<int>(ws, d, V_PIV);
  T* Z = bufp<T>(ws, d, C_TMP2);
  // z U = y :  z_j = (y_j - sum_{i<j} z_i U_ij) / U_jj
  for (int j = 0; j < n; ++j) {
    T s = Z[(long long)j * n + r];
    T s2 = tzero<T>();
    int i = 0;
    for (; i + 1 < j; i += 2) {
      s = s - Z[(long long)i * n + r] * LU[(long long)i * n + j];
      s2 = s2 - Z[(long long)(i + 1) * n + r] * LU[(long long)(i + 1) * n + j];
    }
    for (; i < j; ++i) s = s - Z[(long long)i * n + r] * LU[(long long)i * n + j];
    s = s + s2;
    T ujj = LU[(long long)j * n + j];
    T zj;
    if constexpr (sizeof(T) == sizeof(double)) zj = treal<T>(re(s) / re(ujj));
    else zj = cdiv(*reinterpret_cast<cplx*>(&s), *reinterpret_cast<cplx*>(&ujj));
    Z[(long long)j * n + r] = zj;
  }
  // z L = z1 (unit lower):  z_j = z1_j - sum_{i>j} z_i L_ij
  for (int j = n - 1; j >= 0; --j) {
    T s = Z[(long long)j * n + r];
    for (int i = j + 1; i < n; ++i) s = s - Z[(long long)i * n + r] * LU[(long long)i * n + j];
    Z[(long long)j * n + r] = s;
  }
  // X~ = Z P_{n-1} ... P_0 : swap entries k <-> piv[k], k = n-1 .. 0
  for (int k = n - 1; k >= 0; --k) {
    int p = piv[k];
    if (p != k) {
      T t = Z[(long long)k * n + r];
      Z[(long long)k * n + r] = Z[(long long)p * n + r];
      Z[(long long)p * n + r] = t;
    }
  }
}

template <class T>
void launch_getrf(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk) {
  hipLaunchKernelGGL(k_getrf<T>, dim3(nblk), dim3(1024), 0, s, D, ws, info);
}
template <class T>
void launch_transpose(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, int src,
                      int row0sel, int dst) {
  int tiles = (maxn + 31) / 32;
  int g = tiles * tiles;
  if (g > 256) g = 256;
  hipLaunchKernelGGL(k_transpose<T>, dim3(g, nblk), dim3(256), 0, s, D, ws, info, src, row0sel, dst);
}
template <class T>
void launch_rsolve(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn) {
  hipLaunchKernelGGL(k_rsolve<T>, dim3((maxn + 255) / 256, nblk), dim3(256), 0, s, D, ws, info);
}
template void launch_getrf<double>(hipStream_t, const BlockDesc*, char*, int*, int);
template void launch_getrf<cplx>(hipStream_t, const BlockDesc*, char*, int*, int);
template void launch_transpose<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int);
template void launch_transpose<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int);
template void launch_rsolve<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int);
template void launch_rsolve<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int);

}  // namespace x2c
