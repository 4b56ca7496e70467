// X from the positive-energy subspace (Appendix, Eq. defxmat: X = C_S C_L^-1).
// With Y = [Y_L; Y_S] (m x n) spanning that subspace in the Cholesky-reduced
// basis, X~ = Y_S Y_L^-1 is solved with an LU factorisation (partial
// pivoting) of Y_L; X = sqrt2 c L_T^-H X~ L_S^H follows by two products.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// ---------------------------------------------------------------- blocked
// Blocked LU (panels of LB columns, partial pivoting with whole-row
// interchanges) and blocked right-side triangular solves for X~ = Y_S Y_L^-1.
constexpr int LB = 16;

// Factor panel J (columns LB*J .. +jb, rows LB*J .. n-1) of Y_L in place.
template <class T>
__global__ void __launch_bounds__(256) k_lu_panel(const BlockDesc* D, char* ws, int* info, int J, int bufY, int dsel) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel), j0 = LB * J;
  if (j0 >= n) return;
  const int jb = min(LB, n - j0);
  T* A = bufp<T>(ws, d, bufY);
  int* piv = bufp<int>(ws, d, V_PIV);
  __shared__ double rv[4];
  __shared__ int ri[4];
  __shared__ int s_p, s_fail;
  __shared__ T s_inv;
  __shared__ T rowj[LB];
  if (threadIdx.x == 0) s_fail = 0;
  for (int jj = 0; jj < jb; ++jj) {
    const int j = j0 + jj;
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
      double v = abs1(A[(long long)i * n + j]);
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
      int pp = j;
      for (int w = 0; w < 4; ++w)
        if (rv[w] > bb || (rv[w] == bb && ri[w] < pp)) { bb = rv[w]; pp = ri[w]; }
      s_p = pp;
      piv[j] = pp;
      if (!(bb > 0.0)) s_fail = 1;
    }
    __syncthreads();
    if (s_fail) break;
    const int pp = s_p;
    if (pp != j)
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        T t = A[(long long)j * n + c];
        A[(long long)j * n + c] = A[(long long)pp * n + c];
        A[(long long)pp * n + c] = t;
      }
    __syncthreads();
    if (threadIdx.x == 0) s_inv = tinv(A[(long long)j * n + j]);
    if (threadIdx.x < jb) rowj[threadIdx.x] = A[(long long)j * n + j0 + threadIdx.x];
    __syncthreads();
    const T inv = s_inv;
    const int ncol = jb - jj - 1;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
      long long ri0 = (long long)i * n;
      T l = A[ri0 + j] * inv;
      A[ri0 + j] = l;
      for (int c = 1; c <= ncol; ++c) A[ri0 + j + c] = A[ri0 + j + c] - l * rowj[jj + c];
    }
    __syncthreads();
  }
  if (s_fail && threadIdx.x == 0) info[b] = 3;
}

// U12 = L11^-1 A12 for the block row of panel J (unit lower L11); thread per column.
template <class T>
__global__ void __launch_bounds__(256) k_lu_trsm12(const BlockDesc* D, char* ws, const int* info, int J, int bufY,
                                                   int dsel) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel), j0 = LB * J;
  if (j0 >= n) return;
  const int jb = min(LB, n - j0);
  T* A = bufp<T>(ws, d, bufY);
  __shared__ T L11[LB][LB + 1];
  for (int e = threadIdx.x; e < LB * LB; e += blockDim.x) {
    int i = e / LB, k = e % LB;
    L11[i][k] = (i < jb && k < jb) ? A[(long long)(j0 + i) * n + j0 + k] : tzero<T>();
  }
  __syncthreads();
  const int c = j0 + jb + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if constexpr (is_quat<T>()) {
    // forward substitution in place (a register column of 32 quaternions
    // would not fit): column entries re-read from memory
    for (int i = 1; i < jb; ++i) {
      T acc = A[(long long)(j0 + i) * n + c];
      for (int k = 0; k < i; ++k) acc = acc - L11[i][k] * A[(long long)(j0 + k) * n + c];
      A[(long long)(j0 + i) * n + c] = acc;
    }
    return;
  }
  T col[LB];
#pragma unroll
  for (int i = 0; i < LB; ++i) col[i] = i < jb ? A[(long long)(j0 + i) * n + c] : tzero<T>();
#pragma unroll
  for (int i = 1; i < LB; ++i) {
    T s = col[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = s - L11[i][k] * col[k];
    col[i] = s;
  }
  for (int i = 1; i < jb; ++i) A[(long long)(j0 + i) * n + c] = col[i];
}

// A22 -= L21 U12 (trailing rows/cols >= LB*J + jb), 64 x 64 output tiles.
template <class T>
struct LuTile {
  static constexpr int UT = 64;   // trailing-update output tile
};
template <>
struct LuTile<quat> {
  static constexpr int UT = 32;
};

template <class T>
__global__ void __launch_bounds__(256) k_lu_update(const BlockDesc* D, char* ws, const int* info, int J, int bufY,
                                                   int dsel) {
  constexpr int UT = LuTile<T>::UT, UR = UT / 16;
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel), j0 = LB * J;
  if (j0 >= n) return;
  const int jb = min(LB, n - j0);
  const int t0 = j0 + jb, len = n - t0;
  if (len <= 0) return;
  const int nt = (len + UT - 1) / UT;
  if ((int)blockIdx.x >= nt * nt) return;
  const int r0 = t0 + UT * (blockIdx.x / nt), c0 = t0 + UT * (blockIdx.x % nt);
  T* A = bufp<T>(ws, d, bufY);
  __shared__ T Ls[UT][LB + 1];
  __shared__ T Us[LB][UT + 1];
  for (int e = threadIdx.x; e < UT * LB; e += 256) {
    int i = e / LB, k = e % LB;
    Ls[i][k] = (r0 + i < n && k < jb) ? A[(long long)(r0 + i) * n + j0 + k] : tzero<T>();
    int kk = e / UT, cc = e % UT;
    Us[kk][cc] = (kk < jb && c0 + cc < n) ? A[(long long)(j0 + kk) * n + c0 + cc] : tzero<T>();
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[UR][UR];
#pragma unroll
  for (int i = 0; i < UR; ++i)
#pragma unroll
    for (int j = 0; j < UR; ++j) acc[i][j] = tzero<T>();
#pragma unroll 4
  for (int k = 0; k < LB; ++k) {
    T a[UR], bb[UR];
#pragma unroll
    for (int i = 0; i < UR; ++i) a[i] = Ls[ty + 16 * i][k];
#pragma unroll
    for (int j = 0; j < UR; ++j) bb[j] = Us[k][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < UR; ++i)
#pragma unroll
      for (int j = 0; j < UR; ++j) acc[i][j] = mad(a[i], bb[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < UR; ++i) {
    int r = r0 + ty + 16 * i;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < UR; ++j) {
      int c = c0 + tx + 16 * j;
      if (c >= n) continue;
      long long idx = (long long)r * n + c;
      A[idx] = A[idx] - acc[i][j];
    }
  }
}

// One block column J of the right solves on Z (= Y_S rows, in place):
//   upper: Z_J = (Z_J - Z_{<J} U_{<J,J}) U_JJ^-1        (J ascending)
//   lower: Z_J = (Z_J - Z_{>J} L_{>J,J}) L_JJ^-1, unit L (J descending)
// Work-group: 64 rows x LB columns.
template <class T, bool UPPER>
__global__ void __launch_bounds__(256) k_rsolve_blk(const BlockDesc* D, char* ws, const int* info, int J, int bufY,
                                                    int dsel) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel), j0 = LB * J;
  if (j0 >= n) return;
  const int jb = min(LB, n - j0);
  const int r0 = 64 * blockIdx.x;
  if (r0 >= n) return;
  const T* LU = bufp<T>(ws, d, bufY);
  T* Z = bufp<T>(ws, d, bufY) + (long long)n * n;      // Y_S block
  __shared__ T Zs[64][LB + 1];
  __shared__ T Ms[LB][LB + 1];
  constexpr int CJ = LB / 8;                               // columns per thread
  const int tx = threadIdx.x & 7, ty = threadIdx.x >> 3;   // 8 x 32: cols tx + 8j, rows ty + 32 i
  T acc[2][CJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j) acc[i][j] = tzero<T>();
  const int nJ = (n + LB - 1) / LB;
  const int kbeg = UPPER ? 0 : J + 1, kend = UPPER ? J : nJ;
  for (int kc = kbeg; kc < kend; ++kc) {
    const int k0 = LB * kc, kbk = min(LB, n - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * LB; e += 256) {
      int i = e / LB, k = e % LB;
      Zs[i][k] = (r0 + i < n && k < kbk) ? Z[(long long)(r0 + i) * n + k0 + k] : tzero<T>();
    }
    for (int e = threadIdx.x; e < LB * LB; e += 256) {
      int k = e / LB, c = e % LB;
      Ms[k][c] = (k < kbk && c < jb) ? LU[(long long)(k0 + k) * n + j0 + c] : tzero<T>();
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < LB; ++k) {
      T a0 = Zs[ty][k], a1 = Zs[ty + 32][k];
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        T m = Ms[k][tx + 8 * j];
        acc[0][j] = mad(a0, m, acc[0][j]);
        acc[1][j] = mad(a1, m, acc[1][j]);
      }
    }
  }
  __syncthreads();
  // right-hand side minus the update, then the in-block triangular solve (thread per row)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      int r = r0 + ty + 32 * i, c = tx + 8 * j;
      Zs[ty + 32 * i][c] = (r < n && c < jb) ? Z[(long long)r * n + j0 + c] - acc[i][j] : tzero<T>();
    }
  for (int e = threadIdx.x; e < LB * LB; e += 256) {
    int k = e / LB, c = e % LB;
    Ms[k][c] = (k < jb && c < jb) ? LU[(long long)(j0 + k) * n + j0 + c] : tzero<T>();
  }
  __syncthreads();
  if (threadIdx.x < 64 && r0 + (int)threadIdx.x < n) {
    T* z = Zs[threadIdx.x];
    if (UPPER) {
      for (int j = 0; j < jb; ++j) {
        T s = z[j];
        for (int i = 0; i < j; ++i) s = s - z[i] * Ms[i][j];
        z[j] = rdiv(s, Ms[j][j]);
      }
    } else {
      for (int j = jb - 1; j >= 0; --j) {
        T s = z[j];
        for (int i = j + 1; i < jb; ++i) s = s - z[i] * Ms[i][j];
        z[j] = s;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * LB; e += 256) {
    int i = e / LB, c = e % LB;
    if (r0 + i < n && c < jb) Z[(long long)(r0 + i) * n + j0 + c] = Zs[i][c];
  }
}

// X~ = W P_{n-1} ... P_0 (column interchanges in reverse pivot order), as a
// gather into C_TMP.  One work-group per block.
template <class T>
__global__ void __launch_bounds__(256) k_permute_cols(const BlockDesc* D, char* ws, const int* info, int bufY,
                                                      int dsel, int bufX) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int* piv = bufp<int>(ws, d, V_PIV);
  const T* W = bufp<T>(ws, d, bufY) + (long long)n * n;
  T* X = bufp<T>(ws, d, bufX);
  __shared__ int idx[1024];
  for (int c = threadIdx.x; c < n; c += blockDim.x) idx[c] = c;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = n - 1; k >= 0; --k) {
      int p = piv[k];
      int t = idx[k]; idx[k] = idx[p]; idx[p] = t;
    }
  __syncthreads();
  const long long nn = (long long)n * n;
  for (long long e = threadIdx.x; e < nn; e += blockDim.x) {
    int r = (int)(e / n), c = (int)(e % n);
    X[e] = W[(long long)r * n + idx[c]];
  }
}

template <class T>
void launch_xsolve_blk(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxn, int bufY, int dsel,
                       int bufX) {
  constexpr int UT = LuTile<T>::UT;
  const int nJ = (maxn + LB - 1) / LB;
  for (int J = 0; J < nJ; ++J) {
    hipLaunchKernelGGL(k_lu_panel<T>, dim3(nblk), dim3(256), 0, s, D, ws, info, J, bufY, dsel);
    const int rest = maxn - LB * J - LB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_lu_trsm12<T>, dim3((rest + 255) / 256, nblk), dim3(256), 0, s, D, ws, info, J, bufY,
                         dsel);
      const int nt = (rest + UT - 1) / UT;
      hipLaunchKernelGGL(k_lu_update<T>, dim3(nt * nt, nblk), dim3(256), 0, s, D, ws, info, J, bufY, dsel);
    }
  }
  const int nr = (maxn + 63) / 64;
  for (int J = 0; J < nJ; ++J)
    hipLaunchKernelGGL((k_rsolve_blk<T, true>), dim3(nr, nblk), dim3(256), 0, s, D, ws, info, J, bufY, dsel);
  for (int J = nJ - 1; J >= 0; --J)
    hipLaunchKernelGGL((k_rsolve_blk<T, false>), dim3(nr, nblk), dim3(256), 0, s, D, ws, info, J, bufY, dsel);
  hipLaunchKernelGGL(k_permute_cols<T>, dim3(nblk), dim3(256), 0, s, D, ws, info, bufY, dsel, bufX);
}
template void launch_xsolve_blk<double>(hipStream_t, const BlockDesc*, char*, int*, int, int, int, int, int);
template void launch_xsolve_blk<cplx>(hipStream_t, const BlockDesc*, char*, int*, int, int, int, int, int);
template void launch_xsolve_blk<quat>(hipStream_t, const BlockDesc*, char*, int*, int, int, int, int, int);

}  // namespace x2c
