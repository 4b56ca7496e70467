// Input staging, Cholesky factorisation of S and T, triangular inverses and
// assembly of the Cholesky-reduced modified Dirac matrix.
//
// The modified Dirac equation (Sec. II, Eq. moddiraceq) D C = M C eps with
// D = [[V, T], [T, W/4c^2 - T]] and M = diag(S, T/2c^2) is reduced to a
// standard Hermitian problem with M = L_M L_M^H, L_M = diag(L_S, L_T/(sqrt2 c)):
//   A = L_M^-1 D L_M^-H
//     = [[L_S^-1 V L_S^-H,         sqrt2 c L_S^-1 L_T          ],
//        [sqrt2 c L_T^H L_S^-H,    1/2 L_T^-1 W L_T^-H - 2c^2 I]].
// S, T, V are spin-block diagonal (Eq. defstv) so L_S, L_T and the first three
// blocks are real scalar N x N matrices; W is assembled from W^0..z
// (Eq. defw) after the scalar-level congruence L_T^-1 W^q L_T^-T.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

__global__ void k_init_info(int* info, int nblk) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nblk) info[i] = 0;
}

// Copy S, T, V, W^q into the block workspace and flag non-finite input.
__global__ void k_unpack(const BlockDesc* D, char* ws, int* info, const double* S,
                         const double* T, const double* V, const double* W, int twocomp) {
  const BlockDesc& d = D[blockIdx.y];
  const long long NN = (long long)d.N * d.N;
  const double* Sb = S + d.in_off;
  const double* Tb = T + d.in_off;
  const double* Vb = V + d.in_off;
  const double* Wb = W + (twocomp ? 4 * d.in_off : d.in_off);
  double* s = bufp<double>(ws, d, R_S);
  double* t = bufp<double>(ws, d, R_T);
  double* v = bufp<double>(ws, d, R_V);
  double* ls = bufp<double>(ws, d, R_LS);
  double* lt = bufp<double>(ws, d, R_LT);
  double* w[4] = {bufp<double>(ws, d, R_W0), bufp<double>(ws, d, R_W1), bufp<double>(ws, d, R_W2),
                  bufp<double>(ws, d, R_W3)};
  const int nw = twocomp ? 4 : 1;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NN;
       i += (long long)gridDim.x * blockDim.x) {
    double a = Sb[i], b = Tb[i], c = Vb[i];
    s[i] = a; ls[i] = a;
    t[i] = b; lt[i] = b;
    v[i] = c;
    bad |= !isfinite(a) || !isfinite(b) || !isfinite(c);
    for (int q = 0; q < nw; ++q) {
      double x = Wb[q * NN + i];
      w[q][i] = x;
      bad |= !isfinite(x);
    }
  }
  if (bad) info[blockIdx.y] = 6;
}

// Cholesky S = L L^T (lower, row-major, in place) of the real N x N matrix,
// left-looking by panels of PB columns; one work-group per (block, matrix),
// grid = (2, nblk).  The panel (rows p0.., PB columns) lives in LDS: it is
// first updated with every finished column (k < p0, staged PK at a time),
// then factored column by column.
constexpr int PB = 32, PK = 64;

__global__ void __launch_bounds__(256) k_potrf(const BlockDesc* D, char* ws, int* info) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int which = blockIdx.x;
  const int N = d.N;
  double* A = bufp<double>(ws, d, which == 0 ? R_LS : R_LT);
  extern __shared__ double sm[];
  double* P = sm;                           // N x (PB + 1)
  double* Lt = sm + (size_t)N * (PB + 1);   // PB x (PK + 1)
  __shared__ int fail;
  __shared__ double piv;
  const int t = threadIdx.x, c = t & (PB - 1), g = t >> 5;
  if (t == 0) fail = 0;
  for (int p0 = 0; p0 < N; p0 += PB) {
    const int nb = min(PB, N - p0), rows = N - p0;
    for (int e = t; e < rows * PB; e += 256) {
      const int r = e / PB, cc = e % PB;
      P[r * (PB + 1) + cc] = (cc < nb && cc <= r) ? A[(long long)(p0 + r) * N + p0 + cc] : 0.0;
    }
    for (int kc = 0; kc < p0; kc += PK) {
      const int kn = min(PK, p0 - kc);
      __syncthreads();
      for (int e = t; e < PB * PK; e += 256) {
        const int cc = e / PK, kk = e % PK;
        Lt[cc * (PK + 1) + kk] = (cc < nb && kk < kn) ? A[(long long)(p0 + cc) * N + kc + kk] : 0.0;
      }
      __syncthreads();
      if (c < nb) {
        for (int r = g; r < rows; r += 8) {
          if (c > r) continue;
          const double* Lr = A + (long long)(p0 + r) * N + kc;
          double acc = 0.0;
          for (int kk = 0; kk < kn; ++kk) acc = fma(Lr[kk], Lt[c * (PK + 1) + kk], acc);
          P[r * (PB + 1) + c] -= acc;
        }
      }
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      if (t == 0) {
        const double a = P[j * (PB + 1) + j];
        if (!(a > 0.0) || !isfinite(a)) {
          fail = 1;
        } else {
          piv = sqrt(a);
          P[j * (PB + 1) + j] = piv;
        }
      }
      __syncthreads();
      if (fail) break;
      const double inv = 1.0 / piv;
      for (int r = j + 1 + t; r < rows; r += 256) P[r * (PB + 1) + j] *= inv;
      __syncthreads();
      for (int e = t; e < rows * PB; e += 256) {
        const int r = e / PB, cc = e % PB;
        if (cc > j && cc < nb && r >= cc) P[r * (PB + 1) + cc] -= P[r * (PB + 1) + j] * P[cc * (PB + 1) + j];
      }
      __syncthreads();
    }
    if (fail) break;
    for (int e = t; e < rows * PB; e += 256) {
      const int r = e / PB, cc = e % PB;
      if (cc < nb && cc <= r) A[(long long)(p0 + r) * N + p0 + cc] = P[r * (PB + 1) + cc];
    }
    __syncthreads();
  }
  if (fail) {
    // S failing takes precedence over T failing, whichever work-group ends first
    if (t == 0) {
      if (which == 0) atomicExch(&info[b], 1);
      else atomicCAS(&info[b], 0, 2);
    }
    return;
  }
  // zero the strict upper triangle
  const long long NN = (long long)N * N;
  for (long long e = t; e < NN; e += blockDim.x) {
    const int i = (int)(e / N), k = (int)(e % N);
    if (k > i) A[e] = 0.0;
  }
}

// Inverse X = L^-1 of a real lower-triangular matrix, PB columns per
// work-group (grid = (ceil(N / PB), 2, nblk)).  Rows are taken PB at a time:
// the contribution of the rows already solved is a dense product (all
// threads), the PB x PB diagonal block a short forward substitution.
__global__ void __launch_bounds__(256) k_trtri(const BlockDesc* D, char* ws, const int* info) {
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const int j0 = blockIdx.x * PB;
  if (j0 >= N) return;
  const double* L = bufp<double>(ws, d, blockIdx.y == 0 ? R_LS : R_LT);
  double* X = bufp<double>(ws, d, blockIdx.y == 0 ? R_LSI : R_LTI);
  extern __shared__ double sm[];
  double* xs = sm;                                  // rows j0.. x (PB + 1)
  double* U = sm + (size_t)(N - j0) * (PB + 1);     // PB x (PB + 1)
  double* Ld = U + (size_t)PB * (PB + 1);           // diagonal block of L, PB x (PB + 1)
  const int t = threadIdx.x, c = t & (PB - 1), g = t >> 5;
  const int nc = min(PB, N - j0);
  for (int i0 = j0; i0 < N; i0 += PB) {
    const int ib = min(PB, N - i0);
    for (int e = t; e < PB * PB; e += 256) {
      const int ii = e / PB, kk = e % PB;
      Ld[ii * (PB + 1) + kk] = (ii < ib && kk <= ii) ? L[(long long)(i0 + ii) * N + i0 + kk] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PB / 8; ++q) {
      const int ii = g + 8 * q;
      if (ii < ib) {
        const double* Li = L + (long long)(i0 + ii) * N;
        double acc = 0.0;
        for (int k = j0; k < i0; ++k) acc = fma(Li[k], xs[(k - j0) * (PB + 1) + c], acc);
        U[ii * (PB + 1) + c] = acc;
      }
    }
    __syncthreads();
    // in-block forward substitution, one thread per column, L from LDS
    if (t < PB) {
      for (int ii = 0; ii < ib; ++ii) {
        double acc = ((i0 + ii) == (j0 + c) ? 1.0 : 0.0) - U[ii * (PB + 1) + c];
        for (int kk = 0; kk < ii; ++kk)
          acc = fma(-Ld[ii * (PB + 1) + kk], xs[(i0 + kk - j0) * (PB + 1) + c], acc);
        xs[(i0 + ii - j0) * (PB + 1) + c] = acc / Ld[ii * (PB + 1) + ii];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < N * PB; e += 256) {
    const int i = e / PB, cc = e % PB;
    if (cc < nc) X[(long long)i * N + j0 + cc] = i < j0 ? 0.0 : xs[(i - j0) * (PB + 1) + cc];
  }
}

// Spin expansion of the scalar matrices into the T-typed n x n buffers used
// by the GEMM chain: S, T, V, L_S, L_S^-1, L_T^-1 as diag(A, A) and
// W'' = W/4c^2 - T with W from Eq. defw.  Spin-free: plain copies.
template <class T>
__global__ void k_expand(const BlockDesc* D, char* ws, const int* info, double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, n = d.n;
  const long long nn = (long long)n * n;
  const double q4 = 1.0 / (4.0 * c * c);
  const double* s = bufp<double>(ws, d, R_S);
  const double* t = bufp<double>(ws, d, R_T);
  const double* v = bufp<double>(ws, d, R_V);
  const double* ls = bufp<double>(ws, d, R_LS);
  const double* lsi = bufp<double>(ws, d, R_LSI);
  const double* lti = bufp<double>(ws, d, R_LTI);
  const double* w0 = bufp<double>(ws, d, R_W0);
  const double* wx = bufp<double>(ws, d, R_W1);
  const double* wy = bufp<double>(ws, d, R_W2);
  const double* wz = bufp<double>(ws, d, R_W3);
  T* oS = bufp<T>(ws, d, C_S);
  T* oT = bufp<T>(ws, d, C_T);
  T* oV = bufp<T>(ws, d, C_V);
  T* oW = bufp<T>(ws, d, C_WPP);
  T* oLS = bufp<T>(ws, d, C_LS);
  T* oLSI = bufp<T>(ws, d, C_LSI);
  T* oLTI = bufp<T>(ws, d, C_LTI);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    int si = i / N, sj = j / N;   // spin index (0 = alpha, 1 = beta); always 0 in spin-free mode
    int a = i - si * N, bb = j - sj * N;
    long long k = (long long)a * N + bb;
    bool diag = (si == sj);
    double tv = diag ? t[k] : 0.0;
    oS[e] = treal<T>(diag ? s[k] : 0.0);
    oT[e] = treal<T>(tv);
    oV[e] = treal<T>(diag ? v[k] : 0.0);
    oLS[e] = treal<T>(diag ? ls[k] : 0.0);
    oLSI[e] = treal<T>(diag ? lsi[k] : 0.0);
    oLTI[e] = treal<T>(diag ? lti[k] : 0.0);
    double wr, wi;
    if (n == N) {            // spin-free
      wr = w0[k]; wi = 0.0;
    } else if (si == 0 && sj == 0) {
      wr = w0[k]; wi = wz[k];
    } else if (si == 0) {
      wr = wy[k]; wi = wx[k];
    } else if (sj == 0) {
      wr = -wy[k]; wi = wx[k];
    } else {
      wr = w0[k]; wi = -wz[k];
    }
    oW[e] = tmake<T>(wr * q4 - tv, wi * q4);
  }
}

// A = L_M^-1 D L_M^-H from the reduced scalar blocks.
template <class T>
__global__ void k_assemble_A(const BlockDesc* D, char* ws, const int* info, double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, n = d.n, m = d.m;
  const long long mm = (long long)m * m;
  const double* all = bufp<double>(ws, d, R_ALL);
  const double* bb = bufp<double>(ws, d, R_B);
  const double* w0 = bufp<double>(ws, d, R_WR0);
  const double* wx = bufp<double>(ws, d, R_WR1);
  const double* wy = bufp<double>(ws, d, R_WR2);
  const double* wz = bufp<double>(ws, d, R_WR3);
  T* A = bufp<T>(ws, d, C_A);
  const double sq2c = sqrt(2.0) * c, two_c2 = 2.0 * c * c;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < mm;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e / m), j = (int)(e % m);
    int qi = i / n, qj = j / n;            // 0 = large, 1 = small component
    int ii = i - qi * n, jj = j - qj * n;
    int si = ii / N, sj = jj / N;
    int a = ii - si * N, c2 = jj - sj * N;
    bool sd = (si == sj);
    T val;
    if (qi == 0 && qj == 0) {
      val = treal<T>(sd ? all[(long long)a * N + c2] : 0.0);
    } else if (qi == 0 && qj == 1) {
      val = treal<T>(sd ? sq2c * bb[(long long)a * N + c2] : 0.0);
    } else if (qi == 1 && qj == 0) {
      val = treal<T>(sd ? sq2c * bb[(long long)c2 * N + a] : 0.0);
    } else {
      long long k = (long long)a * N + c2;
      double wr, wi;
      if (n == N) {
        wr = w0[k]; wi = 0.0;
      } else if (si == 0 && sj == 0) {
        wr = w0[k]; wi = wz[k];
      } else if (si == 0) {
        wr = wy[k]; wi = wx[k];
      } else if (sj == 0) {
        wr = -wy[k]; wi = wx[k];
      } else {
        wr = w0[k]; wi = -wz[k];
      }
      val = tmake<T>(0.5 * wr - (ii == jj ? two_c2 : 0.0), 0.5 * wi);
    }
    A[e] = val;
  }
}

// dst = src (same dims), n x n T-typed buffers
template <class T>
__global__ void k_copy(const BlockDesc* D, char* ws, const int* info, int dsel, int src, int dst) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n = seldim(d, dsel);
  const long long nn = (long long)n * n;
  const T* s = bufp<T>(ws, d, src);
  T* o = bufp<T>(ws, d, dst);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    o[e] = s[e];
}

// dst += src + src^H   (n x n)
template <class T>
__global__ void k_add_herm(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n = is_quat<T>() ? d.N : d.n;
  const long long nn = (long long)n * n;
  const T* s = bufp<T>(ws, d, src);
  T* o = bufp<T>(ws, d, dst);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    o[e] = o[e] + s[e] + conjg(s[(long long)j * n + i]);
  }
}

// dst = src^H  (n x n)
template <class T>
__global__ void k_conj_transpose(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n = d.n;
  const T* s = bufp<T>(ws, d, src);
  T* o = bufp<T>(ws, d, dst);
  __shared__ T tile[32][33];
  const int tiles = (n + 31) / 32;
  for (int t = blockIdx.x; t < tiles * tiles; t += gridDim.x) {
    int ti = t / tiles, tj = t % tiles;
    int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int r = ly; r < 32; r += 8) {
      int i = ti * 32 + r, j = tj * 32 + lx;
      if (i < n && j < n) tile[r][lx] = s[(long long)i * n + j];
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {
      int i = tj * 32 + r, j = ti * 32 + lx;   // o[i][j] = conj(s[j][i])
      if (i < n && j < n) o[(long long)i * n + j] = conjg(tile[lx][r]);
    }
    __syncthreads();
  }
}

// Write h (and zero h, eps of failed blocks).
template <class T>
__global__ void k_write_h(const BlockDesc* D, char* ws, const int* info, double* h, double* eps) {
  const BlockDesc& d = D[blockIdx.y];
  const int n = d.n;
  const long long nn = (long long)n * n;
  const bool ok = info[blockIdx.y] == 0;
  const T* src = bufp<T>(ws, d, C_H);
  T* out = reinterpret_cast<T*>(h + d.h_off);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    out[e] = ok ? src[e] : tzero<T>();
  if (!ok)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
      eps[d.eps_off + k] = 0.0;
}

// per-block status from descriptor order to the caller's block order
__global__ void k_scatter_info(const BlockDesc* D, const int* iw, int* info, int nblk) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nblk) info[D[k].orig] = iw[k];
}

// ----------------------------------------------------------------- launchers
void launch_scatter_info(hipStream_t s, const BlockDesc* D, const int* iw, int* info, int nblk) {
  hipLaunchKernelGGL(k_scatter_info, dim3((nblk + 255) / 256), dim3(256), 0, s, D, iw, info, nblk);
}
void launch_init_info(hipStream_t s, int* info, int nblk) {
  hipLaunchKernelGGL(k_init_info, dim3((nblk + 255) / 256), dim3(256), 0, s, info, nblk);
}
void launch_unpack(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN,
                   const double* S, const double* T, const double* V, const double* W, int twocomp) {
  long long nn = (long long)maxN * maxN;
  int gx = (int)((nn + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_unpack, dim3(gx, nblk), dim3(256), 0, s, D, ws, info, S, T, V, W, twocomp);
}
void launch_potrf(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN) {
  const size_t shm = ((size_t)maxN * (PB + 1) + (size_t)PB * (PK + 1)) * sizeof(double);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_potrf), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_potrf, dim3(2, nblk), dim3(256), shm, s, D, ws, info);
}
void launch_trtri(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN) {
  const size_t shm = ((size_t)maxN * (PB + 1) + 2 * (size_t)PB * (PB + 1)) * sizeof(double);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trtri), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_trtri, dim3((maxN + PB - 1) / PB, 2, nblk), dim3(256), shm, s, D, ws, info);
}
static int grid_for(long long elems) {
  long long g = (elems + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return (int)g;
}
template <class T>
void launch_expand(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double c) {
  hipLaunchKernelGGL(k_expand<T>, dim3(grid_for((long long)maxn * maxn), nblk), dim3(256), 0, s, D, ws, info, c);
}
template <class T>
void launch_assemble_A(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxm, double c) {
  hipLaunchKernelGGL(k_assemble_A<T>, dim3(grid_for((long long)maxm * maxm), nblk), dim3(256), 0, s, D, ws, info, c);
}
template <class T>
void launch_copy(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                 int src, int dst) {
  hipLaunchKernelGGL(k_copy<T>, dim3(grid_for((long long)maxdim * maxdim), nblk), dim3(256), 0, s, D, ws, info,
                     dsel, src, dst);
}
template <class T>
void launch_add_herm(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, int src,
                     int dst) {
  hipLaunchKernelGGL(k_add_herm<T>, dim3(grid_for((long long)maxn * maxn), nblk), dim3(256), 0, s, D, ws, info,
                     src, dst);
}
template <class T>
void launch_conj_transpose(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn,
                           int src, int dst) {
  int tiles = (maxn + 31) / 32;
  int g = tiles * tiles;
  if (g > 256) g = 256;
  hipLaunchKernelGGL(k_conj_transpose<T>, dim3(g, nblk), dim3(256), 0, s, D, ws, info, src, dst);
}
template <class T>
void launch_write_h(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double* h,
                    double* eps) {
  hipLaunchKernelGGL(k_write_h<T>, dim3(grid_for((long long)maxn * maxn), nblk), dim3(256), 0, s, D, ws, info, h,
                     eps);
}

#define X2C_INST(T)                                                                                      \
  template void launch_expand<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, double);       \
  template void launch_assemble_A<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, double);   \
  template void launch_copy<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int);  \
  template void launch_add_herm<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);   \
  template void launch_conj_transpose<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int,   \
                                         int);                                                           \
  template void launch_write_h<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, double*, double*);
X2C_INST(double)
X2C_INST(cplx)
template void launch_copy<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int);
template void launch_add_herm<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);

}  // namespace x2c
