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


// ---------------------------------------------------------------- matrix cores
// The same product on the FP64 matrix cores (v_mfma_f64_16x16x4f64): 64 x 64
// tile per work-group, 32 x 32 per wave as 2 x 2 MFMA blocks; operands staged
// through LDS as separate real / imaginary planes, so a complex multiply-add
// is four real MFMAs (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br).  Each lane
// supplies one double of A and one of B per MFMA (lane l: A[l % 16][l / 16],
// B[l / 16][l % 16]; result C[l / 16 + 4 i][l % 16], i < 4), i.e. a quarter
// of the LDS traffic per multiply-add of the register-tiled kernel above.
// herm = 1: the result is Hermitian (as is beta C); only tiles on or below
// the diagonal are computed, and each lower entry is also written, conjugated,
// to its mirror position.  tri: op(A) lower (1) / upper (2), op(B) lower (4)
// / upper (8) triangular with zeros stored outside the triangle; the k range
// of each tile is cut to where both can be non-zero.
typedef __attribute__((ext_vector_type(4))) double d4;
constexpr int GM_T = 64, GM_K = 16, GM_LD = GM_K + 1;

template <class T>
__global__ void __launch_bounds__(256)
k_gemm_mfma(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA, int opA, int bufB, int opB, int bufC,
            T alpha, T beta, int herm, int tri) {
  constexpr bool CP = sizeof(T) == sizeof(cplx);
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int m0 = blockIdx.y * GM_T, n0 = blockIdx.x * GM_T;
  if (m0 >= n || n0 >= n) return;
  if (herm && blockIdx.x > blockIdx.y) return;
  const T* A = bufp<T>(ws, d, bufA);
  const T* B = bufp<T>(ws, d, bufB);
  T* C = bufp<T>(ws, d, bufC);
  __shared__ double Ar[GM_T][GM_LD], Ai[GM_T][GM_LD];       // [row][k]
  __shared__ double Br[GM_K][GM_T + 1], Bi[GM_K][GM_T + 1]; // [k][col]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      ci[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // software pipeline: the next k chunk is fetched into registers while the
  // matrix cores work on the chunk in LDS
  constexpr int NL = GM_T * GM_K / 256;       // elements per thread per operand
  T na[NL], nb[NL];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      int r, kk;
      if (opA == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / GM_T; r = l % GM_T; }
      const int gr = m0 + r, gk = k0 + kk;
      na[q] = (gr < n && gk < n) ? (opA == 0 ? A[(long long)gr * n + gk] : conjg(A[(long long)gk * n + gr]))
                                 : tzero<T>();
      int c;
      if (opB == 0) { kk = l / GM_T; c = l % GM_T; } else { c = l / GM_K; kk = l % GM_K; }
      const int gk2 = k0 + kk, gc = n0 + c;
      nb[q] = (gk2 < n && gc < n) ? (opB == 0 ? B[(long long)gk2 * n + gc] : conjg(B[(long long)gc * n + gk2]))
                                  : tzero<T>();
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      int r, kk;
      if (opA == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / GM_T; r = l % GM_T; }
      Ar[r][kk] = re(na[q]);
      if constexpr (CP) Ai[r][kk] = im(na[q]);
      int c;
      if (opB == 0) { kk = l / GM_T; c = l % GM_T; } else { c = l / GM_K; kk = l % GM_K; }
      Br[kk][c] = re(nb[q]);
      if constexpr (CP) Bi[kk][c] = im(nb[q]);
    }
  };
  int kbeg = 0, kend = n;
  if (tri & 1) kend = min(kend, m0 + GM_T);
  if (tri & 2) kbeg = max(kbeg, m0);
  if (tri & 8) kend = min(kend, n0 + GM_T);
  if (tri & 4) kbeg = max(kbeg, n0);
  kbeg = (kbeg / GM_K) * GM_K;
  fetch(kbeg);
  stash();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += GM_K) {
    const bool more = k0 + GM_K < kend;
    if (more) fetch(k0 + GM_K);
#pragma unroll
    for (int ks = 0; ks < GM_K; ks += 4) {
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = Ar[wr + 16 * x + l16][ks + l4];
        br[x] = Br[ks + l4][wc + 16 * x + l16];
        if constexpr (CP) {
          ai[x] = Ai[wr + 16 * x + l16][ks + l4];
          bi[x] = Bi[ks + l4][wc + 16 * x + l16];
        }
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          cr[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], br[y], cr[x][y], 0, 0, 0);
          if constexpr (CP) {
            cr[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[x], bi[y], cr[x][y], 0, 0, 0);
            ci[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], bi[y], ci[x][y], 0, 0, 0);
            ci[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[x], br[y], ci[x][y], 0, 0, 0);
          }
        }
    }
    __syncthreads();
    if (more) {
      stash();
      __syncthreads();
    }
  }
  const bool use_beta = (re(beta) != 0.0 || im(beta) != 0.0);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = m0 + wr + 16 * x + l4 + 4 * i, c = n0 + wc + 16 * y + l16;
        if (r >= n || c >= n) continue;
        if (herm && c > r) continue;
        T p;
        if constexpr (CP) p = cplx{cr[x][y][i], ci[x][y][i]};
        else p = cr[x][y][i];
        const long long idx = (long long)r * n + c;
        T v = alpha * p;
        if (use_beta) v = mad(beta, C[idx], v);
        C[idx] = v;
        if (herm && c < r) C[(long long)c * n + r] = conjg(v);
      }
}

// Quaternion form of the product (Kramers-structured two-component
// matrices, N x N quaternions A + B j for the complex 2N x 2N matrix).  With
// q = (Re a, Im a, Re b, Im b), left multiplication by x is the real 4 x 4
// matrix with entries qmul_sign(c, d) x_{c xor d}, so a quaternion
// multiply-add is 16 real ones and the N x N quaternion product needs half
// the real multiply-adds of the complex 2N x 2N product.  Operands are staged
// in LDS as four component planes; each wave runs 2 x 2 blocks of 16 x 16
// quaternions, 16 MFMAs per block and k step of 4.  alpha, beta are real.
//
// TS = 64: 64 x 64 output tiles, each wave 2 x 2 blocks of 16 x 16; TS = 32
// (for launches with few tiles): 32 x 32 tiles, one block per wave, four
// times the work-groups.  The k order of every output element is the same
// in both, so are the results.
template <int TS>
__global__ void __launch_bounds__(256, 2)
k_gemm_q_mfma(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA, int opA, int bufB, int opB,
              int bufC, double alpha, double beta, int herm) {
  constexpr int XB = TS / 32;                 // 16 x 16 blocks per wave and dimension
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int m0 = blockIdx.y * TS, n0 = blockIdx.x * TS;
  if (m0 >= n || n0 >= n) return;
  if (herm && blockIdx.x > blockIdx.y) return;
  const bool dtile = herm && blockIdx.x == blockIdx.y;   // diagonal tile of a Hermitian output
  const quat* A = bufp<quat>(ws, d, bufA);
  const quat* B = bufp<quat>(ws, d, bufB);
  quat* C = bufp<quat>(ws, d, bufC);
  __shared__ double As[4][TS][GM_LD];      // [component][row][k]
  __shared__ double Bs[4][GM_K][TS + 1];   // [component][k][col]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wr = (wave >> 1) * 16 * XB, wc = (wave & 1) * 16 * XB;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 acc[XB][XB][4];
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < XB; ++y)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[x][y][c] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int NL = TS * GM_K / 256;
  quat na[NL], nb[NL];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      int r, kk;
      if (opA == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / TS; r = l % TS; }
      const int gr = m0 + r, gk = k0 + kk;
      na[q] = (gr < n && gk < n) ? (opA == 0 ? A[(long long)gr * n + gk] : conjg(A[(long long)gk * n + gr]))
                                 : tzero<quat>();
      int cc;
      if (opB == 0) { kk = l / TS; cc = l % TS; } else { cc = l / GM_K; kk = l % GM_K; }
      const int gk2 = k0 + kk, gc = n0 + cc;
      nb[q] = (gk2 < n && gc < n) ? (opB == 0 ? B[(long long)gk2 * n + gc] : conjg(B[(long long)gc * n + gk2]))
                                  : tzero<quat>();
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      int r, kk;
      if (opA == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / TS; r = l % TS; }
      As[0][r][kk] = na[q].a.x;
      As[1][r][kk] = na[q].a.y;
      As[2][r][kk] = na[q].b.x;
      As[3][r][kk] = na[q].b.y;
      int cc;
      if (opB == 0) { kk = l / TS; cc = l % TS; } else { cc = l / GM_K; kk = l % GM_K; }
      Bs[0][kk][cc] = nb[q].a.x;
      Bs[1][kk][cc] = nb[q].a.y;
      Bs[2][kk][cc] = nb[q].b.x;
      Bs[3][kk][cc] = nb[q].b.y;
    }
  };
  for (int k0 = 0; k0 < n; k0 += GM_K) {
    // two waves per SIMD instead of a register prefetch: the other
    // work-group's matrix-core work covers this one's loads, which go out
    // before the barrier
    fetch(k0);
    __syncthreads();
    stash();
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GM_K; ks += 4) {
      double a[XB][4], bq[XB][4];
#pragma unroll
      for (int x = 0; x < XB; ++x)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          a[x][c] = As[c][wr + 16 * x + l16][ks + l4];
          bq[x][c] = Bs[c][ks + l4][wc + 16 * x + l16];
        }
#pragma unroll
      for (int dd = 0; dd < 4; ++dd)
#pragma unroll
        for (int x = 0; x < XB; ++x)
#pragma unroll
          for (int y = 0; y < XB; ++y)
            if (!(dtile && wc + 16 * y > wr + 16 * x))   // 16 x 16 blocks above the diagonal are not written
#pragma unroll
              for (int c = 0; c < 4; ++c)
                acc[x][y][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    qmul_sign(c, dd) > 0 ? a[x][c ^ dd] : -a[x][c ^ dd], bq[y][dd], acc[x][y][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < XB; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = m0 + wr + 16 * x + l4 + 4 * i, cc = n0 + wc + 16 * y + l16;
        if (r >= n || cc >= n) continue;
        if (herm && cc > r) continue;
        const long long idx = (long long)r * n + cc;
        quat v = {{alpha * acc[x][y][0][i], alpha * acc[x][y][1][i]},
                  {alpha * acc[x][y][2][i], alpha * acc[x][y][3][i]}};
        if (beta != 0.0) v = v + beta * C[idx];
        C[idx] = v;
        if (herm && cc < r) C[(long long)cc * n + r] = conjg(v);
      }
}

void launch_gemm_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                   int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta, int herm) {
  const int t = (maxdim + GM_T - 1) / GM_T;
  // fewer 64 x 64 tiles than two resident work-groups per CU: 32 x 32 tiles
  const long long tiles = (long long)nblk * (herm ? t * (t + 1) / 2 : t * t);
  if (tiles < 2 * 256) {
    const int t2 = (maxdim + 31) / 32;
    hipLaunchKernelGGL(k_gemm_q_mfma<32>, dim3(t2, t2, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA, opA, bufB,
                       opB, bufC, alpha, beta, herm);
    return;
  }
  hipLaunchKernelGGL(k_gemm_q_mfma<64>, dim3(t, t, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA, opA, bufB, opB,
                     bufC, alpha, beta, herm);
}

// Products of a quaternion matrix with a real scalar matrix R (N x N,
// row-major doubles: S, T and the Cholesky factors and inverses, which act on
// both spin components alike).  side 0: C = alpha op(R) Q + beta C; side 1:
// C = alpha Q op(R) + beta C; op(R) = R or R^T.  A real factor multiplies
// each quaternion component separately, so one quaternion multiply-add is 4
// real ones (4 MFMAs per 16 x 16 block and k step, against 16).  tri = 1 / 2:
// op(R) is lower / upper triangular (entries outside the triangle are taken
// as zero, whatever is stored), and the k range of each tile is cut to where
// op(R) can be non-zero.
template <int side>
__global__ void __launch_bounds__(256, 2)
k_gemm_qr_mfma(const BlockDesc* D, char* ws, const int* info, int bufR, int opR, int tri, int bufQ, int bufC,
               double alpha, double beta, int herm) {
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = d.N;
  const int m0 = blockIdx.y * GM_T, n0 = blockIdx.x * GM_T;
  if (m0 >= n || n0 >= n) return;
  if (herm && blockIdx.x > blockIdx.y) return;
  const double* R = bufp<double>(ws, d, bufR);
  const quat* Q = bufp<quat>(ws, d, bufQ);
  quat* C = bufp<quat>(ws, d, bufC);
  // k range where op(R) may be non-zero for this tile
  int kbeg = 0, kend = n;
  if constexpr (side == 0) {     // op(R)[i][k], rows i in [m0, m0 + 64)
    if (tri == 1) kend = min(n, m0 + GM_T);
    if (tri == 2) kbeg = m0;
  } else {                       // op(R)[k][j], columns j in [n0, n0 + 64)
    if (tri == 2) kend = min(n, n0 + GM_T);
    if (tri == 1) kbeg = n0;
  }
  __shared__ double Rs[GM_T * (GM_K + 1)];   // side 0: [row][k] (stride 17); side 1: [k][col] (stride 65)
  __shared__ double Qs[4][GM_T * (GM_K + 1)];   // side 0: [k][col] (stride 65); side 1: [row][k] (stride 17)
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 acc[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[x][y][c] = d4{0.0, 0.0, 0.0, 0.0};
  // element (i, j) of op(R), zero outside its triangle and the matrix
  auto rval = [&](int i, int j) -> double {
    if (i >= n || j >= n || (tri == 1 && j > i) || (tri == 2 && j < i)) return 0.0;
    return opR == 0 ? R[(long long)i * n + j] : R[(long long)j * n + i];
  };
  constexpr int NL = GM_T * GM_K / 256;
  double nr[NL];
  quat nq[NL];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      if constexpr (side == 0) {
        // op(R) rows m0.., k chunk: consecutive threads along k (op N) or rows (op T)
        int r, kk;
        if (opR == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / GM_T; r = l % GM_T; }
        nr[q] = rval(m0 + r, k0 + kk);
        const int kq = l / GM_T, cq = l % GM_T;
        const int gk = k0 + kq, gc = n0 + cq;
        nq[q] = (gk < n && gc < n) ? Q[(long long)gk * n + gc] : tzero<quat>();
      } else {
        int kk, cc;
        if (opR == 0) { kk = l / GM_T; cc = l % GM_T; } else { cc = l / GM_K; kk = l % GM_K; }
        nr[q] = rval(k0 + kk, n0 + cc);
        const int rq = l / GM_K, kq = l % GM_K;
        const int gr = m0 + rq, gk = k0 + kq;
        nq[q] = (gr < n && gk < n) ? Q[(long long)gr * n + gk] : tzero<quat>();
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = t + 256 * q;
      int qi;
      if constexpr (side == 0) {
        int r, kk;
        if (opR == 0) { r = l / GM_K; kk = l % GM_K; } else { kk = l / GM_T; r = l % GM_T; }
        Rs[r * (GM_K + 1) + kk] = nr[q];
        qi = (l / GM_T) * (GM_T + 1) + l % GM_T;            // [k][col]
      } else {
        int kk, cc;
        if (opR == 0) { kk = l / GM_T; cc = l % GM_T; } else { cc = l / GM_K; kk = l % GM_K; }
        Rs[kk * (GM_T + 1) + cc] = nr[q];
        qi = (l / GM_K) * (GM_K + 1) + l % GM_K;            // [row][k]
      }
      Qs[0][qi] = nq[q].a.x;
      Qs[1][qi] = nq[q].a.y;
      Qs[2][qi] = nq[q].b.x;
      Qs[3][qi] = nq[q].b.y;
    }
  };
  kbeg = (kbeg / GM_K) * GM_K;
  for (int k0 = kbeg; k0 < kend; k0 += GM_K) {
    // two waves per SIMD instead of a register prefetch (the loads go out
    // before the barrier)
    fetch(k0);
    __syncthreads();
    stash();
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GM_K; ks += 4) {
      if constexpr (side == 0) {
        double a[2], bq[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          a[x] = Rs[(wr + 16 * x + l16) * (GM_K + 1) + ks + l4];
#pragma unroll
          for (int c = 0; c < 4; ++c) bq[x][c] = Qs[c][(ks + l4) * (GM_T + 1) + wc + 16 * x + l16];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int c = 0; c < 4; ++c)
              acc[x][y][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], bq[y][c], acc[x][y][c], 0, 0, 0);
      } else {
        double aq[2][4], bb[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          bb[x] = Rs[(ks + l4) * (GM_T + 1) + wc + 16 * x + l16];
#pragma unroll
          for (int c = 0; c < 4; ++c) aq[x][c] = Qs[c][(wr + 16 * x + l16) * (GM_K + 1) + ks + l4];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int c = 0; c < 4; ++c)
              acc[x][y][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[x][c], bb[y], acc[x][y][c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = m0 + wr + 16 * x + l4 + 4 * i, cc = n0 + wc + 16 * y + l16;
        if (r >= n || cc >= n) continue;
        if (herm && cc > r) continue;
        const long long idx = (long long)r * n + cc;
        quat v = {{alpha * acc[x][y][0][i], alpha * acc[x][y][1][i]},
                  {alpha * acc[x][y][2][i], alpha * acc[x][y][3][i]}};
        if (beta != 0.0) v = v + beta * C[idx];
        C[idx] = v;
        if (herm && cc < r) C[(long long)cc * n + r] = conjg(v);
      }
}

void launch_gemm_qr(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int side,
                    int bufR, int opR, int tri, int bufQ, int bufC, double alpha, double beta, int herm) {
  int t = (maxN + GM_T - 1) / GM_T;
  if (side == 0)
    hipLaunchKernelGGL(k_gemm_qr_mfma<0>, dim3(t, t, nblk), dim3(256), 0, s, D, ws, info, bufR, opR, tri, bufQ,
                       bufC, alpha, beta, herm);
  else
    hipLaunchKernelGGL(k_gemm_qr_mfma<1>, dim3(t, t, nblk), dim3(256), 0, s, D, ws, info, bufR, opR, tri, bufQ,
                       bufC, alpha, beta, herm);
}

template <class T>
void launch_gemm(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                 int bufA, int opA, int bufB, int opB, int bufC, T alpha, T beta, int herm, int tri) {
  int t = (maxdim + GM_T - 1) / GM_T;
  hipLaunchKernelGGL(k_gemm_mfma<T>, dim3(t, t, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA, opA, bufB, opB,
                     bufC, alpha, beta, herm, tri);
}

template void launch_gemm<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int,
                                  int, double, double, int, int);
template void launch_gemm<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int,
                                int, cplx, cplx, int, int);

}  // namespace x2c
