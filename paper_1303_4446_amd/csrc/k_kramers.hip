// Time-reversal (Kramers) structure of the two-component matrices.
//
// In the spin-orbital basis [all alpha; all beta] every two-component matrix
// of the method (S, T, V, W of Eqs. defstv/defw, the reduced 4c matrix, the
// renormalisation matrix) has the form [[A, B], [-B*, A*]] (Sec. III.A), i.e.
// it is the quaternion matrix A + B j of half the dimension.  Reducing the
// quaternion form instead of the complex one halves the dimension of the
// tridiagonalisation (a real symmetric tridiagonal whose eigenvalues are the
// Kramers pairs) and quarters the bytes it streams.  This file builds the
// quaternion matrices, the unit-quaternion phases that turn the quaternion
// tridiagonal into a real one, and converts quaternion results back to the
// complex spin-orbital layout used by the product chain.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// Quaternion reduced 4c matrix (n x n, n = 2N): index i < N is the large
// component of scalar function i, i >= N the small component of i - N;
// element = (alpha-alpha entry) + (alpha-beta entry) j of the complex matrix
// L_M^-1 D L_M^-H.
__global__ void k_assemble_Aq(const BlockDesc* D, char* ws, const int* info, double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, n = d.n;
  const long long nn = (long long)n * n;
  const double* all = bufp<double>(ws, d, R_ALL);
  const double* bb = bufp<double>(ws, d, R_B);
  const double* w0 = bufp<double>(ws, d, R_WR0);
  const double* wx = bufp<double>(ws, d, R_WR1);
  const double* wy = bufp<double>(ws, d, R_WR2);
  const double* wz = bufp<double>(ws, d, R_WR3);
  quat* A = bufp<quat>(ws, d, C_A);
  const double sq2c = sqrt(2.0) * c, two_c2 = 2.0 * c * c;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const int qi = i / N, qj = j / N;
    const int a = i - qi * N, c2 = j - qj * N;
    quat val = tzero<quat>();
    if (qi == 0 && qj == 0) {
      val.a.x = all[(long long)a * N + c2];
    } else if (qi == 0) {
      val.a.x = sq2c * bb[(long long)a * N + c2];
    } else if (qj == 0) {
      val.a.x = sq2c * bb[(long long)c2 * N + a];
    } else {
      const long long k = (long long)a * N + c2;
      val.a = {0.5 * w0[k] - (a == c2 ? two_c2 : 0.0), 0.5 * wz[k]};
      val.b = {0.5 * wy[k], 0.5 * wx[k]};
    }
    A[e] = val;
  }
}

// delta_0 = 1, delta_{k+1} = e_k delta_k / |e_k|: with D = diag(delta) the
// quaternion tridiagonal T_q satisfies D^H T_q D = tridiag(d, |e|).
__global__ void k_phase_q(const BlockDesc* D, char* ws, const int* info, int nblk, int dsel) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk || info[b]) return;
  const BlockDesc& d = D[b];
  const int dim = seldim(d, dsel);
  const quat* et = bufp<quat>(ws, d, V_ET);
  quat* del = bufp<quat>(ws, d, V_DEL);
  quat cur = treal<quat>(1.0);
  del[0] = cur;
  for (int k = 0; k + 1 < dim; ++k) {
    const quat q = et[k];
    const double a = sqrt(abs2(q));
    if (a > 0.0) {
      cur = q * cur;
      cur = (1.0 / sqrt(abs2(cur))) * cur;   // keep |delta| = 1 to rounding
    }
    del[k + 1] = cur;
  }
}

// complex n x n ([alpha; beta], Kramers-structured) -> quaternion N x N
__global__ void k_cplx_to_quat(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, n = d.n;
  const cplx* C = bufp<cplx>(ws, d, src);
  quat* Q = bufp<quat>(ws, d, dst);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    Q[e] = quat{C[(long long)i * n + j], C[(long long)i * n + N + j]};
  }
}

// quaternion N x N -> complex n x n (blocks [[a, b], [-b*, a*]])
__global__ void k_quat_to_cplx(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, n = d.n;
  const quat* Q = bufp<quat>(ws, d, src);
  cplx* C = bufp<cplx>(ws, d, dst);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const quat q = Q[e];
    C[(long long)i * n + j] = q.a;
    C[(long long)i * n + N + j] = q.b;
    C[(long long)(N + i) * n + j] = cplx{-q.b.x, q.b.y};
    C[(long long)(N + i) * n + N + j] = cplx{q.a.x, -q.a.y};
  }
}

// out[i][j] = delta_i conj(in[j][i])  (N x N quaternions)
__global__ void k_qct_scale(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const quat* in = bufp<quat>(ws, d, src);
  quat* out = bufp<quat>(ws, d, dst);
  const quat* del = bufp<quat>(ws, d, V_DEL);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    out[e] = del[i] * conjg(in[(long long)j * N + i]);
  }
}

// Quaternion (N x N) form of the two-component matrices of the product
// chain that enter as quaternion operands: V (a real scalar matrix, spin
// diagonal) and W'' = W/4c^2 - T with a = (W^0 - 4c^2 T + i W^z)/4c^2 and
// b = (W^y + i W^x)/4c^2 (Eq. defw in the [alpha; beta] order).  T and the
// Cholesky factors enter the products as real matrices directly; S only
// through its Cholesky factor.
__global__ void k_expand_q(const BlockDesc* D, char* ws, const int* info, double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const double q4 = 1.0 / (4.0 * c * c);
  const double* t = bufp<double>(ws, d, R_T);
  const double* v = bufp<double>(ws, d, R_V);
  const double* w0 = bufp<double>(ws, d, R_W0);
  const double* wx = bufp<double>(ws, d, R_W1);
  const double* wy = bufp<double>(ws, d, R_W2);
  const double* wz = bufp<double>(ws, d, R_W3);
  quat* oV = bufp<quat>(ws, d, C_V);
  quat* oW = bufp<quat>(ws, d, C_WPP);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const double tv = t[e];
    oV[e] = treal<quat>(v[e]);
    oW[e] = quat{{w0[e] * q4 - tv, wz[e] * q4}, {wy[e] * q4, wx[e] * q4}};
  }
}

// quaternion N x N identity
__global__ void k_eye_q(const BlockDesc* D, char* ws, const int* info, int buf) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int N = d.N;
  quat* Q = bufp<quat>(ws, d, buf);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x)
    Q[e] = treal<quat>(e / N == e % N ? 1.0 : 0.0);
}

// complex 2N x 2N matrix of time-reversal form [[A, B], [-B*, A*]] at
// in + h_off -> quaternion N x N buffer A + B j (only the blocks A and B,
// the first N rows, are read)
__global__ void k_read_q(const BlockDesc* D, char* ws, const int* info, const double* in, int buf) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int N = d.N, n = d.n;
  const cplx* M = reinterpret_cast<const cplx*>(in + d.h_off);
  quat* Q = bufp<quat>(ws, d, buf);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    Q[e] = quat{M[(long long)i * n + j], M[(long long)i * n + N + j]};
  }
}

// quaternion N x N workspace buffer -> complex 2N x 2N at out + h_off (zero
// for a failed block, whose eigenvalues are zeroed too when eps is given)
__global__ void k_write_q(const BlockDesc* D, char* ws, const int* info, double* out, int buf, double* eps) {
  const BlockDesc& d = D[blockIdx.y];
  const int N = d.N, n = d.n;
  const bool ok = info[blockIdx.y] == 0;
  const quat* Q = bufp<quat>(ws, d, buf);
  cplx* C = reinterpret_cast<cplx*>(out + d.h_off);
  const long long tot = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const quat q = ok ? Q[e] : tzero<quat>();
    C[(long long)i * n + j] = q.a;
    C[(long long)i * n + N + j] = q.b;
    C[(long long)(N + i) * n + j] = cplx{-q.b.x, q.b.y};
    C[(long long)(N + i) * n + N + j] = cplx{q.a.x, -q.a.y};
  }
  if (!ok && eps)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) eps[d.eps_off + k] = 0.0;
}

static int grid_for(long long elems) {
  long long g = (elems + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_assemble_Aq(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double c) {
  hipLaunchKernelGGL(k_assemble_Aq, dim3(grid_for((long long)maxn * maxn), nblk), dim3(256), 0, s, D, ws, info, c);
}
void launch_phase_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int dsel) {
  hipLaunchKernelGGL(k_phase_q, dim3((nblk + 63) / 64), dim3(64), 0, s, D, ws, info, nblk, dsel);
}
void launch_cplx_to_quat(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                         int dst) {
  hipLaunchKernelGGL(k_cplx_to_quat, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, src,
                     dst);
}
void launch_quat_to_cplx(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                         int dst) {
  hipLaunchKernelGGL(k_quat_to_cplx, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, src,
                     dst);
}
void launch_qct_scale(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                      int dst) {
  hipLaunchKernelGGL(k_qct_scale, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, src,
                     dst);
}

void launch_expand_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, double c) {
  hipLaunchKernelGGL(k_expand_q, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, c);
}
void launch_eye_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int buf) {
  hipLaunchKernelGGL(k_eye_q, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, buf);
}
void launch_read_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, const double* in,
                   int buf) {
  hipLaunchKernelGGL(k_read_q, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, in, buf);
}
void launch_write_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, double* out,
                    int buf, double* eps) {
  hipLaunchKernelGGL(k_write_q, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, out, buf,
                     eps);
}

}  // namespace x2c
