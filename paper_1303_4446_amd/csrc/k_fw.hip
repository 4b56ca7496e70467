// Kernels of the free-particle Foldy-Wouthuysen (fpFW) based decouplings,
// BSS and DKHn (Sec. II, "The BSS approach" and "The DKH approach").
//
// Both start in the orthonormal kinetic basis T K = S K t (Eq. orthonormalk):
// with S = L_S L_S^T the reduced kinetic matrix C = L_S^-1 T L_S^-T is
// tridiagonalised by the Householder kernels of the 4c reduction, the
// tridiagonal is diagonalised here by implicit QR steps that accumulate the
// rotations (k_tri_steqr), the reflectors are applied to the rotations and
// K = L_S^-T Z.  From the eigenvalues t: p = sqrt(2t), E_0 = sqrt(c^2 p^2 +
// c^4) and the fpFW factors U_0^A, U_0^B (k_fpfw_vectors); from
// V~ = K^T V K and the W~^q = p^-1 K^T W^q K p^-1 the blocks E_1, O_1, E_1'
// of the fpFW Hamiltonian H^0 (k_fpfw_assemble).  DKHn then only needs
// products of these blocks (the matrix-core GEMMs), the generator
// W_k = O_k / (E_0i + E_0j) (k_dkh_wgen) and weighted sums of terms
// (k_combine); BSS assembles H^0 itself (k_bss_h0) for the 4c eigen-solve of
// the X2C path, whose positive-energy branch gives X'' = C_S'' C_L''^-1.
//
// T = double (spin-free, real N x N) or quat (two-component: the quaternion
// N x N form A + B j of the complex [[A, B], [-B*, A*]] matrices, Sec. III.A;
// the scalar matrices V~, W~^0 enter the quaternion's real part, W~^z its i
// part, W~^y and W~^x the j and k parts, as in Eq. defw).
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// ---------------------------------------------------------------- tridiagonal QR
// Eigen-decomposition T = Z diag(d) Z^T of the real symmetric tridiagonal
// (d, e) of dimension n (dsel).  Implicit QR steps with the Wilkinson shift
// on the lowest unreduced block [p, q] (Golub & Van Loan, symmetric QR),
// deflating |e_k| <= u (|d_k| + |d_k+1|).  One work-group per block: thread
// 0 runs the scalar recurrence of a step and leaves its rotations (c_k, s_k)
// in LDS; every thread then applies them to its rows of Z, Z <- Z G_k
// (columns k, k+1), with Z kept transposed in bufZT so that the threads'
// accesses are coalesced.  Output: eigenvalues in bufD (unordered), Z
// row-major in bufZ.  A block that needs more than 30 n steps gets info 3.
__global__ void __launch_bounds__(256) k_tri_steqr(const BlockDesc* D, char* ws, int* info, int dsel, int bufD,
                                                   int bufE, int bufZT, int bufZ) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  double* dg = bufp<double>(ws, d, bufD);
  const double* eg = bufp<double>(ws, d, bufE);
  double* ZT = bufp<double>(ws, d, bufZT);
  double* Z = bufp<double>(ws, d, bufZ);
  extern __shared__ double sq[];
  double* dd = sq;
  double* ee = sq + n;
  double* cs = ee + n;
  double* sn = cs + n;
  __shared__ int s_p, s_q, s_state;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += blockDim.x) {
    dd[i] = dg[i];
    ee[i] = i < n - 1 ? eg[i] : 0.0;
  }
  const long long nn = (long long)n * n;
  for (long long e = t; e < nn; e += blockDim.x) ZT[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  constexpr double U = 1.1102230246251565e-16;   // 2^-53
  int q = n - 1, steps = 0;                        // thread 0's state
  while (true) {
    if (t == 0) {
      int st = 0, p = 0;
      while (q > 0 && fabs(ee[q - 1]) <= U * (fabs(dd[q - 1]) + fabs(dd[q]))) {
        ee[q - 1] = 0.0;
        --q;
      }
      if (q == 0) {
        st = 1;
      } else if (++steps > 30 * n) {
        st = 2;
      } else {
        p = q - 1;
        while (p > 0 && fabs(ee[p - 1]) > U * (fabs(dd[p - 1]) + fabs(dd[p]))) --p;
        if (p > 0) ee[p - 1] = 0.0;
        // Wilkinson shift from the trailing 2 x 2 of the block
        const double h = 0.5 * (dd[q - 1] - dd[q]);
        const double eq = ee[q - 1];
        const double mu = dd[q] - eq * eq / (h + copysign(hypot(h, eq), h));
        double x = dd[p] - mu, z = ee[p], bulge = 0.0;
        for (int k = p; k < q; ++k) {
          if (k > p) {
            x = ee[k - 1];
            z = bulge;
          }
          const double r = hypot(x, z);
          double c = 1.0, s = 0.0;
          if (r > 0.0) {
            c = x / r;
            s = -z / r;
          }
          if (k > p) ee[k - 1] = r;
          const double a = dd[k], bb = dd[k + 1], ek = ee[k];
          const double cc = c * c, ss = s * s, c2s = 2.0 * c * s;
          dd[k] = cc * a - c2s * ek + ss * bb;
          dd[k + 1] = ss * a + c2s * ek + cc * bb;
          ee[k] = c * s * (a - bb) + (cc - ss) * ek;
          if (k < q - 1) {
            bulge = -s * ee[k + 1];
            ee[k + 1] = c * ee[k + 1];
          }
          cs[k] = c;
          sn[k] = s;
        }
      }
      s_p = p;
      s_q = q;
      s_state = st;
    }
    __syncthreads();
    if (s_state) break;
    const int p = s_p, qq = s_q;
    for (int i = t; i < n; i += blockDim.x) {
      double zk = ZT[(long long)p * n + i];
      for (int k = p; k < qq; ++k) {
        const double c = cs[k], s = sn[k];
        const double zk1 = ZT[(long long)(k + 1) * n + i];
        ZT[(long long)k * n + i] = c * zk - s * zk1;
        zk = s * zk + c * zk1;
      }
      ZT[(long long)qq * n + i] = zk;
    }
    __syncthreads();
  }
  if (s_state == 2) {
    if (t == 0) info[b] = 3;
    return;
  }
  for (int i = t; i < n; i += blockDim.x) dg[i] = dd[i];
  for (long long e = t; e < nn; e += blockDim.x) {
    const int j = (int)(e / n), i = (int)(e % n);
    Z[(long long)i * n + j] = ZT[e];
  }
}

// ---------------------------------------------------------------- fpFW factors
// From the kinetic eigenvalues t (bufD, N of them): the vectors of bufFP,
// [p | E_0 | E_0 - c^2 | U_0^A | U_0^B], each N long.  E_0 - c^2 is taken as
// c^2 p^2 / (E_0 + c^2), which has no cancellation for small p.  A
// non-positive t (T not positive definite) sets info 2.
__global__ void k_fpfw_vectors(const BlockDesc* D, char* ws, int* info, int bufD, int bufFP, double c) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const double* tv = bufp<double>(ws, d, bufD);
  double* fp = bufp<double>(ws, d, bufFP);
  const double c2 = c * c;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double t = tv[i];
    if (!(t > 0.0) || !isfinite(t)) {
      info[b] = 2;
      continue;
    }
    const double p = sqrt(2.0 * t);
    const double E0 = c * sqrt(p * p + c2);
    const double E0m = c2 * p * p / (E0 + c2);
    fp[i] = p;
    fp[N + i] = E0;
    fp[2 * N + i] = E0m;
    fp[3 * N + i] = sqrt((E0 + c2) / (2.0 * E0));
    fp[4 * N + i] = sqrt(E0m / (2.0 * E0));
  }
}

// E_1 = A V~ A + B W~ B, O_1 = A V~ B - B W~ A, E_1' = B V~ B + A W~ A
// (A = U_0^A, B = U_0^B diagonal; the H^0 blocks of the BSS section), with
// W~_ij = (K^T W K)_ij / (p_i p_j).  bufV: K^T V K (real N x N); bufW0:
// K^T W^q K in bufW0 + q, q = 0..3 (two-component) or q = 0.
template <class T>
__global__ void k_fpfw_assemble(const BlockDesc* D, char* ws, const int* info, int bufV, int bufW0, int bufFP,
                                int bufE1, int bufO1, int bufE1p) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const double* fp = bufp<double>(ws, d, bufFP);
  const double* V = bufp<double>(ws, d, bufV);
  const double* W0 = bufp<double>(ws, d, bufW0);
  T* E1 = bufp<T>(ws, d, bufE1);
  T* O1 = bufp<T>(ws, d, bufO1);
  T* E1p = bufp<T>(ws, d, bufE1p);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const double pp = 1.0 / (fp[i] * fp[j]);
    const double Ai = fp[3 * N + i], Aj = fp[3 * N + j], Bi = fp[4 * N + i], Bj = fp[4 * N + j];
    const double v = V[e];
    T w;
    if constexpr (is_quat<T>()) {
      const double* Wx = bufp<double>(ws, d, bufW0 + 1);
      const double* Wy = bufp<double>(ws, d, bufW0 + 2);
      const double* Wz = bufp<double>(ws, d, bufW0 + 3);
      w = quat{{pp * W0[e], pp * Wz[e]}, {pp * Wy[e], pp * Wx[e]}};
    } else {
      w = pp * W0[e];
    }
    E1[e] = treal<T>(Ai * v * Aj) + (Bi * Bj) * w;
    O1[e] = treal<T>(Ai * v * Bj) - (Bi * Aj) * w;
    E1p[e] = treal<T>(Bi * v * Bj) + (Ai * Aj) * w;
  }
}

// W = O / (E_0i + E_0j): the generator of the k-th DKH step, which removes
// the odd term O of order k ([W, diag(E_0 - c^2, -E_0 - c^2)] = -O).
template <class T>
__global__ void k_dkh_wgen(const BlockDesc* D, char* ws, const int* info, int bufO, int bufW, int bufFP) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const double* E0 = bufp<double>(ws, d, bufFP) + N;
  const T* O = bufp<T>(ws, d, bufO);
  T* W = bufp<T>(ws, d, bufW);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    W[e] = (1.0 / (E0[i] + E0[j])) * O[e];
  }
}

// dst = a dst + bs src + bh src^H (N x N; dst is not read when a == 0).
template <class T>
__global__ void k_combine(const BlockDesc* D, char* ws, const int* info, int bufDst, int bufSrc, double a, double bs,
                          double bh) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const T* S = bufp<T>(ws, d, bufSrc);
  T* X = bufp<T>(ws, d, bufDst);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    T v = bs * S[e];
    if (bh != 0.0) v = v + bh * conjg(S[(long long)j * N + i]);
    if (a != 0.0) v = v + a * X[e];
    X[e] = v;
  }
}

// dst = src + diag(s1 * fp[k1] + s0) (N x N; src may equal dst).  k1 selects
// one of the fpFW vectors.
template <class T>
__global__ void k_add_diag(const BlockDesc* D, char* ws, const int* info, int bufDst, int bufSrc, int bufFP, int k1,
                           double s1, double s0) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const double* v = bufp<double>(ws, d, bufFP) + (long long)k1 * N;
  const T* S = bufp<T>(ws, d, bufSrc);
  T* X = bufp<T>(ws, d, bufDst);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    T x = S[e];
    if (i == j) x = x + treal<T>(s1 * v[i] + s0);
    X[e] = x;
  }
}

// BSS: the fpFW 4c matrix H^0 = [[E_1 + E_0 - c^2, O_1], [O_1^H, E_1' - E_0 - c^2]]
// (2N x 2N of the chain's scalar type) in bufA, row stride 2N, for the
// standard Hermitian eigen-solve of the positive-energy branch.
template <class T>
__global__ void k_bss_h0(const BlockDesc* D, char* ws, const int* info, int bufE1, int bufO1, int bufE1p, int bufFP,
                         int bufA, double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N, M = 2 * N;
  const long long mm = (long long)M * M;
  const double* fp = bufp<double>(ws, d, bufFP);
  const T* E1 = bufp<T>(ws, d, bufE1);
  const T* O1 = bufp<T>(ws, d, bufO1);
  const T* E1p = bufp<T>(ws, d, bufE1p);
  T* A = bufp<T>(ws, d, bufA);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < mm;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / M), j = (int)(e % M);
    const int bi = i / N, bj = j / N, a = i - bi * N, cc = j - bj * N;
    T v;
    if (bi == 0 && bj == 0) {
      v = E1[(long long)a * N + cc];
      if (a == cc) v = v + treal<T>(fp[2 * N + a]);
    } else if (bi == 0) {
      v = O1[(long long)a * N + cc];
    } else if (bj == 0) {
      v = conjg(O1[(long long)cc * N + a]);
    } else {
      v = E1p[(long long)a * N + cc];
      if (a == cc) v = v - treal<T>(fp[N + a] + c * c);
    }
    A[e] = v;
  }
}

// BSS decoupling in the kinetic basis from X'' (bufX2): A = U_0^A + U_0^B X''
// and B = 2c p^-1 (U_0^B - U_0^A X''), so that U^L_BSS = K A R'' K^-1 and
// U^S_BSS = K B R'' K^-1 (the BSS decoupling matrices of Sec. II with the
// sign reading of U^S given in the design notes).
template <class T>
__global__ void k_bss_ab(const BlockDesc* D, char* ws, const int* info, int bufX2, int bufFP, int bufA, int bufB,
                         double c) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int N = d.N;
  const long long nn = (long long)N * N;
  const double* fp = bufp<double>(ws, d, bufFP);
  const T* X = bufp<T>(ws, d, bufX2);
  T* A = bufp<T>(ws, d, bufA);
  T* B = bufp<T>(ws, d, bufB);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const double ua = fp[3 * N + i], ub = fp[4 * N + i], s2 = 2.0 * c / fp[i];
    const double dij = i == j ? 1.0 : 0.0;
    const T x = X[e];
    A[e] = treal<T>(ua * dij) + ub * x;
    B[e] = treal<T>(s2 * ub * dij) - (s2 * ua) * x;
  }
}

// ----------------------------------------------------------------- launchers
static int grid_for(long long elems) {
  long long g = (elems + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_tri_steqr(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxdim, int dsel,
                      int bufD, int bufE, int bufZT, int bufZ) {
  const size_t shm = 4 * (size_t)maxdim * sizeof(double);
  hipLaunchKernelGGL(k_tri_steqr, dim3(nblk), dim3(256), shm, s, D, ws, info, dsel, bufD, bufE, bufZT, bufZ);
}
void launch_fpfw_vectors(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int bufD, int bufFP,
                         double c) {
  hipLaunchKernelGGL(k_fpfw_vectors, dim3(nblk), dim3(256), 0, s, D, ws, info, bufD, bufFP, c);
}
template <class T>
void launch_fpfw_assemble(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufV,
                          int bufW0, int bufFP, int bufE1, int bufO1, int bufE1p) {
  hipLaunchKernelGGL(k_fpfw_assemble<T>, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info,
                     bufV, bufW0, bufFP, bufE1, bufO1, bufE1p);
}
template <class T>
void launch_dkh_wgen(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufO,
                     int bufW, int bufFP) {
  hipLaunchKernelGGL(k_dkh_wgen<T>, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, bufO,
                     bufW, bufFP);
}
template <class T>
void launch_combine(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufDst,
                    int bufSrc, double a, double bs, double bh) {
  hipLaunchKernelGGL(k_combine<T>, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, bufDst,
                     bufSrc, a, bs, bh);
}
template <class T>
void launch_add_diag(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufDst,
                     int bufSrc, int bufFP, int k1, double s1, double s0) {
  hipLaunchKernelGGL(k_add_diag<T>, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info,
                     bufDst, bufSrc, bufFP, k1, s1, s0);
}
template <class T>
void launch_bss_h0(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufE1,
                   int bufO1, int bufE1p, int bufFP, int bufA, double c) {
  hipLaunchKernelGGL(k_bss_h0<T>, dim3(grid_for(4LL * maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, bufE1, bufO1,
                     bufE1p, bufFP, bufA, c);
}
template <class T>
void launch_bss_ab(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufX2,
                   int bufFP, int bufA, int bufB, double c) {
  hipLaunchKernelGGL(k_bss_ab<T>, dim3(grid_for((long long)maxN * maxN), nblk), dim3(256), 0, s, D, ws, info, bufX2,
                     bufFP, bufA, bufB, c);
}

#define X2C_FW_INST(T)                                                                                              \
  template void launch_fpfw_assemble<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,  \
                                        int, int, int);                                                             \
  template void launch_dkh_wgen<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int);      \
  template void launch_combine<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, double,     \
                                  double, double);                                                                  \
  template void launch_add_diag<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,  \
                                   double, double);                                                                 \
  template void launch_bss_ab<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,   \
                                 double);                                                                           \
  template void launch_bss_h0<T>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int, \
                                 double);
X2C_FW_INST(double)
X2C_FW_INST(quat)
#undef X2C_FW_INST

}  // namespace x2c
