// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form, Q^H A Q = tridiag(d, e), and application of Q to a block of vectors.
//
// Used twice per DLU block: on the Cholesky-reduced 4c matrix (the "4N
// complex diagonalisation" of Sec. III, Table II) and on the n x n matrix
// whose inverse square root gives the renormalisation (the "2N complex
// diagonalisation", Sec. III).  Reflectors H_k = I - tau_k v_k v_k^H with
// real beta_k (so the off-diagonal e is real), v_k(0) = 1 implicit, the rest
// of v_k stored below the subdiagonal of column k.
//
// One work-group per block.  Each step k keeps the trailing matrix fully
// updated; the rank-2 update of step k and the Hermitian matrix-vector
// product of step k+1 share one pass over the trailing matrix: a thread owns
// a column c, walks its rows, updates A[r][c] and accumulates
// p_c = sum_r conj(A[r][c]) v_r (= (A v)_c for Hermitian A).
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// Reflector for column k (rows k+1..n-1) into vout[0..len).  Returns through
// shared scalars.  All threads call.
template <class T>
__device__ void make_reflector(T* A, int n, int k, T* vout, T* tau_out, double* beta_out, double* red) {
  const int len = n - k - 1;
  double xn2 = 0.0;
  for (int i = 1 + threadIdx.x; i < len; i += blockDim.x) xn2 += abs2(A[(long long)(k + 1 + i) * n + k]);
  xn2 = block_sum(xn2, red);
  T alpha = A[(long long)(k + 1) * n + k];
  double anrm2 = abs2(alpha);
  T tau;
  double beta;
  T scale;
  bool trivial = (xn2 == 0.0 && im(alpha) == 0.0);
  if (trivial) {
    tau = tzero<T>();
    beta = re(alpha);
    scale = tzero<T>();
  } else {
    beta = -copysign(sqrt(anrm2 + xn2), re(alpha));
    tau = tmake<T>((beta - re(alpha)) / beta, -im(alpha) / beta);
    T den = alpha - treal<T>(beta);
    if constexpr (sizeof(T) == sizeof(double)) {
      scale = treal<T>(1.0 / re(den));
    } else {
      scale = crecip(*reinterpret_cast<cplx*>(&den));
    }
  }
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    if (i == 0) {
      vout[0] = treal<T>(1.0);
    } else {
      long long idx = (long long)(k + 1 + i) * n + k;
      T x = trivial ? tzero<T>() : A[idx] * scale;
      vout[i] = x;
      A[idx] = x;
    }
  }
  if (threadIdx.x == 0) {
    *tau_out = tau;
    *beta_out = beta;
  }
  __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(1024) k_hetrd(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                                int bufD, int bufE, int bufTau) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  T* A = bufp<T>(ws, d, bufA);
  double* dd = bufp<double>(ws, d, bufD);
  double* ee = bufp<double>(ws, d, bufE);
  T* taus = bufp<T>(ws, d, bufTau);
  if (n == 1) {
    if (threadIdx.x == 0) dd[0] = re(A[0]);
    return;
  }
  extern __shared__ char smem[];
  T* vcur = reinterpret_cast<T*>(smem);
  T* pcur = vcur + n;
  T* vnext = pcur + n;
  T* pnext = vnext + n;
  __shared__ double red[32];
  __shared__ T sh_tau_next;
  __shared__ double sh_beta_next;
  __shared__ T sh_alpha;

  make_reflector<T>(A, n, 0, vnext, &sh_tau_next, &sh_beta_next, red);
  // initial Hermitian matvec over rows/cols 1..n-1
  for (int c = 1 + threadIdx.x; c < n; c += blockDim.x) {
    T acc = tzero<T>();
    int r = 1;
    for (; r + 3 < n; r += 4) {
      T a0 = A[(long long)r * n + c], a1 = A[(long long)(r + 1) * n + c];
      T a2 = A[(long long)(r + 2) * n + c], a3 = A[(long long)(r + 3) * n + c];
      acc = mad(conjg(a0), vnext[r - 1], acc);
      acc = mad(conjg(a1), vnext[r], acc);
      acc = mad(conjg(a2), vnext[r + 1], acc);
      acc = mad(conjg(a3), vnext[r + 2], acc);
    }
    for (; r < n; ++r) acc = mad(conjg(A[(long long)r * n + c]), vnext[r - 1], acc);
    pnext[c - 1] = acc;
  }
  __syncthreads();

  for (int k = 0; k <= n - 2; ++k) {
    // rotate buffers: current reflector/matvec of step k
    T* t1 = vcur; vcur = vnext; vnext = t1;
    T* t2 = pcur; pcur = pnext; pnext = t2;
    const T tau = sh_tau_next;
    const double beta = sh_beta_next;
    const int len = n - k - 1;
    // p <- tau p;  alpha = -1/2 tau (p^H v);  w = p + alpha v  (stored in pcur)
    double dr = 0.0, di = 0.0;
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      T pt = tau * pcur[i];
      pcur[i] = pt;
      T pv = conjg(pt) * vcur[i];
      dr += re(pv);
      di += im(pv);
    }
    dr = block_sum(dr, red);
    if (sizeof(T) != sizeof(double)) di = block_sum(di, red);
    if (threadIdx.x == 0) sh_alpha = (-0.5 * tau) * tmake<T>(dr, di);
    __syncthreads();
    const T alpha = sh_alpha;
    for (int i = threadIdx.x; i < len; i += blockDim.x) pcur[i] = mad(alpha, vcur[i], pcur[i]);
    if (threadIdx.x == 0) {
      dd[k] = re(A[(long long)k * n + k]);
      ee[k] = beta;
      taus[k] = tau;
    }
    __syncthreads();
    const T* w = pcur;
    if (k == n - 2) {
      if (threadIdx.x == 0) {
        T a = A[(long long)(n - 1) * n + (n - 1)];
        a = a - vcur[0] * conjg(w[0]) - w[0] * conjg(vcur[0]);
        dd[n - 1] = re(a);
      }
      break;
    }
    // update column k+1 (trailing index 0) for rows k+1..n-1
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      long long idx = (long long)(k + 1 + i) * n + (k + 1);
      A[idx] = A[idx] - vcur[i] * conjg(w[0]) - w[i] * conjg(vcur[0]);
    }
    __syncthreads();
    make_reflector<T>(A, n, k + 1, vnext, &sh_tau_next, &sh_beta_next, red);
    // fused pass: rank-2 update of rows/cols k+2.. and the next matvec
    const int base = k + 2;
    for (int c = base + threadIdx.x; c < n; c += blockDim.x) {
      const int jc = c - (k + 1);
      const T wc = conjg(w[jc]);
      const T vc = conjg(vcur[jc]);
      T acc = tzero<T>();
      int r = base;
      for (; r + 3 < n; r += 4) {
        long long i0 = (long long)r * n + c;
        T a0 = A[i0], a1 = A[i0 + n], a2 = A[i0 + 2 * n], a3 = A[i0 + 3 * n];
        int ir = r - (k + 1);
        a0 = a0 - vcur[ir] * wc - w[ir] * vc;
        a1 = a1 - vcur[ir + 1] * wc - w[ir + 1] * vc;
        a2 = a2 - vcur[ir + 2] * wc - w[ir + 2] * vc;
        a3 = a3 - vcur[ir + 3] * wc - w[ir + 3] * vc;
        A[i0] = a0; A[i0 + n] = a1; A[i0 + 2 * n] = a2; A[i0 + 3 * n] = a3;
        int jr = r - base;
        acc = mad(conjg(a0), vnext[jr], acc);
        acc = mad(conjg(a1), vnext[jr + 1], acc);
        acc = mad(conjg(a2), vnext[jr + 2], acc);
        acc = mad(conjg(a3), vnext[jr + 3], acc);
      }
      for (; r < n; ++r) {
        long long i0 = (long long)r * n + c;
        int ir = r - (k + 1);
        T a0 = A[i0] - vcur[ir] * wc - w[ir] * vc;
        A[i0] = a0;
        acc = mad(conjg(a0), vnext[r - base], acc);
      }
      pnext[c - base] = acc;
    }
    __syncthreads();
  }
}

// Y <- Q Y with Q = H_0 H_1 ... H_{n-2} (reflectors stored in bufA/bufTau of
// dimension nr = seldim(dsel)); Y is nr x ncols row-major (ncols =
// seldim(csel)).  grid = (column chunks of 256, nblk).
template <class T>
__global__ void __launch_bounds__(256) k_ormtr(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                               int bufTau, int bufY, int csel) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int nr = seldim(d, dsel);
  const int nc = seldim(d, csel);
  const int c0 = blockIdx.x * 256;
  if (c0 >= nc) return;
  const T* A = bufp<T>(ws, d, bufA);
  const T* taus = bufp<T>(ws, d, bufTau);
  T* Y = bufp<T>(ws, d, bufY);
  extern __shared__ char smem[];
  T* v = reinterpret_cast<T*>(smem);
  const int c = c0 + threadIdx.x;
  const bool act = c < nc;
  for (int k = nr - 2; k >= 0; --k) {
    const int len = nr - k - 1;
    for (int i = threadIdx.x; i < len; i += blockDim.x)
      v[i] = (i == 0) ? treal<T>(1.0) : A[(long long)(k + 1 + i) * nr + k];
    __syncthreads();
    const T tau = taus[k];
    if (act && (re(tau) != 0.0 || im(tau) != 0.0)) {
      T dot = tzero<T>();
      T* Yc = Y + (long long)(k + 1) * nc + c;
      int i = 0;
      for (; i + 3 < len; i += 4) {
        T y0 = Yc[(long long)i * nc], y1 = Yc[(long long)(i + 1) * nc];
        T y2 = Yc[(long long)(i + 2) * nc], y3 = Yc[(long long)(i + 3) * nc];
        dot = mad(conjg(v[i]), y0, dot);
        dot = mad(conjg(v[i + 1]), y1, dot);
        dot = mad(conjg(v[i + 2]), y2, dot);
        dot = mad(conjg(v[i + 3]), y3, dot);
      }
      for (; i < len; ++i) dot = mad(conjg(v[i]), Yc[(long long)i * nc], dot);
      const T f = -(tau * dot);
      for (i = 0; i < len; ++i) Yc[(long long)i * nc] = mad(v[i], f, Yc[(long long)i * nc]);
    }
    __syncthreads();
  }
}

template <class T>
void launch_hetrd(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                  int bufA, int bufD, int bufE, int bufTau) {
  size_t shm = 4 * (size_t)maxdim * sizeof(T);
  hipLaunchKernelGGL(k_hetrd<T>, dim3(nblk), dim3(1024), shm, s, D, ws, info, dsel, bufA, bufD, bufE, bufTau);
}

template <class T>
void launch_ormtr(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int maxcols,
                  int dsel, int bufA, int bufTau, int bufY, int csel) {
  size_t shm = (size_t)maxdim * sizeof(T);
  hipLaunchKernelGGL(k_ormtr<T>, dim3((maxcols + 255) / 256, nblk), dim3(256), shm, s, D, ws, info, dsel, bufA,
                     bufTau, bufY, csel);
}

template void launch_hetrd<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                   int);
template void launch_hetrd<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int);
template void launch_ormtr<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                   int, int);
template void launch_ormtr<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int,
                                 int);

}  // namespace x2c
