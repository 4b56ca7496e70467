// DLU molecular Hamiltonian (Sec. III.A).  U^L and U^S are direct sums of
// atomic blocks (Eq. dlutrans), U^L_AA = R_A and U^S_AA = X_A R_A from the
// atoms' own decoupling (Eq. r2ctransatom), so Eq. utrans splits into atom
// pairs:
//   h_AB = R_A^H [ V_AB + T_AB X_B + X_A^H T_AB + X_A^H (W_AB/4c^2 - T_AB) X_B ] R_B.
// Pairs A >= B are formed together (one launch per product step covers every
// pair); h_BA = h_AB^H fills the other triangle.  Molecular matrices are the
// scalar Ntot x Ntot S, T, V and W^0..z; the two-component h uses the
// molecular spin-orbital order [all alpha; all beta] (Eq. defstv, defw).
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// T-typed n x n workspace buffer of every block -> out + h_off (zero for a
// failed block): the per-atom X and R of the batched build.
template <class T>
__global__ void k_write_buf(const BlockDesc* D, char* ws, const int* info, double* out, int buf) {
  const BlockDesc& d = D[blockIdx.y];
  const long long nn = (long long)d.n * d.n;
  const bool ok = info[blockIdx.y] == 0;
  const T* src = bufp<T>(ws, d, buf);
  T* o = reinterpret_cast<T*>(out + d.h_off);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x)
    o[e] = ok ? src[e] : tzero<T>();
}

template <class T>
void launch_write_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double* out,
                      int buf) {
  long long g = ((long long)maxn * maxn + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_write_buf<T>, dim3((int)g, nblk), dim3(256), 0, s, D, ws, info, out, buf);
}
template void launch_write_buf<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, double*, int);
template void launch_write_buf<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, double*, int);

// n x n T-typed matrix of every block at in + h_off -> workspace buffer
// (zero when in is null)
template <class T>
__global__ void k_read_buf(const BlockDesc* D, char* ws, const int* info, const double* in, int buf) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const long long nn = (long long)d.n * d.n;
  const T* src = in ? reinterpret_cast<const T*>(in + d.h_off) : nullptr;
  T* o = bufp<T>(ws, d, buf);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x)
    o[e] = src ? src[e] : tzero<T>();
}

// dst += src (n x n workspace buffers)
template <class T>
__global__ void k_add_buf(const BlockDesc* D, char* ws, const int* info, int src, int dst) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const long long nn = (long long)d.n * d.n;
  const T* a = bufp<T>(ws, d, src);
  T* o = bufp<T>(ws, d, dst);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x)
    o[e] = o[e] + a[e];
}

template <class T>
void launch_read_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn,
                     const double* in, int buf) {
  long long g = ((long long)maxn * maxn + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_read_buf<T>, dim3((int)g, nblk), dim3(256), 0, s, D, ws, info, in, buf);
}
template <class T>
void launch_add_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, int src,
                    int dst) {
  long long g = ((long long)maxn * maxn + 255) / 256;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_add_buf<T>, dim3((int)g, nblk), dim3(256), 0, s, D, ws, info, src, dst);
}
template void launch_read_buf<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, const double*, int);
template void launch_read_buf<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, const double*, int);
template void launch_add_buf<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);
template void launch_add_buf<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);

// V_AB -> L, T_AB -> Tb, W_AB / 4c^2 - T_AB -> Wb for every pair.
template <class T>
__global__ void k_dlu_gather(const DluPair* P, char* ws, const double* Tm, const double* Vm, const double* Wm,
                             int Ntot, double c) {
  const DluPair& p = P[blockIdx.y];
  constexpr bool TC = sizeof(T) == sizeof(cplx);
  const int NA = TC ? p.nA / 2 : p.nA, NB = TC ? p.nB / 2 : p.nB;
  const long long tot = (long long)p.nA * p.nB;
  const long long NN = (long long)Ntot * Ntot;
  const double q4 = 1.0 / (4.0 * c * c);
  T* Tb = reinterpret_cast<T*>(ws + p.t);
  T* Wb = reinterpret_cast<T*>(ws + p.w);
  T* Lb = reinterpret_cast<T*>(ws + p.l);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / p.nB), j = (int)(e % p.nB);
    const int si = i / NA, sj = j / NB;
    const long long ab = (long long)(p.oA + i - si * NA) * Ntot + (p.oB + j - sj * NB);
    const double tv = Tm[ab], vv = Vm[ab], w0 = Wm[ab];
    if constexpr (TC) {
      const double wx = Wm[NN + ab], wy = Wm[2 * NN + ab], wz = Wm[3 * NN + ab];
      cplx w;
      if (si == 0 && sj == 0) w = cplx{w0, wz};
      else if (si == 0) w = cplx{wy, wx};
      else if (sj == 0) w = cplx{-wy, wx};
      else w = cplx{w0, -wz};
      const double td = si == sj ? tv : 0.0;
      Tb[e] = cplx{td, 0.0};
      Lb[e] = cplx{si == sj ? vv : 0.0, 0.0};
      Wb[e] = cplx{w.x * q4 - td, w.y * q4};
    } else {
      Tb[e] = tv;
      Lb[e] = vv;
      Wb[e] = w0 * q4 - tv;
    }
  }
}

// One product step for every pair (C = alpha op(A) B + beta C), LDS-tiled
// 64 x 64 x 16 with a 4 x 4 register tile.  Steps (all n_A x n_B results):
//   0: L += T_AB X_B      1: L += X_A^H T_AB    2: P = W''_AB X_B
//   3: L += X_A^H P       4: P = L R_B          5: h_AB = R_A^H P  (into Tb)
template <class T>
__global__ void __launch_bounds__(256) k_dlu_gemm(const DluPair* P, int step, char* ws, const T* X, const T* R) {
  const DluPair& p = P[blockIdx.z];
  const int M = p.nA, N = p.nB;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (m0 >= M || n0 >= N) return;
  const T* A;
  const T* B;
  T* C;
  int K, lda, opA;
  bool acc;
  T* Tb = reinterpret_cast<T*>(ws + p.t);
  T* Wb = reinterpret_cast<T*>(ws + p.w);
  T* Lb = reinterpret_cast<T*>(ws + p.l);
  T* Pb = reinterpret_cast<T*>(ws + p.p);
  switch (step) {
    case 0: A = Tb; lda = N; opA = 0; B = X + p.xB; K = N; C = Lb; acc = true; break;
    case 1: A = X + p.xA; lda = M; opA = 1; B = Tb; K = M; C = Lb; acc = true; break;
    case 2: A = Wb; lda = N; opA = 0; B = X + p.xB; K = N; C = Pb; acc = false; break;
    case 3: A = X + p.xA; lda = M; opA = 1; B = Pb; K = M; C = Lb; acc = true; break;
    case 4: A = Lb; lda = N; opA = 0; B = R + p.xB; K = N; C = Pb; acc = false; break;
    default: A = R + p.xA; lda = M; opA = 1; B = Pb; K = M; C = Tb; acc = false; break;
  }
  const int ldb = N;
  __shared__ T As[16][65];
  __shared__ T Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T c4[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c4[i][j] = tzero<T>();
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int l = threadIdx.x; l < 64 * 16; l += 256) {
      int r, kk;
      T v = tzero<T>();
      if (opA == 0) {
        r = l / 16; kk = l % 16;
        const int gr = m0 + r, gk = k0 + kk;
        if (gr < M && gk < K) v = A[(long long)gr * lda + gk];
      } else {
        kk = l / 64; r = l % 64;
        const int gr = m0 + r, gk = k0 + kk;
        if (gr < M && gk < K) v = conjg(A[(long long)gk * lda + gr]);
      }
      As[kk][r] = v;
    }
    for (int l = threadIdx.x; l < 16 * 64; l += 256) {
      const int kk = l / 64, cc = l % 64;
      const int gk = k0 + kk, gc = n0 + cc;
      Bs[kk][cc] = (gk < K && gc < N) ? B[(long long)gk * ldb + gc] : tzero<T>();
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c4[i][j] = mad(a[i], bb[j], c4[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + ty + 16 * i;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = n0 + tx + 16 * j;
      if (cc >= N) continue;
      const long long idx = (long long)r * N + cc;
      C[idx] = acc ? C[idx] + c4[i][j] : c4[i][j];
    }
  }
}

// h_AB (in Tb) -> molecular H; for A != B also h_BA = h_AB^H.
template <class T>
__global__ void k_dlu_scatter(const DluPair* P, char* ws, T* H, int Ntot) {
  const DluPair& p = P[blockIdx.y];
  constexpr bool TC = sizeof(T) == sizeof(cplx);
  const int NA = TC ? p.nA / 2 : p.nA, NB = TC ? p.nB / 2 : p.nB;
  const long long ld = TC ? 2LL * Ntot : (long long)Ntot;
  const T* hb = reinterpret_cast<const T*>(ws + p.t);
  const long long tot = (long long)p.nA * p.nB;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / p.nB), j = (int)(e % p.nB);
    const int si = i / NA, sj = j / NB;
    const long long r = (long long)si * Ntot + p.oA + (i - si * NA);
    const long long cl = (long long)sj * Ntot + p.oB + (j - sj * NB);
    const T v = hb[e];
    H[r * ld + cl] = v;
    if (p.A != p.B) H[cl * ld + r] = conjg(v);
  }
}

template <class T>
void launch_dlu(hipStream_t s, const DluPair* P, int npairs, int maxnA, int maxnB, char* ws, const double* Tm,
                const double* Vm, const double* Wm, int Ntot, double c, const double* X, const double* R, double* H) {
  long long g = ((long long)maxnA * maxnB + 255) / 256;
  if (g > 512) g = 512;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_dlu_gather<T>, dim3((int)g, npairs), dim3(256), 0, s, P, ws, Tm, Vm, Wm, Ntot, c);
  const dim3 gg((maxnB + 63) / 64, (maxnA + 63) / 64, npairs);
  const T* Xt = reinterpret_cast<const T*>(X);
  const T* Rt = reinterpret_cast<const T*>(R);
  for (int step = 0; step < 6; ++step)
    hipLaunchKernelGGL(k_dlu_gemm<T>, gg, dim3(256), 0, s, P, step, ws, Xt, Rt);
  hipLaunchKernelGGL(k_dlu_scatter<T>, dim3((int)g, npairs), dim3(256), 0, s, P, ws, reinterpret_cast<T*>(H), Ntot);
}
template void launch_dlu<double>(hipStream_t, const DluPair*, int, int, int, char*, const double*, const double*,
                                 const double*, int, double, const double*, const double*, double*);
template void launch_dlu<cplx>(hipStream_t, const DluPair*, int, int, int, char*, const double*, const double*,
                               const double*, int, double, const double*, const double*, double*);

}  // namespace x2c
