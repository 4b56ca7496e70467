// Device-wide path of one large block: a whole molecular matrix (the full,
// non-local transformation that the local DLU scheme of Sec. III.A
// approximates by atomic blocks) instead of a batch of atomic blocks.
//
// The per-block kernels of the batched path run one work-group per block and
// column step; a 4c matrix of dimension ~10^4 needs the whole GPU instead,
// and a Householder reduction of it would stream the trailing matrix from
// HBM once per column (hundreds of GB).  This path uses matrix products:
//
//  * the Cholesky factors L_S, L_T and their inverses are blocked in 64 x 64
//    tiles (one launch per panel step: diagonal tile, panel, trailing update;
//    then one launch per tile row of the inverse);
//  * the positive-energy branch (eps + c^2 > 0, Sec. II) of the reduced 4c
//    matrix A is taken from the spectral projector
//      P = (I + sign(A + c^2 I)) / 2,
//    computed by a scaled Newton-Schulz iteration X <- a X - b X^3 on
//    X_0 = (A + c^2 I) / rho, rho the smaller of the Frobenius norm and the
//    largest absolute row sum (two Hermitian products per step);
//  * with the column blocks of P on the large-component unit vectors,
//    X~ = P_SL P_LL^-1: if Y = [Y_L; Y_S] spans the positive branch
//    (orthonormal), P_LL = Y_L Y_L^H, P_SL = Y_S Y_L^H and P_SL P_LL^-1 =
//    Y_S Y_L^-1, the X~ of Eq. defxmat in the reduced basis;
//  * and I + X~^H X~ = (Y_L Y_L^H)^-1 = P_LL^-1, so the Q^-1/2 of the
//    renormalisation (Eq. ulnonortho) is P_LL^(1/2): one coupled
//    Newton-Schulz iteration Y <- Y U, Z <- U Z, U = (3I - Z Y) / 2 on
//    Y_0 = P_LL, Z_0 = I gives both P_LL^(1/2) and P_LL^(-1/2), and
//    X~ = P_SL P_LL^(-1/2) P_LL^(-1/2).
//
// Every iterate is a polynomial in one Hermitian matrix, so every product is
// Hermitian and runs as a lower-triangle product (half the tiles).  The
// iterations stop on the device: a gate word, passed to the product kernels
// in place of the block status, turns the remaining launches of a converged
// iteration into no-ops, so the host enqueues a fixed number of steps and
// never waits.  The element type T is double (spin-free, 4c dimension 2N),
// cplx (two-component, complex form, 4N) or quat (two-component quaternion
// form, 2N quaternions).
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// ---------------------------------------------------------------- blocked Cholesky
constexpr int LT = 64;   // tile edge

// Factor the diagonal tile at k0 of L_S (blockIdx.x = 0) or L_T (1), which
// holds S or T minus the updates of the earlier panels, and write the tile's
// inverse into the diagonal tile of L_S^-1 / L_T^-1.  Rows and columns past
// N are treated as the identity.
__global__ void __launch_bounds__(256) k_lchol_diag(const BlockDesc* D, char* ws, int* info, int k0) {
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b] || k0 >= d.N) return;
  const int which = blockIdx.x, N = d.N;
  double* A = bufp<double>(ws, d, which ? R_LT : R_LS);
  double* X = bufp<double>(ws, d, which ? R_LTI : R_LSI);
  __shared__ double a[LT][LT + 1], x[LT][LT + 1];
  __shared__ int fail;
  const int t = threadIdx.x;
  const int nb = min(LT, N - k0);
  for (int e = t; e < LT * LT; e += 256) {
    const int r = e / LT, c = e % LT;
    double v = 0.0;
    if (r < nb && c < nb) {
      if (c <= r) v = A[(long long)(k0 + r) * N + k0 + c];
    } else if (r == c) {
      v = 1.0;
    }
    a[r][c] = v;
  }
  if (t == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < LT; ++j) {
    if (t == 0) {
      const double p = a[j][j];
      if (!(p > 0.0) || !isfinite(p)) fail = 1;
      else a[j][j] = sqrt(p);
    }
    __syncthreads();
    if (fail) break;
    const double inv = 1.0 / a[j][j];
    for (int r = j + 1 + t; r < LT; r += 256) a[r][j] *= inv;
    __syncthreads();
    for (int e = t; e < LT * LT; e += 256) {
      const int r = e / LT, c = e % LT;
      if (c > j && r >= c) a[r][c] -= a[r][j] * a[c][j];
    }
    __syncthreads();
  }
  if (fail) {
    // S failing takes precedence over T failing
    if (t == 0) {
      if (which == 0) atomicExch(&info[b], 1);
      else atomicCAS(&info[b], 0, 2);
    }
    return;
  }
  // inverse of the lower-triangular tile, one column per thread
  if (t < LT) {
    const int c = t;
    for (int i = 0; i < LT; ++i) {
      if (i < c) {
        x[i][c] = 0.0;
        continue;
      }
      double s = i == c ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s = fma(-a[i][k], x[k][c], s);
      x[i][c] = s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    A[(long long)(k0 + r) * N + k0 + c] = c <= r ? a[r][c] : 0.0;
    X[(long long)(k0 + r) * N + k0 + c] = c <= r ? x[r][c] : 0.0;
  }
}

// 64 x 64 x 64 tile product on 256 threads (4 x 4 outputs each):
// acc[i][j] += sum_q p[tr + 16 i][q] * qt[tc + 16 j][q]  (B given transposed)
__device__ inline void tile_nt(const double (*p)[LT + 1], const double (*qt)[LT + 1], double acc[4][4], int tr,
                               int tc) {
  for (int q = 0; q < LT; ++q) {
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      av[i] = p[tr + 16 * i][q];
      bv[i] = qt[tc + 16 * i][q];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
  }
}

// Panel below the diagonal tile: L_ik = A_ik L_kk^-T, one tile per
// work-group (grid: row tiles below k0, matrix).
__global__ void __launch_bounds__(256) k_lchol_panel(const BlockDesc* D, char* ws, const int* info, int k0) {
  const BlockDesc& d = D[blockIdx.z];
  if (info[blockIdx.z]) return;
  const int N = d.N, which = blockIdx.y;
  const int i0 = k0 + LT * (1 + blockIdx.x);
  if (i0 >= N) return;
  double* A = bufp<double>(ws, d, which ? R_LT : R_LS);
  const double* X = bufp<double>(ws, d, which ? R_LTI : R_LSI);
  __shared__ double a[LT][LT + 1], x[LT][LT + 1];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  const int rb = min(LT, N - i0), kb = min(LT, N - k0);
  for (int e = t; e < LT * LT; e += 256) {
    const int r = e / LT, c = e % LT;
    a[r][c] = (r < rb && c < kb) ? A[(long long)(i0 + r) * N + k0 + c] : 0.0;
    x[r][c] = (r < kb && c <= r) ? X[(long long)(k0 + r) * N + k0 + c] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  tile_nt(a, x, acc, tr, tc);   // (A_ik L_kk^-T)[r][c] = sum_q A_ik[r][q] Linv[c][q]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = tr + 16 * i, c = tc + 16 * j;
      if (r < rb && c < kb) A[(long long)(i0 + r) * N + k0 + c] = acc[i][j];
    }
}

// Trailing update A_ij -= L_ik L_jk^T for the tiles j <= i below the panel
// (grid: lower tile pairs, matrix).
__global__ void __launch_bounds__(256) k_lchol_update(const BlockDesc* D, char* ws, const int* info, int k0) {
  const BlockDesc& d = D[blockIdx.z];
  if (info[blockIdx.z]) return;
  const int N = d.N, which = blockIdx.y;
  const int p = blockIdx.x;
  int ti = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= p) ++ti;
  while (ti * (ti + 1) / 2 > p) --ti;
  const int tj = p - ti * (ti + 1) / 2;
  const int i0 = k0 + LT * (1 + ti), j0 = k0 + LT * (1 + tj);
  if (i0 >= N || j0 >= N) return;
  double* A = bufp<double>(ws, d, which ? R_LT : R_LS);
  __shared__ double li[LT][LT + 1], lj[LT][LT + 1];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  const int rb = min(LT, N - i0), cb = min(LT, N - j0), kb = min(LT, N - k0);
  for (int e = t; e < LT * LT; e += 256) {
    const int r = e / LT, q = e % LT;
    li[r][q] = (r < rb && q < kb) ? A[(long long)(i0 + r) * N + k0 + q] : 0.0;
    lj[r][q] = (r < cb && q < kb) ? A[(long long)(j0 + r) * N + k0 + q] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  tile_nt(li, lj, acc, tr, tc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = tr + 16 * i, c = tc + 16 * j;
      if (r < rb && c < cb) A[(long long)(i0 + r) * N + j0 + c] -= acc[i][j];
    }
}

// Tile row ti of the inverse X = L^-1 (tiles j < ti; the diagonal tiles come
// from k_lchol_diag):  X_ij = -X_ii sum_{j <= k < i} L_ik X_kj.
__global__ void __launch_bounds__(256) k_ltri_row(const BlockDesc* D, char* ws, const int* info, int ti) {
  const BlockDesc& d = D[blockIdx.z];
  if (info[blockIdx.z] || ti * LT >= d.N) return;
  const int N = d.N, which = blockIdx.y, tj = blockIdx.x;
  const double* L = bufp<double>(ws, d, which ? R_LT : R_LS);
  double* X = bufp<double>(ws, d, which ? R_LTI : R_LSI);
  __shared__ double l[LT][LT + 1], xt[LT][LT + 1];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  const int i0 = ti * LT, j0 = tj * LT, rb = min(LT, N - i0);
  double acc[4][4] = {};
  for (int tk = tj; tk < ti; ++tk) {
    const int k0 = tk * LT;
    __syncthreads();
    for (int e = t; e < LT * LT; e += 256) {
      const int r = e / LT, q = e % LT;
      l[r][q] = r < rb ? L[(long long)(i0 + r) * N + k0 + q] : 0.0;
      // transposed: xt[c][q] = X[k0 + q][j0 + c] (tiles k < i are full)
      xt[q][r] = X[(long long)(k0 + r) * N + j0 + q];
    }
    __syncthreads();
    tile_nt(l, xt, acc, tr, tc);
  }
  __syncthreads();
  // s = acc (rows of the sum), then X_ij = -X_ii s
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) xt[tc + 16 * j][tr + 16 * i] = acc[i][j];   // xt[c][r] = s[r][c]
  for (int e = t; e < LT * LT; e += 256) {
    const int r = e / LT, q = e % LT;
    l[r][q] = (r < rb && q <= r) ? X[(long long)(i0 + r) * N + i0 + q] : 0.0;
  }
  __syncthreads();
  double out[4][4] = {};
  tile_nt(l, xt, out, tr, tc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = tr + 16 * i, c = tc + 16 * j;
      if (r < rb) X[(long long)(i0 + r) * N + j0 + c] = -out[i][j];
    }
}

// zero the strict upper triangles of L_S, L_T, L_S^-1, L_T^-1 (blockIdx.y)
__global__ void k_lzero_upper(const BlockDesc* D, char* ws, const int* info) {
  const BlockDesc& d = D[blockIdx.z];
  if (info[blockIdx.z]) return;
  const int ids[4] = {R_LS, R_LT, R_LSI, R_LTI};
  double* A = bufp<double>(ws, d, ids[blockIdx.y]);
  const int N = d.N;
  const long long NN = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < NN; e += (long long)gridDim.x * blockDim.x)
    if (e % N > e / N) A[e] = 0.0;
}

static int egrid(long long tot) {
  long long g = (tot + 255) / 256;
  if (g > NS_PARTS) g = NS_PARTS;
  if (g < 1) g = 1;
  return (int)g;
}

// blocks of different N in one launch sequence: the grids cover the largest,
// tiles past a block's own N exit
void launch_large_cholesky(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN) {
  const int nt = (maxN + LT - 1) / LT;
  for (int k = 0; k < nt; ++k) {
    const int k0 = k * LT, r = nt - k - 1;
    hipLaunchKernelGGL(k_lchol_diag, dim3(2, 1, nblk), dim3(256), 0, s, D, ws, info, k0);
    if (r == 0) break;
    hipLaunchKernelGGL(k_lchol_panel, dim3(r, 2, nblk), dim3(256), 0, s, D, ws, info, k0);
    hipLaunchKernelGGL(k_lchol_update, dim3(r * (r + 1) / 2, 2, nblk), dim3(256), 0, s, D, ws, info, k0);
  }
  for (int i = 1; i < nt; ++i) hipLaunchKernelGGL(k_ltri_row, dim3(i, 2, nblk), dim3(256), 0, s, D, ws, info, i);
  hipLaunchKernelGGL(k_lzero_upper, dim3(egrid((long long)maxN * maxN), 4, nblk), dim3(256), 0, s, D, ws, info);
}

// ---------------------------------------------------------------- Newton-Schulz iterations
// scaled cubic p(x) = a x - b x^3 for a spectrum in [l, 1] (in modulus):
// a^2 = 27 (1 - l) / (4 (1 - l^3)) equalises p(l) and p(1), b = 4 a^3 / 27
// puts the maximum p = 1 at x = 3 / (2a); a >= 3/2 (3/2 is the plain
// Newton-Schulz step, the limit l -> 1).  Small moduli grow by a (up to
// 3 sqrt3 / 2) per step; the new lower bound is min(p(l), p(1)).
__device__ inline void ns_cubic(double l, double& a, double& b, double& lnext) {
  a = sqrt(27.0 * (1.0 - l) / (4.0 * (1.0 - l * l * l)));
  if (!(a >= 1.5)) a = 1.5;
  b = 4.0 * a * a * a / 27.0;
  lnext = fmin(a * l - b * l * l * l, a - b);
  if (!(lnext > 0.0)) lnext = l;
}

__device__ inline NsPar* nspar(char* ws, const BlockDesc& d) { return bufp<NsPar>(ws, d, V_NS); }

// Kernels of the iterations run over the blocks of a launch: one-work-group
// kernels take the block from blockIdx.x, elementwise passes from
// blockIdx.y.  gate[b] is non-zero once block b's iteration has converged or
// the block has failed.

// start of an iteration phase: the gate follows the block status
__global__ void k_ns_begin(const BlockDesc* D, char* ws, const int* info, int* gate) {
  const int b = blockIdx.x;
  NsPar* p = nspar(ws, D[b]);
  gate[b] = info[b];
  p->conv = 0;
  p->iters = 0;
  p->rmax = 0ull;
}

// sum of the partials part[w][0 .. np) in a fixed order (one work-group)
__device__ inline double ns_sum(const NsPar* p, int w, int np, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += p->part[w][i];
  return block_sum(s, sh);
}

// end of a phase: an iteration that did not converge fails the block
__global__ void k_ns_end(const BlockDesc* D, char* ws, int* info, int* gate, int code) {
  const int b = blockIdx.x;
  const NsPar* p = nspar(ws, D[b]);
  if (info[b] == 0 && !p->conv) info[b] = code;
  gate[b] = info[b];
}

// ||A - sigma I||_F^2: one partial per work-group
template <class T>
__global__ void k_ns_fro(const BlockDesc* D, char* ws, const int* gate, int dsel, int buf, double sigma) {
  const int b = blockIdx.y;
  if (gate[b]) return;
  const BlockDesc& d = D[b];
  NsPar* p = nspar(ws, d);
  __shared__ double sh[16];
  const int n = seldim(d, dsel);
  const T* A = bufp<T>(ws, d, buf);
  const long long tot = (long long)n * n;
  double s = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    T v = A[e];
    if (e / n == e % n) v = v - treal<T>(sigma);
    s += abs2(v);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) p->part[0][blockIdx.x] = s;
}

// rho = min(||A - sigma I||_F, largest row sum of |A - sigma I|) (both bound
// the spectral radius from above), X_0 = (A - sigma I) / rho in place, and
// the first lower bound l_0 = gap / rho from the expected half-width of the
// gap
__global__ void k_ns_start(const BlockDesc* D, char* ws, int* gate, double sigma, double gap, int np) {
  const int b = blockIdx.x;
  if (gate[b]) return;
  NsPar* p = nspar(ws, D[b]);
  __shared__ double sh[16];
  const double f2 = ns_sum(p, 0, np, sh);
  if (threadIdx.x != 0) return;
  double rho = fmin(sqrt(f2), __longlong_as_double((long long)p->rmax));
  if (!(rho > 0.0) || !isfinite(rho)) {
    gate[b] = 1;   // no convergence: the phase end fails the block
    return;
  }
  p->sigma = sigma;
  p->rho = rho;
  p->l = fmin(fmax(gap / rho, 1e-14), 0.99);
  p->rmax = 0ull;
}

template <class T>
__global__ void k_ns_shift(const BlockDesc* D, char* ws, const int* gate, int dsel, int buf) {
  const int b = blockIdx.y;
  if (gate[b]) return;
  const BlockDesc& d = D[b];
  const NsPar* p = nspar(ws, d);
  const int n = seldim(d, dsel);
  T* A = bufp<T>(ws, d, buf);
  const double inv = 1.0 / p->rho, sigma = p->sigma;
  const long long tot = (long long)n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    T v = A[e];
    if (e / n == e % n) v = v - treal<T>(sigma);
    A[e] = inv * v;
  }
}

// polynomial factor of one step, in place on U = (product):
//   kind 0 (sign):         U <- a I - b U   (U = X^2; scaled cubic of l)
//   kind 2 (inverse sqrt): U <- (3 I - U) / 2  (U = Z Y)
template <class T>
__global__ void k_ns_poly(const BlockDesc* D, char* ws, const int* gate, int dsel, int buf, int kind) {
  const int b = blockIdx.y;
  if (gate[b]) return;
  const BlockDesc& d = D[b];
  const NsPar* p = nspar(ws, d);
  const int n = seldim(d, dsel);
  T* U = bufp<T>(ws, d, buf);
  double dg, sc;
  if (kind == 0) {
    double a, bc, ln;
    ns_cubic(p->l, a, bc, ln);
    dg = a;
    sc = -bc;
  } else {
    dg = 1.5;
    sc = -0.5;
  }
  const long long tot = (long long)n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    T v = sc * U[e];
    if (e / n == e % n) v = v + treal<T>(dg);
    U[e] = v;
  }
}

// dst <- src; with diff, the work-group's partials of ||src - dst||_F^2 and
// ||src||_F^2
template <class T>
__global__ void k_ns_accept(const BlockDesc* D, char* ws, const int* gate, int dsel, int src, int dst, int diff) {
  const int b = blockIdx.y;
  if (gate[b]) return;
  const BlockDesc& d = D[b];
  NsPar* p = nspar(ws, d);
  __shared__ double sh[16];
  const int n = seldim(d, dsel);
  const T* S = bufp<T>(ws, d, src);
  T* X = bufp<T>(ws, d, dst);
  const long long tot = (long long)n * n;
  double s1 = 0.0, s2 = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const T v = S[e];
    if (diff) {
      s1 += abs2(v - X[e]);
      s2 += abs2(v);
    }
    X[e] = v;
  }
  if (!diff) return;
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    p->part[0][blockIdx.x] = s1;
    p->part[1][blockIdx.x] = s2;
  }
}

// end of a step: relative change d = ||X_new - X||_F / ||X_new||_F; the
// iteration has converged once d <= tol (the next error is O(d^2))
__global__ void k_ns_check(const BlockDesc* D, char* ws, int* gate, int kind, double tol, int np) {
  const int b = blockIdx.x;
  if (gate[b]) return;
  NsPar* p = nspar(ws, D[b]);
  __shared__ double sh[16];
  const double s1 = ns_sum(p, 0, np, sh), s2 = ns_sum(p, 1, np, sh);
  if (threadIdx.x != 0) return;
  p->iters += 1;
  const double dd = sqrt(s1 / fmax(s2, 1e-300));
  if (kind == 0) {
    double a, bc, ln;
    ns_cubic(p->l, a, bc, ln);
    p->l = ln;
  }
  if (dd <= tol) {
    p->conv = 1;
    gate[b] = 1;
  }
}

// trace of the converged sign: the positive and negative branches must be
// equally large (Sec. II), i.e. trace 0 (one work-group)
template <class T>
__global__ void k_ns_trace(const BlockDesc* D, char* ws, int* info, int dsel, int buf) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  __shared__ double sh[16];
  const int n = seldim(d, dsel);
  const T* X = bufp<T>(ws, d, buf);
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += re(X[(long long)i * n + i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0 && !(fabs(s) < 0.5)) info[b] = 4;
}

// P = (I + X) / 2 on the large-component columns: P_LL = (I + X_LL) / 2,
// P_SL = X_SL / 2 (h-sized, dimension h = 4c dimension / 2)
template <class T>
__global__ void k_ns_split(const BlockDesc* D, char* ws, const int* info, int dsel4, int bufX, int bufLL, int bufSL) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n4 = seldim(d, dsel4), h = n4 / 2;
  const T* X = bufp<T>(ws, d, bufX);
  T* PLL = bufp<T>(ws, d, bufLL);
  T* PSL = bufp<T>(ws, d, bufSL);
  const long long tot = (long long)h * h;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / h), j = (int)(e % h);
    T v = 0.5 * X[(long long)i * n4 + j];
    if (i == j) v = v + treal<T>(0.5);
    PLL[e] = v;
    PSL[e] = 0.5 * X[(long long)(h + i) * n4 + j];
  }
}

template <class T>
__global__ void k_ns_eye(const BlockDesc* D, char* ws, const int* info, int dsel, int buf) {
  const BlockDesc& d = D[blockIdx.y];
  if (info[blockIdx.y]) return;
  const int n = seldim(d, dsel);
  T* A = bufp<T>(ws, d, buf);
  const long long tot = (long long)n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x)
    A[e] = treal<T>(e / n == e % n ? 1.0 : 0.0);
}

// largest row sum of the moduli of A - sigma I (>= its spectral radius), one
// wave per row; non-negative doubles order like their bit patterns
template <class T>
__global__ void k_ns_rowmax(const BlockDesc* D, char* ws, const int* gate, int dsel, int buf, double sigma) {
  const int b = blockIdx.y;
  if (gate[b]) return;
  const BlockDesc& d = D[b];
  NsPar* p = nspar(ws, d);
  const int n = seldim(d, dsel);
  const T* A = bufp<T>(ws, d, buf);
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) {
    T v = A[(long long)row * n + j];
    if (j == row) v = v - treal<T>(sigma);
    s += sqrt(abs2(v));
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) atomicMax(&p->rmax, (unsigned long long)__double_as_longlong(s));
}

// eigenvalues are not produced by this path: NaN marks them
__global__ void k_eps_nan(const BlockDesc* D, double* eps) {
  const BlockDesc& d = D[blockIdx.y];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.n; k += gridDim.x * blockDim.x)
    eps[d.eps_off + k] = __longlong_as_double(0x7ff8000000000000ll);
}

// ---------------------------------------------------------------- whole-matrix quaternion products
// C = A B (+ beta C) for one large quaternion matrix (the iterations' products:
// no transposes).  A work-group computes a tile of TR = 16 RB rows x 64
// columns: wave w owns column block w (16 columns) and all RB row blocks of
// 16, 16 MFMAs (v_mfma_f64_16x16x4f64) per 16 x 16 block and k step of 4,
// operands staged in LDS as four component planes, k chunks of 16.  PF: the
// next chunk's operands are loaded into registers while the current one is
// multiplied.  Tiles are enumerated (Hermitian products: only those reaching
// the lower triangle), and consecutive tiles go to one XCD (work-group i runs
// on XCD i mod 8), so that tiles sharing a row panel share an L2.  The row
// height is chosen per launch by the wave-quantisation model of
// launch_gemm_q_big.
typedef __attribute__((ext_vector_type(4))) double d4;
constexpr int BG_K = 16, BG_LD = BG_K + 1, BG_TC = 64;

__host__ __device__ inline int big_row_tiles(int n, int TR, int herm, int ct, int ti) {
  // column tiles of row tile ti
  if (!herm) return ct;
  const int last = min(n - 1, TR * ti + TR - 1);
  return min(ct, last / BG_TC + 1);
}

template <int RB, int PF>
__global__ void __launch_bounds__(256, 2) k_gemm_q_big(const BlockDesc* D, char* ws, const int* gate, int dsel,
                                                       int bufA, int bufB, int bufC, double beta, int herm,
                                                       int ntiles) {
  constexpr int TR = 16 * RB;
  if (gate[0]) return;
  const BlockDesc& d = D[0];
  const int n = seldim(d, dsel);
  const int ct = (n + BG_TC - 1) / BG_TC;
  // XCD-grouped tile index (the grid is a multiple of 8)
  const int per = gridDim.x / 8;
  int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= ntiles) return;
  int ti = 0;
  for (;;) {
    const int c = big_row_tiles(n, TR, herm, ct, ti);
    if (tile < c) break;
    tile -= c;
    ++ti;
  }
  const int m0 = ti * TR, n0 = tile * BG_TC;
  const quat* A = bufp<quat>(ws, d, bufA);
  const quat* B = bufp<quat>(ws, d, bufB);
  quat* C = bufp<quat>(ws, d, bufC);
  __shared__ double As[4][TR][BG_LD];        // [component][row][k]
  __shared__ double Bs[4][BG_K][BG_TC + 1];  // [component][k][col]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 acc[RB][4];
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[x][c] = d4{0.0, 0.0, 0.0, 0.0};
  quat ra[RB], rb[4];
  // chunk k0: thread t loads A rows t / 16 + 16 q, k t % 16, and B row t / 64 + 4 q, column t % 64
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int r = m0 + (t >> 4) + 16 * q, k = k0 + (t & 15);
      ra[q] = (r < n && k < n) ? A[(long long)r * n + k] : tzero<quat>();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + (t >> 6) + 4 * q, c = n0 + (t & 63);
      rb[q] = (k < n && c < n) ? B[(long long)k * n + c] : tzero<quat>();
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int r = (t >> 4) + 16 * q, k = t & 15;
      As[0][r][k] = ra[q].a.x;
      As[1][r][k] = ra[q].a.y;
      As[2][r][k] = ra[q].b.x;
      As[3][r][k] = ra[q].b.y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = (t >> 6) + 4 * q, c = t & 63;
      Bs[0][k][c] = rb[q].a.x;
      Bs[1][k][c] = rb[q].a.y;
      Bs[2][k][c] = rb[q].b.x;
      Bs[3][k][c] = rb[q].b.y;
    }
  };
  const int wc = 16 * wave;
  // (x y)_c = sum_e sigma(c, c xor e) x_e y_(c xor e): the signs sit on the B
  // operand, whose four components per k step are kept in both signs
  auto compute = [&]() {
#pragma unroll 1
    for (int ks = 0; ks < BG_K; ks += 4) {
      double a[RB][4], bp[4], bn[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bp[c] = Bs[c][ks + l4][wc + l16];
        bn[c] = -bp[c];
#pragma unroll
        for (int x = 0; x < RB; ++x) a[x][c] = As[c][16 * x + l16][ks + l4];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < RB; ++x)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[x][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a[x][e], qmul_sign(c, c ^ e) > 0 ? bp[c ^ e] : bn[c ^ e], acc[x][c], 0, 0, 0);
    }
  };
  if (PF) {
    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += BG_K) {
      const bool more = k0 + BG_K < n;
      if (more) fetch(k0 + BG_K);
      compute();
      __syncthreads();
      if (more) {
        stash();
        __syncthreads();
      }
    }
  } else {
    for (int k0 = 0; k0 < n; k0 += BG_K) {
      fetch(k0);          // in flight during the barrier
      __syncthreads();
      stash();
      __syncthreads();
      compute();
    }
  }
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = m0 + 16 * x + l4 + 4 * i, cc = n0 + wc + l16;
      if (r >= n || cc >= n || (herm && cc > r)) continue;
      const long long idx = (long long)r * n + cc;
      quat v = {{acc[x][0][i], acc[x][1][i]}, {acc[x][2][i], acc[x][3][i]}};
      if (beta != 0.0) v = v + beta * C[idx];
      C[idx] = v;
      if (herm && cc < r) C[(long long)cc * n + r] = conjg(v);
    }
}

// tiles of a launch for row blocks RB, and the predicted time: rounds of 512
// resident work-groups (two per CU) times the work of one tile
static long long big_tiles(int n, int RB, int herm) {
  const int TR = 16 * RB, rt = (n + TR - 1) / TR, ct = (n + BG_TC - 1) / BG_TC;
  long long c = 0;
  for (int i = 0; i < rt; ++i) c += big_row_tiles(n, TR, herm, ct, i);
  return c;
}

template <int RB, int PF>
void launch_gemm_q_big_v(hipStream_t s, const BlockDesc* D, char* ws, const int* gate, int n, int dsel, int bufA,
                         int bufB, int bufC, double beta, int herm) {
  const long long t = big_tiles(n, RB, herm);
  const int g = (int)((t + 7) / 8 * 8);
  hipLaunchKernelGGL((k_gemm_q_big<RB, PF>), dim3(g), dim3(256), 0, s, D, ws, gate, dsel, bufA, bufB, bufC, beta,
                     herm, (int)t);
}

void launch_gemm_q_big(hipStream_t s, const BlockDesc* D, char* ws, const int* gate, int n, int dsel, int bufA,
                       int bufB, int bufC, double beta, int herm) {
  // RB = 5 keeps 254 VGPRs without the prefetch registers, RB = 4 fits them:
  // measured on MI355X (quaternion 4992: Hermitian 29.9 ms RB 5 against 31.0
  // RB 4; full 56.6 RB 4 against 59.9 RB 5), the model picks the faster in each
  constexpr long long SLOTS = 512;
  const long long c4 = (big_tiles(n, 4, herm) + SLOTS - 1) / SLOTS * 4;
  const long long c5 = (big_tiles(n, 5, herm) + SLOTS - 1) / SLOTS * 5;
  if (c5 < c4) launch_gemm_q_big_v<5, 0>(s, D, ws, gate, n, dsel, bufA, bufB, bufC, beta, herm);
  else launch_gemm_q_big_v<4, 1>(s, D, ws, gate, n, dsel, bufA, bufB, bufC, beta, herm);
}

// ---------------------------------------------------------------- host side
namespace {
// products of the iterations: a large single block on the whole-matrix
// kernel, anything else on the batched one (the gate array in place of the
// block status)
template <class T>
void gemm(hipStream_t s, const BlockDesc* D, char* ws, const int* gate, int nblk, int maxdim, int dsel, int A, int B,
          int C, int herm) {
  if constexpr (is_quat<T>()) {
    // the whole-matrix kernel for one block large enough to fill the GPU
    // with its tiles (64 x 64 tiles: at least two per CU); else the batched
    // kernel, which takes 32 x 32 tiles when there are few
    const int t = (maxdim + 63) / 64;
    if (nblk == 1 && (herm ? t * (t + 1) / 2 : t * t) >= 2 * 256)
      launch_gemm_q_big(s, D, ws, gate, maxdim, dsel, A, B, C, 0.0, herm);
    else launch_gemm_q(s, D, ws, gate, nblk, maxdim, dsel, A, 0, B, 0, C, 1.0, 0.0, herm);
  } else {
    launch_gemm<T>(s, D, ws, gate, nblk, maxdim, dsel, A, 0, B, 0, C, treal<T>(1.0), tzero<T>(), herm, 0);
  }
}
}  // namespace

template <class T>
void launch_large_sign(hipStream_t s, const BlockDesc* D, char* ws, int* info, int* gate, int nblk, int dsel4,
                       int maxdim4, int bufX, int bufU, int bufN, double c, int maxit, double tol) {
  const long long tot = (long long)maxdim4 * maxdim4;
  const int eg = egrid(tot);
  const dim3 ge(eg, nblk);
  const double sigma = -c * c;
  hipLaunchKernelGGL(k_ns_begin, dim3(nblk), dim3(1), 0, s, D, ws, info, gate);
  hipLaunchKernelGGL(k_ns_fro<T>, ge, dim3(256), 0, s, D, ws, gate, dsel4, bufX, sigma);
  hipLaunchKernelGGL(k_ns_rowmax<T>, dim3((maxdim4 + 3) / 4, nblk), dim3(256), 0, s, D, ws, gate, dsel4, bufX, sigma);
  hipLaunchKernelGGL(k_ns_start, dim3(nblk), dim3(256), 0, s, D, ws, gate, sigma, 0.5 * c * c, eg);
  hipLaunchKernelGGL(k_ns_shift<T>, ge, dim3(256), 0, s, D, ws, gate, dsel4, bufX);
  for (int it = 0; it < maxit; ++it) {
    gemm<T>(s, D, ws, gate, nblk, maxdim4, dsel4, bufX, bufX, bufU, 1);
    hipLaunchKernelGGL(k_ns_poly<T>, ge, dim3(256), 0, s, D, ws, gate, dsel4, bufU, 0);
    gemm<T>(s, D, ws, gate, nblk, maxdim4, dsel4, bufX, bufU, bufN, 1);
    hipLaunchKernelGGL(k_ns_accept<T>, ge, dim3(256), 0, s, D, ws, gate, dsel4, bufN, bufX, 1);
    hipLaunchKernelGGL(k_ns_check, dim3(nblk), dim3(256), 0, s, D, ws, gate, 0, tol, eg);
  }
  hipLaunchKernelGGL(k_ns_end, dim3(nblk), dim3(1), 0, s, D, ws, info, gate, 3);
  hipLaunchKernelGGL(k_ns_trace<T>, dim3(nblk), dim3(256), 0, s, D, ws, info, dsel4, bufX);
}

// X~ and Q^-1/2 from one coupled Newton-Schulz iteration on P_LL: with P an
// orthogonal projector, I + X~^H X~ = P_LL^-1 for X~ = P_SL P_LL^-1, so
// Q^-1/2 = P_LL^(1/2).  Y_0 = P_LL (eigenvalues in (0, 1]), Z_0 = I,
// U = (3I - Z Y) / 2, Y <- Y U, Z <- U Z: Y -> P_LL^(1/2) (into bufQmh),
// Z -> P_LL^(-1/2); then X~ = (P_SL Z) Z.
template <class T>
void launch_large_xrenorm(hipStream_t s, const BlockDesc* D, char* ws, int* info, int* gate, int nblk, int dsel4,
                          int dselh, int maxdimh, int bufX, int bufPSL, int bufZ, int bufU, int bufN, int bufXt,
                          int bufQmh, int maxit, double tol) {
  const long long tot = (long long)maxdimh * maxdimh;
  const int eg = egrid(tot);
  const dim3 ge(eg, nblk);
  hipLaunchKernelGGL(k_ns_split<T>, ge, dim3(256), 0, s, D, ws, info, dsel4, bufX, bufQmh, bufPSL);
  hipLaunchKernelGGL(k_ns_eye<T>, ge, dim3(256), 0, s, D, ws, info, dselh, bufZ);
  hipLaunchKernelGGL(k_ns_begin, dim3(nblk), dim3(1), 0, s, D, ws, info, gate);
  for (int it = 0; it < maxit; ++it) {
    gemm<T>(s, D, ws, gate, nblk, maxdimh, dselh, bufZ, bufQmh, bufU, 1);
    hipLaunchKernelGGL(k_ns_poly<T>, ge, dim3(256), 0, s, D, ws, gate, dselh, bufU, 2);
    gemm<T>(s, D, ws, gate, nblk, maxdimh, dselh, bufQmh, bufU, bufN, 1);
    hipLaunchKernelGGL(k_ns_accept<T>, ge, dim3(256), 0, s, D, ws, gate, dselh, bufN, bufQmh, 0);
    gemm<T>(s, D, ws, gate, nblk, maxdimh, dselh, bufU, bufZ, bufN, 1);
    hipLaunchKernelGGL(k_ns_accept<T>, ge, dim3(256), 0, s, D, ws, gate, dselh, bufN, bufZ, 1);
    hipLaunchKernelGGL(k_ns_check, dim3(nblk), dim3(256), 0, s, D, ws, gate, 2, tol, eg);
  }
  hipLaunchKernelGGL(k_ns_end, dim3(nblk), dim3(1), 0, s, D, ws, info, gate, 3);
  // X~ = (P_SL Z) Z (general products: the gates are the block status again)
  gemm<T>(s, D, ws, gate, nblk, maxdimh, dselh, bufPSL, bufZ, bufN, 0);
  gemm<T>(s, D, ws, gate, nblk, maxdimh, dselh, bufN, bufZ, bufXt, 0);
}

void launch_eps_nan(hipStream_t s, const BlockDesc* D, double* eps, int nblk) {
  hipLaunchKernelGGL(k_eps_nan, dim3(16, nblk), dim3(256), 0, s, D, eps);
}

#define X2C_LARGE_INST(T)                                                                                         \
  template void launch_large_sign<T>(hipStream_t, const BlockDesc*, char*, int*, int*, int, int, int, int, int, int, \
                                     double, int, double);                                                       \
  template void launch_large_xrenorm<T>(hipStream_t, const BlockDesc*, char*, int*, int*, int, int, int, int, int, \
                                        int, int, int, int, int, int, int, double);
X2C_LARGE_INST(double)
X2C_LARGE_INST(cplx)
X2C_LARGE_INST(quat)

}  // namespace x2c
