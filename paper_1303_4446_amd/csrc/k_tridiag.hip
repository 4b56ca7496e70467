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
#include "x2c_tridiag.h"

#include <algorithm>

namespace x2c {

// Reflector for column k (rows k+1..n-1) into vout[0..len).  Returns through
// shared scalars.  All threads call.  col (may be null): LDS copy of the
// column, col[i] = A[k+1+i][k], read instead of A.
template <class T>
__device__ void make_reflector(T* A, int n, int k, T* vout, T* tau_out, double* beta_out, double* red,
                               const T* col = nullptr) {
  const int len = n - k - 1;
  auto ld = [&](int i) { return col ? col[i] : A[(long long)(k + 1 + i) * n + k]; };
  double xn2 = 0.0;
  for (int i = 1 + threadIdx.x; i < len; i += blockDim.x) xn2 += abs2(ld(i));
  xn2 = block_sum(xn2, red);
  T alpha = ld(0);
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
      T x = trivial ? tzero<T>() : ld(i) * scale;
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

// Quaternion Householder reflector for column k (rows k+1..n-1): with
// x0 = A[k+1][k], sigma = (x0/|x0|) ||x||, u = x + sigma e1, the Hermitian
// reflector I - 2 u u^H / u^H u maps x to -sigma e1.  Normalised to
// v = u u0^-1 (v0 = 1) it is I - tau v v^H with real tau = 1 + |x0|/||x||.
// beta_out = -sigma (quaternion sub-diagonal entry).
__device__ void make_reflector_q(quat* A, int n, int k, quat* vout, quat* tau_out, quat* beta_out, double* red,
                                 const quat* col = nullptr) {
  const int len = n - k - 1;
  auto ld = [&](int i) { return col ? col[i] : A[(long long)(k + 1 + i) * n + k]; };
  double xn2 = 0.0;
  for (int i = 1 + threadIdx.x; i < len; i += blockDim.x) xn2 += abs2(ld(i));
  xn2 = block_sum(xn2, red);
  const quat x0 = ld(0);
  const double a0 = sqrt(abs2(x0));
  const double xn = sqrt(a0 * a0 + xn2);
  const bool trivial = (xn2 == 0.0 && x0.a.y == 0.0 && x0.b.x == 0.0 && x0.b.y == 0.0);
  quat tau = tzero<quat>(), beta = x0, uinv = tzero<quat>();
  if (!trivial) {
    const quat ph = a0 > 0.0 ? (1.0 / a0) * x0 : treal<quat>(1.0);
    const quat sig = xn * ph;
    const quat u0 = x0 + sig;
    uinv = (1.0 / abs2(u0)) * conjg(u0);
    tau = treal<quat>(1.0 + a0 / xn);
    beta = -sig;
  }
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    if (i == 0) {
      vout[0] = treal<quat>(1.0);
    } else {
      long long idx = (long long)(k + 1 + i) * n + k;
      quat x = trivial ? tzero<quat>() : ld(i) * uinv;
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

// ---------------------------------------------------------------- blocked
// Blocked reduction over the whole batch (panels of PW columns, lower
// triangle only).  Inside a panel the trailing matrix is left as it was at
// the panel start; with the panel's reflectors V and companion vectors W the
// current trailing matrix is A - V W^H - W V^H.  Per column k:
//   k_tri_col    (one work-group per block): reduce the previous column's
//                matvec, subtract the panel corrections, form w (stored as
//                column of W), update column k with the panel corrections and
//                build reflector k (v_k -> global vector buffer);
//   k_tri_matvec (one work-group per 64 x 64 lower super-tile): each wave
//                stages a 32 x 32 tile in LDS and writes its row sums and
//                (off the diagonal) its transposed column sums with v_k;
// after the panel k_tri_her2k updates the trailing lower triangle.  The tile
// sums are added in a fixed order, so results are bitwise reproducible.

// phase: 0 = first column of a panel (no previous column to finish)
//        1 = finish column k-1 (w), then build column k if it is in the panel
//        2 = finish column k-1 only (last column of the panel)
constexpr int COLT = 256;   // threads of the per-block column kernel
constexpr int CTPR = 4;     // threads per trailing row in its row loop

// sum over the G lanes of an aligned lane group, every lane gets the same
// bits (pairwise tree: lane xor 1, then xor 2, ...)
template <int G, class T>
__device__ inline T group_allsum(T x) {
  constexpr int ND = sizeof(T) / sizeof(double);
  double* p = reinterpret_cast<double*>(&x);
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    double v = p[c];
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
    p[c] = v;
  }
  return x;
}

template <class T>
__global__ void __launch_bounds__(COLT) k_tri_col(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                                 int bufD, int bufE, int bufTau, int bufW, int bufV, int bufHS,
                                                 int bufET, int k0, int i, int phase) {
  constexpr int PW = panel_width<T>();
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  if (k0 >= n - 1 || k0 >= tri_tail_start<T>(n)) return;
  const int kb = min(PW, n - 1 - k0);
  T* A = bufp<T>(ws, d, bufA);
  double* dd = bufp<double>(ws, d, bufD);
  double* ee = bufp<double>(ws, d, bufE);
  T* taus = bufp<T>(ws, d, bufTau);
  T* Wp = bufp<T>(ws, d, bufW);
  T* vg = bufp<T>(ws, d, bufV);
  const T* HS = bufp<T>(ws, d, bufHS);
  const int tid = threadIdx.x;
  extern __shared__ char smem[];
  T* v = reinterpret_cast<T*>(smem);
  T* y = v + n;
  T* colacc = y + n;
  T* acol = colacc + n;                 // column k (rows off..n-1) of A, updated in LDS
  T* tps = acol + n;                    // the matvec's panel dot partials (strips x PW x 2)
  __shared__ double red[32];
  __shared__ T sh_tau;
  __shared__ double sh_beta;
  __shared__ T sh_alpha;
  __shared__ T wk[PW], vk[PW], t1[PW], t2[PW];

  const int k = k0 + i;                 // column to build (if any)
  const bool build = phase != 2 && i < kb;
  if (phase != 0) {
    const int ip = i - 1;              // column being finished
    if (ip >= kb) return;
    const int kp = k0 + ip;
    const int off = kp + 1, len = n - kp - 1;
    const T tau = taus[kp];
    // the matvec's tiling: lead virtual rows, then the len trailing rows
    const int lead = mv_lead<T>(kp), lenp = len + lead;
    // the matvec's super-tile edge for this block and step
    const int st = is_quat<T>() ? mv_st_q(lenp) : 2 * Tiles<T>::HT;
    const int nst = (lenp + st - 1) / st;
    // every load of this part goes out before the first wait: v, column k,
    // row k of the panel and the per-strip panel dot partials (staged in LDS)
    const T* TP = HS + (long long)2 * nst * lenp;
    for (int e = tid; e < nst * PW * 2; e += COLT) tps[e] = TP[e];
    for (int r = tid; r < len; r += COLT) {
      v[r] = vg[r];
      if (build) acol[r] = A[(long long)(off + r) * n + k];
    }
    if (build && tid < ip) {
      wk[tid] = conjg(Wp[(long long)k * PW + tid]);
      vk[tid] = conjg(panel_v(A, n, k0, k, tid));
    }
    __syncthreads();
    // panel dot products t1 = W^H v, t2 = V^H v: the strips' partials in order
    if (tid < ip) {
      T a1 = tzero<T>(), a2 = tzero<T>();
      for (int S = 0; S < nst; ++S) {
        a1 = a1 + tps[(S * PW + tid) * 2];
        a2 = a2 + tps[(S * PW + tid) * 2 + 1];
      }
      t1[tid] = a1;
      t2[tid] = a2;
    }
    __syncthreads();
    // y_r = fixed-order sum of the super-tile partials minus the panel
    // corrections; the same pass accumulates the panel part of the update of
    // the next column.  CTPR threads per row: thread q of the group takes the
    // super-tile partials S = q, q+CTPR, ... and the panel columns j = q,
    // q+CTPR, ... (rows off + r lie below the unit entry of every panel
    // reflector, so V is read as stored); the group's sums are combined by
    // lane exchange in a fixed pattern.  Each group takes two rows per pass
    // and issues the loads of both (the first NSU partials per thread, the
    // panel rows; clamped in-range addresses, masked values) before using
    // any, so that a pass costs one memory round trip.
    constexpr int NSU = 4, PU = PW / CTPR, YR = COLT / CTPR;
    const int q = tid % CTPR;
    auto issue = [&](int r, T (&hp)[NSU], T (&vr)[PU], T (&wr)[PU]) {
      const int rt = r + lead, Sr = rt / st;
      const long long rr = off + r;
#pragma unroll
      for (int u = 0; u < NSU; ++u) {
        const int S = min(q + CTPR * u, nst - 1);
        hp[u] = HS[(long long)(S <= Sr ? S : nst + S) * lenp + rt];
      }
      if (ip > 0) {
#pragma unroll
        for (int u = 0; u < PU; ++u) {
          const int j = min(q + CTPR * u, ip - 1);
          vr[u] = A[rr * n + k0 + j];
          wr[u] = Wp[rr * PW + j];
        }
      }
    };
    auto finish = [&](int r, const T (&hp)[NSU], const T (&vr)[PU], const T (&wr)[PU]) {
      const int rt = r + lead, Sr = rt / st;
      T acc = tzero<T>(), ca = tzero<T>();
#pragma unroll
      for (int u = 0; u < NSU; ++u)
        if (q + CTPR * u < nst) acc = acc + hp[u];
      for (int S = q + CTPR * NSU; S < nst; S += CTPR)   // more than CTPR * NSU strips
        acc = acc + HS[(long long)(S <= Sr ? S : nst + S) * lenp + rt];
      if (ip > 0) {
#pragma unroll
        for (int u = 0; u < PU; ++u) {
          const int j = q + CTPR * u;
          if (j < ip) {
            acc = acc - vr[u] * t1[j] - wr[u] * t2[j];
            ca = ca + vr[u] * wk[j] + wr[u] * vk[j];
          }
        }
      }
      acc = group_allsum<CTPR>(acc);
      ca = group_allsum<CTPR>(ca);
      if (q == 0) {
        y[r] = acc;
        colacc[r] = ca;
      }
    };
    for (int r = tid / CTPR; r < len; r += 2 * YR) {
      T hpa[NSU], vra[PU], wra[PU], hpb[NSU], vrb[PU], wrb[PU];
      const bool two = r + YR < len;      // the same for the CTPR lanes of a row
      issue(r, hpa, vra, wra);
      if (two) issue(r + YR, hpb, vrb, wrb);
      finish(r, hpa, vra, wra);
      if (two) finish(r + YR, hpb, vrb, wrb);
    }
    __syncthreads();   // y, colacc are read below by other threads
    double dr = 0.0, di = 0.0;
    for (int r = tid; r < len; r += COLT) {
      T yt = tau * y[r];
      y[r] = yt;
      T pv = conjg(yt) * v[r];
      dr += re(pv);
      di += im(pv);
    }
    dr = block_sum(dr, red);
    if (sizeof(T) == sizeof(cplx)) di = block_sum(di, red);
    if (tid == 0) {
      if constexpr (is_quat<T>()) sh_alpha = treal<T>(-0.5 * re(tau) * dr);   // y^H v is real
      else sh_alpha = (-0.5 * tau) * tmake<T>(dr, di);
    }
    __syncthreads();
    const T alpha = sh_alpha;
    for (int r = tid; r < len; r += COLT) {
      T w = mad(alpha, v[r], y[r]);
      y[r] = w;
      Wp[(long long)(off + r) * PW + ip] = w;
    }
    __syncthreads();
    if (!build) return;
    // column k = off: A[r][k] -= (panel columns < ip) + v_r conj(w_0) + w_r conj(v_0), v_0 = 1
    const T w0c = conjg(y[0]);
    for (int r = tid; r < len; r += COLT) {
      T a = acol[r] - colacc[r] - v[r] * w0c - y[r];
      if (r == 0) a = treal<T>(re(a));
      acol[r] = a;
      if (r == 0) A[(long long)off * n + k] = a;   // diagonal; the rest is replaced by the reflector
    }
    __syncthreads();
  } else {
    if (!build) return;
    // first column of a panel is current after the previous trailing update
    if (tid == 0) A[(long long)k * n + k] = treal<T>(re(A[(long long)k * n + k]));
    __syncthreads();
  }
  if constexpr (is_quat<T>()) {
    __shared__ T sh_betaq;
    make_reflector_q(A, n, k, vg, &sh_tau, &sh_betaq, red, phase != 0 ? acol + 1 : nullptr);
    if (tid == 0) {
      ee[k] = sqrt(abs2(sh_betaq));
      bufp<T>(ws, d, bufET)[k] = sh_betaq;
    }
  } else {
    make_reflector<T>(A, n, k, vg, &sh_tau, &sh_beta, red, phase != 0 ? acol + 1 : nullptr);
    if (tid == 0) ee[k] = sh_beta;
  }
  // the reflector went straight to the global vector (the old one was read
  // into LDS before the first barrier)
  if (tid == 0) {
    dd[k] = re(A[(long long)k * n + k]);
    taus[k] = sh_tau;
  }
}

// Trailing lower triangle (rows/cols >= k0 + kb): A -= V W^H + W V^H.
// grid = (lower 32 x 32 tiles, nblk).
template <class T>
__global__ void __launch_bounds__(256) k_tri_her2k(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                                   int bufW, int k0) {
  constexpr int TT = Tiles<T>::TT, PW = panel_width<T>();
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  if (k0 >= n - 1) return;
  const int kb = min(PW, n - 1 - k0);
  const int c0 = k0 + kb;
  const int len = n - c0;
  if (len <= 0) return;
  const int nt = (len + TT - 1) / TT;
  const int t = blockIdx.x;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  T* A = bufp<T>(ws, d, bufA);
  const T* Wp = bufp<T>(ws, d, bufW);
  __shared__ T Vr[TT][PW + 1], Wr[TT][PW + 1], Vc[TT][PW + 1], Wc[TT][PW + 1];
  for (int e = threadIdx.x; e < TT * PW; e += 256) {
    int rr = e / PW, j = e % PW;
    int r = c0 + TT * I + rr, c = c0 + TT * J + rr;
    bool okr = r < n && j < kb, okc = c < n && j < kb;
    Vr[rr][j] = okr ? panel_v(A, n, k0, r, j) : tzero<T>();
    Wr[rr][j] = okr ? Wp[(long long)r * PW + j] : tzero<T>();
    Vc[rr][j] = okc ? conjg(panel_v(A, n, k0, c, j)) : tzero<T>();
    Wc[rr][j] = okc ? conjg(Wp[(long long)c * PW + j]) : tzero<T>();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TT * TT; e += 256) {
    int rr = e / TT, cc = e % TT;
    int r = c0 + TT * I + rr, c = c0 + TT * J + cc;
    if (r < n && c < n && c <= r) {
      T s = tzero<T>();
#pragma unroll 8
      for (int j = 0; j < PW; ++j) {
        s = mad(Vr[rr][j], Wc[cc][j], s);
        s = mad(Wr[rr][j], Vc[cc][j], s);
      }
      long long idx = (long long)r * n + c;
      A[idx] = A[idx] - s;
    }
  }
}

// last diagonal entry once every panel is applied
template <class T>
__global__ void k_tri_last(const BlockDesc* D, char* ws, const int* info, int nblk, int dsel, int bufA, int bufD) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk || info[b]) return;
  const BlockDesc& d = D[b];
  const int n = seldim(d, dsel);
  const T* A = bufp<T>(ws, d, bufA);
  bufp<double>(ws, d, bufD)[n - 1] = re(A[(long long)(n - 1) * n + (n - 1)]);
}

// ---------------------------------------------------------------- blocked Q
// Panels of ORB reflectors H_k0 ... H_{k0+ORB-1} = I - V Tf V^H (forward,
// columnwise compact WY form).  k_larft builds the ORB x ORB upper
// triangular factor Tf of every panel:  Tf_ii = tau_i,
// Tf[0:i, i] = -tau_i Tf[0:i, 0:i] (V[:, 0:i]^H v_i).
constexpr int ORB = 32;

template <class T>
__global__ void __launch_bounds__(256) k_larft(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                               int bufTau, int bufTf) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int nr = seldim(d, dsel);
  const int k0 = blockIdx.x * ORB;
  if (k0 >= nr - 1) return;
  const int kb = min(ORB, nr - 1 - k0);
  const T* A = bufp<T>(ws, d, bufA);
  const T* taus = bufp<T>(ws, d, bufTau);
  T* Tf = bufp<T>(ws, d, bufTf) + (long long)blockIdx.x * ORB * ORB;
  constexpr int LR = Tiles<T>::LR;
  static_assert(LR >= ORB, "the T factor reuses the row-chunk buffer");
  __shared__ T Vs[LR][ORB + 1];
  __shared__ T G[ORB][ORB + 1];
  T (*Ts)[ORB + 1] = Vs;            // after the Gram matrix is complete
  // Gram matrix of the panel (strict upper part): thread t owns pairs
  // p = t and t + 256 of the ORB (ORB - 1) / 2 pairs a < c, numbered
  // column by column.  Row chunks of LR: the next chunk is loaded into
  // registers while the current one is reduced.
  constexpr int PER = LR * ORB / 256, NP = ORB * (ORB - 1) / 2;
  static_assert(NP <= 512, "two pairs per thread");
  T acc[2];
  int pa[2], pc[2];
  for (int q = 0; q < 2; ++q) {
    acc[q] = tzero<T>();
    const int p = min((int)threadIdx.x + 256 * q, NP - 1);
    int c = (int)((1.0 + sqrt(1.0 + 8.0 * p)) * 0.5);
    while (c * (c - 1) / 2 > p) --c;
    while ((c + 1) * c / 2 <= p) ++c;
    pa[q] = p - c * (c - 1) / 2;
    pc[q] = c;
  }
  T nv[PER];
  auto fetch = [&](int r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int l = threadIdx.x + 256 * q, rr = l / ORB, a = l % ORB, r = r0 + rr;
      nv[q] = (r < nr && a < kb) ? panel_v(A, nr, k0, r, a) : tzero<T>();
    }
  };
  fetch(k0 + 1);
  for (int r0 = k0 + 1; r0 < nr; r0 += LR) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int l = threadIdx.x + 256 * q;
      Vs[l / ORB][l % ORB] = nv[q];
    }
    __syncthreads();
    if (r0 + LR < nr) fetch(r0 + LR);
    for (int q = 0; q < 2; ++q) {
      if ((int)threadIdx.x + 256 * q < NP) {
        const int a = pa[q], c = pc[q];
        T s = acc[q];
        for (int rr = 0; rr < LR; ++rr) s = mad(conjg(Vs[rr][a]), Vs[rr][c], s);
        acc[q] = s;
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < 2; ++q)
    if ((int)threadIdx.x + 256 * q < NP) G[pa[q]][pc[q]] = acc[q];
  for (int l = threadIdx.x; l < ORB * ORB; l += 256) Ts[l / ORB][l % ORB] = tzero<T>();
  __syncthreads();
  if (threadIdx.x == 0) Ts[0][0] = taus[k0];
  __syncthreads();
  for (int i = 1; i < kb; ++i) {
    const T ti = taus[k0 + i];
    T z = tzero<T>();
    const int a = threadIdx.x;
    if (a < i) {
      for (int j = a; j < i; ++j) z = mad(Ts[a][j], G[j][i], z);
    }
    __syncthreads();
    if (a < i) Ts[a][i] = -(ti * z);
    if (a == i) Ts[i][i] = ti;
    __syncthreads();
  }
  for (int l = threadIdx.x; l < ORB * ORB; l += 256) Tf[l] = Ts[l / ORB][l % ORB];
}

// Y <- Q Y = P_0 (P_1 (... P_last Y)), P_j = I - V_j Tf_j V_j^H.  Work-group:
// CW columns of Y, all panels, 256 threads as (column c, group g of 256/CW).
template <class T>
__global__ void __launch_bounds__(256) k_ormtr_blocked(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                       int bufA, int bufTf, int bufY, int csel) {
  constexpr int CW = Tiles<T>::CW, VR = Tiles<T>::VR, G = 256 / CW, NA = ORB / G;
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int nr = seldim(d, dsel);
  const int nc = seldim(d, csel);
  const int c0 = blockIdx.x * CW;
  if (c0 >= nc || nr < 2) return;
  const T* A = bufp<T>(ws, d, bufA);
  const T* Tfb = bufp<T>(ws, d, bufTf);
  T* Y = bufp<T>(ws, d, bufY);
  __shared__ T Vs[VR][ORB + 1];
  __shared__ T Xs[ORB * CW];        // Y chunk (VR x CW) or W (ORB x CW)
  __shared__ T Ts[ORB][ORB + 1];
  const int cl = threadIdx.x % CW, g = threadIdx.x / CW;
  const int c = c0 + cl;
  const bool cok = c < nc;
  const int np = (nr - 1 + ORB - 1) / ORB;
  for (int j = np - 1; j >= 0; --j) {
    const int k0 = j * ORB;
    const int kb = min(ORB, nr - 1 - k0);
    const int r0 = k0 + 1;
    for (int l = threadIdx.x; l < ORB * ORB; l += 256) Ts[l / ORB][l % ORB] = Tfb[(long long)j * ORB * ORB + l];
    // W = V^H Y  (thread holds W[a][c] for a = g + G i)
    T w[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) w[i] = tzero<T>();
    for (int rc0 = r0; rc0 < nr; rc0 += VR) {
      __syncthreads();
      for (int l = threadIdx.x; l < VR * ORB; l += 256) {
        int rr = l / ORB, a = l % ORB;
        int r = rc0 + rr;
        Vs[rr][a] = (r < nr && a < kb) ? panel_v(A, nr, k0, r, a) : tzero<T>();
      }
      for (int l = threadIdx.x; l < VR * CW; l += 256) {
        int rr = l / CW, cc = l % CW;
        int r = rc0 + rr;
        Xs[l] = (r < nr && c0 + cc < nc) ? Y[(long long)r * nc + c0 + cc] : tzero<T>();
      }
      __syncthreads();
#pragma unroll 4
      for (int rr = 0; rr < VR; ++rr) {
        T y = Xs[rr * CW + cl];
#pragma unroll
        for (int i = 0; i < NA; ++i) w[i] = mad(conjg(Vs[rr][g + G * i]), y, w[i]);
      }
    }
    __syncthreads();
    // W <- Tf W
#pragma unroll
    for (int i = 0; i < NA; ++i) Xs[(g + G * i) * CW + cl] = w[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      int a = g + G * i;
      T s = tzero<T>();
      for (int bb = a; bb < ORB; ++bb) s = mad(Ts[a][bb], Xs[bb * CW + cl], s);
      w[i] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) Xs[(g + G * i) * CW + cl] = w[i];
    // Y -= V W   (W read from LDS: Xs[a * CW + cl])
    for (int rc0 = r0; rc0 < nr; rc0 += VR) {
      __syncthreads();
      for (int l = threadIdx.x; l < VR * ORB; l += 256) {
        int rr = l / ORB, a = l % ORB;
        int r = rc0 + rr;
        Vs[rr][a] = (r < nr && a < kb) ? panel_v(A, nr, k0, r, a) : tzero<T>();
      }
      __syncthreads();
      if (cok) {
        for (int rr = g; rr < VR; rr += G) {
          int r = rc0 + rr;
          if (r >= nr) break;
          T s = tzero<T>();
#pragma unroll 8
          for (int a = 0; a < ORB; ++a) s = mad(Vs[rr][a], Xs[a * CW + cl], s);
          long long idx = (long long)r * nc + c;
          Y[idx] = Y[idx] - s;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- quaternion Q on the matrix cores
// Y <- Q Y for quaternion Y (nr x nc) with the same panels and Tf factors, the
// three products of each panel (W = V^H Y, W <- Tf W, Y -= V W) done as real
// products on v_mfma_f64_16x16x4f64.  A quaternion q = q0 + q1 i + q2 j + q3 k
// (components in storage order a.x, a.y, b.x, b.y) acts on the left as the
// real 4 x 4 matrix L(q), L[c][d] = s(c, d) q_{c xor d}; a quaternion matrix
// product is the real product of the L-blocks of the left factor with the
// right factor's entries as 4-vectors, and L(conj q) = L(q)^T.
// Work-group: 64 columns of Y, wave w owns columns 16 w .. 16 w + 15.  W stays
// in registers: the MFMA result layout (row l/16 + 4 i, column l % 16) holds
// component l/16 of W[a][col] for a = 4 b + i, which is exactly the operand
// layout the next two products read.
__device__ constexpr signed char QSGN[4][4] = {{1, -1, -1, -1}, {1, 1, -1, 1}, {1, 1, 1, -1}, {1, -1, 1, 1}};
typedef __attribute__((ext_vector_type(4))) double qd4;

__global__ void __launch_bounds__(256) k_ormtr_q_mfma(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                      int bufA, int bufTf, int bufY, int csel) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int nr = seldim(d, dsel);
  const int nc = seldim(d, csel);
  const int c0 = blockIdx.x * 64;
  if (c0 >= nc || nr < 2) return;
  const quat* A = bufp<quat>(ws, d, bufA);
  const quat* Tfb = bufp<quat>(ws, d, bufTf);
  double* Y = reinterpret_cast<double*>(bufp<quat>(ws, d, bufY));
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int l16 = lane & 15, l4 = lane >> 4;     // MFMA row / column index and k index
  const int col = c0 + 16 * wave + l16;           // this lane's Y column (B operand, result)
  const bool cok = col < nc;
  constexpr int VRQ = 32;                         // V panel rows per LDS chunk
  // per lane: A-operand row l16 = (quaternion l16 / 4, component c = l16 % 4),
  // k index d = l4; L(q)[c][d] = s(c, d) q_{c xor d}
  const int aq = l16 >> 2, cq = l16 & 3, ix = cq ^ l4;
  const double sgn1 = QSGN[l4][cq], sgn2 = QSGN[cq][l4];
  __shared__ quat Vs[VRQ][ORB + 1];
  __shared__ quat Ts[ORB][ORB + 1];
  const int np = (nr - 1 + ORB - 1) / ORB;
  for (int j = np - 1; j >= 0; --j) {
    const int k0 = j * ORB;
    const int kb = min(ORB, nr - 1 - k0);
    const int r0 = k0 + 1;
    __syncthreads();
    for (int l = t; l < ORB * ORB; l += 256) Ts[l / ORB][l % ORB] = Tfb[(long long)j * ORB * ORB + l];
    // ---- W_real (128 x 16 per wave) = L(V)^T Y_real over the panel rows
    qd4 w[8];
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) w[ob] = qd4{0.0, 0.0, 0.0, 0.0};
    for (int rc = r0; rc < nr; rc += VRQ) {
      const int rend = min(VRQ, nr - rc);
      double ybuf[VRQ];                     // B operands of the chunk: component l4 of Y[r][col]
#pragma unroll
      for (int rr = 0; rr < VRQ; ++rr)      // in flight while the panel rows are staged
        ybuf[rr] = (cok && rr < rend) ? Y[((long long)(rc + rr) * nc + col) * 4 + l4] : 0.0;
      quat vpre[VRQ * ORB / 256];           // the chunk's panel rows, loaded before the barrier
#pragma unroll
      for (int q = 0; q < VRQ * ORB / 256; ++q) {
        const int l = t + 256 * q, rr = l / ORB, a = l % ORB, r = rc + rr;
        vpre[q] = (r < nr && a < kb) ? panel_v(A, nr, k0, r, a) : tzero<quat>();
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < VRQ * ORB / 256; ++q) {
        const int l = t + 256 * q;
        Vs[l / ORB][l % ORB] = vpre[q];
      }
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < VRQ; ++rr) {
        const double y = ybuf[rr];
        const double* vrow = reinterpret_cast<const double*>(&Vs[rr][0]);
#pragma unroll
        for (int ob = 0; ob < 8; ++ob) {
          // A row l16 -> quaternion a = 4 ob + l16/4, component c = l16 % 4; k = d = l4:
          // L(V)^T[c][d] = L(V)[d][c] = s(d, c) V_{c xor d}
          const double av = sgn1 * vrow[4 * (4 * ob + aq) + ix];
          w[ob] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, y, w[ob], 0, 0, 0);
        }
      }
    }
    // ---- W <- Tf W  (Tf upper triangular: only b >= a contributes)
    qd4 w2[8];
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
      w2[ob] = qd4{0.0, 0.0, 0.0, 0.0};
      const double* trow = reinterpret_cast<const double*>(&Ts[4 * ob + aq][0]);
#pragma unroll
      for (int bq = 0; bq < ORB; ++bq) {
        if (bq >= 4 * ob) {
          const double av = sgn2 * trow[4 * bq + ix];                          // L(Tf[a][b])[c][d]
          const double bv = w[bq >> 2][bq & 3];                                 // component l4 of W[b][col]
          w2[ob] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, w2[ob], 0, 0, 0);
        }
      }
    }
    // ---- Y -= L(V) W, four quaternion rows per MFMA block
    for (int rc = r0; rc < nr; rc += VRQ) {
      const int rend = min(VRQ, nr - rc);
      double yv[VRQ];                       // this lane's entries of the chunk, loaded before the products
#pragma unroll
      for (int rr = 0; rr < VRQ; ++rr)
        yv[rr] = (cok && rr < rend) ? Y[((long long)(rc + rr) * nc + col) * 4 + l4] : 0.0;
      quat vpre[VRQ * ORB / 256];           // the chunk's panel rows, loaded before the barrier
#pragma unroll
      for (int q = 0; q < VRQ * ORB / 256; ++q) {
        const int l = t + 256 * q, rr = l / ORB, a = l % ORB, r = rc + rr;
        vpre[q] = (r < nr && a < kb) ? panel_v(A, nr, k0, r, a) : tzero<quat>();
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < VRQ * ORB / 256; ++q) {
        const int l = t + 256 * q;
        Vs[l / ORB][l % ORB] = vpre[q];
      }
      __syncthreads();
#pragma unroll
      for (int rb = 0; rb < VRQ; rb += 4) {
        if (rb >= rend) break;
        qd4 acc = qd4{0.0, 0.0, 0.0, 0.0};
        const double* vrow = reinterpret_cast<const double*>(&Vs[rb + aq][0]);   // quaternion row rb + l16/4
#pragma unroll
        for (int a = 0; a < ORB; ++a) {
          const double av = sgn2 * vrow[4 * a + ix];                            // L(V[r][a])[c][d]
          const double bv = w2[a >> 2][a & 3];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        // result: row l4 + 4 i = (quaternion row rb + i, component l4), column l16
        if (cok) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = rc + rb + i;
            if (rb + i < rend) Y[((long long)r * nc + col) * 4 + l4] = yv[rb + i] - acc[i];
          }
        }
      }
    }
  }
}

template <class T>
void launch_hetrd(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                  int bufA, int bufD, int bufE, int bufTau) {
  size_t shm = 4 * (size_t)maxdim * sizeof(T);
  hipLaunchKernelGGL(k_hetrd<T>, dim3(nblk), dim3(1024), shm, s, D, ws, info, dsel, bufA, bufD, bufE, bufTau);
}

// ---------------------------------------------------------------- quaternion rank-2k update on the matrix cores
// Trailing lower triangle A -= V W^H + W V^H = [V W] [W V]^H for quaternion
// matrices: a product with contraction length 2 PW over 64 x 64 tiles on or
// below the diagonal, operands staged per k chunk of 16 as four component
// planes, 16 MFMAs (one per pair of components, signs of the quaternion
// product) per 16 x 16 block and k step of 4.  grid = (lower tiles, nblk).
constexpr int HQ_T = 64, HQ_K = 16;

__global__ void __launch_bounds__(256, 2) k_tri_her2k_q_mfma(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                          int bufA, int bufW, int k0) {
  constexpr int PW = panel_width<quat>();
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  if (k0 >= n - 1 || k0 >= tri_tail_start<quat>(n)) return;
  const int kb = min(PW, n - 1 - k0);
  const int c0 = k0 + kb;
  const int len = n - c0;
  if (len <= 0) return;
  const int nt = (len + HQ_T - 1) / HQ_T;
  const int t = blockIdx.x;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  quat* A = bufp<quat>(ws, d, bufA);
  const quat* Wp = bufp<quat>(ws, d, bufW);
  const int m0 = c0 + HQ_T * I, n0 = c0 + HQ_T * J;
  __shared__ double As[4][HQ_T][HQ_K + 1];   // [component][row][k]
  __shared__ double Bs[4][HQ_K][HQ_T + 1];   // [component][k][col]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;
  qd4 acc[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[x][y][c] = qd4{0.0, 0.0, 0.0, 0.0};
  // column j of [V W] (wfirst = 0) or [W V] (wfirst = 1) at row `row`; zero
  // beyond the matrix and for panel columns >= kb
  auto opval = [&](int row, int j, int wfirst) -> quat {
    const int half = j >= PW, a = j - PW * half;
    if (row >= n || a >= kb) return tzero<quat>();
    return (half != wfirst) ? Wp[(long long)row * PW + a] : panel_v(A, n, k0, row, a);
  };
  constexpr int NL = HQ_T * HQ_K / 256;
  quat na[NL], nb[NL];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = tid + 256 * q, r = l / HQ_K, kk = l % HQ_K;
      na[q] = opval(m0 + r, kc + kk, 0);
      nb[q] = conjg(opval(n0 + r, kc + kk, 1));
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int l = tid + 256 * q, r = l / HQ_K, kk = l % HQ_K;
      As[0][r][kk] = na[q].a.x;
      As[1][r][kk] = na[q].a.y;
      As[2][r][kk] = na[q].b.x;
      As[3][r][kk] = na[q].b.y;
      Bs[0][kk][r] = nb[q].a.x;
      Bs[1][kk][r] = nb[q].a.y;
      Bs[2][kk][r] = nb[q].b.x;
      Bs[3][kk][r] = nb[q].b.y;
    }
  };
  for (int kc = 0; kc < 2 * PW; kc += HQ_K) {
    // two waves per SIMD instead of a register prefetch (the loads go out
    // before the barrier)
    fetch(kc);
    __syncthreads();
    stash();
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < HQ_K; ks += 4) {
      double a[2][4], bq[2][4];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          a[x][c] = As[c][wr + 16 * x + l16][ks + l4];
          bq[x][c] = Bs[c][ks + l4][wc + 16 * x + l16];
        }
#pragma unroll
      for (int dd = 0; dd < 4; ++dd)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (!(I == J && wc + 16 * y > wr + 16 * x))   // 16 x 16 blocks above the diagonal are not written
#pragma unroll
              for (int c = 0; c < 4; ++c)
                acc[x][y][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    qmul_sign(c, dd) > 0 ? a[x][c ^ dd] : -a[x][c ^ dd], bq[y][dd], acc[x][y][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = m0 + wr + 16 * x + l4 + 4 * i, c = n0 + wc + 16 * y + l16;
        if (r >= n || c > r) continue;
        const long long idx = (long long)r * n + c;
        const quat u = {{acc[x][y][0][i], acc[x][y][1][i]}, {acc[x][y][2][i], acc[x][y][3][i]}};
        A[idx] = A[idx] - u;
      }
}

// ---------------------------------------------------------------- unblocked quaternion tail
// Columns tri_tail_start(n) .. n - 2 of a quaternion reduction by one
// work-group per block.  The trailing matrix (m = n - tri_tail_start(n) <=
// TAIL_MAX + 1 rows, current after the last panel's rank-2k update) is read
// once into LDS as a column-major packed lower triangle and reduced there
// one Householder step at a time: H A H = A - v w^H - w v^H with
// w = tau A v - (tau / 2)(v^H tau A v) v.  The outputs are those of the
// blocked steps: the reflector (below the sub-diagonal of A's column k), tau,
// the real diagonal (also written back to A's diagonal), the quaternion
// sub-diagonal and its modulus.  Row i of the matvec: four threads, columns
// j = q, q + 4, ... (the upper part as conjugates of the lower).
constexpr int TAIL_LDS = (TAIL_MAX + 1) * (TAIL_MAX + 2) / 2;   // packed lower triangle

__global__ void __launch_bounds__(COLT) k_tri_tail_q(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                     int bufA, int bufD, int bufE, int bufTau, int bufET) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int kt = tri_tail_start<quat>(n);
  if (kt > n - 2) return;
  const int m = n - kt;
  quat* A = bufp<quat>(ws, d, bufA);
  double* dd = bufp<double>(ws, d, bufD);
  double* ee = bufp<double>(ws, d, bufE);
  quat* taus = bufp<quat>(ws, d, bufTau);
  quat* et = bufp<quat>(ws, d, bufET);
  const int tid = threadIdx.x;
  __shared__ quat L[TAIL_LDS];
  __shared__ quat v[TAIL_MAX + 1], w[TAIL_MAX + 1];
  __shared__ double red[32];
  __shared__ quat sh_tau, sh_betaq;
  // element (i, j), i >= j, of the trailing matrix
  auto at = [m](int i, int j) { return j * m - j * (j - 1) / 2 + (i - j); };
  for (int e = tid; e < m * m; e += COLT) {            // rows of A: coalesced
    const int i = e / m, j = e - (e / m) * m;
    if (j > i) continue;
    const quat a = A[(long long)(kt + i) * n + kt + j];
    L[at(i, j)] = i == j ? treal<quat>(re(a)) : a;
  }
  __syncthreads();
  for (int c = 0; c <= m - 2; ++c) {
    const int k = kt + c, len = m - c - 1;
    make_reflector_q(A, n, k, v, &sh_tau, &sh_betaq, red, &L[at(c + 1, c)]);   // ends with a barrier
    const quat tau = sh_tau;
    if (tid == 0) {
      const quat dg = L[at(c, c)];
      A[(long long)k * n + k] = dg;
      dd[k] = re(dg);
      taus[k] = tau;
      ee[k] = sqrt(abs2(sh_betaq));
      et[k] = sh_betaq;
    }
    // w = tau A22 v
    for (int r = tid / CTPR; r < len; r += COLT / CTPR) {   // the same r for the CTPR lanes of a group
      const int q = tid % CTPR, i = c + 1 + r;
      quat acc = tzero<quat>();
      for (int t = q; t < len; t += CTPR) {
        const int j = c + 1 + t;
        const quat a = j <= i ? L[at(i, j)] : conjg(L[at(j, i)]);
        acc = mad(a, v[t], acc);
      }
      acc = group_allsum<CTPR>(acc);
      if (q == 0) w[r] = tau * acc;
    }
    __syncthreads();
    double dr = 0.0;
    for (int r = tid; r < len; r += COLT) dr += re(conjg(w[r]) * v[r]);
    dr = block_sum(dr, red);
    const double alpha = -0.5 * re(tau) * dr;                 // y^H v is real
    for (int r = tid; r < len; r += COLT) w[r] = w[r] + alpha * v[r];
    __syncthreads();
    // A22 -= v w^H + w v^H on and below the diagonal (diagonal kept real)
    for (int e = tid; e < len * len; e += COLT) {
      const int r = e / len, t = e - (e / len) * len;
      if (t > r) continue;
      const int idx = at(c + 1 + r, c + 1 + t);
      quat a = L[idx] - v[r] * conjg(w[t]) - w[r] * conjg(v[t]);
      if (r == t) a = treal<quat>(re(a));
      L[idx] = a;
    }
    __syncthreads();
  }
  if (tid == 0) A[(long long)(n - 1) * n + n - 1] = L[at(m - 1, m - 1)];   // read by k_tri_last
}

// Blocked multi-kernel reduction over the batch; falls back to the
// one-work-group reduction when every real or complex block is small.  The
// quaternion reductions run their panels up to tri_tail_start and finish in
// k_tri_tail_q.
template <class T>
void launch_hetrd_mk(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                     int bufA, int bufD, int bufE, int bufTau, int bufW, int bufV, int bufHS, int bufET,
                     int mv_res) {
  constexpr int ST = 2 * Tiles<T>::HT, TT = Tiles<T>::TT, PW = panel_width<T>();   // ST: the smallest edge
  if constexpr (!is_quat<T>()) {
    if (maxdim <= 96) {
      launch_hetrd<T>(s, D, ws, info, nblk, maxdim, dsel, bufA, bufD, bufE, bufTau);
      return;
    }
  }
  // v, y, colacc, acol and the panel dot partials of the column kernel
  const size_t shm = (4 * (size_t)maxdim + (size_t)((maxdim + 3 + ST - 1) / ST) * PW * 2) * sizeof(T);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tri_col<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  // the blocked panels up to the largest block's tail (smaller blocks stop
  // at their own)
  const int kend = std::min(maxdim - 1, tri_tail_start<T>(maxdim));
  for (int k0 = 0; k0 < kend; k0 += PW) {
    const int kbmax = std::min(PW, maxdim - 1 - k0);
    hipLaunchKernelGGL(k_tri_col<T>, dim3(nblk), dim3(COLT), shm, s, D, ws, info, dsel, bufA, bufD, bufE, bufTau, bufW,
                       bufV, bufHS, bufET, k0, 0, 0);
    for (int i = 0; i < kbmax; ++i) {
      const int k = k0 + i;
      const int len = maxdim - k - 1 + mv_lead<T>(k);
      // items per block: the most any block can have at this step (a
      // quaternion block takes its super-tile edge from its own length)
      auto items = [](int l, int e) { const int ns = (l + e - 1) / e; return ns * (ns + 1) / 2; };
      const int nsmax = !is_quat<T>() ? items(len, ST)
                        : std::max(items(len, mv_st_q(len)), items(std::min(len, MV_ST64_LEN), ST));
      hipEvent_t ev0, ev1;
      void* kt = ktrace_begin("k_tri_matvec", &ev0, &ev1);
      launch_matvec<T>(s, D, ws, info, nblk, dsel, bufA, bufV, bufHS, bufW, k0, k, nsmax, ncu, mv_res, ev0, ev1);
      ktrace_end(kt);
      hipLaunchKernelGGL(k_tri_col<T>, dim3(nblk), dim3(COLT), shm, s, D, ws, info, dsel, bufA, bufD, bufE, bufTau,
                         bufW, bufV, bufHS, bufET, k0, i + 1, (i + 1 < kbmax) ? 1 : 2);
    }
    const int len2 = maxdim - (k0 + kbmax);
    if (len2 > 0) {
      if constexpr (is_quat<T>()) {
        const int nt2 = (len2 + HQ_T - 1) / HQ_T;
        hipLaunchKernelGGL(k_tri_her2k_q_mfma, dim3(nt2 * (nt2 + 1) / 2, nblk), dim3(256), 0, s, D, ws, info, dsel,
                           bufA, bufW, k0);
      } else {
        const int nt2 = (len2 + TT - 1) / TT;
        hipLaunchKernelGGL(k_tri_her2k<T>, dim3(nt2 * (nt2 + 1) / 2, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA,
                           bufW, k0);
      }
    }
  }
  if constexpr (is_quat<T>())
    hipLaunchKernelGGL(k_tri_tail_q, dim3(nblk), dim3(COLT), 0, s, D, ws, info, dsel, bufA, bufD, bufE, bufTau,
                       bufET);
  hipLaunchKernelGGL(k_tri_last<T>, dim3((nblk + 255) / 256), dim3(256), 0, s, D, ws, info, nblk, dsel, bufA, bufD);
}
template void launch_hetrd_mk<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                      int, int, int, int, int, int);
template void launch_hetrd_mk<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                    int, int, int, int, int, int);
template void launch_hetrd_mk<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                    int, int, int, int, int, int);

template <class T>
void launch_ormtr_blocked(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim,
                          int maxcols, int dsel, int bufA, int bufTau, int bufTf, int bufY, int csel) {
  int np = (maxdim - 1 + ORB - 1) / ORB;
  if (np < 1) np = 1;
  hipLaunchKernelGGL(k_larft<T>, dim3(np, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA, bufTau, bufTf);
  if constexpr (is_quat<T>()) {
    hipLaunchKernelGGL(k_ormtr_q_mfma, dim3((maxcols + 63) / 64, nblk), dim3(256), 0, s, D, ws, info, dsel, bufA,
                       bufTf, bufY, csel);
  } else {
    constexpr int CW = Tiles<T>::CW;
    hipLaunchKernelGGL(k_ormtr_blocked<T>, dim3((maxcols + CW - 1) / CW, nblk), dim3(256), 0, s, D, ws, info, dsel,
                       bufA, bufTf, bufY, csel);
  }
}
template void launch_ormtr_blocked<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                           int, int, int, int);
template void launch_ormtr_blocked<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                         int, int, int, int);
template void launch_ormtr_blocked<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                         int, int, int, int);
template void launch_hetrd<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                   int);
template void launch_hetrd<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int, int);

}  // namespace x2c
