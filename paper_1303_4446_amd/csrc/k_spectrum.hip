// Spectrum of the tridiagonal matrices and the matrix functions taken on it.
//
// (1) Positive-energy branch of the reduced 4c matrix (Sec. II: eigenvalues
//     with eps + c^2 > 0).  Sturm-sequence counts give the branch size (it
//     must equal n) and, by bisection, the n positive-energy eigenvalues.
// (2) Positive-energy invariant subspace.  X = C_S C_L^-1 (Appendix,
//     Eq. defxmat) depends only on the span of the positive-energy
//     eigenvectors, so instead of individual eigenvectors (ill-determined
//     inside the exactly degenerate Kramers and m_j multiplets) the kernel
//     applies the spectral projector P = (I + sign(T - sigma))/2, sigma = -c^2,
//     to a fixed block of n vectors.  sign() is Zolotarev's best rational
//     approximation on [-1,-l] U [l,1] (coefficients from Jacobi elliptic
//     functions, computed with the arithmetic-geometric mean), evaluated on
//     the tridiagonal by complex shifted tridiagonal solves.
// (3) Inverse square root of the renormalisation matrix (Sec. III:
//     A^-1/2 = C a^-1/2 C^H).  Evaluated as
//     x^-1/2 = (2/pi) int_0^{pi/2} dphi / (x cos^2 phi + sin^2 phi) with the
//     (exponentially convergent, periodic) midpoint rule, i.e. a sum of
//     shifted SPD tridiagonal inverses, again without eigenvectors.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

// 1/q from the hardware reciprocal estimate refined by two Newton steps
// (error a few ulp; |q| >= pivmin keeps it finite)
__device__ inline double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// number of eigenvalues of tridiag(d, e) below x (e2 = e^2)
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Eigenvalues idx0 + k (k < ne, ascending indices) of tridiag(d, e) by
// multisection over the work-group: the threads form groups of
// P = min(blockDim / ne, pmax) (at least 1); each group splits its
// eigenvalue's bracket into P + 1 parts per step with one Sturm count per
// thread.  cbuf / xbuf: blockDim ints / doubles of LDS.  Every thread must
// call it.
__device__ void multisect(const double* d, const double* e2, int m, int idx0, int ne, double lo, double hi,
                          double piv, double* out, int* cbuf, double* xbuf, int pmax = 1 << 30) {
  const int P = max(1, min((int)blockDim.x / max(ne, 1), pmax));
  const int G = blockDim.x / P;
  const int grp = threadIdx.x / P, p = threadIdx.x - grp * P;
  for (int base = 0; base < ne; base += G) {
    const int k = base + grp;
    const bool act = grp < G && k < ne;
    const int idx = idx0 + k;
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      // converged once the bracket is relatively tight or cannot be split
      const double mid = 0.5 * (a + b);
      const bool live = act && mid > a && mid < b && (b - a > 2.2e-16 * fmax(fabs(a), fabs(b)));
      const double x = a + (b - a) * ((double)(p + 1) / (double)(P + 1));
      cbuf[threadIdx.x] = live ? sturm_count(d, e2, m, x, piv) : 0;
      xbuf[threadIdx.x] = x;
      __syncthreads();
      if (live) {
        double na = a, nb = b;
        for (int q = 0; q < P; ++q) {
          if (cbuf[grp * P + q] > idx) {
            nb = xbuf[grp * P + q];
            break;
          }
          na = xbuf[grp * P + q];
        }
        a = na;
        b = nb;
      }
      if (!__syncthreads_or(live)) break;
    }
    if (act && p == 0) out[k] = 0.5 * (a + b);
    __syncthreads();
  }
}

// Gershgorin bounds of tridiag(d, e); block-wide
__device__ inline void gershgorin(const double* d, const double* e, int n, double* lo, double* hi, double* red) {
  double l = 1e300, h = -1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    l = fmin(l, d[i] - r);
    h = fmax(h, d[i] + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_xor(l, o, 64));
    h = fmax(h, __shfl_xor(h, o, 64));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = l;
    red[16 + (threadIdx.x >> 6)] = h;
  }
  __syncthreads();
  l = 1e300; h = -1e300;
  for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) {
    l = fmin(l, red[i]);
    h = fmax(h, red[16 + i]);
  }
  __syncthreads();
  // widen slightly so bisection brackets every eigenvalue
  double span = fmax(h - l, fmax(fabs(l), fabs(h))) * 4e-16 + 1e-300;
  *lo = l - span;
  *hi = h + span;
}

// ---------------------------------------------------------------- Zolotarev
// Jacobi sn, cn of real argument u, modulus k, via the descending Landen
// (arithmetic-geometric mean) sequence a_0 = 1, b_0 = k' , c_0 = k.
struct AGMSeq {
  double a[48], c[48];
  int N;
};
__device__ inline void agm_seq(double kc, double k, AGMSeq& s) {
  double a = 1.0, b = kc, c = k;
  s.a[0] = a; s.c[0] = c;
  int i = 0;
  while (i < 46 && fabs(c) > 1e-17) {
    double an = 0.5 * (a + b);
    c = 0.5 * (a - b);
    b = sqrt(a * b);
    a = an;
    ++i;
    s.a[i] = a; s.c[i] = c;
  }
  s.N = i;
}
__device__ inline void ellip_sn_cn(double u, const AGMSeq& s, double* sn, double* cn) {
  double phi = ldexp(s.a[s.N] * u, s.N);
  for (int i = s.N; i > 0; --i) phi = 0.5 * (phi + asin(s.c[i] / s.a[i] * sin(phi)));
  *sn = sin(phi);
  *cn = cos(phi);
}

// best type (2r+1, 2r) rational approximation of sign on [-1,-l] U [l,1]:
// Z(x) = M x (1 + sum_j a_j / (x^2 + codd_j)); returns the max error.
__device__ double zolotarev(double ell, int r, double* a, double* codd, double* Mout) {
  double cvals[2 * RMAX];
  AGMSeq s;
  const double kp = sqrt((1.0 - ell) * (1.0 + ell));
  agm_seq(ell, kp, s);                                   // modulus kp, complementary ell
  const double Kp = 3.14159265358979323846 / (2.0 * s.a[s.N]);   // K(kp)
  for (int i = 1; i <= 2 * r; ++i) {
    double sn, cn;
    ellip_sn_cn(i * Kp / (2 * r + 1), s, &sn, &cn);
    cvals[i - 1] = ell * ell * sn * sn / (cn * cn);
  }
  for (int j = 0; j < r; ++j) codd[j] = cvals[2 * j];
  for (int j = 0; j < r; ++j) {
    double num = 1.0, den = 1.0;
    for (int k = 0; k < r; ++k) {
      num *= cvals[2 * k + 1] - codd[j];
      if (k != j) den *= codd[k] - codd[j];
    }
    a[j] = num / den;
  }
  auto zhat = [&](double x) {
    double s2 = 1.0;
    for (int j = 0; j < r; ++j) s2 += a[j] / (x * x + codd[j]);
    return x * s2;
  };
  double zl = zhat(ell), z1 = zhat(1.0);
  double M = 2.0 / (zl + z1);
  *Mout = M;
  return fabs(M * z1 - 1.0);
}

// ---------------------------------------------------------------- 4c branch
// Tridiagonal in LDS (d, e, e^2), its Gershgorin interval and the pivot
// floor of the Sturm counts; block-wide, every thread gets the values.
__device__ void tri_setup(const double* dg, const double* eg, int m, double* sd, double* se, double* se2,
                          double* red, double* lo_out, double* hi_out, double* piv_out) {
  __shared__ double s_lo, s_hi, s_piv;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    sd[i] = dg[i];
    if (i < m - 1) {
      se[i] = eg[i];
      se2[i] = eg[i] * eg[i];
    }
  }
  __syncthreads();
  double lo, hi;
  gershgorin(sd, se, m, &lo, &hi, red);
  double emax = 0.0;
  for (int i = threadIdx.x; i < m - 1; i += blockDim.x) emax = fmax(emax, se2[i]);
  for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
  if ((threadIdx.x & 63) == 0) red[32 + (threadIdx.x >> 6)] = emax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) e = fmax(e, red[32 + i]);
    s_piv = 2.2e-308 * fmax(1.0, e) * 16.0;
    s_lo = lo;
    s_hi = hi;
  }
  __syncthreads();
  *lo_out = s_lo;
  *hi_out = s_hi;
  *piv_out = s_piv;
}

// One work-group per block: the branch-size check (info 4), the two
// eigenvalues next to sigma = -c^2 (lambda_{n-1} < sigma < lambda_n) and the
// projector filter parameters.  Zolotarev candidates r = 4, 6, ..., RMAX:
// their 2r elliptic-function values, then their r coefficients, are spread
// over all threads; the smallest r that reaches 1e-13 (or stops improving)
// is kept.  kramers = 1: the tridiagonal is the real form of the quaternion
// reduced matrix (dimension n, one eigenvalue per Kramers pair).
__global__ void __launch_bounds__(1024) k_tri_eig4c(const BlockDesc* D, char* ws, int* info, double c, int kramers) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int m = kramers ? d.n : d.m, n = kramers ? d.n / 2 : d.n;
  double* pf = bufp<double>(ws, d, P_FILT);
  extern __shared__ char smem[];
  double* sd = reinterpret_cast<double*>(smem);
  double* se = sd + m;
  double* se2 = se + m;
  __shared__ double red[64];
  __shared__ double lam[2];
  __shared__ int s_cnt;
  double lo, hi, piv;
  tri_setup(bufp<double>(ws, d, V_D), bufp<double>(ws, d, V_E), m, sd, se, se2, red, &lo, &hi, &piv);
  if (threadIdx.x == 0) s_cnt = sturm_count(sd, se2, m, -c * c, piv);
  __syncthreads();
  if (s_cnt != m - n) {
    if (threadIdx.x == 0) info[b] = 4;
    return;
  }
  __shared__ int cbuf[1024];
  __shared__ double xbuf[1024];
  // 16 counts per eigenvalue and step: a few more steps, far fewer counts
  multisect(sd, se2, m, n - 1, 2, lo, hi, piv, lam, cbuf, xbuf, 16);
  constexpr int NCAND = (RMAX - 4) / 2 + 1;
  // largest accepted sign-approximation error: a leak of relative size e
  // from the other branch moves X by about e kappa(Y_L), well below the
  // FP64 forward error of the path for e <= 1e-11
  constexpr double ZOL_ERR_MAX = 1e-11;
  constexpr int NCV = 2 * NCAND * (NCAND + 3);   // sum over candidates of 2r
  constexpr int NCO = NCAND * (NCAND + 3);       // sum over candidates of r
  __shared__ double zerr[NCAND], zM[NCAND];
  __shared__ double za[NCAND * RMAX], zc[NCAND * RMAX];
  __shared__ double cv[NCV];
  __shared__ AGMSeq agm;
  const double sigma = -c * c;
  const double gam = fmin(lam[1] - sigma, sigma - lam[0]);
  const double rho = fmax(hi - sigma, sigma - lo);
  double ell = 0.9 * gam / rho;
  ell = fmin(fmax(ell, 1e-14), 0.5);
  // candidate q has r = 4 + 2q; its values start at 2q(q+3), its
  // coefficients at q(q+3)
  if (threadIdx.x == 0) agm_seq(ell, sqrt((1.0 - ell) * (1.0 + ell)), agm);   // modulus kp, complementary ell
  __syncthreads();
  const double Kp = 3.14159265358979323846 / (2.0 * agm.a[agm.N]);             // K(kp)
  for (int f = threadIdx.x; f < NCV; f += blockDim.x) {
    int q = 0;
    while (q + 1 < NCAND && 2 * (q + 1) * (q + 4) <= f) ++q;
    const int r = 4 + 2 * q, i = f - 2 * q * (q + 3) + 1;    // i = 1 .. 2r
    double sn, cn;
    ellip_sn_cn(i * Kp / (2 * r + 1), agm, &sn, &cn);
    cv[f] = ell * ell * sn * sn / (cn * cn);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < NCO; g += blockDim.x) {
    int q = 0;
    while (q + 1 < NCAND && (q + 1) * (q + 4) <= g) ++q;
    const int r = 4 + 2 * q, j = g - q * (q + 3);
    const double* cq = cv + 2 * q * (q + 3);
    const double cj = cq[2 * j];
    double num = 1.0, den = 1.0;
    for (int k = 0; k < r; ++k) {
      num *= cq[2 * k + 1] - cj;
      if (k != j) den *= cq[2 * k] - cj;
    }
    za[q * RMAX + j] = num / den;
    zc[q * RMAX + j] = cj;
  }
  __syncthreads();
  if (threadIdx.x < NCAND) {
    const int q = threadIdx.x, r = 4 + 2 * q;
    auto zhat = [&](double x) {
      double s2 = 1.0;
      for (int j = 0; j < r; ++j) s2 += za[q * RMAX + j] / (x * x + zc[q * RMAX + j]);
      return x * s2;
    };
    const double zl = zhat(ell), z1 = zhat(1.0);
    const double M = 2.0 / (zl + z1);
    zM[q] = M;
    zerr[q] = fabs(M * z1 - 1.0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = -1;
    double prev = 1.0;
    for (int t = 0; t < NCAND; ++t) {
      const double err = zerr[t];
      if (best < 0 || err <= prev) best = t;
      if (err < 1e-13 || err > 0.5 * prev) break;
      prev = err;
    }
    // no order reaches the FP64 level: the gap at -c^2 is too narrow relative
    // to the spectral radius for the projector to separate the two branches
    if (!(zerr[best] <= ZOL_ERR_MAX)) info[b] = 3;
    const int rbest = 4 + 2 * best;
    pf[0] = sigma;
    pf[1] = rho;
    pf[2] = zM[best];
    pf[3] = (double)rbest;
    for (int j = 0; j < rbest; ++j) {
      pf[4 + j] = za[best * RMAX + j];
      pf[4 + RMAX + j] = sqrt(zc[best * RMAX + j]);
    }
  }
}

// The n positive-energy eigenvalues (indices n .. 2n-1 of the m = 2n), eps
// ascending, by multisection; grid = (chunks of EPW eigenvalues, blocks).
// kramers = 1: each eigenvalue is written twice (the Kramers pair).
constexpr int EPW = 64;

__global__ void __launch_bounds__(256) k_tri_eps4c(const BlockDesc* D, char* ws, const int* info, double* eps,
                                                   int kramers) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int m = kramers ? d.n : d.m, n = kramers ? d.n / 2 : d.n;
  const int k0 = blockIdx.x * EPW;
  if (k0 >= n) return;
  const int ne = min(EPW, n - k0);
  extern __shared__ char smem[];
  double* sd = reinterpret_cast<double*>(smem);
  double* se = sd + m;
  double* se2 = se + m;
  __shared__ double red[64];
  __shared__ double lam[EPW];
  __shared__ int cbuf[256];
  __shared__ double xbuf[256];
  double lo, hi, piv;
  tri_setup(bufp<double>(ws, d, V_D), bufp<double>(ws, d, V_E), m, sd, se, se2, red, &lo, &hi, &piv);
  multisect(sd, se2, m, n + k0, ne, lo, hi, piv, lam, cbuf, xbuf);
  for (int k = threadIdx.x; k < ne; k += blockDim.x) {
    if (kramers) {
      eps[d.eps_off + 2 * (k0 + k)] = lam[k];
      eps[d.eps_off + 2 * (k0 + k) + 1] = lam[k];
    } else {
      eps[d.eps_off + k0 + k] = lam[k];
    }
  }
}

// LU with partial pivoting of (T_s - i beta_j I), T_s = (T - sigma)/rho, one
// pole per work-group (thread 0).  Factor entry layout (5 complex):
// {dl, 1/du0, du1, du2, (pivot, 0)}.
__global__ void k_filter_factor(const BlockDesc* D, char* ws, const int* info, int kramers) {
  const int b = blockIdx.y, j = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const double* pf = bufp<double>(ws, d, P_FILT);
  const int r = (int)pf[3];
  if (j >= r) return;
  const int m = kramers ? d.n : d.m;
  // the tridiagonal in LDS: the elimination below is one serial chain
  extern __shared__ double ff_sm[];
  double* dg = ff_sm;
  double* eg = ff_sm + m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    dg[i] = bufp<double>(ws, d, V_D)[i];
    eg[i] = i < m - 1 ? bufp<double>(ws, d, V_E)[i] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double sigma = pf[0], rho = pf[1], beta = pf[4 + RMAX + j];
  cplx* F = bufp<cplx>(ws, d, F_FAC) + (long long)j * m * 5;
  const double ir = 1.0 / rho;
  // running diagonal / superdiagonal of the current row (after elimination)
  cplx dcur = {(dg[0] - sigma) * ir, -beta};
  cplx ucur = {m > 1 ? eg[0] * ir : 0.0, 0.0};
  for (int i = 0; i < m - 1; ++i) {
    cplx sub = {eg[i] * ir, 0.0};                  // l_i = A[i+1][i]
    cplx dnext = {(dg[i + 1] - sigma) * ir, -beta};
    cplx unext = {i + 1 < m - 1 ? eg[i + 1] * ir : 0.0, 0.0};
    cplx* f = F + (long long)i * 5;
    if (abs1(dcur) >= abs1(sub)) {
      cplx fact = cdiv(sub, dcur);
      f[0] = fact;
      f[1] = crecip(dcur);
      f[2] = ucur;
      f[3] = {0.0, 0.0};
      f[4] = {0.0, 0.0};
      dcur = dnext - fact * ucur;
      ucur = unext;
    } else {
      // swap rows i and i+1
      cplx fact = cdiv(dcur, sub);
      f[0] = fact;
      f[1] = crecip(sub);
      f[2] = dnext;          // new u1 of row i
      f[3] = unext;          // fill-in u2 of row i
      f[4] = {1.0, 0.0};
      cplx nd = ucur - fact * dnext;
      cplx nu = -(fact * unext);
      dcur = nd;
      ucur = nu;
    }
  }
  cplx* f = F + (long long)(m - 1) * 5;
  f[0] = {0.0, 0.0};
  f[1] = crecip(dcur);
  f[2] = {0.0, 0.0};
  f[3] = {0.0, 0.0};
  f[4] = {0.0, 0.0};
}

// Columns j of Z = 1/2 (E + M [T_s E + sum_q a_q Re((T_s - i beta_q)^-1 E)]),
// E_ij = hash(i, j); the result (real) goes to the T-typed m x n buffer.
// Work-group (column chunk, pole group g, block): group g takes the poles
// q = g, g + G, ... and accumulates into its own real m x n partial (group 0
// also holds T_s E); k_filter_finish adds the G partials in a fixed order.
// Each solve is a forward elimination and a backward substitution along the
// rows, both taken in chunks of FK rows with the chunk's factors of every
// pole of the group staged in LDS and the chunk's entries of E drawn once
// for all poles.  The forward pass (chunks from the top) keeps each pole's
// state at every FK-th row (checkpoints); the backward pass (chunks from the
// bottom) re-runs every pole's forward recurrence over the chunk from its
// checkpoint in registers and substitutes back through the chunk, adding
// a_q Re(x) to the chunk's accumulator in pole order, which is written once
// per chunk.  Between chunks the carries of each pole wait in Z_SCR.
// Partials: in the T-typed output when T is real and G = 1, else in C_TMP
// (free at this point); checkpoints and carries in Z_SCR.
constexpr int FK = FILTER_CK;

template <class T>
__global__ void __launch_bounds__(256) k_filter_solve(const BlockDesc* D, char* ws, const int* info, int kramers,
                                                      int G) {
  const int b = blockIdx.z, g = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int m = kramers ? d.n : d.m, n = kramers ? d.n / 2 : d.n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= n) return;       // whole work-group beyond the columns
  const bool active = j < n;
  const double* pf = bufp<double>(ws, d, P_FILT);
  const double sigma = pf[0], rho = pf[1];
  const int r = (int)pf[3];
  if (g >= r) return;
  const int nq = (r - g + G - 1) / G;             // poles g, g + G, ... of this group
  const double* dg = bufp<double>(ws, d, V_D);
  const double* eg = bufp<double>(ws, d, V_E);
  double* accb = (sizeof(T) == sizeof(double) && G == 1) ? reinterpret_cast<double*>(bufp<T>(ws, d, C_Y))
                                                         : bufp<double>(ws, d, C_TMP);
  double* acc = accb + (long long)g * m * n;
  const int nck = (m + FK - 1) / FK;
  cplx* ckb = bufp<cplx>(ws, d, Z_SCR);                    // [pole][chunk][column]
  cplx* xs = ckb + (long long)RMAX * nck * n;              // [pole][column][2]
  const cplx* Fb = bufp<cplx>(ws, d, F_FAC);
  const double ir = 1.0 / rho;
  extern __shared__ cplx Fs[];          // a chunk of rows of every pole's factors (nq x FK x 5)
  // the chunk's factors of every pole of the group into LDS (all threads)
  auto stage = [&](int i0) {
    __syncthreads();
    for (int e = threadIdx.x; e < nq * FK * 5; e += blockDim.x) {
      const int qi = e / (FK * 5), w = e - qi * FK * 5, i = i0 + w / 5;
      Fs[e] = i < m ? Fb[((long long)(g + G * qi) * m + i) * 5 + w % 5] : cplx{0.0, 0.0};
    }
    __syncthreads();
  };
  // forward: y = L^-1 P b for every pole of the group, chunk by chunk from
  // the top; the carry at rows 0, FK, ... is kept (checkpoints), and between
  // chunks it waits in the carry slot of the pole.  E's entries of a chunk
  // are drawn once for all poles.
  for (int c = 0; c < nck; ++c) {
    const int i0 = c * FK;
    stage(i0);
    if (!active) continue;
    double hb[FK];                      // E_{i+1, j} for the chunk's rows i
#pragma unroll
    for (int u = 0; u < FK; ++u) hb[u] = i0 + u + 1 < m ? hash_uniform(i0 + u + 1, j) : 0.0;
    for (int qi = 0; qi < nq; ++qi) {
      const int q = g + G * qi;
      const cplx* Fc = Fs + qi * FK * 5;
      cplx* xq = xs + ((long long)q * n + j) * 2;
      cplx carry = c == 0 ? cplx{hash_uniform(0, j), 0.0} : xq[0];
      ckb[((long long)q * nck + c) * n + j] = carry;
#pragma unroll
      for (int u = 0; u < FK; ++u) {
        const int i = i0 + u;
        if (i < m - 1) {
          const cplx* f = Fc + u * 5;
          const cplx bnext = {hb[u], 0.0};
          carry = f[4].x != 0.0 ? carry - f[0] * bnext : bnext - f[0] * carry;
        }
      }
      if (c == nck - 1) {
        xq[0] = {0.0, 0.0};             // the backward substitution starts from zero
        xq[1] = {0.0, 0.0};
      } else {
        xq[0] = carry;
      }
    }
  }
  // backward: U x = y chunk by chunk from the bottom; every pole re-runs its
  // forward recurrence over the chunk from the checkpoint in registers and
  // substitutes back; acc = [T_s E (group 0)] + sum_q a_q Re(x), written once
  // per chunk
  for (int c = nck - 1; c >= 0; --c) {
    const int i0 = c * FK;
    stage(i0);
    if (!active) continue;
    double he[FK + 2];                  // E_{i, j} for i = i0 - 1 .. i0 + FK
#pragma unroll
    for (int v = 0; v < FK + 2; ++v) {
      const int i = i0 - 1 + v;
      he[v] = (i >= 0 && i < m) ? hash_uniform(i, j) : 0.0;
    }
    double ab[FK];
#pragma unroll
    for (int u = 0; u < FK; ++u) {
      const int i = i0 + u;
      double t = 0.0;
      if (g == 0 && i < m) {
        t = (dg[i] - sigma) * he[u + 1];
        if (i > 0) t += eg[i - 1] * he[u];
        if (i < m - 1) t += eg[i] * he[u + 2];
        t = t * ir;
      }
      ab[u] = t;
    }
    for (int qi = 0; qi < nq; ++qi) {
      const int q = g + G * qi;
      const cplx* Fc = Fs + qi * FK * 5;
      const double aq = pf[4 + q];
      cplx* xq = xs + ((long long)q * n + j) * 2;
      cplx x1 = xq[0], x2 = xq[1];
      cplx cy = ckb[((long long)q * nck + c) * n + j];
      cplx yb[FK];
#pragma unroll
      for (int u = 0; u < FK; ++u) {
        const int i = i0 + u;
        yb[u] = cy;
        if (i < m - 1) {
          const cplx* f = Fc + u * 5;
          const cplx bnext = {he[u + 2], 0.0};
          const bool sw = f[4].x != 0.0;
          yb[u] = sw ? bnext : cy;
          cy = sw ? cy - f[0] * bnext : bnext - f[0] * cy;
        }
      }
#pragma unroll
      for (int u = FK - 1; u >= 0; --u) {
        const int i = i0 + u;
        if (i < m) {
          const cplx* f = Fc + u * 5;
          const cplx t = yb[u] - f[2] * x1 - f[3] * x2;
          const cplx x = t * f[1];
          ab[u] = ab[u] + aq * x.x;
          x2 = x1;
          x1 = x;
        }
      }
      xq[0] = x1;
      xq[1] = x2;
    }
#pragma unroll
    for (int u = 0; u < FK; ++u) {
      const int i = i0 + u;
      if (i < m) acc[(long long)i * n + j] = ab[u];
    }
  }
}

// Y = 1/2 (E + M sum_g partial_g) (quaternion form: rows scaled by the
// phases, Y_q = D Z).  grid = (chunks of m x n, nblk)
template <class T>
__global__ void k_filter_finish(const BlockDesc* D, char* ws, const int* info, int kramers, int G) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int m = kramers ? d.n : d.m, n = kramers ? d.n / 2 : d.n;
  const double* pf = bufp<double>(ws, d, P_FILT);
  const double M = pf[2];
  const int ng = min(G, (int)pf[3]);
  T* Y = bufp<T>(ws, d, C_Y);
  const double* accb = (sizeof(T) == sizeof(double) && G == 1) ? reinterpret_cast<const double*>(Y)
                                                               : bufp<double>(ws, d, C_TMP);
  const long long tot = (long long)m * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    double sum = accb[e];
    for (int g = 1; g < ng; ++g) sum += accb[(long long)g * tot + e];
    const double z = 0.5 * (hash_uniform(i, j) + M * sum);
    if constexpr (sizeof(T) == sizeof(quat)) Y[e] = z * bufp<quat>(ws, d, V_DEL)[i];
    else Y[e] = treal<T>(z);
  }
}

// ---------------------------------------------------------------- Q^-1/2
// Extreme eigenvalues of tridiag(dq, eq) (must be > 0: info 5), quadrature
// nodes, and the LDL^T factors of (T_Q + s_j I) for every node.
__global__ void __launch_bounds__(256) k_tri_eig_q(const BlockDesc* D, char* ws, int* info, int dsel) {
  const int b = blockIdx.x;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const double* dg = bufp<double>(ws, d, V_DQ);
  const double* eg = bufp<double>(ws, d, V_EQ);
  double* pq = bufp<double>(ws, d, P_QUAD);
  double* fac = bufp<double>(ws, d, Q_FAC);
  extern __shared__ char smem[];
  double* sd = reinterpret_cast<double*>(smem);
  double* se = sd + n;
  double* se2 = se + n;
  __shared__ double red[64];
  __shared__ double s_min, s_max;
  __shared__ int s_nodes;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    sd[i] = dg[i];
    if (i < n - 1) {
      se[i] = eg[i];
      se2[i] = eg[i] * eg[i];
    }
  }
  __syncthreads();
  double lo, hi;
  gershgorin(sd, se, n, &lo, &hi, red);
  const double piv = 2.2e-308 * 16.0 * fmax(1.0, hi * hi);
  __shared__ int cbuf[256];
  __shared__ double xbuf[256];
  multisect(sd, se2, n, 0, 1, lo, hi, piv, &s_min, cbuf, xbuf);
  multisect(sd, se2, n, n - 1, 1, lo, hi, piv, &s_max, cbuf, xbuf);
  __syncthreads();
  if (threadIdx.x == 0) {
    double lmin = s_min, lmax = s_max;
    if (!(lmin > 0.0) || !isfinite(lmax)) {
      info[b] = 5;
      s_nodes = 0;
    } else {
      double s = sqrt(lmin * lmax);
      double kap = lmax / lmin;
      double rate = 4.0 * atanh(pow(kap, -0.25));
      int N = (int)ceil(38.0 / rate) + 2;
      if (N > QMAX) N = QMAX;
      if (N < 2) N = 2;
      pq[0] = N;
      pq[1] = lmin;
      pq[2] = lmax;
      for (int j = 0; j < N; ++j) {
        double phi = (j + 0.5) * 3.14159265358979323846 / (2.0 * N);
        double cph = cos(phi), tph = tan(phi);
        pq[3 + j] = sqrt(s) / (N * cph * cph);
        pq[3 + QMAX + j] = s * tph * tph;
      }
      s_nodes = N;
    }
  }
  __syncthreads();
  const int N = s_nodes;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const double sh = pq[3 + QMAX + j];
    double* f = fac + (long long)j * n * 2;
    double dcur = sd[0] + sh;
    for (int i = 0; i < n - 1; ++i) {
      double l = se[i] / dcur;
      f[2 * i] = l;
      f[2 * i + 1] = 1.0 / dcur;
      dcur = sd[i + 1] + sh - l * se[i];
    }
    f[2 * (n - 1)] = 0.0;
    f[2 * (n - 1) + 1] = 1.0 / dcur;
  }
}

// F = sum_j w_j (T_Q + s_j I)^-1 (symmetric): column k of its lower
// triangle, F[i][k] for i >= k, from the LDL^T factors of every node by a
// forward sweep from row k and a backward sweep down to row k.  Work-group
// (column chunk, node group g, block): group g takes the nodes j = g, g + G,
// ... into its own real n x n partial; the forward sweep keeps its state at
// every IK-th row and the backward sweep re-runs it chunk by chunk in
// registers (as in k_filter_solve).  k_invsqrt_finish adds the partials in a
// fixed order, mirrors the triangle and writes F T-typed into C_TMP
// (quaternion form: rows scaled by the phases, F_q = D F).
// Partials: in C_TMP itself when T is real and G = 1, else at the start of
// the scratch buffer; checkpoints after them.
constexpr int IK = 16;

__device__ inline double* invsqrt_partials(const BlockDesc& d, char* ws, int n, int bufScr, bool real1) {
  return real1 ? bufp<double>(ws, d, C_TMP) : bufp<double>(ws, d, bufScr);
}

template <class T>
__global__ void __launch_bounds__(256) k_invsqrt_cols(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                      int bufScr, int G) {
  const int b = blockIdx.z, g = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* pq = bufp<double>(ws, d, P_QUAD);
  const double* fac = bufp<double>(ws, d, Q_FAC);
  const int nodes = (int)pq[0];
  const bool real1 = sizeof(T) == sizeof(double) && G == 1;
  double* acc = invsqrt_partials(d, ws, n, bufScr, real1) + (long long)g * n * n;
  const int nck = (n + IK - 1) / IK;
  double* ck = (real1 ? bufp<double>(ws, d, bufScr) : invsqrt_partials(d, ws, n, bufScr, false) +
                                                        (long long)G * n * n) +
               (long long)g * nck * n;
  bool fresh = true;
  for (int j = g; j < nodes; j += G) {
    const double* f = fac + (long long)j * n * 2;
    const double w = pq[3 + j];
    // forward L y = e_k from row k (y_k = 1); checkpoints of y at rows
    // i = IK c > k
    double yi = 1.0;
    for (int i = k + 1; i < n; ++i) {
      yi = -f[2 * (i - 1)] * yi;
      if (i % IK == 0) ck[(long long)(i / IK) * n + k] = yi;
    }
    // backward L^T x = D^-1 y, rows n-1 .. k, one chunk of IK rows at a time
    double x = 0.0;
    const int c0 = k / IK;
    for (int c = nck - 1; c >= c0; --c) {
      const int i0 = c * IK;
      const int ib = max(i0, k);                  // first row of the chunk inside the triangle
      double y = ib == k ? 1.0 : ck[(long long)c * n + k];
      double zb[IK], ab[IK];
#pragma unroll
      for (int u = 0; u < IK; ++u) {
        const int i = i0 + u;
        const int ic = min(max(i, k), n - 1);
        ab[u] = fresh ? 0.0 : acc[(long long)ic * n + k];
      }
#pragma unroll
      for (int u = 0; u < IK; ++u) {
        const int i = i0 + u;
        if (i > ib && i < n) y = -f[2 * (i - 1)] * y;
        zb[u] = (i >= ib && i < n) ? y * f[2 * i + 1] : 0.0;
      }
#pragma unroll
      for (int u = IK - 1; u >= 0; --u) {
        const int i = i0 + u;
        if (i >= k && i < n) {
          x = zb[u] - f[2 * i] * x;
          acc[(long long)i * n + k] = ab[u] + w * x;
        }
      }
    }
    fresh = false;
  }
}

template <class T>
__global__ void k_invsqrt_finish(const BlockDesc* D, char* ws, const int* info, int dsel, int bufScr, int G) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int nodes = (int)bufp<double>(ws, d, P_QUAD)[0];
  const int ng = min(G, nodes);
  const bool real1 = sizeof(T) == sizeof(double) && G == 1;
  const double* acc = invsqrt_partials(d, ws, n, bufScr, real1);
  T* F = bufp<T>(ws, d, C_TMP);
  const long long nn = (long long)n * n;
  if (real1) {
    // partial is F itself: mirror the lower triangle
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
      const int i = (int)(e / n), k = (int)(e % n);
      if (k > i) F[e] = treal<T>(acc[(long long)k * n + i]);
    }
    return;
  }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), k = (int)(e % n);
    const long long src = i >= k ? e : (long long)k * n + i;
    double v = acc[src];
    for (int g = 1; g < ng; ++g) v += acc[(long long)g * nn + src];
    if constexpr (sizeof(T) == sizeof(quat)) F[e] = v * bufp<quat>(ws, d, V_DEL)[i];
    else F[e] = treal<T>(v);
  }
}

// ----------------------------------------------------------------- launchers
void launch_tri_eig4c(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxm, double* eps,
                      double c, int kramers) {
  const size_t shm = (size_t)(3 * maxm) * sizeof(double);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tri_eig4c), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tri_eps4c), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(k_tri_eig4c, dim3(nblk), dim3(1024), shm, s, D, ws, info, c, kramers);
  const int maxn = maxm / 2;
  hipLaunchKernelGGL(k_tri_eps4c, dim3((maxn + EPW - 1) / EPW, nblk), dim3(256), shm, s, D, ws, info, eps, kramers);
}
void launch_filter_factor(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int kramers,
                          int maxm_filter) {
  hipLaunchKernelGGL(k_filter_factor, dim3(RMAX, nblk), dim3(64), 2 * (size_t)maxm_filter * sizeof(double), s, D, ws,
                     info, kramers);
}
template <class T>
void launch_filter_solve(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxrhs,
                         int kramers) {
  const int maxm = kramers ? maxrhs * 2 : 2 * maxrhs;      // rows of the tridiagonal
  const int Gs = kramers ? 4 : 1;
  const size_t shm = (size_t)((RMAX + Gs - 1) / Gs) * FK * 5 * sizeof(cplx);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_filter_solve<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  // pole groups: the quaternion form has room for four partials in C_TMP
  const int G = kramers ? 4 : 1;
  hipLaunchKernelGGL(k_filter_solve<T>, dim3((maxrhs + 255) / 256, G, nblk), dim3(256), shm, s, D, ws, info, kramers,
                     G);
  long long gx = ((long long)maxm * maxrhs + 255) / 256;
  if (gx > 256) gx = 256;
  hipLaunchKernelGGL(k_filter_finish<T>, dim3((int)gx, nblk), dim3(256), 0, s, D, ws, info, kramers, G);
}
void launch_tri_eig_q(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxdim, int dsel) {
  size_t shm = (size_t)(3 * maxdim) * sizeof(double);
  hipLaunchKernelGGL(k_tri_eig_q, dim3(nblk), dim3(256), shm, s, D, ws, info, dsel);
}
template <class T>
void launch_invsqrt_cols(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                         int bufScr) {
  // node groups: the quaternion form's scratch (C_QMH) holds four partials
  const int G = is_quat<T>() ? 4 : 1;
  hipLaunchKernelGGL(k_invsqrt_cols<T>, dim3((maxdim + 255) / 256, G, nblk), dim3(256), 0, s, D, ws, info, dsel,
                     bufScr, G);
  long long gx = ((long long)maxdim * maxdim + 255) / 256;
  if (gx > 256) gx = 256;
  hipLaunchKernelGGL(k_invsqrt_finish<T>, dim3((int)gx, nblk), dim3(256), 0, s, D, ws, info, dsel, bufScr, G);
}
template void launch_filter_solve<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int);
template void launch_filter_solve<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int);
template void launch_filter_solve<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int);
template void launch_invsqrt_cols<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);
template void launch_invsqrt_cols<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);
template void launch_invsqrt_cols<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int);

}  // namespace x2c
