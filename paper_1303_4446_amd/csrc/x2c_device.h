// Device-side types and helpers shared by the X2C kernels (gfx950).
//
// Scalar type T is `double` (spin-free mode, real matrices) or `cplx`
// (two-component mode, complex Hermitian matrices in the spin-orbital basis
// [all alpha; all beta], Sec. II Eqs. defstv/defw).  All matrices are
// row-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace x2c {

struct cplx {
  double x, y;
};

// ---------------------------------------------------------------- arithmetic
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cplx operator-(cplx a) { return {-a.x, -a.y}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return {s * a.x, s * a.y}; }
__host__ __device__ inline cplx operator*(cplx a, double s) { return {s * a.x, s * a.y}; }

__host__ __device__ inline double conjg(double a) { return a; }
__host__ __device__ inline cplx conjg(cplx a) { return {a.x, -a.y}; }
__host__ __device__ inline double re(double a) { return a; }
__host__ __device__ inline double re(cplx a) { return a.x; }
__host__ __device__ inline double im(double) { return 0.0; }
__host__ __device__ inline double im(cplx a) { return a.y; }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(cplx a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double abs1(double a) { return fabs(a); }
__host__ __device__ inline double abs1(cplx a) { return fabs(a.x) + fabs(a.y); }

// c + a*b
__device__ inline double mad(double a, double b, double c) { return fma(a, b, c); }
__device__ inline cplx mad(cplx a, cplx b, cplx c) {
  return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
__device__ inline cplx mad(double a, cplx b, cplx c) { return {fma(a, b.x, c.x), fma(a, b.y, c.y)}; }
__device__ inline cplx mad(cplx a, double b, cplx c) { return {fma(a.x, b, c.x), fma(a.y, b, c.y)}; }

// ---------------------------------------------------------------- quaternions
// q = a + b j with complex a, b (j z = conj(z) j).  A time-reversal symmetric
// two-component operator [[A, B], [-B*, A*]] (Sec. III.A) is the quaternion
// matrix A + B j; q corresponds to the 2x2 complex block [[a, b], [-b*, a*]].
struct quat {
  cplx a, b;
};
__host__ __device__ inline quat operator+(quat x, quat y) { return {x.a + y.a, x.b + y.b}; }
__host__ __device__ inline quat operator-(quat x, quat y) { return {x.a - y.a, x.b - y.b}; }
__host__ __device__ inline quat operator-(quat x) { return {-x.a, -x.b}; }
// (a1 + b1 j)(a2 + b2 j) = (a1 a2 - b1 conj(b2)) + (a1 b2 + b1 conj(a2)) j
__host__ __device__ inline quat operator*(quat x, quat y) {
  cplx b2c = {y.b.x, -y.b.y}, a2c = {y.a.x, -y.a.y};
  return {x.a * y.a - x.b * b2c, x.a * y.b + x.b * a2c};
}
// With components q = (Re a, Im a, Re b, Im b), (x y)_c = sum_d
// qmul_sign(c, d) x_{c xor d} y_d: left multiplication by x is a signed
// permutation of x's components as a real 4 x 4 matrix.
constexpr int qmul_sign(int c, int d) {
  return c == 0 ? (d == 0 ? 1 : -1)
                : (d == 0 || d == c || (c == 1 && d == 3) || (c == 2 && d == 1) || (c == 3 && d == 2)) ? 1 : -1;
}
__host__ __device__ inline quat operator*(double s, quat x) { return {s * x.a, s * x.b}; }
__host__ __device__ inline quat operator*(quat x, double s) { return {s * x.a, s * x.b}; }
__host__ __device__ inline quat conjg(quat x) { return {{x.a.x, -x.a.y}, {-x.b.x, -x.b.y}}; }
__host__ __device__ inline double re(quat x) { return x.a.x; }
__host__ __device__ inline double im(quat x) { return x.a.y; }
__host__ __device__ inline double abs2(quat x) { return abs2(x.a) + abs2(x.b); }
__host__ __device__ inline double abs1(quat x) { return abs1(x.a) + abs1(x.b); }
// c + x y as sixteen fused multiply-adds, each component accumulated into c
// (the component form of the product above; signs as source negations)
__device__ inline quat mad(quat x, quat y, quat c) {
  const double xr = x.a.x, xi = x.a.y, xj = x.b.x, xk = x.b.y;
  const double yr = y.a.x, yi = y.a.y, yj = y.b.x, yk = y.b.y;
  quat r;
  r.a.x = fma(-xk, yk, fma(-xj, yj, fma(-xi, yi, fma(xr, yr, c.a.x))));
  r.a.y = fma(xj, yk, fma(-xk, yj, fma(xi, yr, fma(xr, yi, c.a.y))));
  r.b.x = fma(xk, yi, fma(xj, yr, fma(-xi, yk, fma(xr, yj, c.b.x))));
  r.b.y = fma(-xj, yi, fma(xk, yr, fma(xi, yj, fma(xr, yk, c.b.y))));
  return r;
}
__device__ inline quat mad(double s, quat y, quat c) { return {mad(s, y.a, c.a), mad(s, y.b, c.b)}; }

// real components of an element (1 real, 2 complex, 4 quaternion:
// (Re a, Im a, Re b, Im b)) and the largest of their moduli
template <class T>
constexpr int ncomp() {
  return (int)(sizeof(T) / sizeof(double));
}
__host__ __device__ inline double comp(double v, int) { return v; }
__host__ __device__ inline double comp(cplx v, int c) { return c == 0 ? v.x : v.y; }
__host__ __device__ inline double comp(quat v, int c) {
  return c == 0 ? v.a.x : (c == 1 ? v.a.y : (c == 2 ? v.b.x : v.b.y));
}
__host__ __device__ inline double amax(double v) { return fabs(v); }
__host__ __device__ inline double amax(cplx v) { return fmax(fabs(v.x), fabs(v.y)); }
__host__ __device__ inline double amax(quat v) { return fmax(amax(v.a), amax(v.b)); }

template <class T> __host__ __device__ inline T tzero();
template <> __host__ __device__ inline double tzero<double>() { return 0.0; }
template <> __host__ __device__ inline cplx tzero<cplx>() { return {0.0, 0.0}; }
template <> __host__ __device__ inline quat tzero<quat>() { return {{0.0, 0.0}, {0.0, 0.0}}; }
template <class T> __host__ __device__ inline T treal(double a);
template <> __host__ __device__ inline double treal<double>(double a) { return a; }
template <> __host__ __device__ inline cplx treal<cplx>(double a) { return {a, 0.0}; }
template <> __host__ __device__ inline quat treal<quat>(double a) { return {{a, 0.0}, {0.0, 0.0}}; }
template <class T> __host__ __device__ inline T tmake(double a, double b);
template <> __host__ __device__ inline double tmake<double>(double a, double) { return a; }
template <> __host__ __device__ inline cplx tmake<cplx>(double a, double b) { return {a, b}; }
template <> __host__ __device__ inline quat tmake<quat>(double a, double b) { return {{a, b}, {0.0, 0.0}}; }

__device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
  }
}
__device__ inline cplx crecip(cplx b) { return cdiv(cplx{1.0, 0.0}, b); }

template <class T>
constexpr bool is_quat() {
  return sizeof(T) == sizeof(quat);
}

// inverse and right division s u^-1 for every scalar type (quaternion inverse
// = conj(q) / |q|^2; the order matters for quaternions)
__device__ inline double tinv(double u) { return 1.0 / u; }
__device__ inline cplx tinv(cplx u) { return crecip(u); }
__device__ inline quat tinv(quat u) { return (1.0 / abs2(u)) * conjg(u); }
__device__ inline double rdiv(double s, double u) { return s / u; }
__device__ inline cplx rdiv(cplx s, cplx u) { return cdiv(s, u); }
__device__ inline quat rdiv(quat s, quat u) { return s * tinv(u); }

// ---------------------------------------------------------------- workspace
// Named per-block buffers.  Offsets (bytes from the workspace base) are laid
// out by the host plan; every block owns its own region.
enum Buf : int {
  // real N x N
  R_S = 0, R_T, R_V, R_W0, R_W1, R_W2, R_W3,   // input copies
  R_LS, R_LT, R_LSI, R_LTI,                     // Cholesky factors and inverses
  R_TMP, R_ALL, R_B, R_WR0, R_WR1, R_WR2, R_WR3, // reduced blocks
  // T-typed n x n
  C_S, C_T, C_V, C_WPP, C_LS, C_LSI, C_LTI,
  C_X, C_TX, C_Q, C_WX, C_L, C_QMH, C_R, C_LR, C_H, C_TMP, C_TMP2,
  // T-typed m x m and m x n
  C_A, C_Y,
  // complex m x n scratch for the filter solves
  Z_SCR,
  // vectors
  V_D, V_E, V_TAU, V_DQ, V_EQ, V_TAUQ, V_PIV,
  // filter / quadrature parameters and factors
  P_FILT, P_QUAD, F_FAC, Q_FAC,
  // compact-WY factors of the reflector panels (4c and Q)
  W_TF4, W_TFQ,
  // panel companion vectors of the blocked tridiagonalisation (m x 32)
  W_PAN,
  // per-tile matvec sums of the blocked tridiagonalisation
  W_HS,
  // current reflector of the blocked tridiagonalisation (m)
  W_VCUR,
  // quaternion path: sub-diagonal quaternions and the phases making them real
  V_ET, V_DEL,
  // split-precision products: binary exponents of the rows of op(A) and of
  // the columns of op(B)
  V_EXA, V_EXB,
  // split-precision products with int8 slices: the split operands
  Z_SLA, Z_SLB,
  // BSS and DKHn (free-particle FW basis): real N x N reduced kinetic matrix
  // (then its reflectors), rotations (transposed and row-major), K, S K
  R_KC, R_ZT, R_Z, R_K, R_G,
  // fpFW vectors [p | E_0 | E_0 - c^2 | U_0^A | U_0^B] (5 N doubles)
  V_FP,
  // N x N matrices of the scalar type of the chain (quaternion two-component,
  // real spin-free): E_1, O_1, E_1', work, product, X'', h in the kinetic basis
  Q_E1, Q_O1, Q_E1P, Q_M, Q_P, Q_X2, Q_H,
  // device-wide path of a large block: two more 4c-sized matrices for the
  // sign iteration, four h-sized ones for the iteration on P_LL (P_SL, the
  // inverse square root, two products), and the iteration parameters (NsPar)
  C_G1, C_G2, H_A, H_B, H_C, H_D, V_NS,
  // DKHn term and scratch slots (see x2c_dkh_plan.h)
  D_T0,
  NBUF = D_T0 + 48
};

constexpr int RMAX = 48;   // max Zolotarev pole pairs
constexpr int FILTER_CK = 16;   // rows per checkpoint chunk of the projector solves
constexpr int QMAX = 64;   // max quadrature nodes for the inverse square root
// P_FILT layout (doubles): [0]=sigma [1]=rho [2]=M [3]=r [4..4+RMAX)=a_j [4+RMAX..4+2RMAX)=beta_j
constexpr int PF_SIZE = 4 + 2 * RMAX;
// P_QUAD layout: [0]=nodes [1]=lambda_min [2]=lambda_max [3..3+QMAX)=weights [3+QMAX..)=shifts
constexpr int PQ_SIZE = 3 + 2 * QMAX;

// Parameters and reductions of the Newton-Schulz iterations of the
// device-wide path (one per large block, in its V_NS buffer).  `gate` is
// non-zero once the current iteration has converged or the block has
// failed; the product kernels take it in place of the block status.
constexpr int NS_PARTS = 4096;   // work-groups of an elementwise pass, at most
struct NsPar {
  double sigma, rho, l;        // shift, scale, lower bound of the moduli
  unsigned long long rmax;     // largest row sum (bits of a non-negative double)
  int conv, iters;              // converged flag, steps taken (the gates sit in the workspace head)
  // per-work-group partial sums of the last reduction (squares of the step
  // change, of the new iterate), summed in a fixed order: the iteration is
  // reproducible bit for bit
  double part[2][NS_PARTS];
};

struct BlockDesc {
  int N;      // scalar basis functions of the block
  int n;      // dimension of h: N (spin-free) or 2N (two-component)
  int m;      // 4c dimension 2n
  int orig;   // the caller's index of the block (descriptors are sorted by size)
  long long in_off;   // element offset of S, T, V (W: in_off, or 4*in_off in 2c)
  long long h_off;    // double offset into h
  long long eps_off;  // double offset into eps
  long long off[NBUF];
};

// One atom pair (A >= B) of the DLU molecular assembly.
struct DluPair {
  int A, B;           // atoms
  int nA, nB;         // dimensions of their h blocks (N or 2N)
  int oA, oB;         // scalar offsets of their functions in the molecule
  long long xA, xB;   // element offsets of X_A / R_A and X_B / R_B in the X and R arrays
  long long t, w, l, p;   // byte offsets of the pair's work buffers (T_AB / h_AB, W'', L, P)
};

template <class P>
__device__ inline P* bufp(char* ws, const BlockDesc& d, int id) {
  return reinterpret_cast<P*>(ws + d.off[id]);
}

// dimension selector used by the generic kernels
enum Dim : int { DIM_N = 0, DIM_n = 1, DIM_m = 2 };
__device__ inline int seldim(const BlockDesc& d, int s) { return s == DIM_N ? d.N : (s == DIM_n ? d.n : d.m); }

// counter-based hash -> uniform(-1, 1) (SplitMix64 finaliser), used to draw the
// fixed test block of the spectral-projector filter
__host__ __device__ inline double hash_uniform(uint64_t i, uint64_t j) {
  uint64_t z = (i * 0x9E3779B97F4A7C15ull) ^ (j + 0x632BE59BD9B4E019ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// block-wide sum over blockDim.x threads (<= 1024), result broadcast
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  int nw = (blockDim.x + 63) >> 6;
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  __syncthreads();
  return t;
}

}  // namespace x2c
