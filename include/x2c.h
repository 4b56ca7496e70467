/*
 * x2c.h -- C ABI of libx2c: the exact-decoupling (X2C) one-electron
 * Hamiltonian of uncontracted atomic blocks on an AMD MI355X (gfx950).
 *
 * What is computed (Peng, Middendorf, Weigend, Reiher, J. Chem. Phys. 138,
 * 184105 (2013)):  h = H(S, T, V, W) of Sec. II, Eq. r2ctrans, for one block
 * or for a batch of independent atomic blocks as in the local DLU scheme
 * (Sec. III.A, Eqs. dlutrans and r2ctransatom).  Per block:
 *   1. the modified Dirac equation D C = M C eps (Sec. II, Eq. moddiraceq),
 *      D = [[V, T], [T, W/4c^2 - T]], M = diag(S, T/2c^2), is reduced with the
 *      Cholesky factors of S and T to a standard Hermitian problem;
 *   2. its positive-energy branch (eigenvalues with eps + c^2 > 0, Sec. II) is
 *      found: the n eigenvalues and the invariant subspace they span;
 *   3. X = C_S C_L^-1 (Appendix, Eq. defxmat);
 *   4. S~ = S + X^H T X / 2c^2 and the renormalisation
 *      R = S^-1/2 (S^-1/2 S~ S^-1/2)^-1/2 S^1/2 (Sec. II.A, Eq. ulnonortho),
 *      evaluated in the equivalent Cholesky form L_S^-H (L_S^-1 S~ L_S^-H)^-1/2 L_S^H;
 *   5. h = R^H L R with L = V + T X + X^H T + X^H (W/4c^2 - T) X, i.e.
 *      Eq. utrans with U^L = R and U^S = X R (Eq. usnonortho).
 *
 * Modes: spin-free (real N x N matrices, W = W^0; Sec. II scalar
 * approximation) and two-component (2N x 2N complex Hermitian h in the
 * spin-orbital basis [all alpha; all beta], Eq. defstv, with W built from
 * W^0, W^x, W^y, W^z as in Eq. defw).
 *
 * Conventions for every function below:
 *   - All matrices are row-major float64.  Complex matrices are interleaved
 *     (re, im) pairs, i.e. the layout of complex128.
 *   - Every pointer argument except `opts`, `N` (batched) and the offset
 *     arrays is a DEVICE pointer on the current HIP device.  `N`, `in_off`,
 *     `h_off` and `eps_off` of x2c_build_batched are HOST arrays.
 *   - The caller owns every buffer.  The library never frees caller memory
 *     and allocates no device memory of its own on these paths: all scratch
 *     lives in the caller's workspace (size from x2c_workspace_bytes).
 *   - `stream` is a hipStream_t (NULL = default stream); all device work is
 *     enqueued on it.
 *   - Inputs are assumed symmetric (S, T, V, W^0) / antisymmetric
 *     (W^x, W^y, W^z); this is not checked.
 */
#ifndef X2C_H
#define X2C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { X2C_SPINFREE = 1, X2C_TWOCOMP = 2 } x2c_mode;
/* Arithmetic of the products of steps 3-5 (X, S~, L, the renormalisation and
 * h).  X2C_FP64: FP64 products.  X2C_SPLIT_BF16: each FP64 operand row
 * (column) is scaled by a power of two and cut into `ozaki_slices` 7-bit
 * integer slices held exactly in bf16; the slice products run on the bf16
 * matrix cores with exact FP32 partial sums, folded into FP64 (an error-free
 * splitting of FP64 products).  The truncation error of a product entry is
 * about K 2^(-7 s) times the product of the operand row and column maxima
 * (K the inner dimension).  The Cholesky factors, the eigenvalue problems and
 * the inverse square root are FP64 in both modes.  X2C_SPLIT_INT8: the same
 * splitting with int8 slices (the line scaled into (-1/2, 1/2), so each slice
 * holds about 7 bits) on the int8 matrix cores with exact int32 sums; the
 * operands are split once per product. */
typedef enum { X2C_FP64 = 0, X2C_SPLIT_BF16 = 1, X2C_SPLIT_INT8 = 2 } x2c_prec;

/* Reduction of the two Hermitian eigenproblems of a two-component block.
 * Every two-component matrix of the method has the time-reversal form
 * [[A, B], [-B*, A*]] in the [all alpha; all beta] basis (Sec. III.A, Kramers
 * pairs), i.e. it is the quaternion matrix A + B j of half the dimension.
 * The quaternion reduction tridiagonalises that half-size form (one real
 * eigenvalue per Kramers pair); the complex one treats the full complex
 * Hermitian matrix.  Both give the same h to rounding.  Ignored for
 * spin-free blocks. */
typedef enum { X2C_RED_QUATERNION = 0, X2C_RED_COMPLEX = 1 } x2c_reduction;

/* Which path the blocks of a call take (see x2c_max_n for the two paths).
 * X2C_ROUTE_SIZE: by block size, the device-wide path from
 * x2c_device_wide_min_n on, the batched path below (eigenvalues written).
 * X2C_ROUTE_DEVICE_WIDE: every block on the device-wide path (eps NaN).
 * X2C_ROUTE_AUTO: for callers that do not need the eigenvalues: the blocks of
 * batched-path size take the device-wide path together when the batch is
 * small enough for that to be faster, else the batched path.  The estimate:
 * sum over those blocks of N_b^1.5 below 1.7e5 (two-component, quaternion
 * reduction; half that with the complex one) or 1.4e6 (spin-free), where the
 * two paths' times cross for uniform batches of atomic blocks in FP64 on
 * MI355X; x2c_autotune with this route measures the choice for a batch
 * class instead, and later calls of the class follow the measurement.
 * x2c_workspace_bytes with this route covers either path.  eps of a block is
 * NaN whenever it took the device-wide path.
 * BSS and DKHn (batched path only) ignore the route; the no-allocation entry
 * point accepts X2C_ROUTE_SIZE only. */
typedef enum { X2C_ROUTE_SIZE = 0, X2C_ROUTE_DEVICE_WIDE = 1, X2C_ROUTE_AUTO = 2 } x2c_route;

typedef struct {
  int mode;          /* x2c_mode */
  int prec;          /* x2c_prec: arithmetic of the X / L / S~ / R product chain */
  int ozaki_slices;  /* split precision only: slices per operand, 1..8; 0 = automatic (bf16 7, int8 8) */
  double c;          /* speed of light in atomic units (> 0) */
  int reduction;     /* x2c_reduction (two-component only); 0 = quaternion */
  int route;         /* x2c_route; 0 = by block size */
} x2c_options;

/* return codes */
enum {
  X2C_OK = 0,
  X2C_EINVAL = -1,  /* bad argument: NULL pointer, N <= 0 or > x2c_max_n, c <= 0,
                       unknown mode/prec/reduction/route, workspace too small,
                       overlapping layout */
  X2C_EHIP = -2,    /* a HIP runtime call or kernel launch failed */
  X2C_EBLOCK = -3,  /* x2c_build only: the block failed; see its info code */
  X2C_ESCRATCH = -4 /* x2c_build_batched_noalloc only: the batch needs more than the
                       library's static scratch (256 MiB) or has more than 256 blocks */
};

/* per-block status codes (info) */
enum {
  X2C_INFO_OK = 0,
  X2C_INFO_S_NOT_SPD = 1,    /* Cholesky of S failed */
  X2C_INFO_T_NOT_SPD = 2,    /* Cholesky of T failed */
  X2C_INFO_EIGEN = 3,        /* positive-energy subspace not resolved: singular large-component block,
                                or the gap at -c^2 too narrow for the spectral projector (device-wide
                                path: a Newton-Schulz iteration did not converge) */
  X2C_INFO_BRANCH = 4,       /* number of eigenvalues with eps + c^2 > 0 differs from n */
  X2C_INFO_RENORM = 5,       /* L_S^-1 S~ L_S^-H not positive definite */
  X2C_INFO_NONFINITE = 6     /* NaN or Inf in S, T, V or W */
};

/* Largest supported scalar block size N for a mode (0 for an unknown mode):
 * 4096 two-component (4c dimension 16384), 8192 spin-free.  Blocks up to
 * 256 (two-component) / 512 (spin-free) run on the batched path: one
 * work-group per block and column step of the reductions, many blocks at
 * once, eigenvalues eps written out.  Larger blocks (a whole molecular matrix,
 * the full transformation that the DLU scheme of Sec. III.A approximates)
 * run on the device-wide path, all such blocks of a call together, each
 * product spread over the whole GPU (one block: a whole-matrix product
 * kernel; several: the batched one): blocked Cholesky factors, the positive-energy branch from the spectral projector
 * (I + sign(A + c^2 I)) / 2 of the reduced 4c matrix A by a scaled
 * Newton-Schulz iteration, X~ and Q^-1/2 together from one coupled
 * Newton-Schulz iteration on the projector's large-component block; matrix
 * products only.  That path does not compute
 * eigenvalues: eps of such a block is NaN (h, X and R are as on the batched
 * path).  BSS, DKHn, the DLU assembly and x2c_build_batched_noalloc take
 * batched-path sizes only. */
int x2c_max_n(int mode);

/* Smallest N of a block that takes the device-wide path (see x2c_max_n), per
 * mode.  n > 0 sets it (1 .. batched limit + 1), n = 0 restores the default
 * (batched limit + 1), n < 0 only queries.  Returns the previous (or current)
 * value, or X2C_EINVAL for an unknown mode or n above the default.  A setting
 * for the whole process; workspace sizes depend on it.  Not thread-safe with
 * concurrent builds of the same mode. */
int x2c_device_wide_min_n(int mode, int n);

/*
 * Workspace size in bytes needed by x2c_build_batched for `nblk` blocks of
 * scalar sizes N[0..nblk) (host array), or by x2c_build with nblk = 1.
 * Returns 0 for invalid arguments.
 */
size_t x2c_workspace_bytes(const x2c_options* opts, int nblk, const int* N);

/*
 * One block (blocking).
 *   N        scalar basis size (1 <= N <= x2c_max_n(mode)).
 *   S, T, V  N x N each (device).
 *   W        spin-free: W^0 (N x N); two-component: W^0, W^x, W^y, W^z
 *            contiguous (4 x N x N) (device).
 *   h        output: spin-free N x N float64; two-component 2N x 2N complex128 (device).
 *   eps      output: the n positive-energy eigenvalues of Eq. moddiraceq,
 *            ascending, in Hartree (n = N or 2N); NaN on the device-wide
 *            path (device).
 * Synchronises `stream`.  Returns X2C_OK, X2C_EINVAL, X2C_EHIP, or
 * X2C_EBLOCK with *info_out (host, may be NULL) set to the block's info code;
 * on X2C_EBLOCK h and eps are zero.
 */
int x2c_build(const x2c_options* opts, int N, const double* S, const double* T, const double* V,
              const double* W, void* h, double* eps, void* workspace, size_t ws_bytes, void* stream,
              int* info_out);

/*
 * A batch of independent blocks of uneven sizes (stream-ordered, does not
 * synchronise).  Block b has scalar size N[b]:
 *   S, T, V  its N_b x N_b matrix starts at element in_off[b] of each array;
 *   W        spin-free: at in_off[b];  two-component: 4 matrices at 4*in_off[b];
 *   h        output at double offset h_off[b] (N_b^2 doubles spin-free,
 *            2 * (2 N_b)^2 doubles = (2N_b)^2 complex128 two-component);
 *   eps      output at double offset eps_off[b] (n_b doubles);
 *   info     nblk ints (device): per-block status, valid once `stream`
 *            has completed.  A failed block gets zero h and eps; the others
 *            are unaffected.
 * Returns X2C_OK once all work is enqueued, or X2C_EINVAL / X2C_EHIP.
 */
int x2c_build_batched(const x2c_options* opts, int nblk, const int* N, const int64_t* in_off,
                      const double* S, const double* T, const double* V, const double* W,
                      const int64_t* h_off, void* h, const int64_t* eps_off, double* eps, int* info,
                      void* workspace, size_t ws_bytes, void* stream);

/*
 * x2c_build_batched for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layout, per-block info and results as
 * x2c_build_batched (the same kernels, on `stream` only), without the
 * workspace: the scratch lives in a static device array of the library,
 * 256 MiB per GPU, allocated when the library's code is first loaded on a
 * device and held until the process ends.  The batch must fit in it: at
 * most 256 blocks and x2c_workspace_bytes(opts, nblk, N) minus about
 * 0.5 KiB per block of descriptors <= 256 MiB (e.g. one block of any
 * supported size, three two-component blocks of N = 192); otherwise
 * X2C_ESCRATCH is returned before anything is enqueued.  Nothing is
 * allocated, copied from the host or cleared with a memset: descriptors go
 * to the device as kernel arguments, so the call can be captured into a
 * graph.  Every call on a GPU shares that GPU's scratch, which keeps the
 * last call's contents (no part of it needs to start at zero): calls that
 * overlap in time on one GPU (different streams or threads) race and must
 * be serialised by the caller.  Tracing does not record these calls.
 * Returns X2C_OK once enqueued, X2C_EINVAL, X2C_ESCRATCH or X2C_EHIP.
 */
int x2c_build_batched_noalloc(const x2c_options* opts, int nblk, const int* N, const int64_t* in_off,
                              const double* S, const double* T, const double* V, const double* W,
                              const int64_t* h_off, void* h, const int64_t* eps_off, double* eps, int* info,
                              void* stream);

/*
 * x2c_build_batched that also returns each block's decoupling matrices:
 * X_b = C_S C_L^-1 (Appendix, Eq. defxmat) and the renormalisation R_b
 * (Eq. ulnonortho), i.e. U^L_bb = R_b and U^S_bb = X_b R_b (Eq. usnonortho).
 * X and R (device, either may be NULL) use the layout of h: block b's
 * n_b x n_b matrix (float64 or complex128) at double offset h_off[b].
 * A failed block gets zero X and R.  Other arguments and the return value as
 * for x2c_build_batched.
 */
int x2c_build_batched_xr(const x2c_options* opts, int nblk, const int* N, const int64_t* in_off,
                         const double* S, const double* T, const double* V, const double* W,
                         const int64_t* h_off, void* h, const int64_t* eps_off, double* eps, void* X,
                         void* R, int* info, void* workspace, size_t ws_bytes, void* stream);

/*
 * BSS one-electron Hamiltonian of a batch (Sec. II, "The BSS approach",
 * Eq. u1trafo): the free-particle Foldy-Wouthuysen transformation in the
 * orthonormal kinetic basis T K = S K t (Eq. orthonormalk), p = sqrt(2t),
 * E_0 = sqrt(c^2 p^2 + c^4), U_0^A = sqrt((E_0 + c^2)/2E_0),
 * U_0^B = sqrt((E_0 - c^2)/2E_0), gives the 4c matrix
 * H^0 = [[E_1 + E_0 - c^2, O_1], [O_1^H, E_1' - E_0 - c^2]] with
 * E_1 = U_0^A V~ U_0^A + U_0^B W~ U_0^B, O_1 = U_0^A V~ U_0^B - U_0^B W~ U_0^A,
 * E_1' = U_0^B V~ U_0^B + U_0^A W~ U_0^A (V~ = K^T V K, W~ = p^-1 K^T W K p^-1);
 * its positive-energy block X'' = C_S'' C_L''^-1, R'' = (I + X''^H X'')^-1/2
 * and h from Eq. utrans with U^L_BSS = K (U_0^A + U_0^B X'') R'' K^-1 and
 * U^S_BSS = 2c K p^-1 (U_0^B - U_0^A X'') R'' K^-1 and the block's own
 * V, T, W (the same matrix as K^-H R''^H [E + O X'' + X''^H O^H +
 * X''^H E' X''] R'' K^-1, E = E_1 + E_0 - c^2, E' = E_1' - E_0 - c^2).  H^0
 * goes through the eigen-solve that x2c_build_batched applies to its reduced
 * 4c matrix; eps are its positive-energy eigenvalues.
 * Arguments, layout, per-block info and eps (the same positive-energy
 * eigenvalues) as x2c_build_batched; workspace from x2c_bss_workspace_bytes.
 * opts->prec must be X2C_FP64 and, two-component, opts->reduction
 * X2C_RED_QUATERNION (else X2C_EINVAL).  Stream-ordered.
 */
size_t x2c_bss_workspace_bytes(const x2c_options* opts, int nblk, const int* N);
int x2c_bss_batched(const x2c_options* opts, int nblk, const int* N, const int64_t* in_off, const double* S,
                    const double* T, const double* V, const double* W, const int64_t* h_off, void* h,
                    const int64_t* eps_off, double* eps, int* info, void* workspace, size_t ws_bytes, void* stream);

/*
 * DKHn one-electron Hamiltonian of a batch (Sec. II, "The DKH approach",
 * Eq. dkhtrans and Table I): the fpFW Hamiltonian H^0 above is transformed
 * by U_k = exp(W_k), k = 1, 2, ... (exponential parametrisation), W_k the odd
 * anti-Hermitian operator with (W_k)_ij = (O_k)_ij / (E_0i + E_0j) that
 * removes the odd term of order k; h is the electronic block of the even
 * terms through order `order` in the potential, E_0 - c^2 + E_1 + ... + E_n,
 * back-transformed by K^-1.  Products that do not reach that block are
 * skipped (x2c_dkh_products gives their number).
 *   order    1 .. 14.
 *   h        as x2c_build_batched (no eigenvalues are computed).
 * Other arguments as x2c_build_batched; workspace from
 * x2c_dkh_workspace_bytes.  opts->prec must be X2C_FP64 (else X2C_EINVAL);
 * opts->reduction is ignored.  Stream-ordered.
 */
size_t x2c_dkh_workspace_bytes(const x2c_options* opts, int order, int nblk, const int* N);
int x2c_dkh_batched(const x2c_options* opts, int order, int nblk, const int* N, const int64_t* in_off,
                    const double* S, const double* T, const double* V, const double* W, const int64_t* h_off, void* h,
                    int* info, void* workspace, size_t ws_bytes, void* stream);

/* Number of 2c matrix multiplications x2c_dkh_batched performs per block
 * for DKH of the given order (P(n) of Table I), or -1 for an order outside
 * 1 .. 14.  Host only. */
int x2c_dkh_products(int order);

/*
 * Picture-change transformation of one-electron property operators with
 * the blocks' decoupling (Sec. II: U^L and U^S are needed for the picture
 * change of property integrals; U^L_bb = R_b, U^S_bb = X_b R_b, Eqs.
 * ulnonortho, usnonortho).  For a property whose matrix in the basis of
 * the modified Dirac equation (Eq. moddiraceq: large components chi, small
 * components sigma.p chi / 2c) is [[P_LL, P_LS], [P_SL, P_SS]], Eq. utrans
 * with that matrix in place of D gives
 *   P~_b = R^H [ P_LL + P_LS X + X^H P_SL + X^H P_SS X ] R.
 * (A multiplicative operator O has P_LL = O, P_LS = P_SL = 0 and
 * P_SS = W^O / 4c^2 with W^O built from <sigma.p chi|O|sigma.p chi> as in
 * Eq. defw; the Hamiltonian itself is the case D.)
 *   N, p_off host, nblk scalar sizes and double offsets of block b's
 *            n_b x n_b matrices (n_b = N_b spin-free, 2 N_b two-component,
 *            float64 or complex128 row-major), e.g. the h_off of
 *            x2c_build_batched_xr.  The same offsets address PLL, PLS, PSL,
 *            PSS, X, R and out.
 *   PLL, PLS, PSL, PSS  device property blocks; PLS and PSL may be NULL
 *            (zero blocks).
 *   X, R     device, the blocks' decoupling matrices.
 *   out      device output, same layout.
 * The workspace is that of x2c_build_batched for the same blocks (size from
 * x2c_workspace_bytes).  Stream-ordered.  Returns X2C_OK once enqueued,
 * X2C_EINVAL (NULL pointer, N out of range, workspace too small) or
 * X2C_EHIP.  opts->prec and opts->reduction are ignored (FP64 products).
 */
int x2c_picture_change(const x2c_options* opts, int nblk, const int* N, const int64_t* p_off, const double* PLL,
                       const double* PLS, const double* PSL, const double* PSS, const void* X, const void* R,
                       void* out, void* workspace, size_t ws_bytes, void* stream);

/*
 * x2c_picture_change for time-even operators of two-component blocks (the
 * same arguments, layout, workspace and return codes; opts->mode must be
 * X2C_TWOCOMP).  Every two-component matrix of the method has the
 * time-reversal form [[A, B], [-B*, A*]] in the [all alpha; all beta] basis
 * (Sec. III.A, Kramers pairs); so has a time-even property's matrix, e.g.
 * any spin-free multiplicative operator and its W^O (Eq. defw with O in
 * place of V).  The five products then run on the quaternion N x N forms
 * A + B j: half the real multiply-adds of x2c_picture_change.  Only the
 * first N rows (the blocks A and B) of PLL, PLS, PSL, PSS, X and R are read,
 * and out is written whole in that form; a time-odd operator (one whose
 * matrix lacks the form, e.g. a magnetic one) gives a wrong result, which is
 * not detected: use x2c_picture_change for it.
 */
int x2c_picture_change_kramers(const x2c_options* opts, int nblk, const int* N, const int64_t* p_off,
                               const double* PLL, const double* PLS, const double* PSL, const double* PSS,
                               const void* X, const void* R, void* out, void* workspace, size_t ws_bytes,
                               void* stream);

/*
 * Workspace size in bytes for x2c_dlu_assemble with `natom` atoms of scalar
 * sizes N[0..natom) (host).  0 for invalid arguments.
 */
size_t x2c_dlu_workspace_bytes(const x2c_options* opts, int natom, const int* N);

/*
 * Molecular one-electron Hamiltonian in the DLU approximation (Sec. III.A):
 * U^L and U^S are the direct sums of the atoms' R_A and X_A R_A (Eqs.
 * dlutrans, r2ctransatom), and Eq. utrans is applied with the full molecular
 * matrices, pair by pair:
 *   h_AB = R_A^H [V_AB + T_AB X_B + X_A^H T_AB + X_A^H (W_AB/4c^2 - T_AB) X_B] R_B.
 * Stream-ordered (does not synchronise).
 *   N        host, natom scalar sizes; atom A's functions are molecular
 *            scalar indices off_A .. off_A + N[A], off_A = N[0] + .. + N[A-1];
 *            Ntot = sum of N.
 *   T, V     molecular Ntot x Ntot (device, row-major float64).
 *   W        spin-free: W^0 (Ntot x Ntot); two-component: W^0, W^x, W^y, W^z
 *            contiguous (4 x Ntot x Ntot) (device).
 *   u_off    host, natom double offsets of X_A and R_A in X and R (even in
 *            two-component mode), e.g. the h_off of x2c_build_batched_xr.
 *   X, R     device, the atoms' decoupling matrices (n_A x n_A each).
 *   H        output (device): spin-free Ntot x Ntot float64; two-component
 *            2Ntot x 2Ntot complex128 in the molecular spin-orbital order
 *            [all alpha; all beta].  Every entry is written.
 * The caller owns every buffer; the workspace holds the atom-pair products.
 * Returns X2C_OK once enqueued, X2C_EINVAL (NULL pointer, N[A] out of range,
 * odd u_off in two-component mode, workspace too small) or X2C_EHIP.
 */
int x2c_dlu_assemble(const x2c_options* opts, int natom, const int* N, const double* T, const double* V,
                     const double* W, const int64_t* u_off, const void* X, const void* R, void* H,
                     void* workspace, size_t ws_bytes, void* stream);

/* Static description of a return or info code. */
const char* x2c_strerror(int code);

/* Drop cached launch plans, captured graphs, tuned launch shapes held in
 * memory and trace events. */
void x2c_release(void);

/*
 * Graph replay of x2c_build / x2c_build_batched / x2c_build_batched_xr
 * (library infrastructure: all blocks of a batch advance stage by stage).  When
 * on (the default), the first call with a given combination of block sizes,
 * offsets, options and device pointers captures its whole launch sequence
 * into a HIP graph (on a private stream of the library); later calls with the
 * same combination replay that graph on the caller's stream.  Results are
 * identical either way.  Calls made while tracing is enabled run eagerly.
 * Returns the previous setting.
 */
int x2c_graph_enable(int on);

/*
 * Multi-stream execution of a batch (library infrastructure; the per-block
 * problems are independent).  ways in 2..4 (default 4): a call with two or more blocks
 * cuts the batch into min(ways, blocks) parts of about equal work (sum of
 * N^3); the first part runs on the caller's stream, the others on auxiliary
 * streams of the library, forked from and joined back into the caller's
 * stream with events (captured graphs contain every branch).  ways = 1: one
 * stream.  Results are identical either way; calls made while tracing is
 * enabled use one stream.  Other values leave the setting unchanged.  A
 * batch class tuned by x2c_autotune uses its tuned split instead.
 * Returns the previous setting.
 */
int x2c_stream_split(int ways);

/* The launch shape calls with these options and block sizes would use:
 * returns 1 and the tuned shape when x2c_autotune (in this process or, via
 * the cache file, an earlier one on the same GPU architecture) has tuned the
 * class, 0 and the defaults otherwise, X2C_EINVAL for bad arguments.
 * *ways_out / *mv_res_out may be NULL. */
int x2c_tuned_shape(const x2c_options* opts, int nblk, const int* N, int* ways_out, int* mv_res_out);

/*
 * Autotuning of the launch shape of a batch class (library infrastructure).
 * Runs x2c_build_batched on the caller's batch (same arguments, same
 * outputs written) once untimed and `reps` times timed, for every candidate
 * shape: the batch split over 1..4 streams (as x2c_stream_split) times 4 or 8
 * resident work-groups per CU for the persistent matvec of the quaternion
 * reductions.  The fastest (HIP events on `stream`, summed over the reps) is
 * kept for every later call with the same options and block sizes N[] and
 * written to *ways_out and *mv_res_out (either may be NULL); batches of other
 * classes keep x2c_stream_split's setting and 8 work-groups per CU.  The
 * shape is also appended to a cache file keyed by the GPU architecture and
 * the batch class (X2C_TUNE_CACHE if set, an empty value disabling it; else
 * $XDG_CACHE_HOME/libx2c/tune_v1.txt or ~/.cache/libx2c/tune_v1.txt), from
 * which later processes take it.  With X2C_ROUTE_AUTO the shapes are
 * searched on the size route and the device-wide route is then timed
 * against the best of them; the faster route is kept (and cached) for the
 * class, and the outputs written are those of that route.  All launch-shape
 * candidates give identical results.  Blocking: synchronises `stream` once
 * per candidate.  Returns X2C_OK, X2C_EINVAL (arguments as for
 * x2c_build_batched; reps outside 1..100) or X2C_EHIP, in which case the
 * class's previous shape is kept.  Run it with tracing disabled (traced calls
 * use one stream).  x2c_release() forgets the tuned shapes held in
 * memory (the cache file is read again on the next call).
 */
int x2c_autotune(const x2c_options* opts, int nblk, const int* N, const int64_t* in_off, const double* S,
                 const double* T, const double* V, const double* W, const int64_t* h_off, void* h,
                 const int64_t* eps_off, double* eps, int* info, void* workspace, size_t ws_bytes, void* stream,
                 int reps, int* ways_out, int* mv_res_out);

/*
 * Tracing.  x2c_trace_enable(1) makes every later call bracket each of its
 * stages with a pair of HIP events recorded on the call's stream (no device
 * memory is allocated); level 2 also brackets every launch of the
 * tridiagonal-reduction matvec kernel (entry "k_tri_matvec").
 * x2c_trace_enable returns the previous level.
 * x2c_trace_read waits for the recorded events, folds them into per-stage
 * totals and returns the number of stages seen; for 0 <= idx < that number
 * it stores the stage name (static until x2c_trace_reset), the summed
 * device time in ms and the number of calls.  x2c_trace_reset clears the
 * totals.
 */
int x2c_trace_enable(int on);
int x2c_trace_read(int idx, const char** name, double* total_ms, long long* count);
void x2c_trace_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* X2C_H */
