// Host-side launchers of the X2C kernels (internal to libx2c).
#pragma once
#include <hip/hip_runtime.h>

#include "x2c_device.h"

namespace x2c {

// Optional per-launch timing of selected kernels (no-ops unless the library
// trace is enabled at level 2).
// per-launch timing of selected kernels (trace level 2): a pair of events
// for the launch to record at the kernel's own start and end
// (hipExtLaunchKernel), so that launch latency is not counted; both null
// when tracing is off.  ktrace_end files the pair after the launch.
void* ktrace_begin(const char* name, hipEvent_t* start, hipEvent_t* stop);
void ktrace_end(void* h);

void launch_init_info(hipStream_t s, int* info, int nblk);
void launch_scatter_info(hipStream_t s, const BlockDesc* D, const int* iw, int* info, int nblk);
void launch_unpack(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN, const double* S,
                   const double* T, const double* V, const double* W, int twocomp);
void launch_potrf(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN);
void launch_trtri(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN);
template <class T>
void launch_expand(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double c);
template <class T>
void launch_assemble_A(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxm, double c);
template <class T>
void launch_copy(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                 int src, int dst);
template <class T>
void launch_add_herm(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, int src,
                     int dst);
template <class T>
void launch_conj_transpose(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn,
                           int src, int dst);
template <class T>
void launch_write_h(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double* h,
                    double* eps);

// herm = 1: the product is Hermitian (and so is beta C); only the lower
// triangle is computed and mirrored
template <class T>
void launch_gemm(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                 int bufA, int opA, int bufB, int opB, int bufC, T alpha, T beta, int herm = 0, int tri = 0);

// split-precision products (bf16 or int8 slices); T = double, cplx or quat;
// real alpha, beta; herm = 1: Hermitian product (lower tiles, mirrored)
template <class T>
void launch_gemm_split(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                       int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta, int slices,
                       int herm = 0);

template <class T>
void launch_gemm_split_i8(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim,
                          int dsel, int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta,
                          int slices, int herm = 0);

template <class T>
void launch_hetrd(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                  int bufA, int bufD, int bufE, int bufTau);

template <class T>
void launch_hetrd_mk(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                     int bufA, int bufD, int bufE, int bufTau, int bufW, int bufV, int bufHS, int bufET,
                     int mv_res = 8);
template <class T>
void launch_ormtr_blocked(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim,
                          int maxcols, int dsel, int bufA, int bufTau, int bufTf, int bufY, int csel);

void launch_tri_eig4c(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxm, double* eps,
                      double c, int kramers);
void launch_filter_factor(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int kramers,
                          int maxm_filter);
template <class T>
void launch_filter_solve(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxrhs,
                         int kramers);
void launch_tri_eig_q(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxdim, int dsel);
template <class T>
void launch_invsqrt_cols(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                         int bufScr);

void launch_assemble_Aq(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double c);
void launch_phase_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int dsel);
void launch_cplx_to_quat(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                         int dst);
void launch_expand_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, double c);
void launch_eye_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int buf);
void launch_write_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, double* out,
                    int buf, double* eps);
void launch_read_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, const double* in,
                   int buf);
void launch_gemm_qr(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int side,
                    int bufR, int opR, int tri, int bufQ, int bufC, double alpha, double beta, int herm);
void launch_gemm_q(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                   int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta, int herm);
void launch_quat_to_cplx(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                         int dst);
void launch_qct_scale(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int src,
                      int dst);

template <class T>
void launch_write_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, double* out,
                      int buf);
template <class T>
void launch_read_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn,
                     const double* in, int buf);
template <class T>
void launch_add_buf(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxn, int src,
                    int dst);
template <class T>
void launch_dlu(hipStream_t s, const DluPair* P, int npairs, int maxnA, int maxnB, char* ws, const double* Tm,
                const double* Vm, const double* Wm, int Ntot, double c, const double* X, const double* R, double* H);

// X~ = Y_S Y_L^-1 for the (2 dim) x dim matrix Y in bufY (dim selected by
// dsel), result (dim x dim) in bufX
template <class T>
void launch_xsolve_blk(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxn, int bufY, int dsel,
                       int bufX);

// free-particle FW bases of BSS and DKHn (k_fw.hip)
void launch_tri_steqr(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxdim, int dsel,
                      int bufD, int bufE, int bufZT, int bufZ);
void launch_fpfw_vectors(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int bufD, int bufFP,
                         double c);
template <class T>
void launch_fpfw_assemble(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufV,
                          int bufW0, int bufFP, int bufE1, int bufO1, int bufE1p);
template <class T>
void launch_dkh_wgen(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufO,
                     int bufW, int bufFP);
template <class T>
void launch_combine(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufDst,
                    int bufSrc, double a, double bs, double bh);
template <class T>
void launch_add_diag(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufDst,
                     int bufSrc, int bufFP, int k1, double s1, double s0);
template <class T>
void launch_bss_ab(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufX2,
                   int bufFP, int bufA, int bufB, double c);
template <class T>
void launch_bss_h0(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxN, int bufE1,
                   int bufO1, int bufE1p, int bufFP, int bufA, double c);

// device-wide path of the large blocks (k_large.hip), nblk blocks from
// descriptor D on; info and gate point to their status words and iteration
// gates (nblk ints each); maxN, maxdim* are the largest dimensions among them
void launch_large_cholesky(hipStream_t s, const BlockDesc* D, char* ws, int* info, int nblk, int maxN);
// sign(A + c^2 I) of the 4c matrix in bufX (selector dsel4), in place;
// bufU, bufN: 4c-sized scratch
template <class T>
void launch_large_sign(hipStream_t s, const BlockDesc* D, char* ws, int* info, int* gate, int nblk, int dsel4,
                       int maxdim4, int bufX, int bufU, int bufN, double c, int maxit, double tol);
// X~ = P_SL P_LL^-1 into bufXt and Q^-1/2 = P_LL^(1/2) into bufQmh from one
// coupled iteration on P_LL (the converged sign in bufX)
template <class T>
void launch_large_xrenorm(hipStream_t s, const BlockDesc* D, char* ws, int* info, int* gate, int nblk, int dsel4,
                          int dselh, int maxdimh, int bufX, int bufPSL, int bufZ, int bufU, int bufN, int bufXt,
                          int bufQmh, int maxit, double tol);
void launch_eps_nan(hipStream_t s, const BlockDesc* D, double* eps, int nblk);

}  // namespace x2c
