// Split-precision GEMM for the X / L / S~ / R product chain:
//   C_b = alpha op(A_b) op(B_b) + beta C_b  (op in {N, H}, n_b x n_b, batched)
// with FP64 accuracy emulated on bf16 matrix cores (Ozaki-type error-free
// splitting).
//
// Every row i of op(A) is scaled by 2^-ea_i (ea_i = binary exponent of the
// row's largest |entry|, so the scaled row lies in (-1, 1)) and cut into S
// slices of 7 bits: y <- 128 y, q_s = rint(y), y <- y - q_s, so that
// row = 2^ea_i sum_s 2^-7s q_s up to 2^(ea_i - 7S - 1).  Columns of op(B)
// are cut the same way with their own exponents.  Every q_s is an integer of
// magnitude <= 128, exact in bf16, so each bf16 product q_a q_b is exact and
// a sum of up to 2^24 / (S 2^14) such products is exact in the FP32
// accumulator of the matrix core.  With the slices numbered s = 1..S
// (weight 2^-7s; |slice 1| <= 1, |slice s| <= 2^(6-7s) after it), slice pairs
// (a, b) with a + b = g share the weight 2^-7g; the pairs with g <= S + 1
// are kept (in the 0-based loop indices: sa + sb <= S - 1), accumulated
// exactly per g over 128 terms of the inner dimension and folded into FP64
// accumulators, which carry the result.  The dropped pairs (g >= S + 2) add
// at most about (S - 1) 2^(-7S) per inner-dimension term, relative to the
// product of the row and column maxima: the size of the operands' own
// truncation.  Rounding therefore only happens in FP64.
//
// Complex and quaternion operands use the real form with interleaved
// components (F = 2: Re, Im; F = 4: Re a, Im a, Re b, Im b of q = a + b j):
//   A'[F i + c][F k + d] = sigma(c, d) a_ik[c xor d],   B'[F k + d][j] = b_kj[d],
// with sigma the sign pattern of the quaternion product ((x y)_c =
// sum_d sigma(c, d) x_{c xor d} y_d, which restricted to c, d < 2 is the
// complex product), so that (A'B')_{F i + c, j} = component c of (AB)_ij; a
// row exponent covers all components of a row.  herm = 1: the product is
// Hermitian (and so is beta C): only tiles reaching the lower triangle run,
// and each lower element is mirrored.
//
// Tiling (gfx950): 256 threads = 4 waves; the work-group covers 64 rows of
// A' x 64 columns, each wave one 32 x 32 MFMA block (v_mfma_f32_32x32x16_bf16);
// two work-groups fit a CU, so one stages its chunk while the other
// multiplies.  The FP64 tiles are split on the fly into LDS
// (all S slices of a 32-deep k chunk), so HBM traffic equals that of the
// plain FP64 GEMM.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float floatx16;

constexpr int OZ_M = 64, OZ_N = 64, OZ_KC = 32, OZ_LD = OZ_KC + 8;
constexpr int OZ_FLUSH = 4;     // k chunks between folds into FP64 (128 terms)

// binary exponent of the largest |entry| of each row (rows = 1) or column of a
// T-typed n x n matrix; one wave per line.  grid = (ceil(n / 4), nblk)
template <class T>
__global__ void __launch_bounds__(256) k_line_exp(const BlockDesc* D, char* ws, const int* info, int dsel, int buf,
                                                  int rows, int bufE) {
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int line = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (line >= n) return;
  const T* A = bufp<T>(ws, d, buf);
  double mx = 0.0;
  for (int k = lane; k < n; k += 64) mx = fmax(mx, amax(rows ? A[(long long)line * n + k] : A[(long long)k * n + line]));
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) {
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);     // mx < 2^e
    bufp<int>(ws, d, bufE)[line] = e;
  }
}

template <int S>
__device__ inline void split_slices(double x, double scale, __bf16* q) {
  double y = x * scale;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    y *= 128.0;
    const double r = rint(y);
    y -= r;
    q[s] = (__bf16)(float)r;
  }
}

// RF bf16 values to consecutive LDS entries (one store)
template <int RF>
__device__ inline void store_bf(__bf16* p, const __bf16* v) {
  if constexpr (RF == 1) {
    p[0] = v[0];
  } else {
    unsigned int w[RF / 2];
#pragma unroll
    for (int i = 0; i < RF / 2; ++i)
      w[i] = (unsigned int)__builtin_bit_cast(unsigned short, v[2 * i]) |
             ((unsigned int)__builtin_bit_cast(unsigned short, v[2 * i + 1]) << 16);
    if constexpr (RF == 2) *reinterpret_cast<unsigned int*>(p) = w[0];
    else *reinterpret_cast<uint2*>(p) = uint2{w[0], w[1]};
  }
}

template <class T>
__device__ inline T from_comps(const double* v) {
  if constexpr (ncomp<T>() == 1) return v[0];
  else if constexpr (ncomp<T>() == 2) return cplx{v[0], v[1]};
  else return quat{{v[0], v[1]}, {v[2], v[3]}};
}

template <class T, int S>
__global__ void __launch_bounds__(256, 2) k_gemm_split(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                    int bufA, int opA, int bufB, int opB, int bufC, double alpha,
                                                    double beta, int herm, int bufEA, int bufEB) {
  constexpr int RF = ncomp<T>();            // real rows / k per element
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int Mr = RF * n;
  const int m0 = blockIdx.y * OZ_M, n0 = blockIdx.x * OZ_N;   // m0 in rows of A', n0 in columns
  if (m0 >= Mr || n0 >= n) return;
  if (herm && n0 > (m0 + OZ_M) / RF - 1) return;   // tile above the diagonal
  const T* A = bufp<T>(ws, d, bufA);
  const T* B = bufp<T>(ws, d, bufB);
  T* C = bufp<T>(ws, d, bufC);
  const int* ea = bufp<int>(ws, d, bufEA);
  const int* eb = bufp<int>(ws, d, bufEB);

  extern __shared__ __attribute__((aligned(16))) __bf16 oz_sm[];
  __bf16* As = oz_sm;                          // S x OZ_M x OZ_LD
  __bf16* Bs = oz_sm + S * OZ_M * OZ_LD;       // S x OZ_N x OZ_LD
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);   // this wave's 32 x 32 output block

  floatx16 acc[S];
  double acc64[16];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[g][j] = 0.0f;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc64[j] = 0.0;

  // elements of op(A) per chunk: (OZ_M / RF) rows x (OZ_KC / RF) k
  constexpr int AR = OZ_M / RF, AK = OZ_KC / RF, BK = OZ_KC / RF;
  const int Kr = RF * n;
  const int nchunks = (Kr + OZ_KC - 1) / OZ_KC;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int k0 = ch * AK;                   // first element-k of the chunk
    // ---- split op(A) chunk into LDS
#pragma unroll 1
    for (int e = t; e < AR * AK; e += 256) {
      int r, kk;
      if (opA == 0) { r = e / AK; kk = e % AK; } else { kk = e / AR; r = e % AR; }
      const int gi = m0 / RF + r, gk = k0 + kk;
      T v = tzero<T>();
      if (gi < n && gk < n) v = opA == 0 ? A[(long long)gi * n + gk] : conjg(A[(long long)gk * n + gi]);
      const double sc = gi < n ? ldexp(1.0, -ea[gi]) : 0.0;
      __bf16 q[RF][S];
#pragma unroll
      for (int c = 0; c < RF; ++c) split_slices<S>(comp(v, c), sc, q[c]);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int c = 0; c < RF; ++c) {
          __bf16 row[RF];
#pragma unroll
          for (int dd = 0; dd < RF; ++dd) row[dd] = qmul_sign(c, dd) > 0 ? q[c ^ dd][s] : -q[c ^ dd][s];
          store_bf<RF>(As + (s * OZ_M + RF * r + c) * OZ_LD + RF * kk, row);
        }
    }
    // ---- split op(B) chunk into LDS (stored column-major: [col][k])
#pragma unroll 1
    for (int e = t; e < BK * OZ_N; e += 256) {
      int c, kk;
      if (opB == 0) { kk = e / OZ_N; c = e % OZ_N; } else { c = e / BK; kk = e % BK; }
      const int gk = k0 + kk, gj = n0 + c;
      T v = tzero<T>();
      if (gk < n && gj < n) v = opB == 0 ? B[(long long)gk * n + gj] : conjg(B[(long long)gj * n + gk]);
      const double sc = gj < n ? ldexp(1.0, -eb[gj]) : 0.0;
      __bf16 q[RF][S];
#pragma unroll
      for (int cc = 0; cc < RF; ++cc) split_slices<S>(comp(v, cc), sc, q[cc]);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        __bf16 col[RF];
#pragma unroll
        for (int dd = 0; dd < RF; ++dd) col[dd] = q[dd][s];
        store_bf<RF>(Bs + (s * OZ_N + c) * OZ_LD + RF * kk, col);
      }
    }
    __syncthreads();
    // ---- slice-pair products on the matrix cores
#pragma unroll
    for (int ks = 0; ks < OZ_KC / 16; ++ks) {
      bf16x8 af[S];
#pragma unroll
      for (int s = 0; s < S; ++s)
        af[s] = *reinterpret_cast<const bf16x8*>(As + (s * OZ_M + wr + l32) * OZ_LD + 16 * ks + 8 * lhi);
#pragma unroll
      for (int sb = 0; sb < S; ++sb) {
        const bf16x8 bf = *reinterpret_cast<const bf16x8*>(Bs + (sb * OZ_N + wc + l32) * OZ_LD + 16 * ks + 8 * lhi);
#pragma unroll
        for (int sa = 0; sa < S - sb; ++sa)
          acc[sa + sb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[sa], bf, acc[sa + sb], 0, 0, 0);
      }
    }
    __syncthreads();
    // ---- fold the exact FP32 group sums into FP64 (smallest weights first)
    if ((ch + 1) % OZ_FLUSH == 0 || ch + 1 == nchunks) {
#pragma unroll
      for (int g = S - 1; g >= 0; --g) {
        const double w = ldexp(1.0, -7 * (g + 2));
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          acc64[j] = fma((double)acc[g][j], w, acc64[j]);
          acc[g][j] = 0.0f;
        }
      }
    }
  }
  // ---- epilogue: undo the exponents, C = alpha P + beta C (real alpha, beta)
  {
    const int col = n0 + wc + l32;
    if (col >= n) return;
#pragma unroll
    for (int j = 0; j < 16; j += RF) {
      const int rr = m0 + wr + 8 * (j / 4) + 4 * lhi + (j % 4);   // row of A'
      const int i = rr / RF;
      if (i >= n || (herm && col > i)) continue;
      const double sc = ldexp(1.0, ea[i] + eb[col]);
      double vals[RF];
#pragma unroll
      for (int c = 0; c < RF; ++c) vals[c] = acc64[j + c] * sc;
      const long long idx = (long long)i * n + col;
      T v = alpha * from_comps<T>(vals);
      if (beta != 0.0) v = v + beta * C[idx];
      C[idx] = v;
      if (herm && col < i) C[(long long)col * n + i] = conjg(v);
    }
  }
}

template <class T, int S>
static void launch_split_s(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim,
                           int dsel, int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta,
                           int herm) {
  constexpr int RF = ncomp<T>();
  const size_t shm = (size_t)S * (OZ_M + OZ_N) * OZ_LD * sizeof(__bf16);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_split<T, S>), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  dim3 grid((maxdim + OZ_N - 1) / OZ_N, (RF * maxdim + OZ_M - 1) / OZ_M, nblk);
  hipLaunchKernelGGL((k_gemm_split<T, S>), grid, dim3(256), shm, s, D, ws, info, dsel, bufA, opA, bufB, opB, bufC,
                     alpha, beta, herm, (int)V_EXA, (int)V_EXB);
}

template <class T>
void launch_gemm_split(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                       int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta, int slices,
                       int herm) {
  const dim3 lg((maxdim + 3) / 4, nblk);
  hipLaunchKernelGGL(k_line_exp<T>, lg, dim3(256), 0, s, D, ws, info, dsel, bufA, opA == 0 ? 1 : 0, (int)V_EXA);
  hipLaunchKernelGGL(k_line_exp<T>, lg, dim3(256), 0, s, D, ws, info, dsel, bufB, opB == 0 ? 0 : 1, (int)V_EXB);
  switch (slices) {
    case 1: launch_split_s<T, 1>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 2: launch_split_s<T, 2>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 3: launch_split_s<T, 3>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 4: launch_split_s<T, 4>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 5: launch_split_s<T, 5>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 6: launch_split_s<T, 6>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    case 7: launch_split_s<T, 7>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
    default: launch_split_s<T, 8>(s, D, ws, info, nblk, maxdim, dsel, bufA, opA, bufB, opB, bufC, alpha, beta, herm); break;
  }
}

template void launch_gemm_split<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                        int, int, int, double, double, int, int);
template void launch_gemm_split<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                      int, int, double, double, int, int);
template void launch_gemm_split<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                      int, int, double, double, int, int);

}  // namespace x2c
