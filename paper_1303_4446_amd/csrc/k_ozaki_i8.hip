// Split-precision products on the int8 matrix cores.
//
// Same error-free splitting as the bf16 variant, with 8-bit integer slices
// and exact int32 accumulation: every row i of op(A) (column j of op(B)) is
// scaled by 2^-e (e = binary exponent of the line's largest |entry| plus one,
// so the scaled line lies in (-1/2, 1/2)) and cut into S slices
// y <- 128 y, q_s = rint(y), y <- y - q_s, |q_s| <= 64.  The operands are
// split once per product into int8 arrays (K contiguous, K padded to 64);
// the product kernel forms every slice pair (a, b) with a + b = g <= S + 1
// (slices numbered s = 1..S, weight 2^-7s; in the 0-based loop indices
// sa + sb <= S - 1) on v_mfma_i32_32x32x32_i8, one int32 accumulator per g
// (|sum| <= S K 2^12, exact for K < 2^16), and folds them into FP64 at the
// end.  The dropped pairs (g >= S + 2) add at most about (S - 1) 2^(-7S - 2)
// per inner-dimension term relative to the product of the line maxima, the
// size of the operands' own truncation.
//
// Complex and quaternion operands (F = 2, 4 real components): the real form
// has rows F i + c and a K axis of F parts (part d holds component d of
// every k):
//   A'[F i + c] over part d = sigma(c, d) (component c xor d of row i of A),
//   B'[:, j] over part d = component d of column j of B,
// with sigma the sign pattern of the quaternion product (restricted to
// c, d < 2 it is the complex product), so (A'B')_{F i + c, j} = component c
// of (AB)_ij.  The split stores the F component slices of each line once;
// the product kernel builds A' while staging (choosing the component and
// negating bytes where sigma is -1).  herm = 1: Hermitian product, only the
// tiles reaching the lower triangle run and each lower element is mirrored.
#include "x2c_device.h"
#include "x2c_launch.h"

namespace x2c {

typedef __attribute__((ext_vector_type(4))) int i4;
typedef __attribute__((ext_vector_type(16))) int i16;

constexpr int Q8_KC = 64;                  // k chunk (bytes of a slice row)
constexpr int Q8_M = 64, Q8_N = 64;        // rows of A' x columns per work-group (2 x 2 waves of 32 x 32)
constexpr int Q8_LD = Q8_KC + 16;          // LDS row stride in bytes

__host__ __device__ inline int kpad64(int n) { return (n + 63) / 64 * 64; }

// Split the lines of op(X) (side 0: rows of op(A); side 1: columns of op(B))
// into S int8 slices: out[s][part][line][k], part = 0 (Re), 1 (Im, complex
// only), k < kpad64(n) (zero padded); exponent per line in bufE.  One wave
// per line.  grid = (ceil(n / 4), nblk)
template <class T>
__global__ void __launch_bounds__(256) k_split_i8(const BlockDesc* D, char* ws, const int* info, int dsel, int buf,
                                                  int op, int side, int S, int bufOut, int bufE) {
  constexpr int parts = ncomp<T>();
  const int b = blockIdx.y;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int line = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (line >= n) return;
  const T* X = bufp<T>(ws, d, buf);
  // element k of the line: side 0 -> op(A)[line][k]; side 1 -> op(B)[k][line]
  // op N: A[line][k] / B[k][line];  op H: conj(A[k][line]) / conj(B[line][k])
  const bool contiguous = (side == 0) == (op == 0);
  auto elem = [&](int k) -> T {
    const T v = contiguous ? X[(long long)line * n + k] : X[(long long)k * n + line];
    return op == 0 ? v : conjg(v);
  };
  double mx = 0.0;
  for (int k = lane; k < n; k += 64) mx = fmax(mx, amax(elem(k)));
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  int e = 0;
  if (mx > 0.0) frexp(mx, &e);
  e += 1;                                   // scaled line in (-1/2, 1/2)
  if (lane == 0) bufp<int>(ws, d, bufE)[line] = e;
  const double sc = ldexp(1.0, -e);
  const int kp = kpad64(n);
  const long long plane = (long long)n * kp;          // one part of one slice
  signed char* out = bufp<signed char>(ws, d, bufOut);
  for (int k = lane; k < kp; k += 64) {
    const T v = k < n ? elem(k) : tzero<T>();
    for (int p = 0; p < parts; ++p) {
      double y = comp(v, p) * sc;
      for (int s = 0; s < S; ++s) {
        y *= 128.0;
        const double r = rint(y);
        y -= r;
        out[((long long)s * parts + p) * plane + (long long)line * kp + k] = (signed char)(int)r;
      }
    }
  }
}

// bytewise negation of four packed int8 values (|x| <= 64, no overflow)
__device__ inline int neg_bytes(int x) {
  const int y = ~x;
  return ((y & 0x7F7F7F7F) + 0x01010101) ^ (y & 0x80808080);
}

template <class T>
__device__ inline T from_comps_i8(const double* v) {
  if constexpr (ncomp<T>() == 1) return v[0];
  else if constexpr (ncomp<T>() == 2) return cplx{v[0], v[1]};
  else return quat{{v[0], v[1]}, {v[2], v[3]}};
}

template <class T, int S>
__global__ void __launch_bounds__(256, 2) k_gemm_i8(const BlockDesc* D, char* ws, const int* info, int dsel, int bufC,
                                                 double alpha, double beta, int herm, int bufSA, int bufSB, int bufEA,
                                                 int bufEB) {
  constexpr int RF = ncomp<T>();
  const int b = blockIdx.z;
  const BlockDesc& d = D[b];
  if (info[b]) return;
  const int n = seldim(d, dsel);
  const int Mr = RF * n;
  const int m0 = blockIdx.y * Q8_M, n0 = blockIdx.x * Q8_N;   // m0: rows of A'
  if (m0 >= Mr || n0 >= n) return;
  if (herm && n0 > (m0 + Q8_M) / RF - 1) return;   // tile above the diagonal
  const int kp = kpad64(n);
  const long long plane = (long long)n * kp;
  const signed char* SA = bufp<signed char>(ws, d, bufSA);
  const signed char* SB = bufp<signed char>(ws, d, bufSB);
  const int* ea = bufp<int>(ws, d, bufEA);
  const int* eb = bufp<int>(ws, d, bufEB);
  T* C = bufp<T>(ws, d, bufC);

  extern __shared__ __attribute__((aligned(16))) signed char q8_sm[];
  signed char* As = q8_sm;                              // S x Q8_M x Q8_LD
  signed char* Bs = q8_sm + S * Q8_M * Q8_LD;           // S x Q8_N x Q8_LD
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);   // this wave's 32 x 32 output block

  i16 acc[S];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[g][j] = 0;

  const int nk = RF * kp / Q8_KC;            // chunks over the RF-part K axis
  for (int ch = 0; ch < nk; ++ch) {
    const int half = (ch * Q8_KC) / kp;      // K part: the component of B'
    const int kc = ch * Q8_KC - half * kp;   // offset inside the part
    // ---- stage A' rows (16-byte pieces: 4 per row per slice)
    for (int e = t; e < S * Q8_M * 4; e += 256) {
      const int s = e / (Q8_M * 4), rem = e % (Q8_M * 4), rr = rem / 4, piece = rem % 4;
      const int grow = m0 + rr;                 // row of A'
      i4 v = {0, 0, 0, 0};
      if (grow < Mr) {
        const int i = grow / RF, cc = grow % RF;
        // row component cc over K part `half`: component cc xor half of A,
        // negated where the product's sign pattern is -1
        const int part = cc ^ half;
        const bool neg = qmul_sign(cc, half) < 0;
        const signed char* src = SA + ((long long)s * RF + part) * plane + (long long)i * kp + kc + 16 * piece;
        v = *reinterpret_cast<const i4*>(src);
        if (neg) {
#pragma unroll
          for (int w = 0; w < 4; ++w) v[w] = neg_bytes(v[w]);
        }
      }
      *reinterpret_cast<i4*>(As + (s * Q8_M + rr) * Q8_LD + 16 * piece) = v;
    }
    // ---- stage B' columns (K contiguous)
    for (int e = t; e < S * Q8_N * 4; e += 256) {
      const int s = e / (Q8_N * 4), rem = e % (Q8_N * 4), cc = rem / 4, piece = rem % 4;
      const int gcol = n0 + cc;
      i4 v = {0, 0, 0, 0};
      if (gcol < n) {
        const signed char* src = SB + ((long long)s * RF + half) * plane + (long long)gcol * kp + kc + 16 * piece;
        v = *reinterpret_cast<const i4*>(src);
      }
      *reinterpret_cast<i4*>(Bs + (s * Q8_N + cc) * Q8_LD + 16 * piece) = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < Q8_KC / 32; ++ks) {
      i4 af[S];
#pragma unroll
      for (int s = 0; s < S; ++s)
        af[s] = *reinterpret_cast<const i4*>(As + (s * Q8_M + wr + l32) * Q8_LD + 32 * ks + 16 * lhi);
#pragma unroll
      for (int sb = 0; sb < S; ++sb) {
        const i4 bf = *reinterpret_cast<const i4*>(Bs + (sb * Q8_N + wc + l32) * Q8_LD + 32 * ks + 16 * lhi);
#pragma unroll
        for (int sa = 0; sa < S - sb; ++sa)
          acc[sa + sb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[sa], bf, acc[sa + sb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ---- fold the exact group sums into FP64 (smallest weights first) and store
  {
    const int col = n0 + wc + l32;
    double a64[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double sacc = 0.0;
#pragma unroll
      for (int g = S - 1; g >= 0; --g) sacc = fma((double)acc[g][j], ldexp(1.0, -7 * (g + 2)), sacc);
      a64[j] = sacc;
    }
    if (col >= n) return;
#pragma unroll
    for (int j = 0; j < 16; j += RF) {
      const int rr = m0 + wr + 8 * (j / 4) + 4 * lhi + (j % 4);
      const int i = rr / RF;
      if (i >= n || (herm && col > i)) continue;
      const double sc = ldexp(1.0, ea[i] + eb[col]);
      double vals[RF];
#pragma unroll
      for (int c = 0; c < RF; ++c) vals[c] = a64[j + c] * sc;
      const long long idx = (long long)i * n + col;
      T v = alpha * from_comps_i8<T>(vals);
      if (beta != 0.0) v = v + beta * C[idx];
      C[idx] = v;
      if (herm && col < i) C[(long long)col * n + i] = conjg(v);
    }
  }
}

template <class T, int S>
static void launch_i8_s(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim, int dsel,
                        int bufC, double alpha, double beta, int herm) {
  constexpr int RF = ncomp<T>();
  const size_t shm = (size_t)S * (Q8_M + Q8_N) * Q8_LD;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_i8<T, S>), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  dim3 grid((maxdim + Q8_N - 1) / Q8_N, (RF * maxdim + Q8_M - 1) / Q8_M, nblk);
  hipLaunchKernelGGL((k_gemm_i8<T, S>), grid, dim3(256), shm, s, D, ws, info, dsel, bufC, alpha, beta, herm,
                     (int)Z_SLA, (int)Z_SLB, (int)V_EXA, (int)V_EXB);
}

template <class T>
void launch_gemm_split_i8(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int maxdim,
                          int dsel, int bufA, int opA, int bufB, int opB, int bufC, double alpha, double beta,
                          int slices, int herm) {
  const dim3 lg((maxdim + 3) / 4, nblk);
  hipLaunchKernelGGL(k_split_i8<T>, lg, dim3(256), 0, s, D, ws, info, dsel, bufA, opA, 0, slices, (int)Z_SLA,
                     (int)V_EXA);
  hipLaunchKernelGGL(k_split_i8<T>, lg, dim3(256), 0, s, D, ws, info, dsel, bufB, opB, 1, slices, (int)Z_SLB,
                     (int)V_EXB);
  switch (slices) {
    case 1: launch_i8_s<T, 1>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 2: launch_i8_s<T, 2>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 3: launch_i8_s<T, 3>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 4: launch_i8_s<T, 4>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 5: launch_i8_s<T, 5>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 6: launch_i8_s<T, 6>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    case 7: launch_i8_s<T, 7>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
    default: launch_i8_s<T, 8>(s, D, ws, info, nblk, maxdim, dsel, bufC, alpha, beta, herm); break;
  }
}

template void launch_gemm_split_i8<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                           int, int, int, double, double, int, int);
template void launch_gemm_split_i8<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                         int, int, int, double, double, int, int);
template void launch_gemm_split_i8<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int,
                                         int, int, int, double, double, int, int);

}  // namespace x2c
