// Hermitian matrix-vector product of the trailing matrix, one launch per
// column step of the blocked tridiagonalisation over the whole batch (the
// memory-bound kernel of the reduction: the lower triangle is read once).
#include "x2c_device.h"
#include "x2c_launch.h"
#include "x2c_tridiag.h"

#include <hip/hip_ext.h>

namespace x2c {

// Lower-triangle matvec y = A[k+1:, k+1:] v_k, persistent over the batch.
// Work items are (block, lower super-tile (SI, SJ) of 2 HT x 2 HT); a work-group
// walks items blockIdx.x, +gridDim.x, ... and prefetches the next item's
// sub-tile into registers while reducing the current one.  Wave w stages
// sub-tile (w>>1, w&1) in LDS (for a diagonal super-tile the upper sub-tile
// is the conjugate transpose of its mirror, so the block acts as a full
// Hermitian block).  The four waves' sums are combined in a fixed order; the
// super-tile writes its row partial HS[SJ*len + r] and, off the diagonal,
// its column partial HS[(nst + SI)*len + c]; a diagonal super-tile also
// writes its strip's part of the panel dot products (W^H v, V^H v).
struct MvItem {
  int valid, b, SI, SJ, len, n, nst, st;
};

// len (returned) counts the lead virtual rows of the tiling too; ST = 0: the
// block's quaternion super-tile edge mv_st_q(len)
__device__ inline MvItem mv_decode(const BlockDesc* D, const int* info, int dsel, int k, int nblk, int nsmax,
                                   int item, int ST, int lead) {
  MvItem it{0, 0, 0, 0, 0, 0, 0, 0};
  const int b = item / nsmax, st = item - (item / nsmax) * nsmax;
  if (b >= nblk || info[b]) return it;
  const int n = seldim(D[b], dsel);
  if (n - k - 1 <= 0) return it;
  const int len = n - k - 1 + lead;
  if (ST == 0) ST = mv_st_q(len);
  const int nst = (len + ST - 1) / ST;
  if (st >= nst * (nst + 1) / 2) return it;
  int SI = (int)((sqrt(8.0 * st + 1.0) - 1.0) * 0.5);
  while ((SI + 1) * (SI + 2) / 2 <= st) ++SI;
  while (SI * (SI + 1) / 2 > st) --SI;
  it.valid = 1;
  it.b = b;
  it.SI = SI;
  it.SJ = st - SI * (SI + 1) / 2;
  it.len = len;
  it.n = n;
  it.nst = nst;
  it.st = ST;
  return it;
}

template <class T>
__device__ inline void mv_load(const BlockDesc* D, char* ws, int bufA, int k, const MvItem& it, int wi, int wj,
                               int lane, T* regs) {
  constexpr int HT = Tiles<T>::HT, ST = 2 * HT, EPL = HT * HT / 64, RPI = 64 / HT;
  const T* A = bufp<T>(ws, D[it.b], bufA);
  const int off = k + 1, len = it.len, n = it.n;
  const bool diag = it.SI == it.SJ;
  const int rowbase = ST * it.SI + HT * wi, colbase = ST * it.SJ + HT * wj;
  const bool upper = diag && wi < wj, dsub = diag && wi == wj;
  const int lr0 = upper ? colbase : rowbase, lc0 = upper ? rowbase : colbase;
#pragma unroll
  for (int q = 0; q < EPL; ++q) {
    const int ii = lane / HT + RPI * q, jj = lane % HT;
    const int r = lr0 + ii, c = lc0 + jj;
    regs[q] = (r < len && c < len && (!dsub || ii >= jj)) ? A[(long long)(off + r) * n + off + c] : tzero<T>();
  }
}

template <class T>
__global__ void __launch_bounds__(256) k_tri_matvec(const BlockDesc* D, char* ws, const int* info, int dsel, int bufA,
                                                    int bufV, int bufHS, int bufW, int k0, int k, int nblk,
                                                    int nsmax) {
  constexpr int HT = Tiles<T>::HT, ST = 2 * HT, EPL = HT * HT / 64, RPI = 64 / HT;
  constexpr int RPG = ST / 8;          // rows per group in the panel dot products
  static_assert(panel_width<T>() == HB, "eight row groups of 32 panel columns");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  __shared__ T tiles[4][HT][HT + 1];
  __shared__ T comb[4][HT];
  __shared__ T vsh[4][2][HT];
  __shared__ T tpart[8][HB][2];
  T (*tl)[HT + 1] = tiles[wave];
  const int total = nblk * nsmax;
  int item = blockIdx.x;
  MvItem cur = mv_decode(D, info, dsel, k, nblk, nsmax, item, ST, 0);
  T regs[EPL];
  if (cur.valid) mv_load<T>(D, ws, bufA, k, cur, wi, wj, lane, regs);
  while (item < total) {
    const int nitem = item + gridDim.x;
    const MvItem nxt = mv_decode(D, info, dsel, k, nblk, nsmax, nitem, ST, 0);
    T nregs[EPL];
    if (nxt.valid) mv_load<T>(D, ws, bufA, k, nxt, wi, wj, lane, nregs);
    if (cur.valid) {
      const BlockDesc& d = D[cur.b];
      const T* vg = bufp<T>(ws, d, bufV);
      T* HS = bufp<T>(ws, d, bufHS);
      const int len = cur.len, nst = cur.nst, SI = cur.SI, SJ = cur.SJ;
      const bool diag = SI == SJ;
      const int rowbase = ST * SI + HT * wi, colbase = ST * SJ + HT * wj;
      const bool upper = diag && wi < wj, dsub = diag && wi == wj;
      if (lane < HT) {
        const int c = colbase + lane;
        vsh[wave][0][lane] = c < len ? vg[c] : tzero<T>();
      } else if (lane < 2 * HT) {
        const int r = rowbase + lane - HT;
        vsh[wave][1][lane - HT] = r < len ? vg[r] : tzero<T>();
      }
#pragma unroll
      for (int q = 0; q < EPL; ++q) tl[lane / HT + RPI * q][lane % HT] = regs[q];
      wave_sync();
      if (upper) {
        for (int e = lane; e < HT * HT; e += 64) {
          int ii = e / HT, jj = e % HT;
          if (ii < jj) {
            T x = tl[ii][jj];
            tl[ii][jj] = conjg(tl[jj][ii]);
            tl[jj][ii] = conjg(x);
          } else if (ii == jj) {
            tl[ii][ii] = conjg(tl[ii][ii]);
          }
        }
        wave_sync();
      } else if (dsub) {
        for (int e = lane; e < HT * HT; e += 64) {
          int ii = e / HT, jj = e % HT;
          if (ii < jj) tl[ii][jj] = conjg(tl[jj][ii]);
          else if (ii == jj) tl[ii][jj] = treal<T>(re(tl[ii][jj]));
        }
        wave_sync();
      }
      T sum = tzero<T>();
      if (lane < HT) {
#pragma unroll 8
        for (int jj = 0; jj < HT; ++jj) sum = mad(tl[lane][jj], vsh[wave][0][jj], sum);
      } else if (lane < 2 * HT && !diag) {
        const int jj = lane - HT;
#pragma unroll 8
        for (int ii = 0; ii < HT; ++ii) sum = mad(conjg(tl[ii][jj]), vsh[wave][1][ii], sum);
      }
      if (lane < HT && wj == 1) comb[wi][lane] = sum;
      if (lane >= HT && lane < 2 * HT && wi == 1) comb[2 + wj][lane - HT] = sum;
      __syncthreads();
      if (lane < HT && wj == 0) {
        int r = rowbase + lane;
        if (r < len) HS[(long long)SJ * len + r] = sum + comb[wi][lane];
      }
      if (!diag && lane >= HT && lane < 2 * HT && wi == 0) {
        int c = colbase + lane - HT;
        if (c < len) HS[(long long)(nst + SI) * len + c] = sum + comb[2 + wj][lane - HT];
      }
      if (diag) {
        // this strip's part of the panel dot products (j < k - k0):
        // TP[SI][j] = (sum_r conj(W(off+r, j)) v_r, sum_r conj(V(off+r, j)) v_r)
        const int ip = k - k0, off = k + 1, n = cur.n;
        const T* A = bufp<T>(ws, d, bufA);
        const T* Wp = bufp<T>(ws, d, bufW);
        const int j = threadIdx.x & (HB - 1), g = threadIdx.x >> 5;
        T s1 = tzero<T>(), s2 = tzero<T>();
        if (j < ip) {
#pragma unroll
          for (int q = 0; q < RPG; ++q) {
            const int r = ST * SI + RPG * g + q;
            if (r < len) {
              const T vr = vg[r];
              s1 = mad(conjg(Wp[(long long)(off + r) * HB + j]), vr, s1);
              s2 = mad(conjg(panel_v(A, n, k0, off + r, j)), vr, s2);
            }
          }
        }
        tpart[g][j][0] = s1;
        tpart[g][j][1] = s2;
        __syncthreads();
        if (threadIdx.x < HB) {
          T a1 = tzero<T>(), a2 = tzero<T>();
          for (int gg = 0; gg < 8; ++gg) {
            a1 = a1 + tpart[gg][threadIdx.x][0];
            a2 = a2 + tpart[gg][threadIdx.x][1];
          }
          T* TP = HS + (long long)2 * nst * len;
          TP[((long long)SI * HB + threadIdx.x) * 2] = a1;
          TP[((long long)SI * HB + threadIdx.x) * 2 + 1] = a2;
        }
      }
      __syncthreads();
    }
    item = nitem;
    cur = nxt;
#pragma unroll
    for (int q = 0; q < EPL; ++q) regs[q] = nregs[q];
  }
}

// Sum over the four lanes of a quad (lanes 4t..4t+3) with DPP quad
// permutations (no LDS traffic).
__device__ inline double quad_sum(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  double y = x + __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false),
                                  __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false));     // lane ^ 1
  lo = __double2loint(y);
  hi = __double2hiint(y);
  return y + __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false),
                              __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false));      // lane ^ 2
}
__device__ inline quat quad_sum(const quat& q) {
  return quat{cplx{quad_sum(q.a.x), quad_sum(q.a.y)}, cplx{quad_sum(q.b.x), quad_sum(q.b.y)}};
}

// Quaternion matvec, one independent wave per super-tile of st x st (st =
// 64 or 32, mv_st_q; persistent over the batch; work-groups of one wave, so
// no work-group barriers).  The wave walks the super-tile's 32 x 32
// quadrants (three on the diagonal); for each it issues the loads of the four
// 16 x 16 sub-tiles (three on a diagonal quadrant) at once, then stages them
// one by one through its own LDS tile.  Row sums: lane (i, q) covers row i,
// columns 4q..4q+3; column sums: lane (j, q) covers column j, rows
// 4q..4q+3; quads are reduced with DPP and added into the super-tile's row
// and column accumulators in a fixed order.  Output and panel dot products
// as for k_tri_matvec (a diagonal super-tile writes its full Hermitian
// product as the row partial), per strip of st rows.
constexpr int MVW_HT = 16;

__global__ void __launch_bounds__(64) k_tri_matvec_w(const BlockDesc* D, char* ws, const int* info, int dsel,
                                                     int bufA, int bufV, int bufHS, int bufW, int k0, int k,
                                                     int nblk, int nsmax) {
  constexpr int HT = MVW_HT, QT = 2 * HT, EPL = HT * HT / 64;
  const int lane = threadIdx.x;
  __shared__ quat tl[HT][HT + 1];
  __shared__ quat vsh[2][2 * QT];      // [0] row segment, [1] column segment
  __shared__ quat racc[2 * QT], cacc[2 * QT];
  const int total = nblk * nsmax;
  // every other step walks the items in reverse, so that a launch starts on
  // the matrices its predecessor read last (still in the memory-side cache)
  const bool rev = k & 1;
  // tile index r covers matrix row / column off + r; r < lead are virtual
  const int lead = mv_lead<quat>(k), off = k + 1 - lead;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const MvItem it = mv_decode(D, info, dsel, k, nblk, nsmax, rev ? total - 1 - item : item, 0, lead);
    if (!it.valid || k >= tri_tail_start<quat>(it.n)) continue;   // the block's tail kernel takes over
    const BlockDesc& d = D[it.b];
    const quat* A = bufp<quat>(ws, d, bufA);
    const quat* vg = bufp<quat>(ws, d, bufV);
    quat* HS = bufp<quat>(ws, d, bufHS);
    const int len = it.len, n = it.n, nst = it.nst, SI = it.SI, SJ = it.SJ, st = it.st;
    const int nq = st / QT;            // quadrants per side
    const bool diag = SI == SJ;
    const int R0 = st * SI, C0 = st * SJ;
    for (int t = lane; t < 2 * st; t += 64) {
      const int seg = t / st, u = t - seg * st;
      const int g = (seg == 0 ? R0 : C0) + u;
      vsh[seg][u] = (g >= lead && g < len) ? vg[g - lead] : tzero<quat>();
    }
    for (int t = lane; t < st; t += 64) {
      racc[t] = tzero<quat>();
      cacc[t] = tzero<quat>();
    }
    for (int qa = 0; qa < nq; ++qa)
      for (int qb = 0; qb <= (diag ? qa : nq - 1); ++qb) {
        const bool qd = diag && qa == qb;    // quadrant on the matrix diagonal
        const int QR = QT * qa, QC = QT * qb;
        // ---- issue every load of the quadrant
        quat regs[4][EPL];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int a = s >> 1, bb = s & 1;
          const bool skip = qd && a == 0 && bb == 1;
          const bool dsub = qd && a == bb;
#pragma unroll
          for (int q = 0; q < EPL; ++q) {
            const int ii = lane / HT + (64 / HT) * q, jj = lane % HT;
            const int r = R0 + QR + HT * a + ii, c = C0 + QC + HT * bb + jj;
            regs[s][q] = (!skip && r < len && c < len && r >= lead && c >= lead && (!dsub || ii >= jj))
                             ? A[(long long)(off + r) * n + off + c] : tzero<quat>();
          }
        }
        wave_sync();
        // ---- sub-tiles
        const int i4 = lane >> 2, q4 = lane & 3;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int a = s >> 1, bb = s & 1;
          if (qd && a == 0 && bb == 1) continue;
          const bool dsub = qd && a == bb;
#pragma unroll
          for (int q = 0; q < EPL; ++q) tl[lane / HT + (64 / HT) * q][lane % HT] = regs[s][q];
          wave_sync();
          // row sums: row i4, columns 4 q4 .. 4 q4 + 3
          quat rs = tzero<quat>();
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int j = 4 * q4 + t;
            quat e = tl[i4][j];
            if (dsub && j == i4) e = treal<quat>(re(e));
            rs = mad(e, vsh[1][QC + HT * bb + j], rs);
          }
          // column sums: column i4, rows 4 q4 .. 4 q4 + 3 (strictly below the diagonal)
          quat cs = tzero<quat>();
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = 4 * q4 + t;
            if (!dsub || i > i4) cs = mad(conjg(tl[i][i4]), vsh[0][QR + HT * a + i], cs);
          }
          rs = quad_sum(rs);
          cs = quad_sum(cs);
          if (q4 == 0) {
            racc[QR + HT * a + i4] = racc[QR + HT * a + i4] + rs;
            cacc[QC + HT * bb + i4] = cacc[QC + HT * bb + i4] + cs;
          }
          wave_sync();
        }
      }
    // ---- partial sums out
    for (int t = lane; t < st; t += 64) {
      if (diag) {
        const int r = R0 + t;
        if (r < len) HS[(long long)SJ * len + r] = racc[t] + cacc[t];
      } else {
        const int r = R0 + t, c = C0 + t;
        if (r < len) HS[(long long)SJ * len + r] = racc[t];
        if (c < len) HS[(long long)(nst + SI) * len + c] = cacc[t];
      }
    }
    if (diag) {
      // this strip's part of the panel dot products (j < k - k0)
      // lane (g, j): panel column j, rows rg g .. rg g + rg - 1 of the strip
      constexpr int PW = panel_width<quat>(), NG = 64 / PW, PG = 8;
      static_assert(QT / NG % PG == 0, "row groups of PG loads");
      const int rg = st / NG;
      const int ip = k - k0;
      const quat* Wp = bufp<quat>(ws, d, bufW);
      const int j = lane % PW, g = lane / PW;
      quat s1 = tzero<quat>(), s2 = tzero<quat>();
      if (j < ip) {
        // rows off + r lie below the unit entry of every reflector of the
        // panel, so V is read as stored; loads go out in groups of PG rows
        // (clamped in-range addresses, masked values) so that their
        // latencies overlap
#pragma unroll 1
        for (int t0 = 0; t0 < rg; t0 += PG) {
          quat wv[PG], pv[PG];
#pragma unroll
          for (int u = 0; u < PG; ++u) {
            const int r = R0 + rg * g + t0 + u;
            const long long row = off + min(max(r, lead), len - 1);
            wv[u] = Wp[row * PW + j];
            pv[u] = A[row * n + k0 + j];
          }
#pragma unroll
          for (int u = 0; u < PG; ++u) {
            const int r = R0 + rg * g + t0 + u;
            const quat vr = r < len ? vsh[0][rg * g + t0 + u] : tzero<quat>();
            s1 = mad(conjg(wv[u]), vr, s1);
            s2 = mad(conjg(pv[u]), vr, s2);
          }
        }
      }
      // row groups 1 .. NG-1 are added to group 0 in order
      __shared__ quat tsum[NG - 1][2][PW];
      if (g > 0) {
        tsum[g - 1][0][j] = s1;
        tsum[g - 1][1][j] = s2;
      }
      wave_sync();
      if (g == 0) {
#pragma unroll
        for (int h = 0; h < NG - 1; ++h) {
          s1 = s1 + tsum[h][0][j];
          s2 = s2 + tsum[h][1][j];
        }
        quat* TP = HS + (long long)2 * nst * len;
        TP[((long long)SI * PW + j) * 2] = s1;
        TP[((long long)SI * PW + j) * 2 + 1] = s2;
      }
    }
    wave_sync();
  }
}

template <class T>
void launch_matvec(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int dsel, int bufA,
                   int bufV, int bufHS, int bufW, int k0, int k, int nsmax, int ncu, int mv_res, hipEvent_t ev0,
                   hipEvent_t ev1) {
  const long long items = (long long)nsmax * nblk;
  if constexpr (is_quat<T>()) {
    // one-wave work-groups, mv_res (1..8) of them per CU
    const long long res = std::max(1, std::min(8, mv_res));
    const int wgrid = (int)std::min<long long>(items, res * ncu);
    if (ev0)   // traced (never inside a graph capture): start / stop recorded by the launch
      hipExtLaunchKernelGGL(k_tri_matvec_w, dim3(wgrid), dim3(64), 0, s, ev0, ev1, 0, D, ws, info, dsel, bufA, bufV,
                            bufHS, bufW, k0, k, nblk, nsmax);
    else
      hipLaunchKernelGGL(k_tri_matvec_w, dim3(wgrid), dim3(64), 0, s, D, ws, info, dsel, bufA, bufV, bufHS, bufW,
                         k0, k, nblk, nsmax);
  } else {
    const int grid = (int)std::min<long long>(items, 2LL * ncu);    // two resident work-groups per CU (LDS)
    if (ev0)
      hipExtLaunchKernelGGL(k_tri_matvec<T>, dim3(grid), dim3(256), 0, s, ev0, ev1, 0, D, ws, info, dsel, bufA,
                            bufV, bufHS, bufW, k0, k, nblk, nsmax);
    else
      hipLaunchKernelGGL(k_tri_matvec<T>, dim3(grid), dim3(256), 0, s, D, ws, info, dsel, bufA, bufV, bufHS, bufW,
                         k0, k, nblk, nsmax);
  }
}
template void launch_matvec<double>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                    int, int, int, int, int, hipEvent_t, hipEvent_t);
template void launch_matvec<cplx>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                  int, int, int, int, int, hipEvent_t, hipEvent_t);
template void launch_matvec<quat>(hipStream_t, const BlockDesc*, char*, const int*, int, int, int, int, int, int,
                                  int, int, int, int, int, hipEvent_t, hipEvent_t);

}  // namespace x2c
