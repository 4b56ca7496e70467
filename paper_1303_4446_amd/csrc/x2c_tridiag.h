// Shared pieces of the blocked Householder tridiagonalisation kernels
// (internal to libx2c).
#pragma once
#include "x2c_device.h"

namespace x2c {

// Tile sizes per scalar type (quaternions are 32 bytes: smaller tiles keep
// every kernel within the 160 KB of LDS per CU).
template <class T>
struct Tiles {
  static constexpr int HT = 32;   // matvec sub-tile (super-tile / strip = 2 HT)
  static constexpr int TT = 32;   // rank-2k update tile
  static constexpr int LR = 64;   // larft row chunk
  static constexpr int CW = 64;   // back-transformation columns per work-group
  static constexpr int VR = 32;   // back-transformation V row chunk
};
template <>
struct Tiles<quat> {
  static constexpr int HT = 16;
  static constexpr int TT = 16;
  static constexpr int LR = 32;
  static constexpr int CW = 32;
  static constexpr int VR = 16;
};

// panel width (reflectors per panel).  Every column step reads the rows of
// the panel's V and W twice (the panel dot products and the corrections of
// y and of the next column), 4 x width x len elements against the len^2 / 2
// of the trailing triangle, while the rank-2k update after each panel reads
// and writes the triangle once; 16 balances the two for the quaternion
// reductions (whose panel update runs on the matrix cores at either width).
template <class T>
__host__ __device__ constexpr int panel_width() {
  return is_quat<T>() ? 16 : 32;
}
constexpr int HB = 32;   // the widest panel (buffer sizes)

// First column of the unblocked tail of a quaternion reduction: the last
// trailing matrices (at most TAIL_MAX columns) are reduced by one
// work-group per block in one kernel instead of two launches per column; a
// panel boundary, so the blocked part ends with a complete panel and its
// rank-2k update.  Other types: no tail.
constexpr int TAIL_MAX = 64;
template <class T>
__host__ __device__ constexpr int tri_tail_start(int n) {
  if constexpr (is_quat<T>()) {
    const int s = n - 1 - TAIL_MAX, pw = panel_width<T>();
    return s <= 0 ? 0 : (s + pw - 1) / pw * pw;
  } else {
    return 1 << 30;
  }
}

// Super-tile edge of the quaternion matvec for a block whose tile grid at
// this step (virtual lead rows included) has len rows: 64 x 64 items while
// the trailing matrix is long (half the partial sums of 32 x 32 ones), 32 x
// 32 once it is short (finer items).  A function of the block's own length,
// so a block's results do not depend on its batch; the column kernel reads
// the partials with the same edge.
constexpr int MV_ST64_LEN = 192;
__host__ __device__ constexpr int mv_st_q(int len) { return len > MV_ST64_LEN ? 64 : 32; }

// Leading virtual rows / columns of the matvec tiling at column step k.  The
// quaternion tiles start on a 128-byte boundary (4 quaternions): the trailing
// matrix (first row / column k + 1) is preceded by (k + 1) mod 4 zero rows /
// columns in the tile grid, so that no tile row starts inside a cache line.
template <class T>
__host__ __device__ constexpr int mv_lead(int k) {
  return is_quat<T>() ? ((k + 1) & 3) : 0;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element (r, a) of panel V whose first reflector is k0 (dimension nr)
template <class T>
__device__ inline T panel_v(const T* A, int nr, int k0, int r, int a) {
  int row1 = k0 + a + 1;            // row of the implicit unit entry
  if (r < row1) return tzero<T>();
  if (r == row1) return treal<T>(1.0);
  return A[(long long)r * nr + k0 + a];
}

// Hermitian matvec y = A[k+1:, k+1:] v_k of the reduction step k over the
// whole batch (k_matvec.hip); partial sums into bufHS in the layout the
// column kernel reads.  mv_res: resident one-wave work-groups per CU of the
// quaternion kernel's persistent grid (1..8).
template <class T>
void launch_matvec(hipStream_t s, const BlockDesc* D, char* ws, const int* info, int nblk, int dsel, int bufA,
                   int bufV, int bufHS, int bufW, int k0, int k, int nsmax, int ncu, int mv_res,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace x2c
