// Host-only driver of libx2c's C ABI for the sanitizer build: every call
// here runs host logic only (argument checks, workspace layouts, the DKHn
// plan, status strings); none reaches the GPU.  Exits non-zero on a wrong
// result; AddressSanitizer / UndefinedBehaviorSanitizer abort on a fault.
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <vector>

#include "x2c.h"

static int fails = 0;
#define CHECK(cond)                                               \
  do {                                                            \
    if (!(cond)) {                                              \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main() {
  const int P[13] = {1, 4, 9, 17, 26, 38, 55, 79, 104, 132, 169, 217, 266};
  for (int n = 2; n <= 14; ++n) CHECK(x2c_dkh_products(n) == P[n - 2]);
  CHECK(x2c_dkh_products(1) == 0 && x2c_dkh_products(0) == -1 && x2c_dkh_products(15) == -1);
  for (int code = -5; code <= 8; ++code) CHECK(x2c_strerror(code) && std::strlen(x2c_strerror(code)) > 0);
  CHECK(x2c_max_n(X2C_SPINFREE) == 8192 && x2c_max_n(X2C_TWOCOMP) == 4096 && x2c_max_n(7) == 0);
  CHECK(x2c_device_wide_min_n(X2C_SPINFREE, -1) == 513 && x2c_device_wide_min_n(X2C_TWOCOMP, -1) == 257);
  CHECK(x2c_device_wide_min_n(7, -1) == X2C_EINVAL && x2c_device_wide_min_n(X2C_TWOCOMP, 258) == X2C_EINVAL);

  x2c_options o2{X2C_TWOCOMP, X2C_FP64, 0, 137.035999084, X2C_RED_QUATERNION};
  x2c_options o1{X2C_SPINFREE, X2C_FP64, 0, 137.035999084, X2C_RED_QUATERNION};
  // uneven batches of every size class, both modes, each method
  std::vector<int> Ns;
  for (int i = 0; i < 300; ++i) Ns.push_back(1 + (i * 37) % 256);
  for (const x2c_options* o : {&o1, &o2}) {
    const size_t w = x2c_workspace_bytes(o, (int)Ns.size(), Ns.data());
    CHECK(w > 0);
    CHECK(x2c_bss_workspace_bytes(o, (int)Ns.size(), Ns.data()) > w);
    for (int order = 1; order <= 14; ++order) CHECK(x2c_dkh_workspace_bytes(o, order, (int)Ns.size(), Ns.data()) > 0);
    CHECK(x2c_dkh_workspace_bytes(o, 15, (int)Ns.size(), Ns.data()) == 0);
  }
  // invalid sizes, options and pointers are refused before any device work
  int bad[3] = {10, 0, 20};
  CHECK(x2c_workspace_bytes(&o2, 3, bad) == 0);
  int big[1] = {4097};
  CHECK(x2c_workspace_bytes(&o2, 1, big) == 0);
  // device-wide sizes: a whole molecule, and batches that mix both paths
  int wide[3] = {2496, 100, 257};
  CHECK(x2c_workspace_bytes(&o2, 3, wide) > x2c_workspace_bytes(&o2, 1, wide));
  CHECK(x2c_bss_workspace_bytes(&o2, 1, wide) == 0 && x2c_dkh_workspace_bytes(&o2, 2, 1, wide) == 0);
  CHECK(x2c_device_wide_min_n(X2C_TWOCOMP, 100) == 257);
  CHECK(x2c_workspace_bytes(&o2, 3, wide) > 0);
  CHECK(x2c_device_wide_min_n(X2C_TWOCOMP, 0) == 100 && x2c_device_wide_min_n(X2C_TWOCOMP, -1) == 257);
  CHECK(x2c_workspace_bytes(nullptr, 1, big) == 0);
  x2c_options bad_c = o2;
  bad_c.c = -1.0;
  int one[1] = {12};
  CHECK(x2c_workspace_bytes(&bad_c, 1, one) == 0);
  x2c_options split = o2;
  split.prec = X2C_SPLIT_BF16;
  CHECK(x2c_bss_workspace_bytes(&split, 1, one) == 0 && x2c_dkh_workspace_bytes(&split, 2, 1, one) == 0);
  double dummy = 0.0;
  int64_t off[3] = {0, 0, 0};
  int info[3] = {0, 0, 0};
  CHECK(x2c_build_batched(&o2, 1, one, off, nullptr, &dummy, &dummy, &dummy, off, &dummy, off, &dummy, info,
                          &dummy, 8, nullptr) == X2C_EINVAL);
  CHECK(x2c_build_batched(&o2, 3, bad, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, off, &dummy, info,
                          &dummy, 8, nullptr) == X2C_EINVAL);
  int wide1[1] = {300};   // the allocation-free entry takes batched-path sizes only
  CHECK(x2c_build_batched_noalloc(&o2, 1, wide1, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, off, &dummy,
                                  info, nullptr) == X2C_EINVAL);
  CHECK(x2c_build_batched_noalloc(&o2, 257, one, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, off, &dummy,
                                  info, nullptr) == X2C_ESCRATCH);
  CHECK(x2c_dkh_batched(&o2, 0, 1, one, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, info, &dummy, 8,
                        nullptr) == X2C_EINVAL);
  CHECK(x2c_bss_batched(&split, 1, one, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, off, &dummy, info, &dummy,
                        8, nullptr) == X2C_EINVAL);
  CHECK(x2c_dlu_workspace_bytes(&o2, 13, std::vector<int>(13, 192).data()) > 0);
  // routes: every block device-wide, or the faster path for the batch; the
  // allocation-free entry takes the size route only
  x2c_options dw = o2, au = o2, badr = o2;
  dw.route = X2C_ROUTE_DEVICE_WIDE;
  au.route = X2C_ROUTE_AUTO;
  badr.route = 3;
  int ag[1] = {192};
  std::vector<int> ag309(309, 192);
  CHECK(x2c_workspace_bytes(&badr, 1, ag) == 0);
  CHECK(x2c_workspace_bytes(&dw, 1, ag) != x2c_workspace_bytes(&o2, 1, ag));
  CHECK(x2c_workspace_bytes(&au, 1, ag) ==
        std::max(x2c_workspace_bytes(&dw, 1, ag), x2c_workspace_bytes(&o2, 1, ag)));
  CHECK(x2c_workspace_bytes(&au, 309, ag309.data()) ==
        std::max(x2c_workspace_bytes(&dw, 309, ag309.data()), x2c_workspace_bytes(&o2, 309, ag309.data())));
  CHECK(x2c_build_batched_noalloc(&dw, 1, one, off, &dummy, &dummy, &dummy, &dummy, off, &dummy, off, &dummy, info,
                                  nullptr) == X2C_EINVAL);
  std::printf("abi driver: %d failure(s)\n", fails);
  return fails ? 1 : 0;
}
