"""MI355X-native X2C one-electron Hamiltonian for batches of atomic (DLU)
blocks: a thin binding over the HIP library libx2c.so (include/x2c.h)."""
from ._lib import (EBLOCK, EHIP, EINVAL, ESCRATCH, EXPORTED, FP64, OK, RED_COMPLEX, RED_QUATERNION, SPLIT_BF16,  # noqa: F401
                   ROUTE_AUTO, ROUTE_DEVICE_WIDE, ROUTE_SIZE, SPLIT_INT8,
                   SPINFREE, TWOCOMP,
                   Batch, X2CError, autotune, batch_to_device, bss_batched, bss_workspace_bytes, build, build_batched,
                   build_batched_noalloc, build_batched_xr, device_wide_min_n, dkh_batched, dkh_products, dkh_workspace_bytes,
                   dlu_assemble, dlu_workspace_bytes, graph_enable, load, max_n, picture_change, release,
                   stream_split, strerror, trace_enable, trace_read, trace_reset, tuned_shape, unpack_h,
                   workspace_bytes)
