// Launchers of the persistent fused KeyGen kernel (ntrup_persist.h).
// Compiled once per (lanes per key, form): -DNTRUP_LPK=2|4 and
// -DNTRUP_PMIXED=0 (one parameter set per launch, an instance per p) or 1
// (the mixed instance holding every p).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ntrup_host.h"
#include "ntrup_persist.h"

#if !defined(NTRUP_LPK) || !defined(NTRUP_PMIXED)
#error "compile with -DNTRUP_LPK=2|4 -DNTRUP_PMIXED=0|1"
#endif

namespace ntrup {

namespace {

template <int LPK, int... Ps>
int launch_persistent(ntrup_ctx* ctx, const PLaunch& pl, hipStream_t st) {
    auto kernel = keygen_persistent_kernel<LPK, Ps...>;
    int per_cu = 0, cus = 0;
    NTRUP_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0));
    NTRUP_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = std::max(1, std::min(pl.total, std::max(1, per_cu) * cus));
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, st, pl);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

}  // namespace

#if NTRUP_PMIXED
template <int LPK>
int launch_persistent_mixed(ntrup_ctx* ctx, const PLaunch& pl, hipStream_t st) {
    return launch_persistent<LPK, 653, 761, 857, 1277>(ctx, pl, st);
}
template int launch_persistent_mixed<NTRUP_LPK>(ntrup_ctx*, const PLaunch&, hipStream_t);
#else
template <int LPK>
int launch_persistent_single(ntrup_ctx* ctx, int p, const PLaunch& pl, hipStream_t st) {
    switch (p) {
        case 653: return launch_persistent<LPK, 653>(ctx, pl, st);
        case 761: return launch_persistent<LPK, 761>(ctx, pl, st);
        case 857: return launch_persistent<LPK, 857>(ctx, pl, st);
        case 1277: return launch_persistent<LPK, 1277>(ctx, pl, st);
    }
    return NTRUP_EINVAL;
}
template int launch_persistent_single<NTRUP_LPK>(ntrup_ctx*, int, const PLaunch&, hipStream_t);
#endif

}  // namespace ntrup
