// Batched colour sweep: one launch sweeps one colour of many independent
// simulations of one dimension and storage precision, of any (uneven) sizes.
// Members are laid out back to back in the grid: member i owns workgroups
// [block_begin_i, block_begin_i + ceil(count_i / 256)); a workgroup finds its
// member by binary search over block_begin.  Each member may run a different
// sweep kind in the same launch (kinds[launch * members + i], -1 = idle), so
// simulations that start, continue or finish a DP-AVF2 run share launches.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_point.h"
#include "kgs_sweep_body.h"

namespace kgs {
namespace {

constexpr int kBatchBlock = 256;

template <int DIM, typename T>
__global__ void __launch_bounds__(kBatchBlock)
batch_sweep_kernel(const BatchMember *__restrict__ m, int nm, const int *__restrict__ kinds,
                   int launch, int uniform_kind)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m[mid].block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const int kind = kinds ? kinds[static_cast<int64_t>(launch) * nm + lo] : uniform_kind;
    if (kind < 0) return;
    const int64_t t = (b - m[lo].block_begin) * kBatchBlock + threadIdx.x;
    if (t >= m[lo].count) return;
    T *base = static_cast<T *>(m[lo].state);
    const int64_t stride = m[lo].stride;
    const int n = m[lo].n;
    const Coef k = m[lo].k;
    using sweep_detail::sweep_one;
    switch (kind) {
    case PASS_R_BASE: sweep_one<DIM, T, PASS_R_BASE>(base, stride, n, RED, k, t); break;
    case PASS_B_FULL: sweep_one<DIM, T, PASS_B_FULL>(base, stride, n, BLUE, k, t); break;
    case PASS_R_ADJ: sweep_one<DIM, T, PASS_R_ADJ>(base, stride, n, RED, k, t); break;
    case PASS_R_ADJ_BASE: sweep_one<DIM, T, PASS_R_ADJ_BASE>(base, stride, n, RED, k, t); break;
    default: break;
    }
}

}  // namespace

int batch_block() { return kBatchBlock; }

hipError_t launch_batch_sweep(int dim, int precision, const BatchMember *members, int nm,
                              int64_t total_blocks, const int *kinds, int launch,
                              int uniform_kind, hipStream_t s)
{
    if (!members || nm < 1 || total_blocks < 1 || total_blocks > 0x7fffffff || dim < 1 || dim > 3 ||
        (!kinds && (uniform_kind < 0 || uniform_kind > PASS_R_ADJ_BASE)))
        return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(total_blocks)), threads(kBatchBlock);
#define KGS_BATCH(D, T)                                                                         \
    hipLaunchKernelGGL((batch_sweep_kernel<D, T>), grid, threads, 0, s, members, nm, kinds,    \
                       launch, uniform_kind)
    if (precision == 0) {
        if (dim == 1) KGS_BATCH(1, double);
        else if (dim == 2) KGS_BATCH(2, double);
        else KGS_BATCH(3, double);
    } else {
        if (dim == 1) KGS_BATCH(1, float);
        else if (dim == 2) KGS_BATCH(2, float);
        else KGS_BATCH(3, float);
    }
#undef KGS_BATCH
    return hipGetLastError();
}

}  // namespace kgs
