// cs_eval_stamp_noalloc: the region schedule's evaluate-and-stamp with its scratch
// memory in one file-scope device array per GPU, for callers that cannot allocate.
//
// The array's name is a host-side stand-in in host code, not a device address: the
// address is taken once per GPU with hipGetSymbolAddress (with that GPU current) and
// only that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "colorstamp.h"
#include "internal.hpp"
#include "launch.hpp"

namespace cs {
namespace {

constexpr size_t SCRATCH_DOUBLES = CS_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert(CS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a whole number of 256-byte blocks");

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_GPUS = 64;
std::mutex g_mu;
double *g_scratch[MAX_GPUS] = {};

// Device address of this GPU's copy of the array (dev is the current device).
hipError_t scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Zero n 32-bit counters (a kernel rather than a memset node, so that the call can
// be captured into a graph and replayed).
__global__ void k_zero_words(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Offsets in doubles, each section starting on a 256-byte boundary.
inline size_t up32(size_t n) { return (n + 31) & ~(size_t)31; }

cs_status failed(cs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" cs_status cs_eval_stamp_noalloc(cs_circuit *c, const double *x, double ag0, const double *hist,
                                           double *A_val, double *b, void *stream) {
    if (!c) return failed(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return failed(CS_ESTATE, "cs_build_stamp_map must come first");
    if (!c->models_set) return failed(CS_ESTATE, "cs_set_models must come first");
    if (!c->params_set) return failed(CS_ESTATE, "cs_set_params must come first");
    if (!x || !A_val || !b) return failed(CS_EINVAL, "NULL x, A or b");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        return failed(CS_ESTATE, "circuit uploaded to another device");
    if (dev < 0 || dev >= MAX_GPUS) return failed(CS_ENOTSUP, "device index beyond the scratch table");
    if (!c->rp.built || !c->rd.ready || c->rp.cap != c->block)
        return failed(CS_ESTATE,
                      "region tables are not on the device for this block size: one cs_eval_stamp with "
                      "CS_COLOR_REGION must come first");
    // scratch layout: staging values, hub part sums, item counters
    const size_t n_stage = (size_t)c->rp.stage_size;
    const size_t n_chunks = c->rp.hub_of_chunk.size();
    const size_t n_items = c->rp.item.size() / 4;
    const size_t off_part = up32(n_stage);
    const size_t off_count = off_part + up32(n_chunks);
    const size_t n_words = n_items * CNT_STRIDE;
    const size_t need = off_count + (n_words + 1) / 2;
    if (need > SCRATCH_DOUBLES)
        return failed(CS_ENOTSUP, "the circuit needs " + std::to_string(need * sizeof(double)) +
                                      " bytes of scratch; the no-allocation array holds " +
                                      std::to_string((size_t)CS_NOALLOC_SCRATCH_BYTES));
    double *base = nullptr;
    hipError_t e = scratch_address(dev, &base);
    if (e != hipSuccess) return failed(CS_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    if (c->rd.sdp_stale) {
        e = launch_permute_rows(c->h.n_dev, c->rd.cm_pos.p, c->d_sdp.p, c->h.n_dev, NSD, c->rd.sdp.p, s);
        if (e != hipSuccess) return failed(CS_EHIP, std::string("model-constant permute launch: ") + hipGetErrorString(e));
        c->rd.sdp_stale = false;
    }
    uint32_t *words = reinterpret_cast<uint32_t *>(base + off_count);
    KCirc kc = region_kcirc(make_kcirc(c), c->rp, c->rd);
    kc.stage = base;
    kc.hub_part = base + off_part;
    KRegion kr = region_kregion(c->rp, c->rd);
    kr.item_count = words;
    if (n_words > 0) {
        const int grid = (int)std::min<size_t>((n_words + 255) / 256, 1024);
        hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, s, words, (int64_t)n_words);
        e = hipGetLastError();
        if (e != hipSuccess) return failed(CS_EHIP, std::string("counter clear launch: ") + hipGetErrorString(e));
    }
    const KCall call{x, ag0, hist, A_val, b};
    e = launch_region(kc, call, kr, c->block, s);
    if (e != hipSuccess) return failed(CS_EHIP, std::string("region launch: ") + hipGetErrorString(e));
    e = launch_linear_add((int32_t)c->h.linA_idx.size(), c->d_linA_idx.p, c->d_linA_val.p, A_val, s);
    if (e != hipSuccess) return failed(CS_EHIP, std::string("linear-part launch: ") + hipGetErrorString(e));
    return CS_OK;
}
