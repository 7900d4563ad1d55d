// pc_static.hip -- pc_count_batch_static: pc_count_batch in a fixed device
// work area, for callers that cannot allocate device memory.
//
// The batch runner normally takes one stream-ordered allocation per launch
// (converted and ordered catalogue copies, sort scratch, the survivor list,
// descriptors, results) and keeps edge-set tables in an allocating per-device
// cache.  Here all of it, tables included, lives in `scratch`, a file-scope
// device array that every GPU the library runs on holds from the library's
// first use of it until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is taken once per
// device with hipGetSymbolAddress and only that address is handed to kernels
// and copies.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pc.h"
#include "pc_internal.hpp"
#include "pc_runtime.hpp"

namespace pc {

int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
void clear_error();

static __device__ __align__(256) unsigned char scratch[PC_STATIC_SCRATCH_BYTES];

namespace {

struct StaticArea {
    void *ptr = nullptr;  // device address of `scratch` on this device
    std::mutex run_mu;    // one call at a time uses the device's copy
};

std::mutex g_area_mu;
std::map<int, StaticArea *> g_areas;  // never freed: lives as long as `scratch`

int static_area(StaticArea **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_area_mu);
    auto it = g_areas.find(dev);
    if (it == g_areas.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PC_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        auto *a = new StaticArea();
        a->ptr = p;
        it = g_areas.emplace(dev, a).first;
    }
    *out = it->second;
    return PC_OK;
}

}  // namespace
}  // namespace pc

using namespace pc;

extern "C" int pc_count_batch_static(const pc_job *jobs, int32_t n_jobs, int32_t mode, void *stream) {
    clear_error();
    std::vector<BatchJob> v;
    int rc = jobs_from_abi(jobs, n_jobs, &v);
    if (rc) return rc;
    StaticArea *a = nullptr;
    rc = static_area(&a);
    if (rc) return rc;
    BatchOpts o;
    o.ws = a->ptr;
    o.ws_bytes = PC_STATIC_SCRATCH_BYTES;
    // the call returns only after its results are read back, so holding the
    // lock for the whole call keeps two calls of this process from sharing
    // the array at once
    std::lock_guard<std::mutex> lk(a->run_mu);
    return run_batch_opts(v, mode, static_cast<hipStream_t>(stream), nullptr, o);
}
