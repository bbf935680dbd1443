// Host helpers shared by the kernel launchers.
#include <map>
#include <mutex>
#include <utility>

#include <hip/hip_runtime_api.h>

#include "kgs_internal.h"
#include "kgs_plan.h"

namespace kgs {

hipError_t allow_dynamic_lds(const void *kernel, int bytes)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> allowed;  // (device, kernel) -> bytes
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = allowed.find({dev, kernel});
    if (it != allowed.end() && it->second >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) allowed[{dev, kernel}] = bytes;
    return e;
}

int device_cus()
{
    constexpr int kMi355xCus = 256;
    static std::mutex mu;
    static std::map<int, int> cus;  // device -> compute units
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kMi355xCus;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
        c = kMi355xCus;
    cus[dev] = c;
    return c;
}

}  // namespace kgs
