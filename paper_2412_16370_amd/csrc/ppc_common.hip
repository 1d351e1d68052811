// ppc_common.hip -- status strings, version, cached device attributes.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ppc.h"
#include "ppc_host.hpp"

namespace ppc {

static std::mutex g_attr_mu;
static int g_cus[64] = {0};

int device_cus(int device) {
    if (device < 0 || device >= 64) return 256;
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (g_cus[device] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0)
            v = 256;
        g_cus[device] = v;
    }
    return g_cus[device];
}

}  // namespace ppc

extern "C" {

const char *ppc_status_string(int status) {
    switch (status) {
    case PPC_OK: return "PPC_OK";
    case PPC_EINVAL: return "PPC_EINVAL: invalid argument";
    case PPC_ENOMEM: return "PPC_ENOMEM: allocation failed";
    case PPC_EDEVICE: return "PPC_EDEVICE: HIP runtime or launch failure";
    case PPC_EBUSY: return "PPC_EBUSY: not admitted, retry later";
    case PPC_ETIMEDOUT: return "PPC_ETIMEDOUT: a batch passed its deadline on the device";
    default: return "PPC_UNKNOWN";
    }
}

int ppc_version(void) { return 1 * 10000 + 0 * 100 + 0; }

}  // extern "C"
