// Kernel launchers (host side) over the device tables of a plan.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace scasm {

struct DevTables {
    const SubDev* subs = nullptr;
    const TileDev* tiles = nullptr;
    const BlockDev* blocks = nullptr;
    const int32_t* rows = nullptr;
    const double* lval = nullptr;
    const float* lval32 = nullptr;
    const int32_t* piv = nullptr;
    const int32_t* pi = nullptr;
    const int8_t* sgn = nullptr;
    const SyrkItem* syrk = nullptr;
    double* X = nullptr;
    float* X32 = nullptr;
    double* F = nullptr;
    float* F32 = nullptr;
    int64_t ntiles = 0;
    int64_t nsyrk = 0;
};

// Optional per-kernel events: ev[2k] before and ev[2k+1] after kernel k
// (0 = TRSM, 1 = SYRK); null = no timing.
hipError_t launch_assemble_f64(const DevTables& t, hipStream_t stream, hipEvent_t* ev);

}  // namespace scasm
