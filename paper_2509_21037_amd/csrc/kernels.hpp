// Kernel launchers (host side) over the device tables of a plan.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace scasm {

constexpr int kNumTimed = 5;   // timed kernels: TRSM, SYRK, apply, implicit apply, fused assembly

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
    const int32_t* tile_order = nullptr;   // TRSM workgroup -> tile index (-1 = idle)
    double* X = nullptr;
    float* X32 = nullptr;
    double* F = nullptr;
    float* F32 = nullptr;
    const int2* apply_items = nullptr;     // (subdomain, first column) per GEMV workgroup
    const int2* fused = nullptr;           // fused assembly: (kind 0 idle / 1 TRSM / 2 SYRK, index)
    const SyrkItem* syrk_items = nullptr;  // SYRK items in subdomain order (indexed by fused items)
    int32_t* done = nullptr;               // [nsub] TRSM tiles finished (fused assembly)
    int32_t* err = nullptr;                // device error flag
    int64_t ntiles = 0;          // TRSM workgroups (length of tile_order)
    int64_t nsyrk = 0;           // SYRK workgroups (items with sub < 0 are idle)
    int64_t napply = 0;
    int64_t nfused = 0;
    int32_t nsub = 0;
};

// Optional per-kernel events: ev[2k] before and ev[2k+1] after kernel k
// (0 = TRSM, 1 = SYRK); null = no timing.
hipError_t launch_assemble_f64(const DevTables& t, hipStream_t stream, hipEvent_t* ev);

// Single-launch assembly over the fused item list (FP64 or, with X32 set,
// mixed); optional events ev[0] before, ev[1] after.
hipError_t launch_assemble_fused(const DevTables& t, hipStream_t stream, hipEvent_t* ev);

// Mixed precision: FP64 factor -> FP32 copy, and the assembly with FP64
// diagonal solves, FP32 X / updates / SYRK and FP32 F.
hipError_t launch_convert_f32(const double* a, float* b, int64_t n, hipStream_t stream);
hipError_t launch_assemble_mixed(const DevTables& t, hipStream_t stream, hipEvent_t* ev);

struct PcpgArgs {
    const double* G;        // concatenated m_i x k_i column-major blocks
    const int64_t* g_off;   // [nsub] offsets into G
    const int32_t* kdim;    // [nsub] kernel dimension k_i (<= 8)
    const double* GtGinv;   // [nsub][64] (G^T G)^{-1}, k_i x k_i row-major
    const double* d;        // right-hand side (dual layout)
    double* lambda;         // solution (dual layout)
    double *r, *w, *p, *q;  // workspace (dual layout)
    double* ww;             // [nsub]
    double* hist;           // [(iters + 1) * nsub] or null
    int32_t nsub;
    int32_t iters;
};

// Projected CG on every subdomain, `iters` iterations (explicit F apply).
hipError_t launch_pcpg(const DevTables& t, const PcpgArgs& a, hipStream_t stream);

// Implicit apply q = B P^T L^{-T} L^{-1} P B^T p; xwork holds n_i doubles per
// subdomain at xoff[i].
hipError_t launch_apply_implicit(const DevTables& t, const int64_t* xoff, double* xwork, const double* p,
                                 double* q, int32_t nsub, hipStream_t stream, hipEvent_t* ev);

// q = F p for every subdomain (FP32 F when t.F32 is set, else FP64 F);
// optional events ev[0] before, ev[1] after.
hipError_t launch_apply(const DevTables& t, const double* p, double* q, hipStream_t stream, hipEvent_t* ev);

}  // namespace scasm
