// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "wcal.h"

// ------------------------------------------------------------------ plan
struct wcal_plan {
    wcal_problem prob;
    int device = 0;
    int n_cu = 0;
    int64_t rows = 0;
    int32_t max_ns = 0;
    // device tables (plan-owned)
    int32_t* d_ant1 = nullptr;    // [n_bl]
    int32_t* d_ant2 = nullptr;    // [n_bl]
    int64_t* d_row_off = nullptr; // [n_int + 1]
    int32_t* d_ns = nullptr;      // [n_int]
    int32_t* d_order = nullptr;   // [n_int] intervals by decreasing size (LPT order)
    int32_t* d_queue = nullptr;   // [4] work-queue counters
    // DD statistics scratch (plan-owned, sized at creation)
    float* d_stats = nullptr;
    size_t stats_bytes = 0;
    // launch configuration
    int block = 256;              // threads per workgroup of the persistent kernels
    int wg_per_cu = 0;            // resident workgroups per CU (0 = occupancy limit)
};

// ------------------------------------------------------------------ kernel arguments
struct DiArgs {
    const float2* data;      // [rows][nc]
    const float2* model;     // [rows][nc]
    const uint8_t* flags;    // [rows] or null
    float2* gains;           // [n_int][n_ant][nc]   (n_dir == 1)
    const float2* gains_in;  // accumulate/residual: gains read only
    float2* residual;        // [rows][nc] or null
    int32_t* n_iter;         // [n_int]
    uint32_t* status;        // [n_int]
    double* chi2;            // [n_int] or null
    // accumulate outputs
    float2* jhj;             // [n_int][n_ant][blk]
    float2* jhd;             // [n_int][n_ant][nc]
    float2* jhr;             // [n_int][n_ant][nc]
    int32_t* count;          // [n_int][n_ant]
    // tables
    const int32_t* ant1;
    const int32_t* ant2;
    const int64_t* row_off;
    const int32_t* ns;
    const int32_t* order;
    int32_t* queue;
    int32_t n_ant, n_bl, n_int, max_iter, schedule;
    double tol;
};

struct DdArgs {
    const float2* data;      // [rows]
    const float2* model;     // [rows][nd]
    const uint8_t* flags;
    float2* gains;           // [n_int][nd][n_ant]
    const float2* gains_in;
    float2* residual;
    int32_t* n_iter;
    uint32_t* status;
    double* chi2;
    float2* jhj;             // [n_int][n_ant][nd][nd]
    float2* jhd;             // [n_int][n_ant][nd]
    float2* jhr;             // [n_int][n_ant][nd]
    int32_t* count;          // [n_int][n_ant]
    float* stats;            // per-baseline sufficient statistics scratch
    const int32_t* ant1;
    const int32_t* ant2;
    const int64_t* row_off;
    const int32_t* ns;
    const int32_t* order;
    int32_t* queue;
    int32_t n_ant, n_bl, n_int, n_dir, max_iter, schedule, algo;
    double tol;
};

// launchers (return a hipError_t)
hipError_t launch_di_solve(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
hipError_t launch_di_accumulate(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
hipError_t launch_di_residual(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
size_t di_smem_bytes(int n_ant, int nc, int mode, int block);

hipError_t launch_dd_solve(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_dd_accumulate(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_dd_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
size_t dd_stats_bytes(const wcal_problem& p);

hipError_t launch_reset_queue(int32_t* q, hipStream_t s);
