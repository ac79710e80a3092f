// runtime.hpp -- the plan object behind the C ABI and the per-thread error
// message, shared by the per-layer runtime (kernels.hip) and the batched
// executor (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>

#include "plan.hpp"

// devices whose per-device state (kernel attributes, SIMD counts) is cached
constexpr int kMaxDevices = 64;

struct mdpe_plan {
    mdpe::Plan P;
    int device = -1;
    int4 *d_conv = nullptr;
    int2 *d_add = nullptr;
    int2 *d_stage = nullptr;
    int *d_out = nullptr;
    int *d_chains = nullptr;
    int4 *d_corr = nullptr;
    int *d_cbar = nullptr;
    int *d_zbar = nullptr;
    int *d_ybar = nullptr;
    int4 *d_scale = nullptr;
    int4 *d_fconv = nullptr;   // fused layers: jobs by component, then layer
    int *d_foff = nullptr;     // fused layers: per-component layer offsets
    int *d_fchains = nullptr;  // fused layers: the one-job lane schedule
    int4 *d_pjobs = nullptr;   // chain launch: jobs chain after chain
    mdpe::ChainComp *d_pcomps = nullptr;  // chain launch: one per chain
    int *d_pcodes = nullptr;   // chain launch: lane schedules
    int *d_coff = nullptr;     // single launch: convolution layer offsets (int32)
    int *d_aoff = nullptr;     // single launch: addition level offsets (int32)
    int *d_schains = nullptr;  // single launch: the lane schedule of its job groups
};

namespace mdpe {
void set_last_error(const std::string &msg);
const std::string &get_last_error();
}  // namespace mdpe
