// kernels.hip -- HIP kernels for gfx950 and the C ABI of include/mdpe.h.
//
// Data layout in HBM (workspace A): slot-major, then coefficient, then limb:
// A[slot][c][l], one slot = one series = (d+1)*W doubles (W = M, or 2M for
// complex series: real limbs, then imaginary limbs), so a coefficient's
// limbs are contiguous (80 bytes at M = 10) and a series is one contiguous
// block.  User buffers are limb-planar [W][count][d+1]; the staging and
// gather kernels convert.
//
// Kernels
//   stage_kernel         user coeff / z -> input slots of A (+ n_k = 1 copies)
//   conv_layer_kernel    one wavefront per group of J jobs of a layer (four per
//                        workgroup when a launch has one to three wavefronts
//                        per SIMD; or Q wavefronts per job, J = 1, for layers
//                        of few long jobs) stages the jobs' first operands in
//                        LDS (both operands for coefficients of at most two
//                        doubles; none when operands are streamed) and
//                        computes their J*(d+1) output coefficients;
//                        each coefficient is one lane's sequential chain
//                        z_k = x_0 y_k, z_k += x_i y_{k-i} (i = 1..k), spread
//                        over the lanes by a host-made schedule or dealt to the
//                        lanes in turn (Section 2, eq. (1); Section 5, the
//                        convolution kernel); complex series and the
//                        correlations of the reverse pass run on it too
//   scale_kernel         A[dst] := e * A[src] for general exponents (Section 3)
//   add_level_kernel     one thread per coefficient of every pair of a level:
//                        A[t2] := A[t2] + A[t1] (Section 5, the addition kernel)
//   gather_kernel        output slots -> user value / gradient (zeros if absent)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mdpe.h"
#include "conv_core.hpp"
#include "md.hpp"
#include "plan.hpp"
#include "runtime.hpp"

namespace mdpe {

// ------------------------------------------------------------------ kernels

template <int M, bool CX>
__global__ __launch_bounds__(256) void add_level_kernel(double *__restrict__ A, const int2 *__restrict__ pairs,
                                                        long total, int d) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int d1 = d + 1;
    const long p = idx / d1;
    const int c = (int)(idx - p * d1);
    add_item<M, CX>(A, pairs[p], c, d);
}

// A[dst] := e * A[src] at every coefficient of every scale job: one md_mul by
// (e, 0, ..., 0) per part (general exponents, Section 3).
template <int M, bool CX>
__device__ __forceinline__ void scale_item(double *__restrict__ A, int4 t, int c, int d) {
    constexpr int W = kCoef<M, CX>;
    const long S = (long)(d + 1) * W;
    const double *in = A + (long)t.x * S + (long)c * W;
    double *out = A + (long)t.y * S + (long)c * W;
    double E[M], x[M], r[M];
#pragma unroll
    for (int l = 0; l < M; ++l) E[l] = l == 0 ? (double)t.z : 0.0;
#pragma unroll
    for (int part = 0; part < (CX ? 2 : 1); ++part) {
#pragma unroll
        for (int l = 0; l < M; ++l) x[l] = in[part * M + l];
        md_mul<M>(x, E, r);
#pragma unroll
        for (int l = 0; l < M; ++l) out[part * M + l] = r[l];
    }
}

template <int M, bool CX>
__global__ __launch_bounds__(256) void scale_kernel(double *__restrict__ A, const int4 *__restrict__ jobs,
                                                    long total, int d) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int d1 = d + 1;
    const long q = idx / d1;
    scale_item<M, CX>(A, jobs[q], (int)(idx - q * d1), d);
}

__global__ __launch_bounds__(256) void stage_kernel(double *__restrict__ A, const double *__restrict__ coeff,
                                                    const double *__restrict__ z, const int2 *__restrict__ entries,
                                                    long total, int N, int n, int d, int m) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int d1 = d + 1;
    const long e = idx / d1;
    const int c = (int)(idx - e * d1);
    stage_item(A, coeff, z, entries[e], c, N, n, d, m);
}

__global__ __launch_bounds__(256) void gather_kernel(const double *__restrict__ A, double *__restrict__ value,
                                                     double *__restrict__ grad, const int *__restrict__ out_slots,
                                                     int n, int d, int m) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const int d1 = d + 1;
    if (idx >= (long)(1 + n) * d1) return;
    const int o = (int)(idx / d1);
    const int c = (int)(idx - (long)o * d1);
    gather_item(A, value, grad, out_slots[o], o, c, n, d, m);
}

// The whole evaluation in one launch of one workgroup, for plans so small
// that the boundaries between dependent launches (~4.5 us each) would
// dominate: staging, every convolution layer, the scale stage, every addition
// level and the gather, each a phase of the workgroup's threads with a
// workgroup barrier after it.  Each wavefront takes J convolution jobs per
// round in its own LDS region of group_bytes, exactly as a per-layer launch's
// group, so every output bit is that of the per-launch path.  The barrier
// orders a phase's global stores before the next phase's loads within the
// workgroup (one CU; workgroup-scope release and acquire), as between the
// layers of the fused launch; A is read with vector loads only.
struct SingleArgs {
    double *A;
    long ws_doubles;   // > 0: the workspace lives in LDS at lds_ws_off bytes (copied to A at the end)
    int lds_ws_off;
    const double *coeff, *z;
    double *value, *grad;
    const int2 *stage;
    int nstage;
    const int4 *conv;
    const int *conv_off;
    int nl;
    const int *chains;
    int stride, steps, J, simple, group_bytes;
    const int4 *scale;
    int nscale;
    const int2 *add;
    const int *add_off;
    int nlev;
    const int *out;
    int n, N, d;
};

template <int M, bool CX>
__global__ __launch_bounds__(1024) void eval_single_kernel(SingleArgs a) {
    constexpr int W = kCoef<M, CX>;
    extern __shared__ double lds[];
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, waves = nt >> 6;
    const int d1 = a.d + 1;
    // the workspace: in LDS when it fits (every phase after staging then
    // reads and writes LDS only), else the caller's buffer
    double *A = a.ws_doubles > 0 ? (double *)((char *)lds + a.lds_ws_off) : a.A;
    for (long it = tid; it < (long)a.nstage * d1; it += nt) {
        const long e = it / d1;
        stage_item(A, a.coeff, a.z, a.stage[e], (int)(it - e * d1), a.N, a.n, a.d, W);
    }
    __syncthreads();
    double *mine = (double *)((char *)lds + (long)wave * a.group_bytes);
    for (int L = 0; L < a.nl; ++L) {
        const int lo = a.conv_off[L], hi = a.conv_off[L + 1];
        // every wavefront runs the same rounds (conv_group ends its staging
        // with a workgroup barrier, also for a wavefront without a job)
        for (int r = lo; r < hi; r += waves * a.J) {
            const int q = r + wave * a.J;
            const int jn = q < hi ? min(a.J, hi - q) : 0;
            conv_group<M, false, CX, false, false, (CX ? 2 * M : M) <= 2>(A, a.conv + (jn > 0 ? q : lo), jn, a.J, a.d, mine, a.chains,
                                                   a.stride, a.steps, lane, lane, a.simple != 0);
        }
        __syncthreads();
    }
    for (long it = tid; it < (long)a.nscale * d1; it += nt) {
        const long q = it / d1;
        scale_item<M, CX>(A, a.scale[q], (int)(it - q * d1), a.d);
    }
    __syncthreads();
    for (int r = 0; r < a.nlev; ++r) {
        const long hi = (long)a.add_off[r + 1] * d1;
        for (long it = (long)a.add_off[r] * d1 + tid; it < hi; it += nt) {
            const long p = it / d1;
            add_item<M, CX>(A, a.add[p], (int)(it - p * d1), a.d);
        }
        __syncthreads();
    }
    for (long it = tid; it < (long)(1 + a.n) * d1; it += nt) {
        const int o = (int)(it / d1);
        gather_item(A, a.value, a.grad, a.out[o], o, (int)(it - (long)o * d1), a.n, a.d, W);
    }
    // the caller's workspace holds every series afterwards, as after the
    // per-launch path (the reverse pass reads the monomial values there)
    for (long q = tid; q < a.ws_doubles; q += nt) a.A[q] = A[q];
}

// planar [m][count][d+1] series src[e] -> slot dst[e] (skipped when -1), for e < count
__global__ __launch_bounds__(256) void planar_to_slots_kernel(double *__restrict__ A, const double *__restrict__ src,
                                                              int count, const int *__restrict__ dst, long total,
                                                              int d, int m) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int d1 = d + 1;
    const int e = (int)(idx / d1);
    const int c = (int)(idx - (long)e * d1);
    if (dst[e] < 0) return;
    double *to = A + (long)dst[e] * d1 * m + (long)c * m;
    for (int l = 0; l < m; ++l) to[l] = src[((long)l * count + e) * d1 + c];
}

// slot slots[e] (or zeros when -1) -> planar [m][count][d+1] series e of dst
__global__ __launch_bounds__(256) void slots_to_planar_kernel(const double *__restrict__ A, double *__restrict__ dst,
                                                              int count, const int *__restrict__ slots, int d, int m) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const int d1 = d + 1;
    if (idx >= (long)count * d1) return;
    const int e = (int)(idx / d1);
    const int c = (int)(idx - (long)e * d1);
    const int slot = slots[e];
    for (int l = 0; l < m; ++l)
        dst[((long)l * count + e) * d1 + c] = slot >= 0 ? A[(long)slot * d1 * m + (long)c * m + l] : 0.0;
}

// op 0 / 1: md_add / md_mul on planar [M][count]; CX: cmd_add / cmd_mul on [2M][count]
template <int M, bool CX>
__global__ __launch_bounds__(256) void md_elementwise_kernel(int op, long count, const double *__restrict__ x,
                                                             const double *__restrict__ y, double *__restrict__ z) {
    constexpr int W = kCoef<M, CX>;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    double a[W], b[W], r[W];
#pragma unroll
    for (int l = 0; l < W; ++l) {
        a[l] = x[(long)l * count + i];
        b[l] = y[(long)l * count + i];
    }
    if (op == 0)
        coef_add<M, CX>(a, b, r);
    else
        coef_mul<M, CX>(a, b, r);
#pragma unroll
    for (int l = 0; l < W; ++l) z[(long)l * count + i] = r[l];
}

}  // namespace mdpe

// ------------------------------------------------------------------ runtime

namespace mdpe {
static thread_local std::string g_err;
void set_last_error(const std::string &msg) { g_err = msg; }
const std::string &get_last_error() { return g_err; }
}  // namespace mdpe

namespace {

using mdpe::g_err;

size_t conv_lds_bytes(int d, int doubles_per_coef, int J) {
    return (size_t)mdpe::group_lds_bytes(d + 1, doubles_per_coef, J);
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(MDPE_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct mdpe_profiler {
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    size_t used = 0;
    uint32_t classes = 0xfu;  // bit c: time launches of class c (0 stage, 1 conv, 2 add, 3 gather)
};

namespace {

void free_plan(mdpe_plan *p) {
    if (!p) return;
    if (p->device >= 0) {
        DeviceGuard g(p->device);
        (void)hipFree(p->d_conv);
        (void)hipFree(p->d_add);
        (void)hipFree(p->d_stage);
        (void)hipFree(p->d_out);
        (void)hipFree(p->d_chains);
        (void)hipFree(p->d_corr);
        (void)hipFree(p->d_cbar);
        (void)hipFree(p->d_zbar);
        (void)hipFree(p->d_ybar);
        (void)hipFree(p->d_scale);
        (void)hipFree(p->d_fconv);
        (void)hipFree(p->d_foff);
        (void)hipFree(p->d_fchains);
        (void)hipFree(p->d_pjobs);
        (void)hipFree(p->d_pcomps);
        (void)hipFree(p->d_pcodes);
        (void)hipFree(p->d_coff);
        (void)hipFree(p->d_aoff);
        (void)hipFree(p->d_schains);
    }
    delete p;
}

template <class T>
int upload(T **dst, const void *src, size_t bytes) {
    // an empty array still gets a (never read) one-element allocation
    HIP_TRY(hipMalloc((void **)dst, bytes ? bytes : sizeof(T)));
    if (src && bytes) HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return MDPE_OK;
}

int record(mdpe_profiler *prof, int cls, hipStream_t st, bool start) {
    if (!prof || !((prof->classes >> cls) & 1u)) return MDPE_OK;
    if (start) {
        if (prof->used == prof->recs.size()) {
            mdpe_profiler::Rec r{cls, nullptr, nullptr};
            HIP_TRY(hipEventCreate(&r.a));
            HIP_TRY(hipEventCreate(&r.b));
            prof->recs.push_back(r);
        }
        prof->recs[prof->used].cls = cls;
        HIP_TRY(hipEventRecord(prof->recs[prof->used].a, st));
    } else {
        HIP_TRY(hipEventRecord(prof->recs[prof->used].b, st));
        prof->used++;
    }
    return MDPE_OK;
}

#define LAUNCH_CHECK(what)                                                                   \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess) return fail(MDPE_EDEVICE, std::string(what ": ") + hipGetErrorString(e_)); \
    } while (0)

int simd_count(int device) {
    static std::atomic<int> cached[kMaxDevices];
    if (device < 0 || device >= kMaxDevices) return 1024;
    if (!cached[device]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
            cus = 256;
        cached[device] = 4 * cus;
    }
    return cached[device];
}

template <int M, bool CORR, bool CX>
int launch_layer(const mdpe_plan *pl, double *A, const int4 *jobs, int nj, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    const int J = P.lanes.jobs_per_group;
    const int Q = P.lanes.waves_per_job;
    // the LDS limit is a per-device function attribute: raise it once per device
    static std::atomic<bool> attr_set[kMaxDevices];
    const int dv = pl->device >= 0 && pl->device < kMaxDevices ? pl->device : 0;
    if (!attr_set[dv].load()) {
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_layer_kernel<M, CORR, CX, 1, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_layer_kernel<M, CORR, CX, 4, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_layer_kernel<M, CORR, CX, 1, false, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        if constexpr (mdpe::kCoef<M, CX> <= 2)
            HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_layer_kernel<M, CORR, CX, 4, false, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        attr_set[dv].store(true);
    }
    if (nj == 0) return MDPE_OK;
    const int groups = (nj + J - 1) / J;
    int rc = record(prof, 1, st, true);
    if (rc) return rc;
    if (P.streamed) {
        // operands from global memory; only the job descriptors are in LDS
        const size_t group_bytes = conv_lds_bytes(P.d, 0, J);
        const long waves = (long)groups * Q;
        if (waves > 0x7fffffffL) return fail(MDPE_EUNSUPPORTED, "too many wavefronts in one layer");
        hipLaunchKernelGGL((mdpe::conv_layer_kernel<M, CORR, CX, 1, true>), dim3((unsigned)waves), dim3(64),
                           group_bytes, st, A, jobs, nj, P.d, J, pl->d_chains, P.lanes.stride, P.lanes.steps,
                           (int)group_bytes, Q, 0);
    } else {
        const size_t group_bytes =
            (conv_lds_bytes(P.d, mdpe::lds_doubles_per_coef(mdpe::kCoef<M, CX>), J) + 15) / 16 * 16;
        // one wavefront per workgroup, or one per SIMD (see conv_layer_kernel)
        const long waves = (long)groups * Q;
        if (waves > 0x7fffffffL) return fail(MDPE_EUNSUPPORTED, "too many wavefronts in one layer");
        const int simds = simd_count(pl->device);
        const int wpb =
            (waves > simds && waves <= 3 * simds && 4 * group_bytes <= (size_t)mdpe::kMaxLdsBytes) ? 4 : 1;
        const long blocks = (waves + wpb - 1) / wpb;
        // Jobs over Q wavefronts whose coefficients (of at most two doubles)
        // are dealt: four-wavefront workgroups, so that no SIMD gets two of
        // them while another idles (p2 2d, d = 64: 1.09 -> 0.78 ms).  Other
        // multi-wavefront plans measured equal or slower that way (deca
        // double +22%: the 256-thread bound slows a lone wavefront).
        const bool dealt4 = mdpe::kCoef<M, CX> <= 2 && Q > 1 && P.simple &&
                            4 * group_bytes <= (size_t)mdpe::kMaxLdsBytes;
        if (dealt4) {
            if constexpr (mdpe::kCoef<M, CX> <= 2)
                hipLaunchKernelGGL((mdpe::conv_layer_kernel<M, CORR, CX, 4, false, true>),
                                   dim3((unsigned)((waves + 3) / 4)), dim3(256), 4 * group_bytes, st, A, jobs, nj, P.d,
                                   J, pl->d_chains, P.lanes.stride, P.lanes.steps, (int)group_bytes, Q, 1);
        } else if (Q > 1)
            hipLaunchKernelGGL((mdpe::conv_layer_kernel<M, CORR, CX, 1, false, true>), dim3((unsigned)waves), dim3(64),
                               group_bytes, st, A, jobs, nj, P.d, J, pl->d_chains, P.lanes.stride, P.lanes.steps,
                               (int)group_bytes, Q, P.simple ? 1 : 0);
        else if (wpb == 4)
            hipLaunchKernelGGL((mdpe::conv_layer_kernel<M, CORR, CX, 4, false>), dim3((unsigned)blocks), dim3(256),
                               4 * group_bytes, st, A, jobs, nj, P.d, J, pl->d_chains, P.lanes.stride, P.lanes.steps,
                               (int)group_bytes, 1, P.simple ? 1 : 0);
        else
            hipLaunchKernelGGL((mdpe::conv_layer_kernel<M, CORR, CX, 1, false>), dim3((unsigned)blocks), dim3(64),
                               group_bytes, st, A, jobs, nj, P.d, J, pl->d_chains, P.lanes.stride, P.lanes.steps,
                               (int)group_bytes, 1, P.simple ? 1 : 0);
    }
    LAUNCH_CHECK("conv_layer_kernel");
    return record(prof, 1, st, false);
}

// fused layers: one workgroup per component, up to four wavefronts each
// (fewer where their LDS would not fit)
template <int M, bool CX>
int launch_fused(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    const int J = P.fused_lanes.jobs_per_group;  // 1: one job per wavefront
    const size_t group_bytes = (conv_lds_bytes(P.d, mdpe::lds_doubles_per_coef(mdpe::kCoef<M, CX>), J) + 15) / 16 * 16;
    int waves = P.fused_waves;
    while (waves > 1 && waves * group_bytes > (size_t)mdpe::kMaxLdsBytes) --waves;
    static std::atomic<bool> attr_set[kMaxDevices];
    const int dv = pl->device >= 0 && pl->device < kMaxDevices ? pl->device : 0;
    if (!attr_set[dv].load()) {
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_fused_kernel<M, CX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        attr_set[dv].store(true);
    }
    int rc = record(prof, 1, st, true);
    if (rc) return rc;
    hipLaunchKernelGGL((mdpe::conv_fused_kernel<M, CX>), dim3((unsigned)P.fused_components), dim3(64 * waves),
                       waves * group_bytes, st, A, pl->d_fconv, pl->d_foff, P.n_layers(), P.d, J, pl->d_fchains,
                       P.fused_lanes.stride, P.fused_lanes.steps, (int)group_bytes, P.fused_simple ? 1 : 0);
    LAUNCH_CHECK("conv_fused_kernel");
    return record(prof, 1, st, false);
}

// chain launch: one workgroup of pipe_waves wavefronts per chain
template <int M, bool CX>
int launch_chain(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    const long SS = (long)(P.d + 1) * mdpe::kCoef<M, CX>;
    const size_t lds = (size_t)mdpe::conv_lds_jobs_offset((long)P.pipe_ring * SS) +
                       (size_t)P.pipe_layers * sizeof(mdpe::JobOffsets);
    if (lds > (size_t)mdpe::kMaxLdsBytes) return fail(MDPE_EUNSUPPORTED, "chain launch: LDS beyond one workgroup's");
    static std::atomic<bool> attr_set[kMaxDevices];
    const int dv = pl->device >= 0 && pl->device < kMaxDevices ? pl->device : 0;
    if (!attr_set[dv].load()) {
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_chain_kernel<M, CX, 4>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_chain_kernel<M, CX, 8>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_chain_kernel<M, CX, 12>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::conv_chain_kernel<M, CX, 16>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        attr_set[dv].store(true);
    }
    const unsigned chains = (unsigned)P.pipe_comps.size();
    int rc = record(prof, 1, st, true);
    if (rc) return rc;
    if (P.pipe_waves == 4)
        hipLaunchKernelGGL((mdpe::conv_chain_kernel<M, CX, 4>), dim3(chains), dim3(256), lds, st, A, pl->d_pjobs,
                           pl->d_pcomps, pl->d_pcodes, P.d, P.pipe_ring, P.pipe_window);
    else if (P.pipe_waves == 8)
        hipLaunchKernelGGL((mdpe::conv_chain_kernel<M, CX, 8>), dim3(chains), dim3(512), lds, st, A, pl->d_pjobs,
                           pl->d_pcomps, pl->d_pcodes, P.d, P.pipe_ring, P.pipe_window);
    else if (P.pipe_waves == 12)
        hipLaunchKernelGGL((mdpe::conv_chain_kernel<M, CX, 12>), dim3(chains), dim3(768), lds, st, A, pl->d_pjobs,
                           pl->d_pcomps, pl->d_pcodes, P.d, P.pipe_ring, P.pipe_window);
    else if (P.pipe_waves == 16)
        hipLaunchKernelGGL((mdpe::conv_chain_kernel<M, CX, 16>), dim3(chains), dim3(1024), lds, st, A, pl->d_pjobs,
                           pl->d_pcomps, pl->d_pcodes, P.d, P.pipe_ring, P.pipe_window);
    else
        return fail(MDPE_EUNSUPPORTED, "chain launch: 4, 8, 12 or 16 wavefronts per chain");
    LAUNCH_CHECK("conv_chain_kernel");
    return record(prof, 1, st, false);
}

template <int M, bool CX>
int launch_conv(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    if (P.fused_components > 0) return launch_fused<M, CX>(pl, A, st, prof);
    if (P.pipe_layers > 0) {
        int rc = launch_chain<M, CX>(pl, A, st, prof);
        if (rc) return rc;
    }
    for (int L = P.pipe_layers + 1; L <= P.n_layers(); ++L) {
        const long off = P.conv_off[L - 1];
        int rc = launch_layer<M, false, CX>(pl, A, pl->d_conv + off, (int)(P.conv_off[L] - off), st, prof);
        if (rc) return rc;
    }
    return MDPE_OK;
}

template <int M, bool CX>
int launch_add(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    for (int r = 1; r <= P.n_levels(); ++r) {
        const long off = P.add_off[r - 1];
        const long np = P.add_off[r] - off;
        if (np == 0) continue;
        const long total = np * (P.d + 1);
        int rc = record(prof, 2, st, true);
        if (rc) return rc;
        hipLaunchKernelGGL((mdpe::add_level_kernel<M, CX>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A,
                           pl->d_add + off, total, P.d);
        LAUNCH_CHECK("add_level_kernel");
        if ((rc = record(prof, 2, st, false))) return rc;
    }
    return MDPE_OK;
}

template <int M, bool CX>
int launch_scale(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    if (P.scale.empty()) return MDPE_OK;
    const long total = (long)P.scale.size() * (P.d + 1);
    int rc = record(prof, 2, st, true);
    if (rc) return rc;
    hipLaunchKernelGGL((mdpe::scale_kernel<M, CX>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A,
                       pl->d_scale, total, P.d);
    LAUNCH_CHECK("scale_kernel");
    return record(prof, 2, st, false);
}

// single launch: the whole evaluation in one workgroup of single_waves wavefronts
template <int M, bool CX>
int launch_single(const mdpe_plan *pl, double *A, const double *coeff, const double *z, double *value, double *grad,
                  hipStream_t st, mdpe_profiler *prof) {
    const mdpe::Plan &P = pl->P;
    const int J = P.single_lanes.jobs_per_group;
    const size_t gb = (conv_lds_bytes(P.d, mdpe::lds_doubles_per_coef(mdpe::kCoef<M, CX>), J) + 15) / 16 * 16;
    size_t lds = gb * (size_t)P.single_waves;
    // the workspace in LDS too when it fits beside the job groups
    const long ws_doubles = P.n_series * (long)(P.d + 1) * mdpe::kCoef<M, CX>;
    const bool ws_lds = lds + (size_t)ws_doubles * sizeof(double) <= (size_t)mdpe::kMaxLdsBytes;
    const int ws_off = (int)lds;
    if (ws_lds) lds += (size_t)ws_doubles * sizeof(double);
    if (lds > (size_t)mdpe::kMaxLdsBytes) return fail(MDPE_EUNSUPPORTED, "single launch: LDS beyond one workgroup's");
    static std::atomic<bool> attr_set[kMaxDevices];
    const int dv = pl->device >= 0 && pl->device < kMaxDevices ? pl->device : 0;
    if (!attr_set[dv].load()) {
        HIP_TRY(hipFuncSetAttribute((const void *)mdpe::eval_single_kernel<M, CX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mdpe::kMaxLdsBytes));
        attr_set[dv].store(true);
    }
    mdpe::SingleArgs a;
    a.A = A;
    a.ws_doubles = ws_lds ? ws_doubles : 0;
    a.lds_ws_off = ws_off;
    a.coeff = coeff;
    a.z = z;
    a.value = value;
    a.grad = grad;
    a.stage = pl->d_stage;
    a.nstage = (int)P.stage.size();
    a.conv = pl->d_conv;
    a.conv_off = pl->d_coff;
    a.nl = P.n_layers();
    a.chains = pl->d_schains;
    a.stride = P.single_lanes.stride;
    a.steps = P.single_lanes.steps;
    a.J = J;
    a.simple = P.single_simple ? 1 : 0;
    a.group_bytes = (int)gb;
    a.scale = pl->d_scale;
    a.nscale = (int)P.scale.size();
    a.add = pl->d_add;
    a.add_off = pl->d_aoff;
    a.nlev = P.n_levels();
    a.out = pl->d_out;
    a.n = P.n;
    a.N = P.N;
    a.d = P.d;
    int rc = record(prof, 1, st, true);
    if (rc) return rc;
    hipLaunchKernelGGL((mdpe::eval_single_kernel<M, CX>), dim3(1), dim3(64 * P.single_waves), lds, st, a);
    LAUNCH_CHECK("eval_single_kernel");
    return record(prof, 1, st, false);
}

template <int M>
int run_single(const mdpe_plan *pl, double *A, const double *coeff, const double *z, double *value, double *grad,
               hipStream_t st, mdpe_profiler *prof) {
    return pl->P.complex_series() ? launch_single<M, true>(pl, A, coeff, z, value, grad, st, prof)
                                  : launch_single<M, false>(pl, A, coeff, z, value, grad, st, prof);
}

template <int M, bool CX>
int run_field(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    int rc;
    if ((rc = launch_conv<M, CX>(pl, A, st, prof))) return rc;
    if ((rc = launch_scale<M, CX>(pl, A, st, prof))) return rc;
    return launch_add<M, CX>(pl, A, st, prof);
}

template <int M>
int run_md(const mdpe_plan *pl, double *A, hipStream_t st, mdpe_profiler *prof) {
    return pl->P.complex_series() ? run_field<M, true>(pl, A, st, prof) : run_field<M, false>(pl, A, st, prof);
}

int eval_impl(const mdpe_plan *pl, const double *coeff, const double *z, double *value, double *grad,
              void *workspace, void *stream, mdpe_profiler *prof) {
    if (!pl) return fail(MDPE_EINVAL, "plan is NULL");
    if (pl->device < 0) return fail(MDPE_EINVAL, "host-only plan (device -1) cannot evaluate");
    const mdpe::Plan &P = pl->P;
    if (!coeff || !z || !value || !grad || !workspace)
        return fail(MDPE_EINVAL, "NULL buffer (coeff, z, value, grad and workspace are required)");
    if (((uintptr_t)workspace) % 256) return fail(MDPE_EINVAL, "workspace must be 256-byte aligned");
    DeviceGuard g(pl->device);
    if (!g.ok) return fail(MDPE_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    double *A = (double *)workspace;
    const int d1 = P.d + 1;
    int rc;
    if (P.single) {
        switch (P.m) {
            case 1: return run_single<1>(pl, A, coeff, z, value, grad, st, prof);
            case 2: return run_single<2>(pl, A, coeff, z, value, grad, st, prof);
            case 3: return run_single<3>(pl, A, coeff, z, value, grad, st, prof);
            case 4: return run_single<4>(pl, A, coeff, z, value, grad, st, prof);
            case 5: return run_single<5>(pl, A, coeff, z, value, grad, st, prof);
            case 8: return run_single<8>(pl, A, coeff, z, value, grad, st, prof);
            case 10: return run_single<10>(pl, A, coeff, z, value, grad, st, prof);
            default: return fail(MDPE_EUNSUPPORTED, "unsupported m");
        }
    }
    {
        const long total = (long)P.stage.size() * d1;
        if ((rc = record(prof, 0, st, true))) return rc;
        hipLaunchKernelGGL(mdpe::stage_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, coeff, z,
                           pl->d_stage, total, P.N, P.n, P.d, P.w);
        LAUNCH_CHECK("stage_kernel");
        if ((rc = record(prof, 0, st, false))) return rc;
    }
    switch (P.m) {
        case 1: rc = run_md<1>(pl, A, st, prof); break;
        case 2: rc = run_md<2>(pl, A, st, prof); break;
        case 3: rc = run_md<3>(pl, A, st, prof); break;
        case 4: rc = run_md<4>(pl, A, st, prof); break;
        case 5: rc = run_md<5>(pl, A, st, prof); break;
        case 8: rc = run_md<8>(pl, A, st, prof); break;
        case 10: rc = run_md<10>(pl, A, st, prof); break;
        default: return fail(MDPE_EUNSUPPORTED, "unsupported m");
    }
    if (rc) return rc;
    {
        const long total = (long)(1 + P.n) * d1;
        if ((rc = record(prof, 3, st, true))) return rc;
        hipLaunchKernelGGL(mdpe::gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, value,
                           grad, pl->d_out, P.n, P.d, P.w);
        LAUNCH_CHECK("gather_kernel");
        if ((rc = record(prof, 3, st, false))) return rc;
    }
    return MDPE_OK;
}

int adjoint_impl(const mdpe_plan *pl, const double *ybar, void *workspace, const double *grad, double *coeff_bar,
                 double *z_bar, void *stream, mdpe_profiler *prof) {
    if (!pl) return fail(MDPE_EINVAL, "plan is NULL");
    if (pl->device < 0) return fail(MDPE_EINVAL, "host-only plan (device -1) cannot evaluate");
    const mdpe::Plan &P = pl->P;
    if (!(P.flags & mdpe::kKeepMonomialValues))
        return fail(MDPE_EINVAL, "the plan was built without MDPE_KEEP_MONOMIAL_VALUES");
    if (!ybar || !workspace || !grad || !coeff_bar || !z_bar) return fail(MDPE_EINVAL, "NULL buffer");
    if (((uintptr_t)workspace) % 256) return fail(MDPE_EINVAL, "workspace must be 256-byte aligned");
    DeviceGuard g(pl->device);
    if (!g.ok) return fail(MDPE_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    double *A = (double *)workspace;
    const int d1 = P.d + 1;
    int rc;
    if ((rc = record(prof, 0, st, true))) return rc;
    hipLaunchKernelGGL(mdpe::planar_to_slots_kernel, dim3((unsigned)((d1 + 255) / 256)), dim3(256), 0, st, A, ybar, 1,
                       pl->d_ybar, (long)d1, P.d, P.m);
    LAUNCH_CHECK("planar_to_slots_kernel");
    {
        // the caller's gradient g_i into the slots the correlations read
        const long tg = (long)P.n * d1;
        hipLaunchKernelGGL(mdpe::planar_to_slots_kernel, dim3((unsigned)((tg + 255) / 256)), dim3(256), 0, st, A, grad,
                           P.n, pl->d_out + 1, tg, P.d, P.m);
        LAUNCH_CHECK("planar_to_slots_kernel");
    }
    if ((rc = record(prof, 0, st, false))) return rc;
    const int nj = (int)P.corr.size();
    switch (P.m) {
        case 1: rc = launch_layer<1, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 2: rc = launch_layer<2, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 3: rc = launch_layer<3, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 4: rc = launch_layer<4, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 5: rc = launch_layer<5, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 8: rc = launch_layer<8, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        case 10: rc = launch_layer<10, true, false>(pl, A, pl->d_corr, nj, st, prof); break;
        default: return fail(MDPE_EUNSUPPORTED, "unsupported m");
    }
    if (rc) return rc;
    if ((rc = record(prof, 3, st, true))) return rc;
    {
        const long tc = (long)(P.N + 1) * d1, tz = (long)P.n * d1;
        hipLaunchKernelGGL(mdpe::slots_to_planar_kernel, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0, st, A,
                           coeff_bar, P.N + 1, pl->d_cbar, P.d, P.m);
        LAUNCH_CHECK("slots_to_planar_kernel");
        hipLaunchKernelGGL(mdpe::slots_to_planar_kernel, dim3((unsigned)((tz + 255) / 256)), dim3(256), 0, st, A,
                           z_bar, P.n, pl->d_zbar, P.d, P.m);
        LAUNCH_CHECK("slots_to_planar_kernel");
    }
    return record(prof, 3, st, false);
}

template <int M>
void launch_elementwise(int op, long count, const double *x, const double *y, double *z, hipStream_t st) {
    const dim3 grid((unsigned)((count + 255) / 256));
    if (op >= 2)
        hipLaunchKernelGGL((mdpe::md_elementwise_kernel<M, true>), grid, dim3(256), 0, st, op - 2, count, x, y, z);
    else
        hipLaunchKernelGGL((mdpe::md_elementwise_kernel<M, false>), grid, dim3(256), 0, st, op, count, x, y, z);
}

}  // namespace

// ------------------------------------------------- allocation-free entry --
// eval_and_diff_noalloc runs on a workspace the library holds from load to
// process end: one fixed array per device, sized for plans of up to
// kScratchBytes of workspace (64 MiB: every series slot of p2 at quad double
// and d = 64, 50.6 MB, or of p1 at octo double and d = 32 with the monomial
// values kept).  Every call on a device shares that device's copy; calls that
// overlap on one device race.  Nothing in it must start at zero: staging
// writes the inputs, and every convolution and addition writes its output
// slot before any job reads it.
namespace {
constexpr int64_t kScratchBytes = 64ll << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

// The array's device address on `device` (each device holds its own copy).
// Looked up once per device, with that device current; host code uses this
// address, never the array's name, wherever it needs the array's memory.
int scratch_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices];
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        DeviceGuard g(device);
        if (!g.ok) return fail(MDPE_EDEVICE, "cannot select the plan's device");
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MDPE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[device] = p;
    }
    *out = addr[device];
    return MDPE_OK;
}
}  // namespace

extern "C" {

int plan_polynomial(const mdpe_poly_desc *desc, int device, mdpe_plan **out) {
    if (!desc || !out) return fail(MDPE_EINVAL, "desc and out are required");
    *out = nullptr;
    if (desc->flags & ~(uint32_t)(MDPE_KEEP_MONOMIAL_VALUES | MDPE_COMPLEX | MDPE_STREAM_OPERANDS | MDPE_STAGE_OPERANDS |
                                MDPE_ASAP_LAYERS | MDPE_FUSED_LAYERS | MDPE_LAYER_LAUNCHES | MDPE_CHAIN_LAUNCH |
                                MDPE_NO_CHAIN_LAUNCH | MDPE_SINGLE_LAUNCH))
        return fail(MDPE_EINVAL, "unknown flags");
    if (device < -1) return fail(MDPE_EINVAL, "device must be >= -1");
    std::unique_ptr<mdpe_plan> pl(new (std::nothrow) mdpe_plan());
    if (!pl) return fail(MDPE_ENOMEM, "host allocation failed");
    bool unsupported = false;
    std::string err;
    try {
        err = mdpe::build_plan(desc->n, desc->N, desc->d, desc->m, desc->nvars, desc->vars, desc->exps, desc->flags, pl->P,
                               &unsupported);
    } catch (const std::bad_alloc &) {
        return fail(MDPE_ENOMEM, "host allocation failed while planning");
    }
    if (!err.empty()) return fail(unsupported ? MDPE_EUNSUPPORTED : MDPE_EINVAL, err);
    if (device >= 0) {
        int ndev = 0;
        HIP_TRY(hipGetDeviceCount(&ndev));
        if (device >= ndev) return fail(MDPE_EINVAL, "no such device");
        DeviceGuard g(device);
        if (!g.ok) return fail(MDPE_EDEVICE, "cannot select device");
        pl->device = device;
        const mdpe::Plan &P = pl->P;
        std::vector<int4> conv(P.conv.size());
        for (size_t q = 0; q < P.conv.size(); ++q) conv[q] = make_int4(P.conv[q][0], P.conv[q][1], P.conv[q][2], 0);
        std::vector<int4> corr(P.corr.size());
        for (size_t q = 0; q < P.corr.size(); ++q) corr[q] = make_int4(P.corr[q][0], P.corr[q][1], P.corr[q][2], 0);
        std::vector<int4> scale(P.scale.size());
        for (size_t q = 0; q < P.scale.size(); ++q) scale[q] = make_int4(P.scale[q][0], P.scale[q][1], P.scale[q][2], 0);
        std::vector<int4> fconv(P.fused_conv.size());
        for (size_t q = 0; q < P.fused_conv.size(); ++q)
            fconv[q] = make_int4(P.fused_conv[q][0], P.fused_conv[q][1], P.fused_conv[q][2], 0);
        std::vector<int4> pjobs(P.pipe_jobs.size());
        for (size_t q = 0; q < P.pipe_jobs.size(); ++q)
            pjobs[q] = make_int4(P.pipe_jobs[q][0], P.pipe_jobs[q][1], P.pipe_jobs[q][2], 0);
        std::vector<int32_t> coff(P.conv_off.begin(), P.conv_off.end()), aoff(P.add_off.begin(), P.add_off.end());
        std::vector<int2> add(P.add.size()), stage(P.stage.size());
        for (size_t q = 0; q < P.add.size(); ++q) add[q] = make_int2(P.add[q][0], P.add[q][1]);
        for (size_t q = 0; q < P.stage.size(); ++q) stage[q] = make_int2(P.stage[q][0], P.stage[q][1]);
        int rc;
        mdpe_plan *raw = pl.get();
        if ((rc = upload(&raw->d_conv, conv.data(), conv.size() * sizeof(int4))) ||
            (rc = upload(&raw->d_add, add.data(), add.size() * sizeof(int2))) ||
            (rc = upload(&raw->d_stage, stage.data(), stage.size() * sizeof(int2))) ||
            (rc = upload(&raw->d_out, P.out_slots.data(), P.out_slots.size() * sizeof(int))) ||
            (rc = upload(&raw->d_chains, P.lanes.chains.data(), P.lanes.chains.size() * sizeof(int))) ||
            (rc = upload(&raw->d_corr, corr.data(), corr.size() * sizeof(int4))) ||
            (rc = upload(&raw->d_cbar, P.coeff_bar_slots.data(), P.coeff_bar_slots.size() * sizeof(int))) ||
            (rc = upload(&raw->d_zbar, P.z_bar_slots.data(), P.z_bar_slots.size() * sizeof(int))) ||
            (rc = upload(&raw->d_ybar, &P.ybar_slot, sizeof(int))) ||
            (rc = upload(&raw->d_scale, scale.data(), scale.size() * sizeof(int4))) ||
            (rc = upload(&raw->d_fconv, fconv.data(), fconv.size() * sizeof(int4))) ||
            (rc = upload(&raw->d_foff, P.fused_off.data(), P.fused_off.size() * sizeof(int))) ||
            (rc = upload(&raw->d_fchains, P.fused_lanes.chains.data(), P.fused_lanes.chains.size() * sizeof(int))) ||
            (rc = upload(&raw->d_pjobs, pjobs.data(), pjobs.size() * sizeof(int4))) ||
            (rc = upload(&raw->d_pcomps, P.pipe_comps.data(), P.pipe_comps.size() * sizeof(mdpe::ChainComp))) ||
            (rc = upload(&raw->d_pcodes, P.pipe_codes.data(), P.pipe_codes.size() * sizeof(int))) ||
            (rc = upload(&raw->d_coff, coff.data(), coff.size() * sizeof(int))) ||
            (rc = upload(&raw->d_aoff, aoff.data(), aoff.size() * sizeof(int))) ||
            (rc = upload(&raw->d_schains, P.single_lanes.chains.data(), P.single_lanes.chains.size() * sizeof(int)))) {
            std::string keep = g_err;
            free_plan(pl.release());
            g_err = keep;
            return rc;
        }
    }
    *out = pl.release();
    return MDPE_OK;
}

int plan_info(const mdpe_plan *pl, mdpe_plan_info *o) {
    if (!pl || !o) return fail(MDPE_EINVAL, "plan and out are required");
    const mdpe::Plan &P = pl->P;
    o->n_series = P.n_series;
    o->n_conv = (int64_t)P.conv.size();
    o->n_add = (int64_t)P.add.size();
    o->n_layers = P.n_layers();
    o->n_levels = P.n_levels();
    o->workspace_bytes = P.n_series * (int64_t)(P.d + 1) * P.w * (int64_t)sizeof(double);
    o->jobs_per_group = P.lanes.jobs_per_group;
    o->lane_steps = P.lanes.steps;
    o->n_reverse = (int64_t)P.corr.size();
    o->n_scale = (int64_t)P.scale.size();
    o->waves_per_job = P.lanes.waves_per_job;
    o->streamed = P.streamed ? 1 : 0;
    o->simple_dealing = P.simple ? 1 : 0;
    o->balanced_layers = P.balanced ? 1 : 0;
    o->fused_components = P.fused_components;
    o->fused_waves = P.fused_waves;
    o->chain_layers = P.pipe_layers;
    o->chain_count = (int32_t)P.pipe_comps.size();
    o->chain_waves = P.pipe_waves;
    o->chain_window = P.pipe_window;
    o->chain_ring = P.pipe_ring;
    o->single_launch = P.single ? 1 : 0;
    o->single_waves = P.single_waves;
    o->flags = P.flags;
    o->n = P.n;
    o->N = P.N;
    o->d = P.d;
    o->m = P.m;
    return MDPE_OK;
}

int plan_layer_sizes(const mdpe_plan *pl, int32_t *conv_sizes, int32_t *add_sizes) {
    if (!pl) return fail(MDPE_EINVAL, "plan is NULL");
    const mdpe::Plan &P = pl->P;
    if (conv_sizes)
        for (int L = 0; L < P.n_layers(); ++L) conv_sizes[L] = (int32_t)(P.conv_off[L + 1] - P.conv_off[L]);
    if (add_sizes)
        for (int r = 0; r < P.n_levels(); ++r) add_sizes[r] = (int32_t)(P.add_off[r + 1] - P.add_off[r]);
    return MDPE_OK;
}

int plan_fused_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    if (P.fused_components == 0) return fail(MDPE_EINVAL, "the plan does not fuse its layers (MDPE_FUSED_LAYERS)");
    const int nl = P.n_layers();
    for (int32_t c = 0; c < P.fused_components; ++c)
        for (int L = 1; L <= nl; ++L)
            for (int32_t q = P.fused_off[(size_t)c * (nl + 1) + L - 1]; q < P.fused_off[(size_t)c * (nl + 1) + L]; ++q) {
                rows[5 * q] = c;
                rows[5 * q + 1] = L;
                rows[5 * q + 2] = P.fused_conv[q][0];
                rows[5 * q + 3] = P.fused_conv[q][1];
                rows[5 * q + 4] = P.fused_conv[q][2];
            }
    return MDPE_OK;
}

int plan_conv_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    for (int L = 1; L <= P.n_layers(); ++L)
        for (int64_t q = P.conv_off[L - 1]; q < P.conv_off[L]; ++q) {
            rows[4 * q] = L;
            rows[4 * q + 1] = P.conv[q][0];
            rows[4 * q + 2] = P.conv[q][1];
            rows[4 * q + 3] = P.conv[q][2];
        }
    return MDPE_OK;
}

int plan_add_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    for (int r = 1; r <= P.n_levels(); ++r)
        for (int64_t q = P.add_off[r - 1]; q < P.add_off[r]; ++q) {
            rows[3 * q] = r;
            rows[3 * q + 1] = P.add[q][0];
            rows[3 * q + 2] = P.add[q][1];
        }
    return MDPE_OK;
}

int plan_outputs(const mdpe_plan *pl, int32_t *out_slots) {
    if (!pl || !out_slots) return fail(MDPE_EINVAL, "plan and out_slots are required");
    std::memcpy(out_slots, pl->P.out_slots.data(), pl->P.out_slots.size() * sizeof(int32_t));
    return MDPE_OK;
}

int plan_scale_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    for (size_t q = 0; q < P.scale.size(); ++q)
        for (int r = 0; r < 3; ++r) rows[3 * q + r] = P.scale[q][r];
    return MDPE_OK;
}

int eval_and_diff(const mdpe_plan *pl, const double *coeff, const double *z, double *value, double *grad,
                  void *workspace, void *stream) {
    return eval_impl(pl, coeff, z, value, grad, workspace, stream, nullptr);
}

int eval_and_diff_noalloc(const mdpe_plan *pl, const double *coeff, const double *z, double *value, double *grad,
                          void *stream) {
    if (!pl) return fail(MDPE_EINVAL, "plan is NULL");
    if (pl->device < 0 || pl->device >= kMaxDevices)
        return fail(MDPE_EINVAL, "eval_and_diff_noalloc needs a device plan on devices 0..63");
    const mdpe::Plan &P = pl->P;
    const int64_t need = P.n_series * (int64_t)(P.d + 1) * P.w * (int64_t)sizeof(double);
    if (need > kScratchBytes)
        return fail(MDPE_EUNSUPPORTED, "eval_and_diff_noalloc: the plan needs a workspace of " + std::to_string(need) +
                                           " bytes, above the library's fixed " + std::to_string(kScratchBytes) +
                                           "; use eval_and_diff with a workspace of the caller");
    void *ws = nullptr;
    int rc = scratch_address(pl->device, &ws);
    if (rc) return rc;
    return eval_impl(pl, coeff, z, value, grad, ws, stream, nullptr);
}

int eval_and_diff_profiled(const mdpe_plan *pl, const double *coeff, const double *z, double *value, double *grad,
                           void *workspace, void *stream, mdpe_profiler *prof) {
    if (!prof) return fail(MDPE_EINVAL, "profiler is NULL");
    return eval_impl(pl, coeff, z, value, grad, workspace, stream, prof);
}

int profiler_create(mdpe_profiler **out) {
    if (!out) return fail(MDPE_EINVAL, "out is NULL");
    *out = new (std::nothrow) mdpe_profiler();
    return *out ? MDPE_OK : fail(MDPE_ENOMEM, "host allocation failed");
}

int profiler_set_classes(mdpe_profiler *prof, uint32_t classes) {
    if (!prof) return fail(MDPE_EINVAL, "profiler is NULL");
    if (classes & ~0xfu) return fail(MDPE_EINVAL, "unknown launch classes");
    if (prof->used) return fail(MDPE_EINVAL, "read the recorded events first");
    prof->classes = classes;
    return MDPE_OK;
}

int profiler_read(mdpe_profiler *prof, mdpe_times *o) {
    if (!prof || !o) return fail(MDPE_EINVAL, "profiler and out are required");
    for (size_t q = 0; q < prof->used; ++q) {
        auto &r = prof->recs[q];
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        switch (r.cls) {
            case 0: o->stage_ms += ms; o->n_stage++; break;
            case 1: o->cnv_ms += ms; o->n_cnv++; break;
            case 2: o->add_ms += ms; o->n_add++; break;
            default: o->gather_ms += ms; o->n_gather++; break;
        }
    }
    prof->used = 0;
    return MDPE_OK;
}

void profiler_destroy(mdpe_profiler *prof) {
    if (!prof) return;
    for (auto &r : prof->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    delete prof;
}

int md_elementwise(int op, int m, int64_t count, const double *x, const double *y, double *z, void *stream) {
    if (op < 0 || op > 3) return fail(MDPE_EINVAL, "op must be 0 (add), 1 (mul), 2 (complex add) or 3 (complex mul)");
    if (count < 0) return fail(MDPE_EINVAL, "count < 0");
    if (count == 0) return MDPE_OK;
    if (!x || !y || !z) return fail(MDPE_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    switch (m) {
        case 1: launch_elementwise<1>(op, (long)count, x, y, z, st); break;
        case 2: launch_elementwise<2>(op, (long)count, x, y, z, st); break;
        case 3: launch_elementwise<3>(op, (long)count, x, y, z, st); break;
        case 4: launch_elementwise<4>(op, (long)count, x, y, z, st); break;
        case 5: launch_elementwise<5>(op, (long)count, x, y, z, st); break;
        case 8: launch_elementwise<8>(op, (long)count, x, y, z, st); break;
        case 10: launch_elementwise<10>(op, (long)count, x, y, z, st); break;
        default: return fail(MDPE_EUNSUPPORTED, "unsupported m");
    }
    LAUNCH_CHECK("md_elementwise_kernel");
    return MDPE_OK;
}

int eval_adjoint(const mdpe_plan *pl, const double *ybar, void *workspace, const double *grad, double *coeff_bar,
                 double *z_bar, void *stream) {
    return adjoint_impl(pl, ybar, workspace, grad, coeff_bar, z_bar, stream, nullptr);
}

int eval_adjoint_profiled(const mdpe_plan *pl, const double *ybar, void *workspace, const double *grad,
                          double *coeff_bar, double *z_bar, void *stream, mdpe_profiler *prof) {
    if (!prof) return fail(MDPE_EINVAL, "profiler is NULL");
    return adjoint_impl(pl, ybar, workspace, grad, coeff_bar, z_bar, stream, prof);
}

int plan_reverse_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    for (size_t q = 0; q < P.corr.size(); ++q)
        for (int r = 0; r < 3; ++r) rows[3 * q + r] = P.corr[q][r];
    return MDPE_OK;
}

int plan_chain_jobs(const mdpe_plan *pl, int32_t *rows) {
    if (!pl || !rows) return fail(MDPE_EINVAL, "plan and rows are required");
    const mdpe::Plan &P = pl->P;
    if (P.pipe_layers == 0) return fail(MDPE_EINVAL, "the plan has no chain launch (MDPE_CHAIN_LAUNCH)");
    for (size_t c = 0; c < P.pipe_comps.size(); ++c) {
        const mdpe::ChainComp &cc = P.pipe_comps[c];
        for (int32_t q = 0; q < cc.len; ++q) {
            const auto &t = P.pipe_jobs[(size_t)cc.first + q];
            int32_t *r = rows + 5 * ((size_t)cc.first + q);
            r[0] = (int32_t)c;
            r[1] = q;
            r[2] = t[0];
            r[3] = t[1];
            r[4] = t[2];
        }
    }
    return MDPE_OK;
}

int chain_schedule(int32_t L, int32_t d, int32_t waves, int32_t window, int32_t ring, int32_t *codes,
                   int64_t capacity, int32_t *stride, int32_t *steps) {
    if (L < 1 || L > mdpe::kMaxChainLength || d < 0 || d > 4095 || waves < 4 || waves > 16 || waves % 4 || window < 1 ||
        ring < 2 || !stride || !steps || capacity < 0)
        return fail(MDPE_EINVAL, "need 1 <= L <= 2048, 0 <= d <= 4095, waves 4, 8, 12 or 16, window >= 1, ring >= 2");
    std::vector<int32_t> cs;
    int st = 0;
    try {
        *steps = mdpe::make_chain_schedule(L, d, waves, window, ring, cs, &st);
    } catch (const std::bad_alloc &) {
        return fail(MDPE_ENOMEM, "host allocation failed");
    }
    *stride = st;
    if (codes) {
        if ((int64_t)cs.size() > capacity) return fail(MDPE_EINVAL, "codes: capacity below 64 * waves * stride");
        std::memcpy(codes, cs.data(), cs.size() * sizeof(int32_t));
    }
    return MDPE_OK;
}

int check_chain_schedule(int32_t L, int32_t d, int32_t waves, int32_t window, int32_t ring, int32_t steps,
                         const int32_t *codes, int32_t stride) {
    std::string e;
    try {
        e = mdpe::check_chain_schedule(L, d, waves, window, ring, steps, codes, stride);
    } catch (const std::bad_alloc &) {
        return fail(MDPE_ENOMEM, "host allocation failed");
    }
    if (!e.empty()) return fail(MDPE_EINVAL, e);
    return MDPE_OK;
}

int check_plan_jobs(int32_t n, int32_t N, int64_t n_series, const int32_t *conv_rows, int64_t n_conv,
                    const int32_t *add_rows, int64_t n_add, const int32_t *out_slots, const int32_t *extra_staged,
                    int64_t n_extra, int32_t waves_per_job, int32_t streamed) {
    if (n < 1 || N < 0 || n_series < 1 + (int64_t)N + n || n_series > INT32_MAX)
        return fail(MDPE_EINVAL, "need n >= 1, N >= 0 and 1 + N + n <= n_series < 2^31");
    if (n_conv < 0 || n_add < 0 || n_extra < 0 || waves_per_job < 1)
        return fail(MDPE_EINVAL, "negative count, or waves_per_job < 1");
    if ((n_conv && !conv_rows) || (n_add && !add_rows) || (n_extra && !extra_staged))
        return fail(MDPE_EINVAL, "NULL rows");
    mdpe::Plan P;
    P.n = n;
    P.N = N;
    P.n_series = n_series;
    P.streamed = streamed != 0;
    P.lanes.waves_per_job = waves_per_job;
    for (int32_t s = 0; s < 1 + N + n; ++s) P.stage.push_back({s, s});
    for (int64_t q = 0; q < n_extra; ++q) {
        if (extra_staged[q] < 0 || extra_staged[q] >= n_series) return fail(MDPE_EINVAL, "staged slot out of range");
        P.stage.push_back({extra_staged[q], 0});
    }
    // rows grouped by layer / level, numbered from 1 in nondecreasing order
    // off[L-1] .. off[L]: the rows of layer (level) L
    auto group = [&](const int32_t *rows, int64_t count, int width, std::vector<int64_t> &off) -> bool {
        off.assign(1, 0);
        int32_t cur = 1;
        for (int64_t q = 0; q < count; ++q) {
            const int32_t L = rows[width * q];
            if (L < cur) return false;
            for (; cur < L; ++cur) off.push_back(q);
        }
        if (count > 0) off.push_back(count);
        return true;
    };
    if (!group(conv_rows, n_conv, 4, P.conv_off)) return fail(MDPE_EINVAL, "conv rows: layers must start at 1 and not decrease");
    if (!group(add_rows, n_add, 3, P.add_off)) return fail(MDPE_EINVAL, "add rows: levels must start at 1 and not decrease");
    for (int64_t q = 0; q < n_conv; ++q) P.conv.push_back({conv_rows[4 * q + 1], conv_rows[4 * q + 2], conv_rows[4 * q + 3]});
    for (int64_t q = 0; q < n_add; ++q) P.add.push_back({add_rows[3 * q + 1], add_rows[3 * q + 2]});
    if (out_slots)
        for (int32_t o = 0; o <= n; ++o) {
            if (out_slots[o] < -1 || out_slots[o] >= n_series) return fail(MDPE_EINVAL, "output slot out of range");
            P.out_slots.push_back(out_slots[o]);
        }
    std::string e = mdpe::check_hazards(P);
    if (!e.empty()) return fail(MDPE_EINVAL, e);
    return MDPE_OK;
}

void plan_destroy(mdpe_plan *pl) { free_plan(pl); }

const char *last_error_string(void) { return g_err.c_str(); }

}  // extern "C"
