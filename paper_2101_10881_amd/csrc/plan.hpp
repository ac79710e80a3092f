// plan.hpp -- host-side data staging (Section 5 of the paper): series slots,
// convolution triplets per layer, addition pairs per level, output slots,
// hazard check and the lane schedule of the convolution kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace mdpe {

constexpr int kLanes = 64;             // one wavefront per convolution workgroup
constexpr int kMaxLdsBytes = 163840;   // LDS one gfx950 workgroup may allocate
constexpr int kLdsBudget = 65536;      // LDS a workgroup aims to stay under (>= 2 per CU)
constexpr int kMaxExponent = 64;

struct LaneSchedule {
    int jobs_per_group = 1;            // J: convolution jobs staged per workgroup
    int waves_per_job = 1;             // Q: wavefronts sharing one job's coefficients (J = 1 when Q > 1)
    int steps = 0;                     // multiply-add steps of the busiest lane
    int stride = 0;                    // entries per lane in `chains`
    // chains[row*stride + s]: (job << 16) | k for the s-th output coefficient
    // schedule row `row` computes, -1 after its last one; row q*64 + lane is
    // lane `lane` of the q-th of the Q wavefronts of a group.
    std::vector<int32_t> chains;
};

// The convolution kernel stages both operands of a job in LDS when a
// coefficient is at most two doubles (short steps: the second operand's
// latency from L2 would dominate), else only the first.  Doubles of LDS per
// coefficient of a job:
__host__ __device__ constexpr bool stages_second_operand(int w) { return w <= 2; }
__host__ __device__ constexpr int lds_doubles_per_coef(int w) { return stages_second_operand(w) ? 2 * w : w; }

// A job's three series as offsets (in doubles) into A: first operand, second
// operand, output.  Kept in LDS, so that a lane starting a chain finds its
// operands' addresses with one LDS read and an add.
struct JobOffsets {
    long x, y, z, unused;
};

// LDS layout of one wavefront's group: X[J][d+1][W] doubles (the first
// operands), Y[J][d+1][W] (the second operands, only when
// stages_second_operand(W)), then the J JobOffsets (16-byte aligned).
// `doubles_per_coef` is lds_doubles_per_coef(W), or 0 for streamed operands.
__host__ __device__ inline long conv_lds_jobs_offset(long xdoubles) { return (xdoubles * 8 + 15) / 16 * 16; }
__host__ __device__ inline long group_lds_bytes(long d1, int doubles_per_coef, int J) {
    return conv_lds_jobs_offset((long)J * d1 * doubles_per_coef) + (long)J * (long)sizeof(JobOffsets);
}

constexpr uint32_t kKeepMonomialValues = 1u;
constexpr uint32_t kComplex = 2u;          // complex series: real limbs, then imaginary limbs
constexpr uint32_t kStreamOperands = 4u;   // read both convolution operands from global memory
constexpr uint32_t kStageOperands = 8u;    // stage them in LDS (no automatic streaming)
constexpr uint32_t kAsapLayers = 16u;      // every convolution at its earliest layer (no balancing)
constexpr uint32_t kFusedLayers = 32u;     // all convolution layers in one launch, per independent component
constexpr uint32_t kLayerLaunches = 64u;   // one launch per convolution layer (no automatic fusing)
constexpr uint32_t kChainLaunch = 128u;    // first-operand chains in one pipelined launch (see Plan::pipe_*)
constexpr uint32_t kNoChainLaunch = 256u;  // never the chain launch (the plan chooses the rest)
constexpr uint32_t kSingleLaunch = 512u;   // the whole evaluation in one launch of one workgroup

// Chain launch: the code of an idle stretch in a lane's entry list (job field)
constexpr int32_t kIdleJob = 0x7FFF;    // codes stay positive; chain jobs are numbered below it
constexpr int kMaxChainLength = 2048;      // jobs of one chain (their descriptors sit in LDS)

// One chain of the chain launch: its jobs pipe_jobs[first .. first+len), its
// lane schedule at pipe_codes[code_off], `stride` entries per row, `steps`
// steps (a multiple of the barrier window).
struct ChainComp {
    int32_t first, len, code_off, stride, steps, pad0, pad1, pad2;
};

struct Plan {
    int n = 0, N = 0, d = 0, m = 0;
    int w = 0;                         // doubles per coefficient: m, or 2m for complex series
    uint32_t flags = 0;
    int64_t n_series = 0;
    // convolution jobs {t1, t2, t3} in launch order; layer L spans
    // conv[conv_off[L-1] .. conv_off[L])
    std::vector<std::array<int32_t, 3>> conv;
    std::vector<int64_t> conv_off;
    // addition jobs {t1, t2}: A[t2] += A[t1]; level r spans add[add_off[r-1] .. add_off[r])
    std::vector<std::array<int32_t, 2>> add;
    std::vector<int64_t> add_off;
    std::vector<int32_t> out_slots;    // [1+n]: value slot, then d/dz_i slot or -1
    // staging copies {slot, source}: source s < N+1 is coeff series s, else z series s-N-1
    std::vector<std::array<int32_t, 2>> stage;
    // general exponents: scale jobs {src, dst, e}, A[dst] := e * A[src] per
    // coefficient, run after the last convolution layer, before the additions
    std::vector<std::array<int32_t, 3>> scale;
    LaneSchedule lanes;
    // reverse pass (flags & kKeepMonomialValues): one layer of correlation jobs
    // {t1 = ybar slot, t2 = M_k or gradient slot, t3 = output slot}
    int32_t ybar_slot = -1;
    std::vector<std::array<int32_t, 3>> corr;
    std::vector<int32_t> coeff_bar_slots;   // [N+1]: ybar slot, then abar_k slots
    std::vector<int32_t> z_bar_slots;       // [n]: zbar_i slot or -1 (absent variable)

    bool complex_series() const { return (flags & kComplex) != 0; }
    // streamed operands: chosen when a job's operands would not fit in LDS, or
    // asked for; then no convolution writes its own first operand
    bool streamed = false;
    // staged coefficients of at most two doubles: deal coefficients to lanes
    // in turn instead of following the lane schedule (when estimated faster)
    bool simple = false;
    // jobs with slack moved to later layers to fill whole rounds of the SIMDs
    bool balanced = false;
    // fused layers (kFusedLayers, staged operands): the convolutions split into
    // independent components (no slot written by a job of one is read or
    // written by a job of another); fused_conv holds them by component, then
    // layer, and component c's layer L (1-based) spans
    // fused_conv[fused_off[c * (n_layers + 1) + L - 1] .. fused_off[c * (n_layers + 1) + L]).
    // One workgroup of fused_waves wavefronts runs a component, one job per
    // wavefront at a time, with the one-job lane schedule fused_lanes.
    std::vector<std::array<int32_t, 3>> fused_conv;
    std::vector<int32_t> fused_off;
    int32_t fused_components = 0;
    int32_t fused_waves = 0;
    LaneSchedule fused_lanes;
    bool fused_simple = false;
    // Chain launch (kChainLaunch, or chosen by the cost model): chains of
    // convolutions where each job's first operand is the previous job's
    // output and its second a staged input series (p2's forward and backward
    // products).  Coefficient i of a product is final once its own i+1 terms
    // are summed, and the next product of the chain reads its first operand
    // in increasing i, so consecutive jobs of a chain overlap.  Layer
    // L <= pipe_layers holds the jobs at position L of their chain; one
    // launch runs them all, one workgroup of pipe_waves wavefronts per chain,
    // with a workgroup barrier every pipe_window steps; the layers after
    // pipe_layers launch one by one.
    // pipe_jobs: the chain jobs {t1, t2, t3}, chain after chain, in chain order;
    // pipe_comps: one per chain;
    // pipe_codes: per schedule (chains of one length share one), 64 *
    // pipe_waves rows of `stride` entries: (job << 16) | k for coefficient k
    // of the chain's job-th product (k+1 steps), or (kIdleJob << 16) | (g-1)
    // for g idle steps, then -1.
    // pipe_ring: LDS slots of first operands per chain (job j's in slot j mod pipe_ring).
    int pipe_layers = 0;
    int pipe_waves = 0, pipe_window = 0, pipe_ring = 0;
    std::vector<std::array<int32_t, 3>> pipe_jobs;
    std::vector<ChainComp> pipe_comps;
    std::vector<int32_t> pipe_codes;
    // Single launch (kSingleLaunch, or chosen by the cost model for plans so
    // small that kernel boundaries dominate): one workgroup of single_waves
    // wavefronts runs staging, every convolution layer (single_lanes.jobs_per_group
    // jobs per wavefront and round), the scale stage, every addition level
    // and the gather, with a workgroup barrier after each.
    bool single = false;
    int single_waves = 0;
    LaneSchedule single_lanes;
    bool single_simple = false;
    int n_layers() const { return (int)conv_off.size() - 1; }
    int n_levels() const { return (int)add_off.size() - 1; }
};

// Returns "" on success, else a message; *unsupported distinguishes limits
// of this implementation from invalid input.
// exps: NULL (every exponent one) or [sum nvars] exponents in 1..kMaxExponent.
std::string build_plan(int n, int N, int d, int m, const int32_t *nvars, const int32_t *vars, const int32_t *exps,
                       uint32_t flags, Plan &out, bool *unsupported);

LaneSchedule make_lane_schedule(int d, int jobs_per_group, int waves_per_job = 1);
LaneSchedule make_paired_schedule(int d, int waves_per_job);
// Streamed operands: wavefronts per job for degree d, and whether the paired
// schedule is used (large d, where first-fit would be slow to build).
int stream_waves_per_job(int d, bool *paired);
// Whether a group of J jobs of degree d with w doubles per coefficient is
// estimated faster dealt to the lanes in turn than by the lane schedule.
bool prefer_simple_dealing(int d, int J, int w, int schedule_steps);
// Steps of a group of J jobs of degree d dealt to the lanes of Q wavefronts in
// turn (the slowest wavefront's).
int dealt_steps(int d, int J, int Q = 1);
int choose_jobs_per_group(int d, int w);
// The rules every plan meets (Section 5: the jobs of one layer are
// independent): a job reads only slots written at an earlier stage (inputs,
// an earlier layer or level); no two jobs of a stage write one slot, and no
// job reads a slot another job of its stage writes; a convolution never
// writes its second operand, nor its first when operands are streamed or a
// job spans several wavefronts; output slots are written.  Returns "" or
// what is violated, naming the stage.
std::string check_hazards(const Plan &P);

// Chain launch schedule for one chain of L jobs of degree d on W wavefronts
// with a workgroup barrier every S steps and first operands in B LDS slots:
// codes (64W rows of *stride entries, the encoding of Plan::pipe_codes).
// Returns the steps (an even multiple of S).
int make_chain_schedule(int L, int d, int W, int S, int B, std::vector<int32_t> &codes, int *stride);
// Checks a chain schedule against the kernel's timing: every coefficient of
// every job exactly once, within `steps`; the first operand of step t is read
// from LDS in iteration t-1 (the prologue, iteration -1, for step 0), a
// coefficient's result is stored in the iteration of its last step, and a
// barrier follows every iteration s with (s+1) % S == 0.  Every read of a
// job's first operand must come after the barrier that follows the store of
// that coefficient by the previous job, and before the barrier that precedes
// its overwriting (B slots later).  Returns "" or what is wrong.
std::string check_chain_schedule(int L, int d, int W, int S, int B, int steps, const int32_t *codes, int stride);

}  // namespace mdpe
