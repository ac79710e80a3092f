// conv_core.hpp -- device building blocks shared by the per-layer kernels
// and the persistent batched executor: one wavefront's convolution (or
// correlation) group, and one coefficient of an addition job.
#pragma once

#include <hip/hip_runtime.h>

#include "md.hpp"
#include "plan.hpp"

namespace mdpe {

// One lane's position in its list of output coefficients, with the addresses
// of the operand coefficients of its current term and of its output.
struct ChainState {
    const int *cp;  // the lane's chain list entry after the current one (stays on the terminator)
    int code;   // (job << 16) | k, or -1 when the lane is done
    int next;   // *cp: the code after it
    int j, k, i;
    bool live;  // computes a real coefficient (job j exists in this group)
    const double *x, *y;  // first and second operand coefficient of term i
    double *out;          // the output coefficient
};

__device__ __forceinline__ void chain_decode(ChainState &st, int jn) {
    if (st.code >= 0) {
        st.j = st.code >> 16;
        st.k = st.code & 0xffff;
        st.live = st.j < jn;
    } else {
        st.j = 0;
        st.k = 0;
        st.live = false;
    }
    st.i = 0;
}


// CORR = false: convolution z_k = sum_{i=0..k} x_i y_{k-i} (eq. (1)).
// CORR = true:  correlation z_s = sum_{j=0..d-s} x_{s+j} y_j (the reverse pass);
//               chain code k then denotes s = d-k, with k+1 terms, x index d-k+i
//               and y index i, so the same lane schedule balances both.
// CX = true: complex series, W = 2M doubles per coefficient (cmd_mul, cmd_add).
// One 64-lane wavefront computes jn <= J jobs jobs[0..jn) (the output
// coefficients of each spread over the lanes by the schedule `chains`).
// lds must hold group_lds_bytes(d+1, lds_doubles_per_coef(W), J) bytes (0
// doubles per coefficient when streamed).  Ends with the wavefront's stores
// issued (not necessarily complete).
// XS = true (streamed operands, for degrees whose operands do not fit in LDS):
// both operands are read from global memory and only the job descriptors are
// in LDS; the planner then guarantees that no job writes its first operand.
// `row` selects the lane's row of the schedule (q*64 + lane for the q-th of
// the nrows / 64 wavefronts sharing a job).  `simple` (coefficients of at
// most two doubles, staged operands): deal the coefficients to the lanes in
// turn instead of following the schedule (see below).
// CODE_AHEAD: load the code of a lane's next chain at every step, outside
// the chain-start branch, instead of inside it.  Measured on lone wavefronts
// (p2's layers): 15-18% faster for jobs spread over several wavefronts
// (p2 10d, d = 152), 15% slower for groups of several jobs per wavefront
// (p2 10d, d = 63; p1 8d, d = 32), equal on p1 10d at d = 152; the kernel
// chooses per instantiation.
// DESC_FIRST: how the operands are staged (below).  Descriptors first, with a
// small group copied in one flat round, takes 16 products of three of eight
// variables at two doubles and d = 8 (a single launch) from 0.027 to 0.018 ms.
// Elsewhere it measured even or slower (per-layer launches of p1 at eight
// doubles and d = 32, the batched kernel), and in the fused and single-launch
// kernels it took 20-40 more registers from three doubles on; only the single
// launch at one or two doubles per coefficient uses it.
template <int M, bool CORR, bool CX = false, bool XS = false, bool CODE_AHEAD = false, bool DESC_FIRST = false>
__device__ __forceinline__ void conv_group(double *__restrict__ A, const int4 *__restrict__ jobs, int jn, int J,
                                           int d, double *lds, const int *__restrict__ chains, int stride,
                                           int steps, int lane, int row, bool simple = false, int nrows = kLanes) {
    constexpr int W = kCoef<M, CX>;
    constexpr bool YL = !XS && stages_second_operand(W);
    const long S = (long)(d + 1) * W;
    double *X = lds;
    double *Y = lds + J * S;  // used when YL
    JobOffsets *jd = (JobOffsets *)((char *)lds + (XS ? 0 : conv_lds_jobs_offset(J * (YL ? 2 : 1) * S)));
    // Stage the first operand of every job in LDS: it is read by all lanes and
    // may be the job's own output (the in-place b := b * a of Section 3).  The
    // second operand is never the output (the planner checks) and is streamed
    // from global memory -- mostly one of the shared input series, so it stays
    // in L2 -- except for coefficients of at most two doubles, where a step is
    // so short that its latency would dominate: then it is staged too.  The
    // first operand is read one step ahead of its use, the second two steps.
    if (!DESC_FIRST) {
        // job by job: lane 0 writes the descriptor, all lanes copy the operands
        for (int j = 0; j < jn; ++j) {
            const int4 t = jobs[j];
            if (!XS) {
                const double *xs = A + (long)t.x * S;
                for (long q = lane; q < S; q += 64) X[j * S + q] = xs[q];
            }
            if (YL) {
                const double *ys = A + (long)t.y * S;
                for (long q = lane; q < S; q += 64) Y[j * S + q] = ys[q];
            }
            if (lane == 0) jd[j] = JobOffsets{(long)t.x * S, (long)t.y * S, (long)t.z * S, 0};
        }
        __syncthreads();
    } else {
        // The descriptors first, one per lane; then a group whose staged doubles
        // fit one round of kStageLoads per lane (many small jobs, as at low
        // degree) is copied as one flat range with all its loads in flight
        // before the LDS stores: a few memory latencies instead of one per job.
        // (X and Y are job-major with stride S: flat element g is double g mod S
        // of job g / S.)  Larger groups are copied job by job.
        for (int j = lane; j < jn; j += 64) {
            const int4 t = jobs[j];
            jd[j] = JobOffsets{(long)t.x * S, (long)t.y * S, (long)t.z * S, 0};
        }
        __syncthreads();
        constexpr int kStageLoads = YL ? 4 : 8;
        const int Si = (int)S, total = jn * Si;
        if (!XS && total <= 64 * kStageLoads) {
            const int sj = 64 / Si, sq = 64 - sj * Si;
            int j = lane / Si, q = lane - j * Si;
            double vx[kStageLoads], vy[kStageLoads];
#pragma unroll
            for (int u = 0; u < kStageLoads; ++u) {
                if (lane + 64 * u < total) {
                    const JobOffsets &o = jd[j];
                    vx[u] = A[o.x + q];
                    if (YL) vy[u] = A[o.y + q];
                }
                j += sj;
                q += sq;
                if (q >= Si) {
                    q -= Si;
                    ++j;
                }
            }
#pragma unroll
            for (int u = 0; u < kStageLoads; ++u)
                if (lane + 64 * u < total) {
                    X[lane + 64 * u] = vx[u];
                    if (YL) Y[lane + 64 * u] = vy[u];
                }
        } else if (!XS) {
            for (int j = 0; j < jn; ++j) {
                const JobOffsets &o = jd[j];
                for (long q = lane; q < S; q += 64) X[j * S + q] = A[o.x + q];
                if (YL)
                    for (long q = lane; q < S; q += 64) Y[j * S + q] = A[o.y + q];
            }
        }
        if (!XS) __syncthreads();  // every wavefront of the workgroup, whichever copy it took
    }
    if (jn <= 0) return;  // a wavefront past the last group (after the workgroup barriers)

    if constexpr (W <= 2 && !XS) {
        if (simple) {
            // Coefficients of one or two doubles: a multiply-add is a handful of
            // operations, so the lane schedule's bookkeeping can dominate.
            // Instead the group's (job, coefficient) items are dealt to the
            // lanes in turn and each lane sums its coefficient's terms in the
            // specified order from the staged operands: more lane-steps, far
            // fewer instructions per step (the planner weighs the two).  With
            // several wavefronts per group, row r of the nrows = 64Q takes
            // items r, r + 64Q, ...
            const int d1 = d + 1;
            for (int t = row; t < jn * d1; t += nrows) {
                const int j = t / d1;
                const int k = t - j * d1;
                const double *x = X + (long)j * S;
                const double *y = Y + (long)j * S;
                double *out = A + jd[j].z + (long)(CORR ? d - k : k) * W;
                // CORR: z_s = sum_{i=0..d-s} x_{s+i} y_i with s = d - k (k+1 terms)
                const int x0 = CORR ? d - k : 0;
                double acc[W], pr[W], xa[W], ya[W];
#pragma unroll
                for (int l = 0; l < W; ++l) {
                    xa[l] = x[x0 * W + l];
                    ya[l] = y[(CORR ? 0 : k) * W + l];
                }
                coef_mul<M, CX>(xa, ya, acc);
                for (int i = 1; i <= k; ++i) {
#pragma unroll
                    for (int l = 0; l < W; ++l) {
                        xa[l] = x[(x0 + i) * W + l];
                        ya[l] = y[(CORR ? i : k - i) * W + l];
                    }
                    coef_mul<M, CX>(xa, ya, pr);
                    coef_add<M, CX>(acc, pr, acc);
                }
#pragma unroll
                for (int l = 0; l < W; ++l) out[l] = acc[l];
            }
            return;
        }
    }

    const int *my = chains + (long)row * stride;
    auto xidx = [&](int k, int i) { return CORR ? d - k + i : i; };
    auto yidx = [&](int k, int i) { return CORR ? i : k - i; };
    // Addresses of a chain's first term and of its output coefficient: LDS,
    // or global memory when streamed.  A lane with no chain (code -1, or a job
    // past the group's last) gets those of job 0's coefficient, so every lane
    // may load at every step and no load needs a guard; such lanes never store.
    auto start = [&](ChainState &t) {
        const int j = t.live ? t.j : 0;
        const JobOffsets &jb = jd[j];
        t.x = XS ? A + jb.x + (long)xidx(t.k, 0) * W : X + j * S + xidx(t.k, 0) * W;
        t.y = YL ? Y + j * S + yidx(t.k, 0) * W : A + jb.y + (long)yidx(t.k, 0) * W;
        t.out = A + jb.z + (long)(CORR ? d - t.k : t.k) * W;
    };
    // Next position in the lane's chain list.  The code after the current
    // chain's is loaded a chain ahead of its use (at a chain's start, or at
    // every step with CODE_AHEAD); the list pointer stops on the -1
    // terminator, so the list is never read past.
    auto advance = [&](const ChainState &cur, ChainState &nxt) {
        nxt = cur;
        if (cur.i == cur.k) {
            nxt.code = cur.next;
            if (nxt.code >= 0) ++nxt.cp;
            if (!CODE_AHEAD) nxt.next = *nxt.cp;
            chain_decode(nxt, jn);
            start(nxt);
        } else {
            nxt.i = cur.i + 1;
            nxt.x += W;
            nxt.y += CORR ? W : -W;
        }
        if (CODE_AHEAD) nxt.next = *nxt.cp;
    };

    // Software pipeline over the lane's steps: iteration s accumulates the
    // product of step s while it computes the product of step s+1 (the two are
    // independent) and loads the second operand of step s+2 (and, streamed,
    // the first).
    ChainState st;
    st.code = my[0];
    st.cp = my + (st.code >= 0 ? 1 : 0);
    st.next = *st.cp;
    chain_decode(st, jn);
    start(st);
    double p[W];
    {
        double x0[W], y0[W];
#pragma unroll
        for (int l = 0; l < W; ++l) {
            x0[l] = st.x[l];
            y0[l] = st.y[l];
        }
        coef_mul<M, CX>(x0, y0, p);
    }
    ChainState nx;
    advance(st, nx);
    double yn[W], xn[W];
#pragma unroll
    for (int l = 0; l < W; ++l) {
        yn[l] = nx.y[l];
        if (XS) xn[l] = nx.x[l];
    }
    double acc[W];
#pragma unroll
    for (int l = 0; l < W; ++l) acc[l] = 0.0;
    // Two steps per iteration up to five doubles per coefficient: the copies
    // between the pipeline's buffers become register renames (m = 4: 60 -> 44
    // VALU and 76 -> 48 SALU instructions per step besides the md
    // operations).  Measured slower from eight doubles on (octo double: 5-6%
    // on p2 and at d = 32), where the body is long anyway, and at five with
    // jobs over several wavefronts (penta double p2, d = 152: 8.39 -> 8.96 ms,
    // while one-wavefront groups gain 2-6%).
    constexpr int kUnroll = (W <= 4 || (W == 5 && !CODE_AHEAD)) ? 2 : 1;
#pragma unroll kUnroll
    for (int s = 0; s < steps; ++s) {
        ChainState n2;
        advance(nx, n2);
        double x1[W], y1[W];
#pragma unroll
        for (int l = 0; l < W; ++l) {
            y1[l] = yn[l];
            x1[l] = XS ? xn[l] : nx.x[l];
            yn[l] = n2.y[l];
            if (XS) xn[l] = n2.x[l];
        }
        double pn[W], r[W];
        coef_mul<M, CX>(x1, y1, pn);   // step s+1 (unused past the lane's last step)
        coef_add<M, CX>(acc, p, r);    // step s; a chain's first term replaces acc
        const bool first = st.i == 0;
#pragma unroll
        for (int l = 0; l < W; ++l) acc[l] = first ? p[l] : r[l];
        if (st.i == st.k && st.live) {
#pragma unroll
            for (int l = 0; l < W; ++l) st.out[l] = acc[l];
        }
        st = nx;
        nx = n2;
#pragma unroll
        for (int l = 0; l < W; ++l) p[l] = pn[l];
    }
}

// WPB wavefronts per workgroup (1 or 4), each with its own group of J jobs and
// its own LDS region of group_bytes.  Four-wavefront workgroups put one
// wavefront on each SIMD of a CU; the launcher uses them when a layer has
// between one and three wavefronts per SIMD, where single-wavefront workgroups
// can pile three onto one SIMD while another stays idle.  (A separate
// instantiation: the 256-thread launch bound alone slows a lone wavefront.)
// Q wavefronts share each group (Q > 1 for few jobs per layer at a large
// degree, and for streamed operands); wavefront w takes group w / Q, schedule
// part w % Q.
// MQ = false: one wavefront per group (Q = 1), the mapping without a division
// (a separate instantiation so that the common case's code is unchanged).
template <int M, bool CORR, bool CX = false, int WPB = 1, bool XS = false, bool MQ = XS>
__global__ __launch_bounds__(64 * WPB) void conv_layer_kernel(double *__restrict__ A, const int4 *__restrict__ jobs,
                                                              int njobs, int d, int J, const int *__restrict__ chains,
                                                              int stride, int steps, int group_bytes, int Q,
                                                              int simple) {
    extern __shared__ double lds[];
    const int wave = WPB == 1 ? 0 : (int)(threadIdx.x >> 6);
    const int wv = blockIdx.x * WPB + wave;
    const int g = MQ ? wv / Q : wv;
    const int part = MQ ? wv - g * Q : 0;
    const int g0 = g * J;
    const int lane = threadIdx.x & 63;
    conv_group<M, CORR, CX, XS, MQ>(A, jobs + g0, min(J, njobs - g0), J, d, (double *)((char *)lds + wave * group_bytes),
                                    chains, stride, steps, lane, part * 64 + lane, simple != 0, (MQ ? Q : 1) * 64);
}

// Every convolution layer of a plan in one launch.  The jobs fall into
// independent components (no slot written by a job of one is read or written
// by a job of another), and a component's jobs depend only on its own earlier
// layers.  Workgroup c runs component c layer by layer: in each round its
// wavefronts take one job each (wavefront w the w-th of the round), and a
// workgroup barrier ends every layer, after which the layer's stores are
// visible to the whole workgroup.  Every wavefront runs the same rounds (a
// wavefront without a job still meets conv_group's barrier), so the barriers
// match.  Each job runs exactly as in conv_layer_kernel with one job per
// group, so the output bits are those of the per-layer launches.
// J (jobs per wavefront, 1 from the planner) is read from the argument from
// four doubles per coefficient on and fixed at compile time below: measured
// 5-9% faster that way at four and ten doubles (p2 4d d = 64: 2.52 -> 2.37
// ms; 10d d = 8: 2.97 -> 2.69) and 1-4% slower at two and three, the same
// bits -- a difference in the generated code only.
template <int M, bool CX = false>
__global__ __launch_bounds__(256) void conv_fused_kernel(double *__restrict__ A, const int4 *__restrict__ jobs,
                                                          const int *__restrict__ off, int nl, int d, int J,
                                                          const int *__restrict__ chains, int stride, int steps,
                                                          int group_bytes, int simple) {
    extern __shared__ double lds[];
    const int waves = (int)(blockDim.x >> 6);
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int *o = off + (long)blockIdx.x * (nl + 1);
    double *mine = (double *)((char *)lds + wave * group_bytes);
    for (int L = 0; L < nl; ++L) {
        const int a = o[L], b = o[L + 1];
        const int jj = kCoef<M, CX> >= 4 ? J : 1;
        for (int r = a; r < b; r += waves * jj) {
            const int q = r + wave * jj;
            const int jn = q < b ? min(jj, b - q) : 0;
            conv_group<M, false, CX, false, false>(A, jobs + (jn > 0 ? q : a), jn, jj, d, mine, chains, stride,
                                                   steps, lane, lane, simple != 0);
        }
        __syncthreads();
    }
}

// A workgroup barrier that orders LDS accesses only: the LDS stores and
// reads issued before it complete before any wavefront passes it, while
// global loads in flight (second operands prefetched two steps ahead) and
// global stores (read by later launches only) are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The chain launch.  Workgroup c runs chain c: products where each job's
// first operand is the previous job's output and its second a staged input
// series (the forward and backward products of Section 3).  Its lanes follow
// the chain's schedule `codes` (rows of (job << 16) | k for coefficient k of
// the chain's job-th product, k+1 steps; (kIdleJob << 16) | (g-1) for g idle
// steps; -1 after the last): each coefficient is one lane's sequential sum of
// its k+1 terms in the specified order, as in conv_group, so every bit is that
// of the per-layer launches.  Job j's first operand sits in LDS slot j mod B:
// job 0's is staged from A, every later job's is stored there coefficient by
// coefficient by the job before it, beside its store to A.  Coefficient i of
// a product is final after its own i+1 terms and the next product reads its
// first operand in increasing i, so consecutive products overlap.  A
// workgroup barrier on LDS after every S steps orders those stores and reads: the
// host checks that the schedule reads each coefficient only in a window after
// that of its store, and overwrites a slot only in a window after that of its
// last read (check_chain_schedule).  Second operands stream from A two steps
// ahead; lanes without a coefficient compute on job 0's first terms and
// store nothing.
template <int M, bool CX, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void conv_chain_kernel(double *__restrict__ A, const int4 *__restrict__ jobs,
                                                                const ChainComp *__restrict__ comps,
                                                                const int *__restrict__ codes, int d, int B, int S) {
    constexpr int W = kCoef<M, CX>;
    extern __shared__ double lds[];
    const ChainComp cc = comps[blockIdx.x];
    const long SS = (long)(d + 1) * W;
    double *ring = lds;
    // per job: x = LDS offset of its first operand, y and z = offsets in A,
    // unused = LDS offset of the next job's first operand (-1 for the last)
    JobOffsets *jd = (JobOffsets *)((char *)lds + conv_lds_jobs_offset((long)B * SS));
    const int tid = (int)threadIdx.x;
    {
        const int4 t0 = jobs[cc.first];
        const double *xs = A + (long)t0.x * SS;
        for (long q = tid; q < SS; q += 64 * WAVES) ring[q] = xs[q];
        for (int j = tid; j < cc.len; j += 64 * WAVES) {
            const int4 t = jobs[cc.first + j];
            jd[j] = JobOffsets{(long)(j % B) * SS, (long)t.y * SS, (long)t.z * SS,
                               j + 1 < cc.len ? (long)((j + 1) % B) * SS : -1L};
        }
    }
    __syncthreads();

    struct St {
        const int *cp;  // the row entry after the current one (stays on the terminator)
        int code, next, k, i;
        bool live;      // a coefficient of a job (not idle, not past the row's end)
        const double *x, *y;
        double *out, *rout;
    };
    auto decode = [&](St &t) {
        int j = 0;
        if (t.code >= 0) {
            j = t.code >> 16;
            t.k = t.code & 0xffff;
            t.live = j != kIdleJob;
        } else {
            t.k = 0;
            t.live = false;
        }
        t.i = 0;
        const JobOffsets &jb = jd[t.live ? j : 0];
        const long kk = t.live ? t.k : 0;
        t.x = ring + jb.x;
        t.y = A + jb.y + kk * W;
        t.out = A + jb.z + kk * W;
        t.rout = jb.unused >= 0 ? ring + jb.unused + kk * W : nullptr;
    };
    auto advance = [&](const St &cur, St &nxt) {
        nxt = cur;
        if (cur.i == cur.k) {
            nxt.code = cur.next;
            if (nxt.code >= 0) ++nxt.cp;
            nxt.next = *nxt.cp;
            decode(nxt);
        } else {
            nxt.i = cur.i + 1;
            if (cur.live) {
                nxt.x += W;
                nxt.y -= W;
            }
        }
    };

    const int *my = codes + cc.code_off + (long)tid * cc.stride;
    St st;
    st.code = my[0];
    st.cp = my + (st.code >= 0 ? 1 : 0);
    st.next = *st.cp;
    decode(st);
    double p[W];
    {
        double x0[W], y0[W];
#pragma unroll
        for (int l = 0; l < W; ++l) {
            x0[l] = st.x[l];
            y0[l] = st.y[l];
        }
        coef_mul<M, CX>(x0, y0, p);
    }
    St nx;
    advance(st, nx);
    double yn[W], acc[W];
#pragma unroll
    for (int l = 0; l < W; ++l) {
        yn[l] = nx.y[l];
        acc[l] = 0.0;
    }
    int until_barrier = S;
    auto step = [&]() {
        St n2;
        advance(nx, n2);
        double x1[W], y1[W];
#pragma unroll
        for (int l = 0; l < W; ++l) {
            y1[l] = yn[l];
            x1[l] = nx.x[l];
            yn[l] = n2.y[l];
        }
        double pn[W], r[W];
        coef_mul<M, CX>(x1, y1, pn);  // step s+1
        coef_add<M, CX>(acc, p, r);   // step s; a coefficient's first term replaces acc
        const bool first = st.i == 0;
#pragma unroll
        for (int l = 0; l < W; ++l) acc[l] = first ? p[l] : r[l];
        if (st.i == st.k && st.live) {
#pragma unroll
            for (int l = 0; l < W; ++l) st.out[l] = acc[l];
            if (st.rout) {
#pragma unroll
                for (int l = 0; l < W; ++l) st.rout[l] = acc[l];
            }
        }
        st = nx;
        nx = n2;
#pragma unroll
        for (int l = 0; l < W; ++l) p[l] = pn[l];
        if (--until_barrier == 0) {
            lds_barrier();
            until_barrier = S;
        }
    };
    // Two steps per iteration up to four doubles per coefficient, as in
    // conv_group (the pipeline's copies become renames); the planner makes
    // every chain's step count even.
    constexpr int kU = W <= 4 ? 2 : 1;
    for (int s = 0; s < cc.steps; s += kU) {
        step();
        if constexpr (kU == 2) step();
    }
}

// A[t2] := A[t2] + A[t1] at coefficient c (Section 5, the addition job).
template <int M, bool CX = false>
__device__ __forceinline__ void add_item(double *__restrict__ A, int2 t, int c, int d) {
    constexpr int W = kCoef<M, CX>;
    const long S = (long)(d + 1) * W;
    double *up = A + (long)t.y * S + (long)c * W;
    const double *in = A + (long)t.x * S + (long)c * W;
    double x[W], y[W], z[W];
#pragma unroll
    for (int l = 0; l < W; ++l) {
        x[l] = up[l];
        y[l] = in[l];
    }
    coef_add<M, CX>(x, y, z);
#pragma unroll
    for (int l = 0; l < W; ++l) up[l] = z[l];
}

// user coefficient / input series -> staged slot (entry (slot, source) at coefficient c)
__device__ __forceinline__ void stage_item(double *__restrict__ A, const double *__restrict__ coeff,
                                           const double *__restrict__ z, int2 en, int c, int N, int n, int d, int m) {
    const int d1 = d + 1;
    double *dst = A + (long)en.x * d1 * m + (long)c * m;
    if (en.y <= N) {
        for (int l = 0; l < m; ++l) dst[l] = coeff[((long)l * (N + 1) + en.y) * d1 + c];
    } else {
        const int i = en.y - N - 1;
        for (int l = 0; l < m; ++l) dst[l] = z[((long)l * n + i) * d1 + c];
    }
}

// output o (0 = value, 1+i = d/dz_i) at coefficient c -> user buffers
__device__ __forceinline__ void gather_item(const double *__restrict__ A, double *__restrict__ value,
                                            double *__restrict__ grad, int slot, int o, int c, int n, int d, int m) {
    const int d1 = d + 1;
    for (int l = 0; l < m; ++l) {
        const double v = slot >= 0 ? A[(long)slot * d1 * m + (long)c * m + l] : 0.0;
        if (o == 0)
            value[(long)l * d1 + c] = v;
        else
            grad[((long)l * n + (o - 1)) * d1 + c] = v;
    }
}

}  // namespace mdpe
