// conv_core.hpp -- device building blocks shared by the per-layer kernels
// and the persistent batched executor: one wavefront's convolution (or
// correlation) group, and one coefficient of an addition job.
#pragma once

#include <hip/hip_runtime.h>

#include "md.hpp"
#include "plan.hpp"

namespace mdpe {

// One lane's position in its list of output coefficients.
struct ChainState {
    int c;      // index in the lane's chain list
    int code;   // (job << 16) | k, or -1 when the lane is done
    int j, k, i;
    bool live;  // computes a real coefficient (job j exists in this group)
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

// LDS layout of one wavefront's group: X[J][d+1][W] doubles (the first
// operands), Y[J][d+1][W] (the second operands, only when
// stages_second_operand(W)), then the J job descriptors (16-byte aligned).
__host__ __device__ inline long conv_lds_jobs_offset(long xdoubles) { return (xdoubles * 8 + 15) / 16 * 16; }

// CORR = false: convolution z_k = sum_{i=0..k} x_i y_{k-i} (eq. (1)).
// CORR = true:  correlation z_s = sum_{j=0..d-s} x_{s+j} y_j (the reverse pass);
//               chain code k then denotes s = d-k, with k+1 terms, x index d-k+i
//               and y index i, so the same lane schedule balances both.
// CX = true: complex series, W = 2M doubles per coefficient (cmd_mul, cmd_add).
// One 64-lane wavefront computes jn <= J jobs jobs[0..jn) (the output
// coefficients of each spread over the lanes by the schedule `chains`).
// lds must hold conv_lds_jobs_offset(J*(d+1)*lds_doubles_per_coef(W)) + J*16
// bytes.  Ends with the wavefront's stores issued (not necessarily complete).
// XS = true (streamed operands, for degrees whose operands do not fit in LDS):
// both operands are read from global memory and only the job descriptors are
// in LDS; the planner then guarantees that no job writes its first operand.
// `row` selects the lane's row of the schedule (q*64 + lane for the q-th of
// the wavefronts sharing a job).  `simple` (coefficients of at most two
// doubles, staged operands): deal the coefficients to the lanes in turn
// instead of following the schedule (see below).
template <int M, bool CORR, bool CX = false, bool XS = false>
__device__ __forceinline__ void conv_group(double *__restrict__ A, const int4 *__restrict__ jobs, int jn, int J,
                                           int d, double *lds, const int *__restrict__ chains, int stride,
                                           int steps, int lane, int row, bool simple = false) {
    constexpr int W = kCoef<M, CX>;
    constexpr bool YL = !XS && stages_second_operand(W);
    const long S = (long)(d + 1) * W;
    double *X = lds;
    double *Y = lds + J * S;  // used when YL
    int4 *jd = (int4 *)((char *)lds + (XS ? 0 : conv_lds_jobs_offset(J * (YL ? 2 : 1) * S)));
    // Stage the first operand of every job in LDS: it is read by all lanes and
    // may be the job's own output (the in-place b := b * a of Section 3).  The
    // second operand is never the output (the planner checks) and is streamed
    // from global memory -- mostly one of the shared input series, so it stays
    // in L2 -- except for coefficients of at most two doubles, where a step is
    // so short that its latency would dominate: then it is staged too.  The
    // first operand is read one step ahead of its use, the second two steps.
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
        if (lane == 0) jd[j] = t;
    }
    __syncthreads();
    if (jn <= 0) return;  // a wavefront past the last group (after the workgroup barrier)

    if constexpr (W <= 2 && !XS) {
        if (simple) {
            // Coefficients of one or two doubles: a multiply-add is a handful of
            // operations, so the lane schedule's bookkeeping can dominate.
            // Instead the group's (job, coefficient) items are dealt to the
            // lanes in turn and each lane sums its coefficient's terms in the
            // specified order from the staged operands: more lane-steps, far
            // fewer instructions per step (the planner weighs the two).
            const int d1 = d + 1;
            for (int t = lane; t < jn * d1; t += 64) {
                const int j = t / d1;
                const int k = t - j * d1;
                const double *x = X + (long)j * S;
                const double *y = Y + (long)j * S;
                double *out = A + (long)jd[j].z * S + (long)(CORR ? d - k : k) * W;
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
    // Next position in the lane's chain list (reads the -1 terminator at most).
    auto advance = [&](const ChainState &cur, ChainState &nxt, int4 &nj) {
        nxt = cur;
        if (cur.i == cur.k) {
            if (cur.code >= 0) nxt.code = my[++nxt.c];
            chain_decode(nxt, jn);
            if (nxt.live) nj = jd[nxt.j];
        } else {
            nxt.i = cur.i + 1;
        }
    };
    auto xidx = [&](int k, int i) { return CORR ? d - k + i : i; };
    auto yidx = [&](int k, int i) { return CORR ? i : k - i; };

    // Software pipeline over the lane's steps: iteration s accumulates the
    // product of step s while it computes the product of step s+1 (the two are
    // independent, and sit in one basic block so the scheduler can interleave
    // them) and loads the second operand of step s+2.
    ChainState st;
    st.c = 0;
    st.code = my[0];
    chain_decode(st, jn);
    int4 job = jd[st.live ? st.j : 0];
    // the first operand of a position: LDS, or global memory when streamed
    auto xaddr = [&](const ChainState &t, const int4 &jb) -> const double * {
        return XS ? A + (long)jb.x * S + (long)xidx(t.k, t.i) * W : X + t.j * S + xidx(t.k, t.i) * W;
    };
    double p[W];
    {
        const double *xp = xaddr(st, job);
        const double *yp = YL ? Y + st.j * S + yidx(st.k, 0) * W : A + (long)job.y * S + (long)yidx(st.k, 0) * W;
        double x0[W], y0[W];
#pragma unroll
        for (int l = 0; l < W; ++l) {
            x0[l] = XS ? (st.live ? xp[l] : 0.0) : xp[l];
            y0[l] = st.live ? yp[l] : 0.0;
        }
        coef_mul<M, CX>(x0, y0, p);
    }
    ChainState nx;
    int4 njob = job;
    advance(st, nx, njob);
    double yn[W], xn[W];
    {
        const double *yp = YL ? Y + nx.j * S + yidx(nx.k, nx.i) * W : A + (long)njob.y * S + (long)yidx(nx.k, nx.i) * W;
        const bool fetch = nx.live && 1 < steps;
#pragma unroll
        for (int l = 0; l < W; ++l) yn[l] = fetch ? yp[l] : 0.0;
        if (XS) {  // streamed: x is read two steps ahead too
            const double *xp = xaddr(nx, njob);
#pragma unroll
            for (int l = 0; l < W; ++l) xn[l] = fetch ? xp[l] : 0.0;
        }
    }
    double acc[W];
#pragma unroll
    for (int l = 0; l < W; ++l) acc[l] = 0.0;
    for (int s = 0; s < steps; ++s) {
        ChainState n2;
        int4 n2job = njob;
        advance(nx, n2, n2job);
        double x1[W], y1[W];
#pragma unroll
        for (int l = 0; l < W; ++l) y1[l] = yn[l];
        {
            const bool fetch = n2.live && s + 2 < steps;
            if (XS) {
                const double *xp = xaddr(n2, n2job);
#pragma unroll
                for (int l = 0; l < W; ++l) {
                    x1[l] = xn[l];
                    xn[l] = fetch ? xp[l] : 0.0;
                }
            } else {
                const double *xp = xaddr(nx, njob);
#pragma unroll
                for (int l = 0; l < W; ++l) x1[l] = xp[l];
            }
            const double *yp = YL ? Y + n2.j * S + yidx(n2.k, n2.i) * W
                                  : A + (long)n2job.y * S + (long)yidx(n2.k, n2.i) * W;
#pragma unroll
            for (int l = 0; l < W; ++l) yn[l] = fetch ? yp[l] : 0.0;
        }
        double pn[W], r[W];
        coef_mul<M, CX>(x1, y1, pn);   // step s+1 (unused past the lane's last step)
        coef_add<M, CX>(acc, p, r);    // step s; a chain's first term replaces acc
        const bool first = st.i == 0;
#pragma unroll
        for (int l = 0; l < W; ++l) acc[l] = first ? p[l] : r[l];
        if (st.i == st.k && st.live) {
            double *out = A + (long)job.z * S + (long)(CORR ? d - st.k : st.k) * W;
#pragma unroll
            for (int l = 0; l < W; ++l) out[l] = acc[l];
        }
        st = nx;
        job = njob;
        nx = n2;
        njob = n2job;
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
    conv_group<M, CORR, CX, XS>(A, jobs + g0, min(J, njobs - g0), J, d, (double *)((char *)lds + wave * group_bytes),
                                chains, stride, steps, lane, part * 64 + lane, simple != 0);
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
