// plan.cpp -- the data staging algorithm of Section 5 of the paper.
//
// Slots (one slot = one series of d+1 coefficients; slot s starts at
// s*(d+1) in the paper's array A, Fig. 1):
//   a_0 = 0, a_k = k (k = 1..N), z_i = N + i (i = 1..n),
//   f_{k,j} = 1+N+n + alpha_k + j-1,
//   b_{k,j} = 1+N+n + alpha_{N+1} + beta_k + j-1,
//   c_{k,j} = 1+N+n + alpha_{N+1} + beta_{N+1} + gamma_k + j-1,
// with alpha, beta, gamma the prefix sums of n_l, max(1, n_l-2), max(0, n_l-2)
// (Section 5; the slot count is e/(d+1) of eq. (6)).
//
// Convolution jobs per monomial (Section 3, statement list and eq. (2);
// Section 5, steps 1-7) with the readings: forward chain by z_{i_j};
// c_j = f_j * b_{n-2-j} at layer max(j, n-2-j)+1; b_{n-2} := b_{n-2} * a and
// c_{n-2} = f_{n-2} * z_{i_n} at layer n-1; n = 2: b_1 = z_{i_2} * a; n = 1:
// the derivative is a_k itself, copied into its b slot at staging time.
//
// Addition jobs: per output list a pairwise tree, adjacent pairs with the odd
// element carried, the later element updated (Section 5, the addition
// recursion, read through the worked example after eq. (5)).
//
// General exponents (Section 3): a table of powers z_i^p := z_i^{p-1} * z_i,
// the common factor a_k * prod z^(e-1) in front of the monomial's jobs, and a
// scale stage (A[dst] := e * A[src]) for the partial derivatives.  Streamed
// operands (degrees beyond one workgroup's LDS, or estimated faster): no job
// writes its own first operand, and a job may span several wavefronts.
#include "plan.hpp"

#include <cmath>

#include <algorithm>
#include <numeric>
#include <unordered_map>

namespace mdpe {

static bool supported_m(int m) { return m == 1 || m == 2 || m == 3 || m == 4 || m == 5 || m == 8 || m == 10; }

int choose_jobs_per_group(int d, int w) {
    // Enough jobs per wavefront that the average lane load, J(d+1)(d+2)/2/64,
    // covers the longest output coefficient (d+1 multiply-adds); within the
    // LDS budget.
    int need = (2 * kLanes + (d + 2) - 1) / (d + 2);
    need = std::max(1, std::min(need, kLanes));
    long per_job = (long)(d + 1) * lds_doubles_per_coef(w) * 8;
    long cap = std::max(1L, (long)kLdsBudget / per_job);
    return (int)std::max(1L, std::min((long)need, cap));
}

LaneSchedule make_lane_schedule(int d, int J, int Q) {
    // Assign the J*(d+1) output coefficients (coefficient k costs k+1
    // multiply-adds) to the 64*Q lanes of Q wavefronts: first-fit-decreasing
    // into lanes of capacity C, for the smallest C >= max(ceil(total/lanes),
    // d+1) that fits.  Each coefficient stays whole on one lane, so its
    // operation order is the specified one whatever lane computes it.
    LaneSchedule s;
    s.jobs_per_group = J;
    s.waves_per_job = Q;
    const int lanes = kLanes * Q;
    std::vector<std::pair<int, int>> items;  // (length, code)
    long total = 0;
    for (int j = 0; j < J; ++j)
        for (int k = 0; k <= d; ++k) {
            items.push_back({k + 1, (j << 16) | k});
            total += k + 1;
        }
    std::stable_sort(items.begin(), items.end(), [](auto &a, auto &b) { return a.first > b.first; });
    std::vector<long> load;
    std::vector<std::vector<int32_t>> lists;
    for (long cap = std::max((total + lanes - 1) / lanes, (long)d + 1);; ++cap) {
        load.assign(lanes, 0);
        lists.assign(lanes, {});
        bool ok = true;
        for (auto &it : items) {
            int l = 0;
            while (l < lanes && load[l] + it.first > cap) ++l;
            if (l == lanes) {
                ok = false;
                break;
            }
            load[l] += it.first;
            lists[l].push_back(it.second);
        }
        if (ok) break;
    }
    size_t stride = 1;
    for (auto &l : lists) stride = std::max(stride, l.size() + 1);
    s.stride = (int)stride;
    s.steps = (int)*std::max_element(load.begin(), load.end());
    s.chains.assign((size_t)lanes * stride, -1);
    for (int l = 0; l < lanes; ++l)
        for (size_t q = 0; q < lists[l].size(); ++q) s.chains[(size_t)l * stride + q] = lists[l][q];
    return s;
}

LaneSchedule make_paired_schedule(int d, int Q) {
    // One job over the 64*Q lanes of Q wavefronts for large d: coefficients k
    // and d-k (k+1 and d-k+1 terms, d+2 together) share a lane, one pair per
    // lane; the middle coefficient of an even d is alone.  Q*64 must be at
    // least the number of pairs, ceil((d+1)/2).
    LaneSchedule s;
    s.jobs_per_group = 1;
    s.waves_per_job = Q;
    const int lanes = kLanes * Q;
    s.stride = 3;
    s.chains.assign((size_t)lanes * 3, -1);
    int steps = 0;
    for (int k = 0, l = 0; k <= d - k; ++k, ++l) {
        s.chains[(size_t)l * 3] = d - k;                    // the longer coefficient first
        if (k != d - k) s.chains[(size_t)l * 3 + 1] = k;
        steps = std::max(steps, (d - k + 1) + (k != d - k ? k + 1 : 0));
    }
    s.steps = steps;
    return s;
}

int stream_waves_per_job(int d, bool *paired) {
    const int pairs = (d + 2) / 2;
    *paired = d + 1 > 4096;
    if (*paired) return (pairs + kLanes - 1) / kLanes;
    return std::max(1, pairs / kLanes);
}

int dealt_steps(int d, int J, int Q) {
    // steps of dealing J*(d+1) coefficients to the 64*Q lanes of Q wavefronts
    // in turn (item t to lane t mod 64Q): each round of 64 items of a
    // wavefront costs its longest coefficient; the slowest wavefront counts
    const long items = (long)J * (d + 1);
    long worst = 0;
    for (int q = 0; q < Q; ++q) {
        long steps = 0;
        for (long r = (long)q * kLanes; r < items; r += (long)kLanes * Q) {
            int longest = 0;
            for (long t = r; t < std::min(items, r + kLanes); ++t) longest = std::max(longest, (int)(t % (d + 1)) + 1);
            steps += longest;
        }
        worst = std::max(worst, steps);
    }
    return (int)std::min(worst, (long)INT32_MAX);
}

bool prefer_simple_dealing(int d, int J, int w, int schedule_steps) {
    // a dealt step costs about 0.15 (w = 1) or 0.4-0.5 (w = 2) schedule steps
    // (measured on p2 at d = 152; 0.5 keeps the marginal cases of the batched
    // configuration on the schedule)
    if (w > 2) return false;
    return dealt_steps(d, J) * (w == 1 ? 0.15 : 0.5) < schedule_steps;
}

// Pairwise tree over `items`; pushes the jobs of round r into rounds[r].
static int tree_rounds(std::vector<int32_t> live, std::vector<std::vector<std::array<int32_t, 2>>> &rounds) {
    int r = 0;
    while (live.size() > 1) {
        if ((int)rounds.size() <= r) rounds.emplace_back();
        std::vector<int32_t> next;
        size_t pairs = live.size() / 2;
        for (size_t p = 0; p < pairs; ++p) {
            rounds[r].push_back({live[2 * p], live[2 * p + 1]});
            next.push_back(live[2 * p + 1]);
        }
        if (live.size() % 2) next.push_back(live.back());
        live.swap(next);
        ++r;
    }
    return live.empty() ? -1 : live[0];
}

std::string check_hazards(const Plan &P) {
    // Each slot's last writer stage: inputs at stage 0, conv layer L at stage
    // L, addition level r at stage n_layers + r.  A job may read a slot only
    // when it was written at an earlier stage, and two jobs of one stage may
    // not touch a slot that one of them writes.
    std::vector<int> written(P.n_series, -1);
    for (int s = 0; s < 1 + P.N + P.n; ++s) written[s] = 0;
    for (auto &c : P.stage) written[c[0]] = 0;
    auto stage_check = [&](int stage, const std::vector<std::array<int32_t, 3>> &jobs) -> std::string {
        std::unordered_map<int32_t, int> writer;
        for (size_t q = 0; q < jobs.size(); ++q) {
            int32_t w = jobs[q][2];
            // the second operand of a convolution is streamed while outputs are
            // written, so it may never be the job's own output
            const bool conv_stage = stage <= P.n_layers() || stage > P.n_layers() + 1 + P.n_levels();
            if (conv_stage && jobs[q][1] == w) return "second operand is the output";
            // nor the first one when it is streamed, or when a job spans several
            // wavefronts (each stages it on its own, not necessarily before
            // another wavefront of the job stores)
            if (conv_stage && (P.streamed || P.lanes.waves_per_job > 1) && jobs[q][0] == w)
                return "first operand is the output (streamed, or a job over several wavefronts)";
            if (w < 0 || w >= P.n_series) return "slot out of range";
            if (!writer.emplace(w, (int)q).second) return "two jobs write one slot";
        }
        for (size_t q = 0; q < jobs.size(); ++q)
            for (int r = 0; r < 2; ++r) {
                int32_t s = jobs[q][r];
                if (s < 0 || s >= P.n_series) return "slot out of range";
                auto it = writer.find(s);
                if (it != writer.end() && it->second != (int)q) return "read of a slot written in the same stage";
                if (written[s] < 0 || written[s] >= stage) return "read before write";
            }
        for (auto &j : jobs) written[j[2]] = stage;
        return "";
    };
    for (int L = 1; L <= P.n_layers(); ++L) {
        std::vector<std::array<int32_t, 3>> jobs(P.conv.begin() + P.conv_off[L - 1], P.conv.begin() + P.conv_off[L]);
        auto e = stage_check(L, jobs);
        if (!e.empty()) return "conv layer " + std::to_string(L) + ": " + e;
    }
    {
        // the scale stage: job {src, dst, e} reads src and writes dst
        std::vector<std::array<int32_t, 3>> jobs;
        for (auto &c : P.scale) {
            if (c[2] < 2 || c[2] > kMaxExponent) return "scale job with a bad exponent";
            jobs.push_back({c[0], c[0], c[1]});
        }
        auto e = stage_check(P.n_layers() + 1, jobs);
        if (!e.empty()) return "scale stage: " + e;
    }
    for (int r = 1; r <= P.n_levels(); ++r) {
        std::vector<std::array<int32_t, 3>> jobs;
        for (int64_t q = P.add_off[r - 1]; q < P.add_off[r]; ++q) jobs.push_back({P.add[q][0], P.add[q][1], P.add[q][1]});
        auto e = stage_check(P.n_layers() + 1 + r, jobs);
        if (!e.empty()) return "add level " + std::to_string(r) + ": " + e;
    }
    for (auto s : P.out_slots)
        if (s >= 0 && written[s] < 0) return "output slot never written";
    if (!P.corr.empty() || P.ybar_slot >= 0) {
        const int stage = P.n_layers() + P.n_levels() + 2;
        written[P.ybar_slot] = stage - 1;  // staged before the reverse layer
        auto e = stage_check(stage, P.corr);
        if (!e.empty()) return "reverse layer: " + e;
    }
    return "";
}

static std::string build_plan_mode(int n, int N, int d, int m, const int32_t *nvars, const int32_t *vars,
                                   const int32_t *exps, uint32_t flags, bool stream, bool no_inplace, Plan &P,
                                   bool *unsupported);

// Relative cost of a layer plan: each layer takes about ceil(wavefronts /
// SIMDs) wavefront lifetimes (a SIMD's throughput hardly depends on how many
// wavefronts share it), a streamed step costing ~1.2 staged steps (p1 10d: 15.2
// vs 12.9 ms at equal steps).
constexpr long kSimds = 1024;  // MI355X: 256 CUs x 4 SIMDs

static double layer_cost(const Plan &P, int waves_per_job, int jobs_per_group, int steps, double step_cost,
                         int from_layer = 1) {
    double c = 0;
    for (int L = from_layer; L <= P.n_layers(); ++L) {
        const long jobs = P.conv_off[L] - P.conv_off[L - 1];
        const long waves = (jobs + jobs_per_group - 1) / jobs_per_group * waves_per_job;
        c += std::ceil(waves / (double)kSimds) * steps * step_cost;
    }
    return c;
}

// Staged operands: jobs per wavefront J and wavefronts per job Q for the
// layers from_layer.. (the others are launched otherwise).
static void choose_staged_lanes(Plan &P, int from_layer) {
    const int d = P.d, w = P.w;
    // Candidates, by the layer cost model: J jobs per wavefront by the lane
    // schedule (J0 halved down to 1), one job over Q = 2..4 wavefronts,
    // and for coefficients of at most two doubles the same J dealt to the
    // lanes in turn (steps weighted by their lower cost).  Fewer jobs per
    // wavefront or several wavefronts per job pay when layers have fewer
    // wavefronts than the chip has SIMDs (deep chains such as p2).
    // (A candidate replaces the default only when estimated 10% faster: the
    // model ignores staging and per-wavefront costs, e.g. p2 4d d = 64's two jobs
    // per wavefront measure 4% faster than one although it predicts the
    // opposite.)  Dealt steps weigh 0.15 (m = 1) or 0.4 (m = 2): measured
    // on p2 at d = 152.
    const int J0 = choose_jobs_per_group(d, w);
    double best = -1;
    auto consider = [&](LaneSchedule &&ls, bool simple, double c) {
        if (best < 0 || c < 0.9 * best) {
            best = c;
            P.lanes = std::move(ls);
            P.simple = simple;
        }
    };
    for (int J = J0;; J /= 2) {
        LaneSchedule ls = make_lane_schedule(d, J);
        const double c = layer_cost(P, 1, J, ls.steps, 1.0, from_layer);
        if (w <= 2) {
            const double sc = layer_cost(P, 1, J, dealt_steps(d, J), w == 1 ? 0.15 : 0.4, from_layer);
            if (sc < c) {
                consider(std::move(ls), true, sc);
                if (J == 1) break;
                continue;
            }
        }
        consider(std::move(ls), false, c);
        if (J == 1) break;
    }
    for (int Q = 2; Q <= 4 && d + 1 >= kLanes; ++Q) {
        LaneSchedule ls = make_lane_schedule(d, 1, Q);
        const double c = layer_cost(P, Q, 1, ls.steps, 1.0, from_layer);
        consider(std::move(ls), false, c);
    }
    // one job's coefficients dealt over Q wavefronts (deep chains of small
    // layers, such as p2, at one or two doubles per coefficient)
    for (int Q = 2; Q <= 4 && w <= 2 && d + 1 > (Q - 1) * kLanes; ++Q)
        consider(make_lane_schedule(d, 1, Q), true, layer_cost(P, Q, 1, dealt_steps(d, 1, Q), w == 1 ? 0.15 : 0.4, from_layer));
}

// Layer balancing.  The layering above puts every convolution at its
// earliest layer; many jobs have slack (b_1 of a four-variable monomial is
// needed only by b_2, c_1 by nothing but the additions), and any layering
// that keeps each job after the jobs it depends on gives the same bits.  A
// layer costs about ceil(wavefronts / SIMDs) rounds, so the pass moves jobs
// with slack to later layers until each layer but the last fills whole rounds
// of `per_round` jobs where it can (p1: 3640/5460/5460/1820 jobs, 18 rounds
// of 1024, become 3072/4096/6144/3068, 16 rounds).  The depth stays the same.
//
// Dependencies come from slot accesses in the old layer order: a job depends
// on the last writer of each slot it reads (read after write), on the last
// writer of the slot it writes (write after write) and on every job that read
// that slot since (write after read; a job's in-place read of its own output
// is no dependency).  latest[j] is the last layer j can take with its
// dependants still fitting below the depth.  Layer by layer, the ready jobs
// (all dependencies placed earlier) are taken least slack first, then by
// their old order: all whose latest layer this is, and beyond them as many
// whole rounds as the ready jobs fill (or the rest of the round the
// mandatory ones start).  Within a layer jobs keep their old relative order.
// Returns false (P unchanged) if nothing moved.
static bool balance_layers(Plan &P, long per_round) {
    const int D = P.n_layers();
    const long nj = (long)P.conv.size();
    if (D < 2 || nj == 0 || per_round < 1) return false;
    std::vector<int> old_layer(nj);
    for (int L = 1; L <= D; ++L)
        for (int64_t j = P.conv_off[L - 1]; j < P.conv_off[L]; ++j) old_layer[j] = L;
    // edges (from, to) with from in an earlier old layer than to
    std::vector<std::pair<int, int>> edges;
    std::vector<int> last_writer(P.n_series, -1);
    std::vector<int> reader_head(P.n_series, -1);  // readers since the last write, as linked lists
    std::vector<int> reader_job, reader_next;
    for (int L = 1; L <= D; ++L) {
        const long lo = P.conv_off[L - 1], hi = P.conv_off[L];
        for (long j = lo; j < hi; ++j) {
            const auto &t = P.conv[j];
            for (int r = 0; r < 2; ++r)
                if (last_writer[t[r]] >= 0) edges.push_back({last_writer[t[r]], (int)j});
            if (last_writer[t[2]] >= 0) edges.push_back({last_writer[t[2]], (int)j});
            for (int q = reader_head[t[2]]; q >= 0; q = reader_next[q])
                if (reader_job[q] != (int)j) edges.push_back({reader_job[q], (int)j});
        }
        for (long j = lo; j < hi; ++j)
            for (int r = 0; r < 2; ++r) {
                const int32_t s = P.conv[j][r];
                if (r == 1 && s == P.conv[j][0]) continue;
                reader_job.push_back((int)j);
                reader_next.push_back(reader_head[s]);
                reader_head[s] = (int)reader_job.size() - 1;
            }
        for (long j = lo; j < hi; ++j) {
            last_writer[P.conv[j][2]] = (int)j;
            reader_head[P.conv[j][2]] = -1;
        }
    }
    // successor lists (CSR)
    std::vector<int> sbeg(nj + 1, 0), succ(edges.size()), npred(nj, 0);
    for (auto &e : edges) {
        if (old_layer[e.first] >= old_layer[e.second]) return false;  // not a valid layering: leave it
        sbeg[e.first + 1]++;
        npred[e.second]++;
    }
    for (long j = 0; j < nj; ++j) sbeg[j + 1] += sbeg[j];
    {
        std::vector<int> fill(sbeg.begin(), sbeg.end() - 1);
        for (auto &e : edges) succ[fill[e.first]++] = e.second;
    }
    std::vector<int> latest(nj, D);
    for (long j = nj - 1; j >= 0; --j)
        for (int q = sbeg[j]; q < sbeg[j + 1]; ++q) latest[j] = std::min(latest[j], latest[succ[q]] - 1);
    std::vector<int> layer(nj, 0), ready, next;
    for (long j = 0; j < nj; ++j)
        if (npred[j] == 0) ready.push_back((int)j);
    long placed = 0;
    for (int L = 1; L <= D; ++L) {
        std::sort(ready.begin(), ready.end(), [&](int a, int b) {
            return latest[a] != latest[b] ? latest[a] < latest[b] : a < b;
        });
        const long nr = (long)ready.size();
        long mand = 0;
        while (mand < nr && latest[ready[mand]] <= L) ++mand;
        long take = nr;
        if (L < D) {
            const long whole = nr / per_round * per_round;
            take = whole >= mand ? whole : std::min(nr, (mand + per_round - 1) / per_round * per_round);
            if (take == 0) take = nr;
        }
        next.clear();
        for (long q = 0; q < nr; ++q) {
            const int j = ready[q];
            if (q >= take) {
                next.push_back(j);
                continue;
            }
            layer[j] = L;
            ++placed;
            for (int s = sbeg[j]; s < sbeg[j + 1]; ++s)
                if (--npred[succ[s]] == 0) next.push_back(succ[s]);
        }
        ready.swap(next);
    }
    if (placed != nj || !ready.empty()) return false;
    bool moved = false;
    for (long j = 0; j < nj; ++j) moved |= layer[j] != old_layer[j];
    if (!moved) return false;
    std::vector<std::array<int32_t, 3>> conv;
    conv.reserve(nj);
    std::vector<int64_t> off{0};
    for (int L = 1; L <= D; ++L) {
        for (long j = 0; j < nj; ++j)
            if (layer[j] == L) conv.push_back(P.conv[j]);
        off.push_back((int64_t)conv.size());
    }
    P.conv.swap(conv);
    P.conv_off.swap(off);
    return true;
}

// Fused layers: split the convolutions into independent components.  Two jobs
// depend on each other only through a slot that some convolution writes (the
// staged inputs a_k and z_i are read-only), so a union of every job's output
// slot with each operand slot that is also written puts every read after
// write, write after write and write after read pair in one component.  The
// layers inside a component keep the plan's order.
// Returns the most jobs of one component in one layer (0 if nothing was fused).
static int fuse_layers(Plan &P) {
    const int nl = P.n_layers();
    const size_t nj = P.conv.size();
    if (nl < 1 || nj == 0) return 0;
    std::vector<int64_t> parent(P.n_series);
    for (int64_t s = 0; s < P.n_series; ++s) parent[s] = s;
    auto find = [&](int64_t s) {
        while (parent[s] != s) s = parent[s] = parent[parent[s]];
        return s;
    };
    std::vector<char> written(P.n_series, 0);
    for (const auto &t : P.conv) written[t[2]] = 1;
    for (const auto &t : P.conv)
        for (int o = 0; o < 2; ++o)
            if (written[t[o]]) {
                const int64_t a = find(t[o]), b = find(t[2]);
                if (a != b) parent[a] = b;
            }
    std::vector<int32_t> comp_of_root(P.n_series, -1), comp(nj);
    int32_t C = 0;
    for (size_t j = 0; j < nj; ++j) {
        const int64_t r = find(P.conv[j][2]);
        if (comp_of_root[r] < 0) comp_of_root[r] = C++;
        comp[j] = comp_of_root[r];
    }
    std::vector<int> layer(nj);
    for (int L = 1; L <= nl; ++L)
        for (int64_t j = P.conv_off[L - 1]; j < P.conv_off[L]; ++j) layer[j] = L;
    // counting sort by (component, layer), stable inside each bucket
    std::vector<int32_t> cnt((size_t)C * (nl + 1) + 1, 0);
    for (size_t j = 0; j < nj; ++j) cnt[(size_t)comp[j] * (nl + 1) + layer[j]]++;
    int widest = 0;
    for (int32_t x : cnt) widest = std::max(widest, (int)x);
    P.fused_off.assign((size_t)C * (nl + 1), 0);
    int32_t acc = 0;
    for (int32_t c = 0; c < C; ++c) {
        P.fused_off[(size_t)c * (nl + 1)] = acc;
        for (int L = 1; L <= nl; ++L) {
            acc += cnt[(size_t)c * (nl + 1) + L];
            P.fused_off[(size_t)c * (nl + 1) + L] = acc;
        }
    }
    std::vector<int32_t> pos(P.fused_off);
    P.fused_conv.assign(nj, {0, 0, 0});
    for (size_t j = 0; j < nj; ++j) {
        const size_t key = (size_t)comp[j] * (nl + 1) + layer[j] - 1;
        P.fused_conv[pos[key]++] = P.conv[j];
    }
    P.fused_components = C;
    P.fused_lanes = make_lane_schedule(P.d, 1);
    P.fused_simple = prefer_simple_dealing(P.d, 1, P.w, P.fused_lanes.steps);
    // up to four wavefronts (one per SIMD of a CU); the launcher lowers this
    // where their LDS would not fit
    P.fused_waves = std::min(4, std::max(1, widest));
    return widest;
}

static void unfuse(Plan &P) {
    P.fused_conv.clear();
    P.fused_off.clear();
    P.fused_components = P.fused_waves = 0;
    P.fused_lanes = LaneSchedule();
    P.fused_simple = false;
}

// Fuse the layers by default where each layer is a short step that the per-layer
// kernel boundary (~4.5 us on MI355X) would dominate: deep plans, one
// wavefront per job, and either small layers (under half a round of the
// SIMDs) at small coefficients or low degree, or coefficients of one double
// (two up to d = 63).  Measured, fused against per-layer: p2 (64 layers of
// 378 jobs) 3.9x at one double and d = 8, 1.7x at d = 63, 1.5x at two doubles
// and d = 63, 1.0x at four doubles and d = 63-95, 1.2x at ten doubles and
// d = 8, slower beyond (ten doubles at d = 31: 0.95x); p1 (4 layers of
// 3072-6144 jobs) 1.14-1.2x at one double, 1.12-1.13x at two up to d = 63,
// 0.99x at d = 152, 0.87x at four doubles and d = 8.  Slower too wherever the
// plan spreads a job over several wavefronts or packs many short jobs into one
// (p3 at d = 8: 0.2x).  On p2 beyond four doubles (wall time): five doubles
// 1.17x at d = 15, 1.0x at d = 31; ten doubles 1.14x at d = 15, 1.05x at
// d = 31; eight doubles 1.2x at d = 8 but 0.99x at d = 15 and 0.89x at d = 31
// (the other widths take eight doubles' limit).  The caller also requires
// every component's layer to fit one round of four wavefronts.
static bool fuse_by_default(const Plan &P) {
    if (P.streamed || P.lanes.waves_per_job != 1 || P.n_layers() < 4) return false;
    if (P.w == 1 || (P.w == 2 && P.d <= 63)) return true;
    for (int L = 1; L <= P.n_layers(); ++L)
        if (P.conv_off[L] - P.conv_off[L - 1] > 512) return false;
    return P.d <= (P.w <= 4 ? 127 : (P.w == 5 || P.w == 10) ? 31 : 8);
}

// ------------------------------------------------------------ chain launch
// Timing of the chain kernel (conv_chain_kernel): every lane of a chain's
// workgroup runs the same steps.  The first operand of step t is read from
// LDS in iteration t-1 (in the prologue, iteration -1, for t = 0); a
// coefficient is stored -- to A and, for the chain's next product, to the LDS
// slot of that product's first operand -- in the iteration of its last step;
// a workgroup barrier follows iteration s when (s+1) % S == 0.  A store and a
// read of one LDS coefficient are therefore ordered exactly when their
// windows floor(iteration / S) differ.

static inline int chain_window(int it, int S) { return it >= 0 ? it / S : -1; }

int make_chain_schedule(int L, int d, int W, int S, int B, std::vector<int32_t> &codes, int *stride) {
    // Jobs in chain order, each job's coefficients longest first; each at the
    // earliest step its first operand allows (every x_i read after the window
    // of its store by the previous job; its own store into the LDS slot of
    // job l+1 after the last read of the product that slot held, B jobs
    // earlier), on the lane free by then with the least idle time before it,
    // else on the lane that frees first.
    const int lanes = kLanes * W, d1 = d + 1;
    std::vector<int> lane_free(lanes, 0);
    std::vector<std::vector<int32_t>> lists(lanes);
    std::vector<int> store((size_t)L * d1, 0);
    std::vector<int> last_read(L, -1);
    for (int l = 0; l < L; ++l) {
        for (int k = d; k >= 0; --k) {
            int s0 = 0;
            if (l > 0)
                for (int i = 0; i <= k; ++i)
                    s0 = std::max(s0, S * (chain_window(store[(size_t)(l - 1) * d1 + i], S) + 1) - i + 1);
            if (l + 1 < L && l + 1 - B >= 0) s0 = std::max(s0, S * (chain_window(last_read[l + 1 - B], S) + 1) - k);
            int best = -1;
            for (int q = 0; q < lanes; ++q)
                if (lane_free[q] <= s0 && (best < 0 || lane_free[q] > lane_free[best])) best = q;
            if (best < 0) {
                best = 0;
                for (int q = 1; q < lanes; ++q)
                    if (lane_free[q] < lane_free[best]) best = q;
            }
            const int start = std::max(s0, lane_free[best]);
            for (int g = start - lane_free[best]; g > 0;) {
                const int q = std::min(g, 0x10000);
                lists[best].push_back((kIdleJob << 16) | (q - 1));
                g -= q;
            }
            lists[best].push_back((l << 16) | k);
            lane_free[best] = start + k + 1;
            store[(size_t)l * d1 + k] = start + k;
            last_read[l] = std::max(last_read[l], start + k - 1);
        }
    }
    // a multiple of the window, and even (the kernel may run two steps per iteration)
    const int q = S % 2 ? 2 * S : S;
    int steps = *std::max_element(lane_free.begin(), lane_free.end());
    steps = (steps + q - 1) / q * q;
    size_t st = 1;
    for (auto &x : lists) st = std::max(st, x.size() + 1);
    *stride = (int)st;
    codes.assign((size_t)lanes * st, -1);
    for (int q = 0; q < lanes; ++q) std::copy(lists[q].begin(), lists[q].end(), codes.begin() + (size_t)q * st);
    return steps;
}

std::string check_chain_schedule(int L, int d, int W, int S, int B, int steps, const int32_t *codes, int stride) {
    if (L < 1 || L > kMaxChainLength || d < 0 || W < 1 || W > 16 || S < 1 || B < 2 || steps < 0 || steps % S ||
        stride < 1 || !codes)
        return "bad chain schedule parameters";
    const int lanes = kLanes * W, d1 = d + 1;
    std::vector<int> start((size_t)L * d1, -1);
    for (int q = 0; q < lanes; ++q) {
        const int32_t *row = codes + (size_t)q * stride;
        long t = 0;
        int e = 0;
        for (; e < stride && row[e] >= 0; ++e) {
            const int j = row[e] >> 16, k = row[e] & 0xffff;
            if (j == kIdleJob) {
                t += k + 1;
                continue;
            }
            if (j >= L || k > d) return "code out of range";
            const size_t key = (size_t)j * d1 + k;
            if (start[key] >= 0) return "coefficient scheduled twice";
            start[key] = (int)t;
            t += k + 1;
        }
        if (e == stride) return "row without its terminator";
        if (t > steps) return "row longer than the steps";
    }
    for (int v : start)
        if (v < 0) return "coefficient never scheduled";
    for (int l = 0; l < L; ++l)
        for (int k = 0; k <= d; ++k) {
            const int s = start[(size_t)l * d1 + k];
            for (int i = 0; i <= k; ++i) {
                const int rd = s + i - 1;  // iteration that reads x_i
                // job 0's first operand is staged before the first barrier
                if (l > 0 && chain_window(rd, S) <= chain_window(start[(size_t)(l - 1) * d1 + i] + i, S))
                    return "job " + std::to_string(l) + " coefficient " + std::to_string(k) +
                           ": first operand read before the barrier after its store";
                // job l-1+B stores the first operand of job l+B into the same slot
                const int wj = l - 1 + B;
                if (wj + 1 < L && chain_window(start[(size_t)wj * d1 + i] + i, S) <= chain_window(rd, S))
                    return "job " + std::to_string(l) + " coefficient " + std::to_string(k) +
                           ": first operand overwritten before the barrier after its read";
            }
        }
    return "";
}

// Chains of the plan's convolutions: a job whose second operand is a staged
// input (written by no convolution) starts a chain when its first operand is
// one too, and continues the chain of its first operand's writer when it is
// the first such job to read that output.  Jobs in launch (topological)
// order; chains[c] lists job indices in chain order.  Requires one writer per
// slot (no in-place jobs).
static bool find_chains(const Plan &P, std::vector<std::vector<int64_t>> &chains) {
    const size_t nj = P.conv.size();
    std::vector<int64_t> writer(P.n_series, -1);
    for (size_t j = 0; j < nj; ++j) {
        if (writer[P.conv[j][2]] >= 0) return false;
        writer[P.conv[j][2]] = (int64_t)j;
    }
    std::vector<int64_t> chain_of(nj, -1);
    chains.clear();
    for (size_t j = 0; j < nj; ++j) {
        const auto &t = P.conv[j];
        if (writer[t[1]] >= 0 || t[0] == t[2]) continue;
        const int64_t p = writer[t[0]];
        if (p < 0) {
            chain_of[j] = (int64_t)chains.size();
            chains.push_back({(int64_t)j});
        } else if (chain_of[p] >= 0 && chains[chain_of[p]].back() == p &&
                   (int)chains[chain_of[p]].size() < kMaxChainLength) {
            chain_of[j] = chain_of[p];
            chains[chain_of[p]].push_back((int64_t)j);
        }
    }
    return !chains.empty();
}

// Rebuilds P's convolution layers for the chain launch with W wavefronts per
// chain, a barrier every S steps and B LDS slots of first operands: layer L
// <= pipe_layers holds the jobs at position L of their chain, the other jobs
// follow at their earliest layers.  Returns the estimated cost (in wavefront
// steps per SIMD, the unit of layer_cost) or -1 when no chain launch applies.
static double make_chain_plan(Plan &P, const std::vector<std::vector<int64_t>> &chains, int W, int S, int B) {
    const size_t nj = P.conv.size();
    int Lmax = 0;
    std::vector<char> in_chain(nj, 0);
    for (auto &c : chains) {
        Lmax = std::max(Lmax, (int)c.size());
        for (int64_t j : c) in_chain[j] = 1;
    }
    // the other jobs at their earliest layers after the chain launch
    std::vector<int> wlayer(P.n_series, 0);
    std::vector<int> rest_layer(nj, 0);
    int rest_layers = 0;
    for (size_t j = 0; j < nj; ++j) {
        if (in_chain[j]) continue;
        const auto &t = P.conv[j];
        const int L = std::max(wlayer[t[0]], wlayer[t[1]]) + 1;
        rest_layer[j] = L;
        wlayer[t[2]] = std::max(wlayer[t[2]], L);
        rest_layers = std::max(rest_layers, L);
    }
    std::vector<std::array<int32_t, 3>> conv;
    std::vector<int64_t> off{0};
    for (int L = 0; L < Lmax; ++L) {
        for (auto &c : chains)
            if ((int)c.size() > L) conv.push_back(P.conv[c[L]]);
        off.push_back((int64_t)conv.size());
    }
    for (int L = 1; L <= rest_layers; ++L) {
        for (size_t j = 0; j < nj; ++j)
            if (!in_chain[j] && rest_layer[j] == L) conv.push_back(P.conv[j]);
        off.push_back((int64_t)conv.size());
    }
    if (conv.size() != nj) return -1;
    // one schedule per chain length
    std::vector<ChainComp> comps;
    std::vector<std::array<int32_t, 3>> pjobs;
    std::vector<int32_t> codes;
    std::vector<std::array<int, 3>> sched(Lmax + 1, {-1, 0, 0});  // length -> {code_off, stride, steps}
    int worst = 0;
    for (auto &c : chains) {
        const int len = (int)c.size();
        if (sched[len][0] < 0) {
            std::vector<int32_t> cs;
            int stride = 0;
            const int steps = make_chain_schedule(len, P.d, W, S, B, cs, &stride);
            if (!check_chain_schedule(len, P.d, W, S, B, steps, cs.data(), stride).empty()) return -1;
            if (codes.size() + cs.size() > (size_t)INT32_MAX / 2) return -1;
            sched[len] = {(int)codes.size(), stride, steps};
            codes.insert(codes.end(), cs.begin(), cs.end());
        }
        comps.push_back(ChainComp{(int32_t)pjobs.size(), len, sched[len][0], sched[len][1], sched[len][2], 0, 0, 0});
        worst = std::max(worst, sched[len][2]);
        for (int64_t j : c) pjobs.push_back(P.conv[j]);
    }
    P.conv.swap(conv);
    P.conv_off.swap(off);
    P.pipe_layers = Lmax;
    P.pipe_waves = W;
    P.pipe_window = S;
    P.pipe_ring = B;
    P.pipe_jobs.swap(pjobs);
    P.pipe_comps.swap(comps);
    P.pipe_codes.swap(codes);
    P.balanced = false;
    choose_staged_lanes(P, Lmax + 1);
    // a chain's workgroup holds a CU: k = W/4 wavefronts per SIMD, ceil(chains
    // / CUs) rounds.  A lone wavefront keeps its SIMD's VALU about half busy
    // (counters on c2: 0.49); k of them share it at eff(k) of k times the
    // lone step's cost (measured on p2 at d = 31..152 and four, eight and ten
    // doubles, the same schedules at 4..16 wavefronts: eff(2) = 0.80, eff(3)
    // = 0.73, eff(4) = 0.70 up to five doubles per coefficient; 0.89, 0.81,
    // 0.74 from eight on, where one step is long enough to fill the pipeline
    // better).
    const long cus = kSimds / 4;
    const double rounds = std::ceil((double)chains.size() / cus);
    const int k = std::max(1, W / 4);
    static const double eff_short[5] = {1.0, 1.0, 0.80, 0.73, 0.70}, eff_long[5] = {1.0, 1.0, 0.89, 0.81, 0.74};
    const double eff = P.w >= 8 ? eff_long[std::min(k, 4)] : eff_short[std::min(k, 4)];
    // a chain step at one double per coefficient costs about 0.55 of a
    // schedule step (measured on p2 at d = 8..152 against the dealt plans)
    const double step = P.w == 1 ? 0.55 : 1.0;
    const double chain_cost = rounds * worst * k * eff * (1.0 + 0.02 * 4.0 / S) * step;
    // the layers after the chains (p2's cross products), dealt or by the lane
    // schedule as choose_staged_lanes set them, weighed as the plan without a
    // chain launch weighs its steps
    const int Q = P.lanes.waves_per_job, J = P.lanes.jobs_per_group;
    const double rest = P.simple ? layer_cost(P, Q, J, dealt_steps(P.d, J, Q), P.w == 1 ? 0.15 : 0.4, Lmax + 1)
                                 : layer_cost(P, Q, J, P.lanes.steps, 1.0, Lmax + 1);
    return chain_cost + rest;
}

// LDS slots of first operands a chain workgroup gets: up to 96 KiB of LDS
// (one workgroup per CU then), at least two, at most the longest chain.
static int chain_ring_slots(const Plan &P, int Lmax) {
    const long per = (long)(P.d + 1) * P.w * 8;
    const long jobs = (long)Lmax * 32;
    const long fit = (98304 - jobs) / per;
    return (int)std::min<long>(std::max(Lmax, 2), fit);
}

// The chain launch for a plan without in-place jobs: the cheapest of W = 4,
// 8, 12, 16 wavefronts and barriers every S = 1, 2, 4 steps, applied when forced or
// estimated under 0.9 of `other` (the cost of the plan without it).  On p2
// (64 products per chain) that is every precision from two doubles on at
// d = 8..191 (measured 1.3-7.4x faster) and one double at d = 31..152
// (1.1-1.6x); one double at d = 191 keeps its dealt per-layer plan (the chain
// launch measured 7% slower there).  Returns whether P now holds a chain
// launch.
static constexpr bool kChainByDefault = true;

static bool choose_chain_launch(Plan &P, bool forced, double other) {
    if (P.streamed) return false;
    std::vector<std::vector<int64_t>> chains;
    if (!find_chains(P, chains)) return false;
    int Lmax = 0;
    long members = 0;
    for (auto &c : chains) {
        Lmax = std::max(Lmax, (int)c.size());
        members += (long)c.size();
    }
    if (!forced && (Lmax < 16 || 4 * members < (long)P.conv.size())) return false;
    const int B = chain_ring_slots(P, Lmax);
    if (B < 2) return false;
    double best = -1;
    int bw = 0, bs = 0;
    // up to 16 wavefronts (1024 threads, at most 128 VGPRs each: not for ten
    // doubles per coefficient, whose chain kernel needs 134)
    for (int W : {4, 8, 12, 16})
        for (int S : {1, 2, 4}) {
            if (W == 16 && P.w > 8) continue;
            Plan T = P;
            const double c = make_chain_plan(T, chains, W, S, B);
            if (c >= 0 && (best < 0 || c < best)) {
                best = c;
                bw = W;
                bs = S;
            }
        }
    if (best < 0 || (!forced && best >= 0.9 * other)) return false;
    return make_chain_plan(P, chains, bw, bs, B) >= 0;
}

// ----------------------------------------------------------- single launch
// FP64 instructions of one md_add / md_mul of the specification (two_sum = 6
// additions, two_prod = 1 mul + 1 fma; the closed forms of the accounting).
static long md_instr(bool mul, int m) {
    const long rs = m >= 2 ? 2 * m - 3 : 0;
    if (!mul) return 6 * ((long)m * (m - 1) / 2 + rs) + m;
    long ntp = m >= 2 ? (m - 1) + (long)(m - 2) * (m - 1) / 2 : 0;
    long tse = m >= 2 ? (long)(m - 2) * (m - 1) / 2 : 0;
    long tsp = 0, plain = m - 1;
    for (int k = 1; k < m - 1; ++k) {
        tsp += (long)k * (2 * m - 3 - 2 * k);
        plain += 2 * k;
    }
    return 6 * (tse + tsp + rs) + plain + (ntp + 1) + (ntp + 2 * (m - 1));
}

// Estimated microseconds of a plan's evaluation: per-launch (the kernel
// boundary of ~4.5 us between dependent launches, measured on MI355X, plus
// each launch's rounds of the SIMDs) against one workgroup of `waves`
// wavefronts that runs every stage.  A multiply-add step of one wavefront
// costs its md instructions plus ~50 of bookkeeping, 4 cycles each at
// ~2.2 GHz; a wavefront sharing its SIMD with k-1 others takes k times as
// long.  Dealt coefficients (w <= 2) take the measured weight of their steps.
struct SingleCost {
    double multi_us, single_us;
    int waves;
    LaneSchedule lanes;
    bool simple;
};

static SingleCost single_launch_cost(const Plan &P) {
    const bool cx = P.complex_series();
    const long mul = cx ? 4 * md_instr(true, P.m) + 2 * md_instr(false, P.m) : md_instr(true, P.m);
    const long add = (cx ? 2 : 1) * md_instr(false, P.m);
    const double step_us = (double)(mul + add + 50) * 4 / 2200.0;
    const double add_us = (double)(add + 20) * 4 / 2200.0;
    const double boundary_us = 4.5;
    const long d1 = P.d + 1;
    SingleCost c{0, 0, 0, LaneSchedule(), false};
    // per launch
    const int J = P.lanes.jobs_per_group, Q = P.lanes.waves_per_job;
    const double lsteps = P.simple ? dealt_steps(P.d, J, Q) * (P.w == 1 ? 0.15 : 0.4) : (double)P.lanes.steps;
    long launches = 2 + P.n_layers() + P.n_levels() + (P.scale.empty() ? 0 : 1);
    c.multi_us = launches * boundary_us;
    for (int L = 1; L <= P.n_layers(); ++L) {
        const long waves = (P.conv_off[L] - P.conv_off[L - 1] + J - 1) / J * Q;
        c.multi_us += std::ceil(waves / (double)kSimds) * lsteps * step_us;
    }
    for (int r = 1; r <= P.n_levels(); ++r) {
        const long items = (P.add_off[r] - P.add_off[r - 1]) * d1;
        c.multi_us += std::ceil(items / (256.0 * kSimds)) * add_us;
    }
    // one workgroup: the cheapest of 4, 8 and 16 wavefronts, one-wavefront
    // groups of J0 (or fewer) jobs within the LDS of the workgroup
    c.single_us = -1;
    const long stage_items = (long)P.stage.size() * d1, gather_items = (long)(1 + P.n) * d1;
    for (int W : {4, 8, 16}) {
        const int lds_per_coef = lds_doubles_per_coef(P.w);
        for (int Js = choose_jobs_per_group(P.d, P.w);; Js = std::max(1, Js / 2)) {
            const long bytes = (group_lds_bytes(d1, lds_per_coef, Js) + 15) / 16 * 16;
            if (bytes * W <= kMaxLdsBytes) {
                const LaneSchedule ls = make_lane_schedule(P.d, Js);
                const bool simple = prefer_simple_dealing(P.d, Js, P.w, ls.steps);
                const double st = simple ? dealt_steps(P.d, Js) * (P.w == 1 ? 0.15 : 0.5) : (double)ls.steps;
                const double share = W / 4.0;  // wavefronts per SIMD
                double u = boundary_us;
                for (int L = 1; L <= P.n_layers(); ++L) {
                    const long jobs = P.conv_off[L] - P.conv_off[L - 1];
                    u += std::ceil(jobs / (double)(W * Js)) * st * step_us * share + 0.5;
                }
                const double threads = 64.0 * W;
                for (int r = 1; r <= P.n_levels(); ++r)
                    u += std::ceil((P.add_off[r] - P.add_off[r - 1]) * d1 / threads) * add_us * share + 0.5;
                u += std::ceil((double)P.scale.size() * d1 / threads) * step_us * share;
                u += std::ceil((stage_items + gather_items) / threads) * 0.2 + 1.0;
                if (c.single_us < 0 || u < c.single_us) {
                    c.single_us = u;
                    c.waves = W;
                    c.lanes = ls;
                    c.simple = simple;
                }
                break;
            }
            if (Js == 1) break;
        }
    }
    return c;
}

static bool choose_single_launch(Plan &P, bool forced) {
    if (P.streamed || P.pipe_layers > 0 || P.fused_components > 0) return false;
    const SingleCost c = single_launch_cost(P);
    if (c.single_us < 0 || (!forced && c.single_us >= 0.7 * c.multi_us)) return false;
    P.single = true;
    P.single_waves = c.waves;
    P.single_lanes = c.lanes;
    P.single_simple = c.simple;
    return true;
}

static std::string build_plan_launches(int n, int N, int d, int m, const int32_t *nvars, const int32_t *vars,
                                       const int32_t *exps, uint32_t flags, Plan &P, bool *unsupported) {
    // Staged operands unless asked otherwise, or unless they do not fit in
    // LDS, or unless streaming with several wavefronts per job is estimated
    // to be faster (large d with few jobs per layer).
    std::string err = build_plan_mode(n, N, d, m, nvars, vars, exps, flags, false, false, P, unsupported);
    if (!err.empty()) return err;
    // The chain launch (deep chains of products, p2's above all), when asked
    // for or estimated well under the layered or fused plan.  Its plans give
    // the in-place products fresh output slots: a chain's products overlap,
    // so b_{n-2} must stay readable while b_{n-2} * a_k is stored.
    const bool chain_forced = (flags & kChainLaunch) != 0;
    if (!P.streamed && !(flags & (kFusedLayers | kLayerLaunches | kNoChainLaunch)) &&
        (chain_forced || (kChainByDefault && P.n_layers() >= 16))) {
        // the plan without it, in the layer cost model's units: dealt steps
        // weigh what choose_staged_lanes gives them
        const int Q = P.lanes.waves_per_job, J = P.lanes.jobs_per_group;
        double other = P.simple ? layer_cost(P, Q, J, dealt_steps(d, J, Q), P.w == 1 ? 0.15 : 0.4)
                                : layer_cost(P, Q, J, P.lanes.steps, 1.0);
        if (fuse_by_default(P)) {
            const LaneSchedule one = make_lane_schedule(d, 1);
            const double per = prefer_simple_dealing(d, 1, P.w, one.steps) ? dealt_steps(d, 1) * (P.w == 1 ? 0.15 : 0.5)
                                                                           : (double)one.steps;
            other = std::min(other, P.n_layers() * per);
        }
        Plan C;
        bool uns = false;
        std::string e2 = build_plan_mode(n, N, d, m, nvars, vars, exps, flags, false, true, C, &uns);
        if (e2.empty() && choose_chain_launch(C, chain_forced, other)) {
            auto h = check_hazards(C);
            if (!h.empty()) return "internal planner error (chain launch): " + h;
            P = std::move(C);
            return "";
        }
    }
    if (chain_forced) {
        *unsupported = true;
        return "MDPE_CHAIN_LAUNCH: no chain of products to pipeline, or its first operands do not fit in LDS";
    }
    auto fuse = [&]() {
        if (P.streamed) return err;
        if (flags & kFusedLayers)
            fuse_layers(P);
        else if (!(flags & (kLayerLaunches | kSingleLaunch)) && fuse_by_default(P) && fuse_layers(P) > 4)
            unfuse(P);  // a component would need several rounds per layer
        return err;
    };
    if (P.streamed || (flags & kStageOperands)) return fuse();
    bool paired = false;
    const int Q = stream_waves_per_job(d, &paired);
    if (Q >= 2 && !(flags & kFusedLayers)) {
        const LaneSchedule ss = paired ? make_paired_schedule(d, Q) : make_lane_schedule(d, 1, Q);
        if (layer_cost(P, Q, 1, ss.steps, 1.2) < layer_cost(P, 1, P.lanes.jobs_per_group, P.lanes.steps, 1.0))
            return build_plan_mode(n, N, d, m, nvars, vars, exps, flags, true, false, P, unsupported);
    }
    return fuse();
}

// The plan's launch structure (per layer, fused, chain launch or streamed),
// then, for plans so small that kernel boundaries dominate, the single launch.
std::string build_plan(int n, int N, int d, int m, const int32_t *nvars, const int32_t *vars, const int32_t *exps,
                       uint32_t flags, Plan &P, bool *unsupported) {
    const bool forced = (flags & kSingleLaunch) != 0;
    std::string err = build_plan_launches(n, N, d, m, nvars, vars, exps, forced ? flags | kNoChainLaunch : flags, P,
                                          unsupported);
    if (!err.empty()) return err;
    P.flags = flags;
    if (forced || !(flags & (kLayerLaunches | kFusedLayers | kChainLaunch | kStreamOperands))) {
        if (!choose_single_launch(P, forced) && forced) {
            *unsupported = true;
            return "MDPE_SINGLE_LAUNCH: a job group does not fit in the workgroup's LDS";
        }
    }
    return "";
}

static std::string build_plan_mode(int n, int N, int d, int m, const int32_t *nvars, const int32_t *vars,
                                   const int32_t *exps, uint32_t flags, bool stream, bool no_inplace, Plan &P,
                                   bool *unsupported) {
    *unsupported = false;
    if (flags & ~(kKeepMonomialValues | kComplex | kStreamOperands | kStageOperands | kAsapLayers | kFusedLayers |
                  kLayerLaunches | kChainLaunch | kNoChainLaunch | kSingleLaunch))
        return "unknown flags";
    if ((flags & kChainLaunch) && (flags & (kFusedLayers | kLayerLaunches | kStreamOperands | kNoChainLaunch)))
        return "MDPE_CHAIN_LAUNCH excludes MDPE_FUSED_LAYERS, MDPE_LAYER_LAUNCHES, MDPE_STREAM_OPERANDS and "
               "MDPE_NO_CHAIN_LAUNCH";
    if ((flags & kSingleLaunch) && (flags & (kFusedLayers | kLayerLaunches | kStreamOperands | kChainLaunch)))
        return "MDPE_SINGLE_LAUNCH excludes MDPE_FUSED_LAYERS, MDPE_LAYER_LAUNCHES, MDPE_STREAM_OPERANDS and "
               "MDPE_CHAIN_LAUNCH";
    if ((flags & kFusedLayers) && (flags & kLayerLaunches)) return "MDPE_FUSED_LAYERS and MDPE_LAYER_LAUNCHES exclude each other";
    if ((flags & kStreamOperands) && (flags & kStageOperands)) return "MDPE_STREAM_OPERANDS and MDPE_STAGE_OPERANDS exclude each other";
    const bool keep = (flags & kKeepMonomialValues) != 0;
    const bool cx = (flags & kComplex) != 0;
    if (keep && cx) {
        *unsupported = true;
        return "the reverse pass (MDPE_KEEP_MONOMIAL_VALUES) is for real series only";
    }
    if (n < 1 || N < 0 || d < 0) return "need n >= 1, N >= 0, d >= 0";
    if (!supported_m(m)) {
        *unsupported = true;
        return "m must be one of 1, 2, 3, 4, 5, 8, 10";
    }
    if (N > 0 && (!nvars || !vars)) return "nvars/vars missing";
    int64_t tot = 0, nb = 0, nc = 0;
    int nmax = 0;
    for (int k = 0; k < N; ++k) {
        int nk = nvars[k];
        if (nk < 1 || nk > n) return "monomial " + std::to_string(k) + ": n_k out of range";
        for (int j = 0; j < nk; ++j) {
            int v = vars[tot + j];
            if (v < 0 || v >= n) return "monomial " + std::to_string(k) + ": variable out of range";
            if (j > 0 && v <= vars[tot + j - 1]) return "monomial " + std::to_string(k) + ": variables not strictly increasing";
        }
        tot += nk;
        nb += std::max(1, nk - 2);
        nc += std::max(0, nk - 2);
        nmax = std::max(nmax, nk);
    }
    // General exponents (Section 3): a table of powers z_i^p, p = 2..maxp[i],
    // and one common-factor slot per monomial with an exponent above one.
    std::vector<int> maxp(n, 0);
    int64_t nfac = 0;
    if (exps) {
        int64_t q = 0;
        for (int k = 0; k < N; ++k) {
            bool any = false;
            for (int j = 0; j < nvars[k]; ++j, ++q) {
                const int e = exps[q];
                if (e < 1 || e > kMaxExponent) return "monomial " + std::to_string(k) + ": exponent out of range 1..64";
                maxp[vars[q]] = std::max(maxp[vars[q]], e - 1);
                any |= e >= 2;
            }
            nfac += any;
        }
    }
    int64_t npow = 0;
    std::vector<int64_t> powoff(n, 0);  // slot of z_i^p is pbase + powoff[i] + p - 2
    for (int i = 0; i < n; ++i) {
        powoff[i] = npow;
        npow += std::max(0, maxp[i] - 1);
    }
    if (keep && nfac > 0) {
        *unsupported = true;
        return "the reverse pass (MDPE_KEEP_MONOMIAL_VALUES) is for multilinear monomials only";
    }
    const int64_t base = 1 + (int64_t)N + n;
    int64_t nmono2 = 0;  // monomials with n_k >= 2: they get an M_k slot when kept
    for (int k = 0; k < N; ++k) nmono2 += nvars[k] >= 2;
    const int64_t pbase = base + tot + nb + nc;  // powers, then common factors
    const int64_t fbase = pbase + npow;
    const int64_t mbase = fbase + nfac;
    const int w = cx ? 2 * m : m;
    // Streamed operands when a job's LDS operands would not fit in one
    // workgroup's LDS, or when asked for.  Then no convolution may write its
    // own first operand: b_{n-2} * a and every common-factor step after the
    // first get fresh output slots, after all others.  The same holds for
    // staged operands when one job is spread over several wavefronts
    // (no_inplace): each wavefront stages the first operand on its own, and
    // the wavefronts of a job need not share a workgroup, so one of them could
    // store output coefficients before another has read them.
    const bool fits = (long)(d + 1) * lds_doubles_per_coef(w) * 8 <= kMaxLdsBytes - 32768;
    if ((flags & kStageOperands) && !fits) {
        *unsupported = true;
        return "MDPE_STAGE_OPERANDS: a job's operands do not fit in one workgroup's LDS "
               "((d+1)*w*8 <= 131072 bytes, w = m doubles per coefficient, 2m complex; twice that when w <= 2)";
    }
    const bool streamed = stream || (flags & kStreamOperands) || !fits;
    const bool fresh_out = streamed || no_inplace;
    int64_t n3 = 0, nfac_extra = 0;
    for (int k = 0, q = 0; k < N; q += nvars[k], ++k) {
        n3 += nvars[k] >= 3;
        int cnt = 0;
        for (int j = 0; exps && j < nvars[k]; ++j) cnt += exps[q + j] >= 2;
        nfac_extra += std::max(0, cnt - 1);
    }
    const int64_t xbase = mbase + (keep ? nmono2 + 1 + N + n : 0);
    const int64_t nser = xbase + (fresh_out ? n3 + nfac_extra : 0);
    if (nser > INT32_MAX / 2) {
        *unsupported = true;
        return "too many series for 32-bit slot indices";
    }
    if (d + 1 > 65535) {
        *unsupported = true;
        return "d too large";
    }
    P = Plan();
    P.n = n;
    P.N = N;
    P.d = d;
    P.m = m;
    P.w = w;
    P.flags = flags;
    P.n_series = nser;
    P.streamed = streamed;
    int64_t xpos = 0;
    auto fresh = [&]() { return (int32_t)(xbase + xpos++); };

    std::vector<std::vector<std::array<int32_t, 3>>> layers(std::max(nmax, 1));
    auto add_job = [&](int layer, int32_t t1, int32_t t2, int32_t t3) {
        if ((int)layers.size() < layer) layers.resize(layer);
        layers[layer - 1].push_back({t1, t2, t3});
    };
    std::vector<int32_t> value_list{0};
    std::vector<std::vector<int32_t>> grad_lists(n);
    std::vector<int32_t> mono_slot(N, -1);  // slot holding M_k = prod of the monomial's variables
    for (int s = 0; s < 1 + N + n; ++s) P.stage.push_back({s, s});

    // table of powers: z_i^p := z_i^{p-1} * z_i at layer p-1, ready after it
    auto pow_slot = [&](int i, int p) {
        return p == 1 ? (int32_t)(1 + N + i) : (int32_t)(pbase + powoff[i] + p - 2);
    };
    for (int i = 0; i < n; ++i)
        for (int p = 2; p <= maxp[i]; ++p) add_job(p - 1, pow_slot(i, p - 1), (int32_t)(1 + N + i), pow_slot(i, p));

    int64_t alpha = 0, beta = 0, gamma = 0, pos = 0, mpos = 0, fpos = 0;
    for (int k = 0; k < N; ++k) {
        const int nk = nvars[k];
        const int32_t *v = vars + pos;
        const int32_t *e = exps ? exps + pos : nullptr;
        // common factor a_k * prod_j z_{i_j}^{e_j - 1}, in increasing j; the
        // monomial's own jobs follow it, `shift` layers later
        int32_t a_slot = (int32_t)(k + 1);
        int shift = 0;
        for (int j = 0; e && j < nk; ++j) {
            if (e[j] < 2) continue;
            const int32_t fac = fresh_out && a_slot != (int32_t)(k + 1) ? fresh() : (int32_t)(fbase + fpos);
            const int ready = e[j] - 1 >= 2 ? e[j] - 2 : 0;
            shift = std::max(shift, ready) + 1;
            add_job(shift, a_slot, pow_slot(v[j], e[j] - 1), fac);
            a_slot = fac;
        }
        if (a_slot != (int32_t)(k + 1)) ++fpos;
        auto A = [&](void) { return a_slot; };
        auto Z = [&](int i) { return (int32_t)(1 + N + v[i - 1]); };  // z_{i_i}, 1-based position
        auto F = [&](int j) { return (int32_t)(base + alpha + j - 1); };
        auto B = [&](int j) { return (int32_t)(base + tot + beta + j - 1); };
        auto C = [&](int j) { return (int32_t)(base + tot + nb + gamma + j - 1); };
        auto job = [&](int layer, int32_t t1, int32_t t2, int32_t t3) { add_job(layer + shift, t1, t2, t3); };
        // a z^e factor's partial derivative is e times the multilinear one
        auto scale = [&](int j0, int32_t src, int32_t dst) {
            if (e && e[j0] >= 2) P.scale.push_back({src, dst, e[j0]});
        };
        if (nk == 1) {
            job(1, A(), Z(1), F(1));
            if (e && e[0] >= 2)
                scale(0, A(), B(1));
            else
                P.stage.push_back({B(1), (int32_t)(k + 1)});
            value_list.push_back(F(1));
            grad_lists[v[0]].push_back(B(1));
            mono_slot[k] = Z(1);
        } else {
            job(1, A(), Z(1), F(1));
            for (int j = 2; j <= nk; ++j) job(j, F(j - 1), Z(j), F(j));
            if (nk == 2) {
                job(1, Z(2), A(), B(1));
                grad_lists[v[0]].push_back(B(1));
                grad_lists[v[1]].push_back(F(1));
                scale(0, B(1), B(1));
                scale(1, F(1), F(1));
                if (keep) {
                    mono_slot[k] = (int32_t)(mbase + mpos++);
                    job(1, Z(2), Z(1), mono_slot[k]);  // M_k = z_{i_2} * z_{i_1}
                }
            } else {
                job(1, Z(nk), Z(nk - 1), B(1));
                for (int j = 2; j <= nk - 2; ++j) job(j, B(j - 1), Z(nk - j), B(j));
                // b_{n-2} := b_{n-2} * a_k, in place unless operands are streamed
                // or a job spans several wavefronts
                const int32_t bfin = fresh_out ? fresh() : B(nk - 2);
                if (keep) {
                    // M_k = b_{n-2} * z_{i_1} reads the backward product before its
                    // multiplication by a_k, which therefore moves one layer later
                    mono_slot[k] = (int32_t)(mbase + mpos++);
                    job(nk - 1, B(nk - 2), Z(1), mono_slot[k]);
                    job(nk, B(nk - 2), A(), bfin);
                } else {
                    job(nk - 1, B(nk - 2), A(), bfin);
                }
                for (int j = 1; j <= nk - 3; ++j) job(std::max(j, nk - 2 - j) + 1, F(j), B(nk - 2 - j), C(j));
                job(nk - 1, F(nk - 2), Z(nk), C(nk - 2));
                grad_lists[v[0]].push_back(bfin);
                for (int j = 1; j <= nk - 2; ++j) grad_lists[v[j]].push_back(C(j));
                grad_lists[v[nk - 1]].push_back(F(nk - 1));
                scale(0, bfin, bfin);
                for (int j = 1; j <= nk - 2; ++j) scale(j, C(j), C(j));
                scale(nk - 1, F(nk - 1), F(nk - 1));
            }
            value_list.push_back(F(nk));
        }
        alpha += nk;
        beta += std::max(1, nk - 2);
        gamma += std::max(0, nk - 2);
        pos += nk;
    }

    P.conv_off.push_back(0);
    if (N > 0)
        for (auto &L : layers) {
            P.conv.insert(P.conv.end(), L.begin(), L.end());
            P.conv_off.push_back((int64_t)P.conv.size());
        }

    std::vector<std::vector<std::array<int32_t, 2>>> rounds;
    P.out_slots.push_back(tree_rounds(value_list, rounds));
    for (int i = 0; i < n; ++i) P.out_slots.push_back(tree_rounds(grad_lists[i], rounds));
    P.add_off.push_back(0);
    for (auto &r : rounds) {
        P.add.insert(P.add.end(), r.begin(), r.end());
        P.add_off.push_back((int64_t)P.add.size());
    }

    if (keep) {
        // reverse pass: abar_k = corr(ybar, M_k), zbar_i = corr(ybar, dp/dz_i)
        int64_t q = mbase + nmono2;
        P.ybar_slot = (int32_t)q++;
        P.coeff_bar_slots.push_back(P.ybar_slot);
        for (int k = 0; k < N; ++k) {
            int32_t out = (int32_t)q++;
            P.corr.push_back({P.ybar_slot, mono_slot[k], out});
            P.coeff_bar_slots.push_back(out);
        }
        for (int i = 0; i < n; ++i) {
            int32_t out = (int32_t)q++;
            int32_t g = P.out_slots[1 + i];
            if (g >= 0) P.corr.push_back({P.ybar_slot, g, out});
            P.z_bar_slots.push_back(g >= 0 ? out : -1);
        }
    }

    if (xpos != nser - xbase) return "internal planner error: fresh slot count";
    if (streamed) {
        bool paired = false;
        const int Q = stream_waves_per_job(d, &paired);
        if (paired)
            P.lanes = make_paired_schedule(d, Q);
        else
            P.lanes = make_lane_schedule(d, Q > 1 ? 1 : std::max(1, std::min(kLanes, (2 * kLanes + d + 1) / (d + 2))), Q);
    } else {
        choose_staged_lanes(P, 1);
        // A job over several wavefronts may not write its own first operand
        // (see no_inplace above): rebuild with fresh output slots for the
        // in-place jobs.  The jobs and layers are the same, so is the choice.
        if (P.lanes.waves_per_job > 1 && !no_inplace) {
            bool inplace = false;
            for (const auto &t : P.conv) inplace |= t[0] == t[2];
            if (inplace) return build_plan_mode(n, N, d, m, nvars, vars, exps, flags, false, true, P, unsupported);
        }
    }
    // after the lane choice: the check depends on the wavefronts per job
    auto err = check_hazards(P);
    if (!err.empty()) return "internal planner error: " + err;
    if (!(flags & kAsapLayers)) {
        const int J = P.lanes.jobs_per_group, Q = P.lanes.waves_per_job;
        const double before = layer_cost(P, Q, J, P.lanes.steps, 1.0);
        auto conv = P.conv;
        auto off = P.conv_off;
        if (balance_layers(P, std::max(1L, kSimds * J / Q))) {
            if (layer_cost(P, Q, J, P.lanes.steps, 1.0) < before) {
                P.balanced = true;
                auto e = check_hazards(P);
                if (!e.empty()) return "internal planner error after layer balancing: " + e;
            } else {
                P.conv.swap(conv);
                P.conv_off.swap(off);
            }
        }
    }
    return "";
}

}  // namespace mdpe
