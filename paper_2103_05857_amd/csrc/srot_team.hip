// Block-step chain (Alg. 1) for rows wider than 4096 columns, spread over a
// team of workgroups: stored FP32 / FP64 cost or the fused squared-Euclidean
// cost, up to 65536 columns.
//
// The steps stay strictly sequential and exact; what is split is the row.
// Member w of a team of W = ceil(n / 1024) workgroups owns the columns
// [1024 w, 1024 w + 1024); its thread tid owns the four adjacent columns
// 1024 w + 4 tid + e, e < 4, and keeps their residual entries r_j (and, for
// the fused cost, their target points) in registers for the whole launch.
// A step on row i (eq. RelaxedGradient, eq. SemiRelaxedSubproblemImplement,
// eq. SemiRelaxedBCFWStep):
//   1. every thread forms v_j = c_ij + w r_j on its columns; each wave finds
//      its lowest-index minimum and, relative to it, its line-search partials
//      over the row's support (P = sum t (v - min), Q = sum of t^2 off the
//      argmin, the entry at the argmin, sum t); the member merges its four
//      waves through LDS;
//   2. wave 1 publishes that record to the team while a fifth wave, the
//      exchange wave, reads every member's record of the step: tagged 64-bit
//      words written and read with device-scope atomics, so no cache
//      maintenance is needed and a word is taken only once it carries this
//      step's tag; every member merges the W records in the same order and
//      obtains the same G, j*, num, den and step size, bit for bit.  The
//      exchange wave issues no other memory operation, so its spinning
//      never waits on the column waves' prefetches or stores;
//   3. every thread updates its own columns: t_ij, r_j, the plan entries
//      (plain stores: each entry has one owner) and the support-mask bits of
//      the handle's ownership layout (device-scope atomic or / and, since
//      several members share a mask word).
// Row data (the thread's four plan entries, cost entries or the source
// point, a_i) is requested TEAM_DA steps ahead.  The entries of a row that a
// later step of the window updates are patched in registers; a request
// issued after the update follows the owner thread's own stores in program
// order and so reads the new values.
//
// Records are double-buffered by step parity: a member writes the record of
// step s + 2 only after its exchange wave has read every member's record of
// step s + 1, which each member publishes only after reading step s.  Every wait is
// bounded: after TEAM_SPIN_LIMIT polls, or once another member has given up,
// a member raises the team error flag and stops (the plan is then left
// inconsistent and the caller reports the failure; the flag stays set).
// ---------------------------------------------------------------------------
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <type_traits>

#include "../../include/srot.h"
#include "srot_internal.h"
#include "srot_device.h"

namespace srot {

namespace {

constexpr int TEAM_NT = 256;             // column threads of a member
constexpr int TEAM_NW = TEAM_NT / 64;     // column waves
constexpr int TEAM_BLOCK = TEAM_NT + 64;  // plus the exchange wave
constexpr int TEAM_CPT = 4;
constexpr int TEAM_DA = 4;
constexpr int TEAM_SPIN_LIMIT = 1 << 22;
constexpr int TEAM_POLL_SLEEP = 4;  // s_sleep units (64 cycles) between the exchange wave's samples

struct Part {
    double v, P, Q, tj, Ts;
    int j;
};

// Merge of two members' (or waves') parts: the lower (v, j) wins; moving the
// reference minimum down to the winner's adds (v_loser - v) * Ts_loser to
// P, and the loser's entry at its own argmin joins Q.  Symmetric in its
// arguments, so every lane of a butterfly ends with the same bits.
__device__ __forceinline__ Part part_merge(const Part &A, const Part &B)
{
    const bool bw = (B.v < A.v) || (B.v == A.v && B.j < A.j);
    const Part &W = bw ? B : A;
    const Part &L = bw ? A : B;
    Part o;
    o.v = W.v; o.j = W.j; o.tj = W.tj;
    o.Q = (A.Q + B.Q) + L.tj * L.tj;
    const double pa = (A.Ts != 0.0) ? (A.v - W.v) * A.Ts : 0.0;
    const double pb = (B.Ts != 0.0) ? (B.v - W.v) * B.Ts : 0.0;
    o.P = (A.P + B.P) + (pa + pb);
    o.Ts = A.Ts + B.Ts;
    return o;
}

template <typename CT>
struct TeamSlot {
    int i;
    double a;
    double t[TEAM_CPT];
    CT c[TEAM_CPT];
    float x[3];
};

// A member's record of step s, in 64-bit words written with single stores:
//   w0 = tag << 48 | j << 32 | low half of v,   w1 = tag << 48 | long << 32 | high half of v,
// with tag = (s + 1) mod 2^16 (a slot of the double buffer is rewritten every
// two steps, so an older record there never carries the current tag, and
// the buffer is zeroed before each launch) and j < 65536.  When the member
// holds support entries of the row (long = 1), w2..w9 carry P, Q, tj, Ts as
// halves under a 32-bit tag (s + 1).
__device__ __forceinline__ unsigned short_tag(int64_t s) { return (unsigned)((s + 1) & 0xffff); }

__device__ __forceinline__ unsigned long long rec_word(const Part &p, int q, int64_t s, bool lng)
{
    const double d = (q < 2) ? p.v : (q < 4) ? p.P : (q < 6) ? p.Q : (q < 8) ? p.tj : p.Ts;
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    const unsigned half = (q & 1) ? (unsigned)(u >> 32) : (unsigned)u;
    if (q < 2) {
        const unsigned mid = (q == 0) ? ((unsigned)p.j & 0xffffu) : (lng ? 1u : 0u);
        return ((unsigned long long)short_tag(s) << 48) | ((unsigned long long)mid << 32) | half;
    }
    return ((unsigned long long)(unsigned)(s + 1) << 32) | half;
}

__device__ __forceinline__ double join_f64(unsigned long long lo, unsigned long long hi)
{
    return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}

// Lowest-index minimum over the lanes, when the column indices grow with
// the lane (so the first lane holding the minimum holds the lowest one).
__device__ __forceinline__ void lane_ordered_argmin(double &v, int &j)
{
    const double mn = wave_min(v);
    const unsigned long long hit = __ballot(v == mn);
    const int l = __ffsll((long long)hit) - 1;
    j = __builtin_amdgcn_readlane(j, l);
    v = mn;
}

// The exchange of step s (wave TEAM_NW, the exchange wave): after the
// member's waves have left their parts in LDS (barrier 1), wait for every
// member's record of the step, merge them, and leave the step size and the
// vertex in LDS for barrier 2 (vertex -1: the exchange failed).  This wave
// issues no other memory operation, so its waits cover only its own polls.
template <bool TRACE>
__device__ __forceinline__ void team_exchange(const unsigned long long *__restrict__ buf, int nwg, int64_t s,
                                              int rule, int64_t k, int32_t m, double w, double ai,
                                              int32_t *__restrict__ err, double *s_gamma, int *s_jstar,
                                              bool write_trace, __amdgpu_buffer_rsrc_t rs_tj,
                                              __amdgpu_buffer_rsrc_t rs_tg)
{
    const int lane = threadIdx.x & 63;
    const unsigned tag16 = short_tag(s);
    const unsigned tag32 = (unsigned)(s + 1);
    auto ready2 = [&](unsigned long long a, unsigned long long b) {
        return (unsigned)(a >> 48) == tag16 && (unsigned)(b >> 48) == tag16;
    };
    double v = INFINITY, P = 0.0, Q = 0.0, tj = 0.0, Ts = 0.0;
    int j = 0x7fffffff, lng = 0, bad = 0;
    if (lane < nwg) {
        const unsigned long long *src = buf + (size_t)lane * TEAM_REC_STRIDE;
        // four samples of (w0, w1) in flight, issued a quarter of a round
        // trip apart; each is checked when it returns and issued again
        unsigned long long a0, b0, a1, b1, a2, b2, a3, b3;
        auto ld = [&](int q) { return __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
        a0 = ld(0); b0 = ld(1);
        __builtin_amdgcn_s_sleep(TEAM_POLL_SLEEP);
        a1 = ld(0); b1 = ld(1);
        __builtin_amdgcn_s_sleep(TEAM_POLL_SLEEP);
        a2 = ld(0); b2 = ld(1);
        __builtin_amdgcn_s_sleep(TEAM_POLL_SLEEP);
        a3 = ld(0); b3 = ld(1);
        unsigned long long ga = 0, gb = 0;
        for (int spins = 0;; spins += 4) {
            if (ready2(a0, b0)) { ga = a0; gb = b0; break; }
            a0 = ld(0); b0 = ld(1);
            if (ready2(a1, b1)) { ga = a1; gb = b1; break; }
            a1 = ld(0); b1 = ld(1);
            if (ready2(a2, b2)) { ga = a2; gb = b2; break; }
            a2 = ld(0); b2 = ld(1);
            if (ready2(a3, b3)) { ga = a3; gb = b3; break; }
            a3 = ld(0); b3 = ld(1);
            if (spins > TEAM_SPIN_LIMIT ||
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                bad = 1;
                break;
            }
        }
        if (!bad) {
            v = join_f64(ga, gb);
            j = (int)((ga >> 32) & 0xffffu);
            lng = (int)((gb >> 32) & 1u);
        }
        if (!bad && lng) {
            // the support partials: rare, read once they carry the tag
            int spins = 0;
            for (;;) {
                unsigned long long wv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) wv[q] = ld(2 + q);
                bool ok = true;
#pragma unroll
                for (int q = 0; q < 8; ++q) ok &= (unsigned)(wv[q] >> 32) == tag32;
                if (ok) {
                    P = join_f64(wv[0], wv[1]);
                    Q = join_f64(wv[2], wv[3]);
                    tj = join_f64(wv[4], wv[5]);
                    Ts = join_f64(wv[6], wv[7]);
                    break;
                }
                if (++spins > TEAM_SPIN_LIMIT ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    bad = 1;
                    break;
                }
            }
        }
    }
    if (__any(bad)) {
        if (lane == 0) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *s_jstar = -1;
        }
        return;
    }
    // G and j*: members own increasing column ranges, so the lowest-index
    // minimum is the first member holding the minimum; then num = sum of
    // P + (v - G) Ts, the squares off j* and the entry at j*, over the
    // members that hold support entries
    const int jm = j;
    double G = v;
    int jstar = j;
    lane_ordered_argmin(G, jstar);
    double x3[3] = {0.0, 0.0, 0.0};
    if (__any(lng)) {
        x3[0] = P + ((Ts != 0.0) ? (v - G) * Ts : 0.0);
        x3[1] = Q + ((jm != jstar) ? tj * tj : 0.0);
        x3[2] = (jm == jstar) ? tj : 0.0;
        wave_sum<3>(x3);
    }
    const double gamma = step_size(rule, k, m, w, x3[0], x3[1], x3[2], ai);
    if (lane == 0) {
        *s_gamma = gamma;
        *s_jstar = jstar;
    }
    if constexpr (TRACE) {
        const bool wr = write_trace && lane == 0;
        buf_store_u32((unsigned)jstar, rs_tj, wr ? (unsigned)s * 4u : kOOB);
        buf_store_f64(gamma, rs_tg, wr ? (unsigned)s * 8u : kOOB);
    }
}

template <int COST, bool TRACE>
__global__ __launch_bounds__(TEAM_BLOCK) void chain_team_kernel(ProblemView P, double *__restrict__ T,
                                                                double *__restrict__ rg,
                                                                uint32_t *__restrict__ M, Ownership own,
                                                                const int32_t *__restrict__ idx, int64_t k0,
                                                                int64_t nsteps, int rule,
                                                                int32_t *__restrict__ trace_j,
                                                                double *__restrict__ trace_gamma,
                                                                unsigned long long *__restrict__ rec,
                                                                int32_t *__restrict__ err,
                                                                int64_t *__restrict__ stats)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F64, double, float>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    __shared__ Part s_part[2][TEAM_NW];
    __shared__ double s_ai[2];
    __shared__ double s_gamma[2];
    __shared__ int s_jstar[2];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nwg = (int)gridDim.x, w_id = (int)blockIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;

    if (wid == TEAM_NW) {
        // ---- the exchange wave: two barriers per step, like the column waves
        const __amdgpu_buffer_rsrc_t rs_tj = buf_rsrc(trace_j, (TRACE && trace_j) ? (unsigned)nsteps * 4u : 0u);
        const __amdgpu_buffer_rsrc_t rs_tg = buf_rsrc(trace_gamma, (TRACE && trace_gamma) ? (unsigned)nsteps * 8u : 0u);
        for (int64_t s = 0; s < nsteps; ++s) {
            const int par = (int)(s & 1);
            __syncthreads();
            team_exchange<TRACE>(rec + (size_t)par * TEAM_MAX_MEMBERS * TEAM_REC_STRIDE, nwg, s, rule, k0 + s, m,
                                 w, s_ai[par], err, &s_gamma[par], &s_jstar[par], w_id == 0, rs_tj, rs_tg);
            __syncthreads();
            if (s_jstar[par] < 0) break;
        }
        return;
    }

    // ---- the column waves
    const int jb = w_id * (TEAM_NT * TEAM_CPT) + tid * TEAM_CPT;  // first of this thread's columns
    const unsigned row_bytes = (unsigned)n * 8u;
    const unsigned crow_bytes = (unsigned)n * (unsigned)sizeof(CT);
    const CT *__restrict__ C = (const CT *)P.C;

    bool valid[TEAM_CPT];
    double r[TEAM_CPT];
    float y[TEAM_CPT][3];
#pragma unroll
    for (int e = 0; e < TEAM_CPT; ++e) {
        const int j = jb + e;
        valid[e] = j < n;
        r[e] = valid[e] ? rg[j] : 0.0;
        if constexpr (FUSED) {
#pragma unroll
            for (int d = 0; d < 3; ++d) y[e][d] = valid[e] ? P.Y[3 * j + d] : 0.f;
        }
    }

    TeamSlot<CT> ring[TEAM_DA];
    // row i's a_i, this thread's plan entries and cost entries (or the
    // source point); entries past column n - 1 read as zero.  (i is held in
    // a vector register, so a_i and x_i are vector loads, counted by vmcnt;
    // the buffer descriptors take its uniform copy.)
    auto issue_row = [&](TeamSlot<CT> &S, int i) {
        S.i = i;
        S.a = P.a[i];
        const int iu = __builtin_amdgcn_readfirstlane(i);
        const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + (size_t)iu * (size_t)n, row_bytes);
#pragma unroll
        for (int e = 0; e < TEAM_CPT; ++e) S.t[e] = buf_load_f64(rt, valid[e] ? (unsigned)(jb + e) * 8u : kOOB);
        if constexpr (FUSED) {
            S.x[0] = P.X[3 * i + 0]; S.x[1] = P.X[3 * i + 1]; S.x[2] = P.X[3 * i + 2];
        } else {
            const __amdgpu_buffer_rsrc_t rc = buf_rsrc(C + (size_t)iu * (size_t)n, crow_bytes);
#pragma unroll
            for (int e = 0; e < TEAM_CPT; ++e) {
                const unsigned off = valid[e] ? (unsigned)(jb + e) * (unsigned)sizeof(CT) : kOOB;
                if constexpr (sizeof(CT) == 4)
                    S.c[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)off, 0, 0));
                else
                    S.c[e] = buf_load_f64(rc, off);
            }
        }
    };

    // block indices through vector loads: those of the next group of
    // TEAM_DA steps are requested at the start of a group, so they have
    // long arrived when the group's end hands them on
    const int32_t *__restrict__ idxv = idx + in_vgpr(0);
    const int64_t last = nsteps - 1;
    int nidx[TEAM_DA];
#pragma unroll
    for (int u = 0; u < TEAM_DA; ++u) {
        issue_row(ring[u], idxv[u < last ? u : last]);
        nidx[u] = idxv[TEAM_DA + u < last ? TEAM_DA + u : last];
    }
    // nothing in flight when the loop starts: the wait counts of the loop
    // then follow its own requests only
    drain_memory();
    bool failed = false;

    for (int64_t s0 = 0; s0 < nsteps && !failed; s0 += TEAM_DA) {
        int nidx_next[TEAM_DA];
#pragma unroll
        for (int u = 0; u < TEAM_DA; ++u) {
            const int64_t sn = s0 + 2 * TEAM_DA + u;
            nidx_next[u] = idxv[sn < last ? sn : last];
        }
#pragma unroll
        for (int q = 0; q < TEAM_DA; ++q) {
            const int64_t s = s0 + q;
            if (s >= nsteps || failed) break;
            TeamSlot<CT> &S = ring[q];
            const int i = __builtin_amdgcn_readfirstlane(S.i);
            const double ai = S.a;

            // ---- 1. gradient entries, the wave's LMO candidate and partials
            double v[TEAM_CPT];
#pragma unroll
            for (int e = 0; e < TEAM_CPT; ++e) {
                double c;
                if constexpr (FUSED) c = sqdist(S.x[0], S.x[1], S.x[2], y[e][0], y[e][1], y[e][2]);
                else c = (double)S.c[e];
                const double ve = c + w * r[e];
                v[e] = valid[e] ? ve : INFINITY;
            }
            const double best = fmin(fmin(v[0], v[1]), fmin(v[2], v[3]));
            int bj = jb + 3;
#pragma unroll
            for (int e = TEAM_CPT - 2; e >= 0; --e) bj = (v[e] == best) ? jb + e : bj;
            // the thread's columns grow with the lane: the first lane holding
            // the wave minimum holds its lowest column
            Part wp;
            wp.v = best;
            wp.j = bj;
            lane_ordered_argmin(wp.v, wp.j);
            {
                double p = 0.0, q2 = 0.0, tj = 0.0, ts = 0.0;
#pragma unroll
                for (int e = 0; e < TEAM_CPT; ++e) {
                    const double t = S.t[e];
                    const bool at_j = (jb + e) == wp.j;
                    p += (t != 0.0) ? t * (v[e] - wp.v) : 0.0;
                    q2 += at_j ? 0.0 : t * t;
                    tj += at_j ? t : 0.0;
                    ts += t;
                }
                // each sum over the lanes holding support entries, in lane order
                unsigned long long act = __ballot(ts != 0.0);
                double sp = 0.0, sq = 0.0, sj = 0.0, ss = 0.0;
                while (act) {
                    const int l = __ffsll((long long)act) - 1;
                    act &= act - 1ull;
                    sp += readlane_f64(p, l);
                    sq += readlane_f64(q2, l);
                    sj += readlane_f64(tj, l);
                    ss += readlane_f64(ts, l);
                }
                wp.P = sp; wp.Q = sq; wp.tj = sj; wp.Ts = ss;
            }
            const int par = (int)(s & 1);
            if (lane == 0) {
                s_part[par][wid] = wp;
                if (wid == 0) s_ai[par] = ai;
            }
            __syncthreads();

            // ---- 2. publish the member's record (wave 1); the exchange wave
            // polls and merges meanwhile
            if (wid == 1) {
                Part t4[TEAM_NW];
#pragma unroll
                for (int k = 0; k < TEAM_NW; ++k) t4[k] = s_part[par][k];
                const Part mp = part_merge(part_merge(t4[0], t4[1]), part_merge(t4[2], t4[3]));
                unsigned long long *dst =
                    rec + (size_t)par * TEAM_MAX_MEMBERS * TEAM_REC_STRIDE + (size_t)w_id * TEAM_REC_STRIDE;
                const bool lng = mp.Ts != 0.0;
                if (lane < (lng ? 10 : 2))
                    __hip_atomic_store(dst + lane, rec_word(mp, lane, s, lng), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            const int jstar = s_jstar[par];
            if (jstar < 0) {
                failed = true;
                break;
            }
            const double gamma = s_gamma[par];

            // ---- 3. update of this thread's columns: t, r, plan, masks
            const double gadd = gamma * ai;
            const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + (size_t)i * (size_t)n, row_bytes);
            double tn[TEAM_CPT];
#pragma unroll
            for (int e = 0; e < TEAM_CPT; ++e) {
                const int j = jb + e;
                const double t = S.t[e];
                tn[e] = blend(t, gamma, (j == jstar) ? gadd : 0.0);
                const bool put = valid[e] && tn[e] != t;
                r[e] = put ? r[e] + (tn[e] - t) : r[e];
                buf_store_f64(tn[e], rt, put ? (unsigned)j * 8u : kOOB);
                if (put && ((t == 0.0) != (tn[e] == 0.0))) {
                    // the support-mask bit of column j in the handle's layout
                    const int jg = j / own.vec;
                    const int ts = jg % own.nt;
                    const int u = (jg / own.nt) * own.vec + (j % own.vec);
                    uint32_t *word = M + ((size_t)i * own.words + (u >> 5)) * own.nt + ts;
                    if (tn[e] != 0.0)
                        __hip_atomic_fetch_or(word, 1u << (u & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else
                        __hip_atomic_fetch_and(word, ~(1u << (u & 31)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // requests of later steps in the window read this row before the
            // update: patch them
#pragma unroll
            for (int q2 = 1; q2 < TEAM_DA; ++q2) {
                TeamSlot<CT> &R = ring[(q + q2) % TEAM_DA];
                if (__builtin_amdgcn_readfirstlane(R.i) == i) {
#pragma unroll
                    for (int e = 0; e < TEAM_CPT; ++e) R.t[e] = tn[e];
                }
            }
            // row of step s + TEAM_DA
            issue_row(ring[q], nidx[q]);
        }
#pragma unroll
        for (int u = 0; u < TEAM_DA; ++u) nidx[u] = nidx_next[u];
    }
    if (failed) return;
#pragma unroll
    for (int e = 0; e < TEAM_CPT; ++e)
        if (valid[e]) rg[jb + e] = r[e];
    if (w_id == 0 && tid == 0) stats[2] = SROT_CHAIN_TEAM;
}

// Zeroes the exchange records before a launch, so that tags (the step
// number within the launch, from 1) never match a record of an earlier
// launch.  A kernel rather than a memset, so that the launch sequence can
// be captured in a graph.  The team error flag is not cleared here: once
// set it stays set (later launches stop at their first wait) until the
// handle's state is rewritten (srot_set_state) or the handle is made again.
__global__ void team_clear_kernel(unsigned long long *__restrict__ rec, int words)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x) rec[k] = 0ull;
}

}  // namespace

int team_members(int64_t n) { return (int)((n + TEAM_NT * TEAM_CPT - 1) / (TEAM_NT * TEAM_CPT)); }

bool team_chain_supported(const ProblemView &P)
{
    const char *env = getenv("SROT_TEAM_CHAIN");
    if (env && strcmp(env, "0") == 0) return false;
    return P.n > 4096 && team_members(P.n) <= TEAM_MAX_MEMBERS;
}

template <int COST>
static hipError_t launch_team_cost(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                                   int64_t nsteps, int rule, int32_t *tj, double *tg, hipStream_t st)
{
    const int nwg = team_members(P.n);
    const int words = 2 * TEAM_MAX_MEMBERS * TEAM_REC_STRIDE;
    hipLaunchKernelGGL(team_clear_kernel, dim3(8), dim3(256), 0, st, S.team_rec, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tj || tg)
        hipLaunchKernelGGL((chain_team_kernel<COST, true>), dim3(nwg), dim3(TEAM_BLOCK), 0, st, P, S.T, S.r, S.mask,
                           S.own, idx, k0, nsteps, rule, tj, tg, S.team_rec, S.flags + 6, S.slow_steps);
    else
        hipLaunchKernelGGL((chain_team_kernel<COST, false>), dim3(nwg), dim3(TEAM_BLOCK), 0, st, P, S.T, S.r, S.mask,
                           S.own, idx, k0, nsteps, rule, tj, tg, S.team_rec, S.flags + 6, S.slow_steps);
    return hipGetLastError();
}

hipError_t launch_chain_team(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                             int64_t nsteps, int rule, int32_t *tj, double *tg, hipStream_t st)
{
    switch (P.cost) {
    case SROT_COST_F32: return launch_team_cost<SROT_COST_F32>(P, S, idx, k0, nsteps, rule, tj, tg, st);
    case SROT_COST_F64: return launch_team_cost<SROT_COST_F64>(P, S, idx, k0, nsteps, rule, tj, tg, st);
    default: return launch_team_cost<SROT_COST_SQEUCLID>(P, S, idx, k0, nsteps, rule, tj, tg, st);
    }
}

}  // namespace srot
