// Batched BCFW for many independent problems of uneven sizes (gfx950).
//
// Each problem is solved start to finish by one workgroup: initial plan
// (every row at its first vertex), then passes of m block steps (Alg. 1)
// with the block indices drawn on the device from the counter-based Philox
// stream, the duality-gap sweep (Thm 2) every gap_every passes and the stop
// test g <= eps -- no host round trip until every problem is done.  The
// per-problem work reuses the single-problem chain (chain_run), so a
// problem solved here follows the same trajectory as srot_solve with the
// same tile shape and seed.
//
// Each problem has a tile shape (threads x columns per thread x vector
// width): either the single-problem default for its width or, with
// srot_init_batched(tune = 1), the fastest candidate measured on the widest
// problem of its default shape.  Shapes of one workgroup size (and, at 256
// threads, one vector width) form a launch class: one launch of
// batch_solve_kernel per class, one workgroup per problem, which switches
// to the problem's shape.  The (at most four) class launches are
// independent nodes of one hipGraph, instantiated once and replayed by
// every srot_solve_batched call; four launches fit the four hardware queues
// a process gets by default, so they all run at once (launches that share
// a queue would run one after another).  Within a class the workgroups
// start in launch order: the largest problems first, and from the second
// solve on the longest-running ones of the previous solve (per-problem
// run times come from the device clock), so that the slowest problem of a
// batch starts at once instead of behind the short ones.
//
// Workspace (caller-owned): problem table, launch order, results, then per
// problem r (n), block indices (m), support masks (m x 256 words) and the
// dense FP64 plan (m x n).  The plan is never cleared: every kernel reads
// t_ij only where the support mask has its bit set.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/srot.h"
#include "srot_device.h"
#include "srot_internal.h"

namespace srot {

struct BatchProblem {
    int32_t m, n;
    int64_t c_off;    // elements of C before this problem's cost matrix
    int64_t a_off;    // entries of a before this problem's weights
    int64_t b_off;    // entries of b before this problem's weights
    int64_t T_off;    // doubles of the plan arena
    int64_t r_off;    // doubles of the residual arena
    int64_t M_off;    // words of the mask arena
    int64_t idx_off;  // entries of the index arena
    int32_t tile;     // tile id (the instantiation that solves it)
    int32_t pad;
};

struct BatchResult {
    double g, f, D;
    int64_t passes;
    int32_t status, pad;
    int64_t ticks;  // the workgroup's run time, in ticks of the constant-rate device clock
};

struct BatchParams {
    double w, eps;
    uint64_t seed;
    int64_t max_passes;
    int32_t gap_every, rule;
};

namespace {

constexpr int kMaskNT = 256;  // mask words reserved per row (the widest tile used here)

// Duality-gap sweep of one problem by one workgroup (Thm 2, eq. AppenEq:Gi,
// dual of App. D).  Wave `wid` takes rows in groups of BG_R: rows
// wid * BG_R + k, then NW * BG_R further on, ...  For a group the wave
// requests the rows' support-mask words first, then streams the cost rows
// in batches of U columns per lane (all R rows at once, each r_j read once
// for the R rows), so a batch is one round of memory latency; the support
// entries (the first BG_KS per lane and row, found from the mask words) are
// requested before the first batch is consumed.  Per row: the lowest-index
// argmin of c_ij + w r_j, then t_ij (v_ij - G_i) and t_ij c_ij summed over
// the support.  A wave adds its rows in row order, the waves are added in
// wave order; the result is the same in every thread.
constexpr int BG_R = 4;   // rows per wave and group
constexpr int BG_KS = 2;  // support entries per lane and row gathered ahead

template <int NT, int CPT, int VEC>
__device__ void batch_gap(const ProblemView &P, const double *__restrict__ T,
                          const double *__restrict__ rg, const uint32_t *__restrict__ M,
                          double &g_out, double &f_out, double &D_out)
{
    constexpr int NW = NT / 64;
    constexpr int WPL = NT / 64;  // mask words per lane and row
    // vectors of VEC columns per lane and batch: up to 16 columns
    constexpr int PER_LANE = (NT * CPT) / (64 * VEC);
    constexpr int U = PER_LANE < 16 / VEC ? (PER_LANE > 0 ? PER_LANE : 1) : 16 / VEC;
    using CV = typename std::conditional<VEC == 4, float4, float>::type;
    __shared__ double s_w[NW][3];
    __shared__ double s_rb[NW][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = P.m, n = P.n;
    const int nv = n / VEC;  // whole vectors (VEC = 4 only with n % 4 == 0)
    const double w = P.w;
    const float *__restrict__ C = (const float *)P.C;
    double aG = 0.0, lin = 0.0, gs = 0.0;
    for (int i0 = wid * BG_R; i0 < m; i0 += NW * BG_R) {
        int ir[BG_R];
#pragma unroll
        for (int k = 0; k < BG_R; ++k) ir[k] = i0 + k < m ? i0 + k : m - 1;
        uint32_t mw[BG_R][WPL];
#pragma unroll
        for (int k = 0; k < BG_R; ++k)
#pragma unroll
            for (int q = 0; q < WPL; ++q)
                mw[k][q] = i0 + k < m ? M[(size_t)ir[k] * NT + lane + 64 * q] : 0u;
        // support entries: the lane's slots in increasing order, bits low to high
        int sj[BG_R][BG_KS];
        bool more[BG_R];
#pragma unroll
        for (int k = 0; k < BG_R; ++k) {
            int found = 0;
            more[k] = false;
#pragma unroll
            for (int e = 0; e < BG_KS; ++e) sj[k][e] = -1;
#pragma unroll
            for (int q = 0; q < WPL; ++q) {
                uint32_t mk = mw[k][q];
                while (mk) {
                    const int u = __ffs(mk) - 1;
                    mk &= mk - 1u;
                    if (found < BG_KS) {
#pragma unroll
                        for (int e = 0; e < BG_KS; ++e)
                            sj[k][e] = e == found ? owned_col<NT, VEC>(u, lane + 64 * q) : sj[k][e];
                        ++found;
                    } else {
                        more[k] = true;
                    }
                }
            }
        }
        double st[BG_R][BG_KS], sc[BG_R][BG_KS], sr[BG_R][BG_KS];
#pragma unroll
        for (int k = 0; k < BG_R; ++k)
#pragma unroll
            for (int e = 0; e < BG_KS; ++e) {
                const int j = sj[k][e] >= 0 ? sj[k][e] : 0;
                st[k][e] = T[(size_t)ir[k] * (size_t)n + j];
                sc[k][e] = (double)C[(size_t)ir[k] * (size_t)n + j];
                sr[k][e] = rg[j];
            }
        double best[BG_R];
        int bj[BG_R];
#pragma unroll
        for (int k = 0; k < BG_R; ++k) { best[k] = INFINITY; bj[k] = 0x7fffffff; }
        for (int q0 = 0; q0 < nv; q0 += 64 * U) {
            CV cv[BG_R][U];
            double rv[U][VEC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * 64 + lane;
                const int qc = q < nv ? q : nv - 1;  // clamped: read, then masked
#pragma unroll
                for (int k = 0; k < BG_R; ++k)
                    cv[k][u] = reinterpret_cast<const CV *>(C + (size_t)ir[k] * (size_t)n)[qc];
                if constexpr (VEC == 4) {
                    const double2 r0 = reinterpret_cast<const double2 *>(rg)[2 * qc];
                    const double2 r1 = reinterpret_cast<const double2 *>(rg)[2 * qc + 1];
                    rv[u][0] = r0.x; rv[u][1] = r0.y; rv[u][2] = r1.x; rv[u][3] = r1.y;
                } else {
                    rv[u][0] = rg[qc];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * 64 + lane;
#pragma unroll
                for (int k = 0; k < BG_R; ++k) {
                    float c[VEC];
                    if constexpr (VEC == 4) {
                        c[0] = cv[k][u].x; c[1] = cv[k][u].y; c[2] = cv[k][u].z; c[3] = cv[k][u].w;
                    } else {
                        c[0] = cv[k][u];
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const double v = q < nv ? (double)c[e] + w * rv[u][e] : INFINITY;
                        if (v < best[k]) { best[k] = v; bj[k] = q * VEC + e; }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < BG_R; ++k) {
            if (i0 + k >= m) break;  // uniform over the wave
            const int i = i0 + k;
            double G = best[k];
            int J = bj[k];
            wave_argmin(G, J);
            double x[2] = {0.0, 0.0};
#pragma unroll
            for (int e = 0; e < BG_KS; ++e) {
                if (sj[k][e] >= 0) {
                    x[0] += st[k][e] * (sc[k][e] + w * sr[k][e] - G);
                    x[1] += st[k][e] * sc[k][e];
                }
            }
            if (__any(more[k])) {
                // the lane's support entries after its first BG_KS, same order
                int seen = 0;
#pragma unroll
                for (int q = 0; q < WPL; ++q) {
                    uint32_t mk = mw[k][q];
                    while (mk) {
                        const int u = __ffs(mk) - 1;
                        mk &= mk - 1u;
                        if (seen++ < BG_KS) continue;
                        const int j = owned_col<NT, VEC>(u, lane + 64 * q);
                        const double t = T[(size_t)i * (size_t)n + j];
                        const double c = (double)C[(size_t)i * (size_t)n + j];
                        x[0] += t * (c + w * rg[j] - G);
                        x[1] += t * c;
                    }
                }
            }
            wave_sum<2>(x);
            aG += P.a[i] * G;
            lin += x[1];
            gs += x[0];
        }
    }
    if (lane == 0) { s_w[wid][0] = aG; s_w[wid][1] = lin; s_w[wid][2] = gs; }
    double rb[2] = {0.0, 0.0};
#pragma unroll 4
    for (int j = threadIdx.x; j < n; j += NT) {
        rb[0] += rg[j] * rg[j];
        rb[1] += P.b[j] * rg[j];
    }
    block_sum<NW, 2>(rb, s_rb);  // its barrier also publishes s_w
    if (NW == 1) __syncthreads();
    double tot[3] = {s_w[0][0], s_w[0][1], s_w[0][2]};
#pragma unroll
    for (int k = 1; k < NW; ++k) {
        tot[0] += s_w[k][0]; tot[1] += s_w[k][1]; tot[2] += s_w[k][2];
    }
    g_out = tot[2];
    f_out = tot[1] + 0.5 * w * rb[0];
    D_out = tot[0] - w * rb[1] - 0.5 * w * rb[0];
    __syncthreads();  // s_w and s_rb are rewritten by the next sweep
}

// One problem from its initial plan to the stop test, by the workgroup.
template <int NT, int CPT, int VEC>
__device__ __forceinline__ void batch_solve_one(const float *__restrict__ C, const double *__restrict__ a,
                                                const double *__restrict__ b, double *__restrict__ Tar,
                                                double *__restrict__ rar, uint32_t *__restrict__ Mar,
                                                int32_t *__restrict__ idxar, const BatchProblem &bp, int32_t p,
                                                const BatchParams &prm, BatchResult *__restrict__ res)
{
    constexpr int COST = SROT_COST_F32;
    const int tid = threadIdx.x;
    const uint64_t t_start = wall_clock64();
    ProblemView P;
    P.m = bp.m; P.n = bp.n; P.cost = COST;
    P.C = C + bp.c_off;
    P.X = nullptr; P.Y = nullptr; P.Y4 = nullptr;
    P.a = a + bp.a_off;
    P.b = b + bp.b_off;
    P.w = prm.w;
    const int m = bp.m, n = bp.n;
    double *__restrict__ T = Tar + bp.T_off;
    double *__restrict__ rg = rar + bp.r_off;
    uint32_t *__restrict__ M = Mar + bp.M_off;
    int32_t *__restrict__ idx = idxar + bp.idx_off;

    // initial plan t_i = a_i e_0: column 0 is owned by thread 0 (bit 0)
    for (int i = tid; i < m; i += NT) T[(size_t)i * (size_t)n] = P.a[i];
    for (int i = 0; i < m; ++i) M[(size_t)i * NT + tid] = (tid == 0) ? 1u : 0u;
    // r = T^T 1 - b, each column summed in row order
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        if (j >= n) continue;
        double s = 0.0;
        if (j == 0)
            for (int i = 0; i < m; ++i) s += P.a[i];
        rg[j] = s - P.b[j];
    }

    double g = INFINITY, f = NAN, D = NAN;
    int64_t passes = 0, k = 0;
    int32_t status = SROT_NOT_CONVERGED;
    for (int64_t pass = 0; pass < prm.max_passes; ++pass) {
        __syncthreads();  // every read of the previous pass's indices (and of T) is done
        for (int s = tid; s < m; s += NT)
            idx[s] = (int32_t)__umul64hi(philox_output(prm.seed, (uint64_t)(k + s)), (uint64_t)m);
        __syncthreads();
        chain_run<NT, CPT, VEC, COST, false>(P, T, rg, M, idx, k, m, prm.rule, nullptr, nullptr);
        k += m;
        passes = pass + 1;
        if (passes % prm.gap_every == 0 || passes == prm.max_passes) {
            __syncthreads();  // the sweep reads every thread's columns of r, T and the masks
            batch_gap<NT, CPT, VEC>(P, T, rg, M, g, f, D);
            if (g <= prm.eps) { status = SROT_OK; break; }
        }
    }
    if (tid == 0) {
        BatchResult out;
        out.g = g; out.f = f; out.D = D; out.passes = passes; out.status = status; out.pad = 0;
        out.ticks = (int64_t)(wall_clock64() - t_start);
        res[p] = out;
    }
}

// Dense copy of one problem's plan: zeros off the support.
__global__ void batch_plan_kernel(const double *__restrict__ T, const uint32_t *__restrict__ M,
                                  int32_t m, int32_t n, Ownership own, double *__restrict__ out)
{
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        for (int ts = threadIdx.x; ts < own.nt; ts += blockDim.x) {
            const uint32_t word = M[(size_t)i * own.nt + ts];
            for (int u = 0; u < own.cpt; ++u) {
                const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                if (j < n) out[(size_t)i * n + j] = ((word >> u) & 1u) ? T[(size_t)i * n + j] : 0.0;
            }
        }
    }
}

// Flags NaN/Inf in a problem's cost or weights and negative weights.
__global__ void batch_validate_kernel(const float *__restrict__ C, const double *__restrict__ a,
                                      const double *__restrict__ b,
                                      const BatchProblem *__restrict__ probs,
                                      int32_t *__restrict__ flag)
{
    const BatchProblem bp = probs[blockIdx.y];
    const size_t mn = (size_t)bp.m * (size_t)bp.n;
    bool bad = false;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < mn; e += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(C[bp.c_off + e]);
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < bp.m; i += blockDim.x) bad |= !(a[bp.a_off + i] >= 0.0) || !isfinite(a[bp.a_off + i]);
        for (int j = threadIdx.x; j < bp.n; j += blockDim.x) bad |= !(b[bp.b_off + j] >= 0.0) || !isfinite(b[bp.b_off + j]);
    }
    if (bad) atomicOr(flag, 1);
}

struct Tile {
    int nt, cpt, vec;
    bool operator==(const Tile &o) const { return nt == o.nt && cpt == o.cpt && vec == o.vec; }
};

// Tile shapes compiled for the batched kernel (one mask word per thread),
// numbered in this order.
#define SROT_BATCH_TILES(X) \
    X(0, 64, 2, 1) X(1, 64, 4, 1) X(2, 128, 4, 1) X(3, 256, 4, 1) X(4, 256, 8, 1) X(5, 256, 16, 1) \
    X(6, 64, 4, 4) X(7, 128, 4, 4) X(8, 256, 4, 4) X(9, 256, 8, 4) X(10, 256, 16, 4)

int tile_id(const Tile &t)
{
#define SROT_TID(ID_, NT_, CPT_, VEC_) \
    if (t.nt == NT_ && t.cpt == CPT_ && t.vec == VEC_) return ID_;
    SROT_BATCH_TILES(SROT_TID)
#undef SROT_TID
    return -1;
}

// Launch classes: the tiles of one class share a kernel (and its
// workgroup size), which picks the problem's tile at run time.  Four
// classes keep the whole batch within four concurrent launches.
constexpr int kClasses = 4;
int tile_class(const Tile &t) { return t.nt == 64 ? 0 : t.nt == 128 ? 1 : t.vec == 1 ? 2 : 3; }
constexpr int class_nt(int c) { return c == 0 ? 64 : c == 1 ? 128 : 256; }

// A workgroup per problem: order[blockIdx.x] names it, its tile id (one of
// the class's) selects the instantiation.
template <int NT, int V4>
__global__ __launch_bounds__(NT) void batch_solve_kernel(const float *__restrict__ C,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         double *__restrict__ Tar,
                                                         double *__restrict__ rar,
                                                         uint32_t *__restrict__ Mar,
                                                         int32_t *__restrict__ idxar,
                                                         const BatchProblem *__restrict__ probs,
                                                         const int32_t *__restrict__ order,
                                                         BatchParams prm,
                                                         BatchResult *__restrict__ res)
{
    const int32_t p = order[blockIdx.x];
    const BatchProblem bp = probs[p];
    bool solved = false;
    switch (bp.tile) {
#define SROT_BCASE(ID_, NT_, CPT_, VEC_)                                                      \
    case ID_:                                                                                \
        if constexpr (NT_ == NT && (NT != 256 || (VEC_ == 4) == (V4 != 0))) {                \
            batch_solve_one<NT_, CPT_, VEC_>(C, a, b, Tar, rar, Mar, idxar, bp, p, prm, res); \
            solved = true;                                                                   \
        }                                                                                    \
        break;
        SROT_BATCH_TILES(SROT_BCASE)
#undef SROT_BCASE
    default:
        break;
    }
    if (!solved && threadIdx.x == 0) {
        // a tile outside this launch's class (not produced by the host):
        // reported, never left as an earlier solve's result
        BatchResult out;
        out.g = NAN; out.f = NAN; out.D = NAN; out.passes = 0; out.status = SROT_EINVAL; out.pad = 0;
        out.ticks = 0;
        res[p] = out;
    }
}

const void *class_kernel(int c)
{
    switch (c) {
    case 0: return (const void *)&batch_solve_kernel<64, 0>;
    case 1: return (const void *)&batch_solve_kernel<128, 0>;
    case 2: return (const void *)&batch_solve_kernel<256, 0>;
    default: return (const void *)&batch_solve_kernel<256, 1>;
    }
}

std::vector<Tile> tile_candidates(int64_t n, bool vec4)
{
    std::vector<Tile> out;
#define SROT_BC(ID_, NT_, CPT_, VEC_) \
    if ((int64_t)NT_ * CPT_ >= n && (VEC_ == 1 || vec4)) out.push_back(Tile{NT_, CPT_, VEC_});
    SROT_BATCH_TILES(SROT_BC)
#undef SROT_BC
    return out;
}

}  // namespace
}  // namespace srot

using srot::BatchParams;
using srot::BatchProblem;
using srot::BatchResult;
using srot::Tile;
using srot::fail;

struct srot_batch {
    int32_t count;
    srot_options opt;
    hipStream_t stream;
    const float *C;
    const double *a, *b;
    BatchProblem *d_probs;
    int32_t *d_order;
    BatchResult *d_res;
    double *T, *r;
    uint32_t *M;
    int32_t *idx;
    std::vector<BatchProblem> probs;
    std::vector<Tile> tile;                 // per problem
    std::vector<std::pair<Tile, std::pair<int, int>>> groups;  // tile, (first, count) in the order array
    std::vector<float> tune_ms;             // per group: measured ms per block step (0 = not tuned)
    std::vector<int32_t> order;             // launch order: the classes' segments back to back
    int cls_first[srot::kClasses] = {}, cls_count[srot::kClasses] = {};
    int tune_cached = 0;                    // groups whose tile came from the tuning cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

#define SROT_HIP_B(call)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(SROT_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    size_t probs, order, res, r, idx, M, T, total;
    std::vector<int64_t> r_off, idx_off, M_off, T_off;
};

BatchLayout batch_layout(int32_t count, const int64_t *m, const int64_t *n)
{
    BatchLayout L;
    size_t off = 0;
    L.probs = off; off = al(off + sizeof(BatchProblem) * (size_t)count);
    L.order = off; off = al(off + sizeof(int32_t) * (size_t)count);
    L.res = off; off = al(off + sizeof(BatchResult) * (size_t)count);
    int64_t nr = 0, ni = 0, nm = 0, nT = 0;
    for (int32_t p = 0; p < count; ++p) {
        L.r_off.push_back(nr); nr += (n[p] + 3) & ~int64_t(3);          // 32-byte aligned
        L.idx_off.push_back(ni); ni += (m[p] + 3) & ~int64_t(3);
        L.M_off.push_back(nm); nm += m[p] * srot::kMaskNT;
        L.T_off.push_back(nT); nT += (m[p] * n[p] + 31) & ~int64_t(31);  // 256-byte aligned
    }
    L.r = off; off = al(off + sizeof(double) * (size_t)nr);
    L.idx = off; off = al(off + sizeof(int32_t) * (size_t)ni);
    L.M = off; off = al(off + sizeof(uint32_t) * (size_t)nm);
    L.T = off; off = al(off + sizeof(double) * (size_t)nT);
    L.total = off;
    return L;
}

bool batch_sizes_ok(int32_t count, const int64_t *m, const int64_t *n)
{
    if (count < 1 || !m || !n) return false;
    for (int32_t p = 0; p < count; ++p)
        if (m[p] < 1 || n[p] < 1 || m[p] > 0x7fffffff || n[p] > 4096) return false;
    return true;
}

BatchParams params_of(const srot_options &o)
{
    BatchParams prm;
    prm.w = o.w; prm.eps = o.eps; prm.seed = o.seed; prm.max_passes = o.max_passes;
    prm.gap_every = o.gap_every; prm.rule = o.step_rule;
    return prm;
}

hipError_t launch_class(srot_batch *h, int cls, int first, int cnt, const BatchParams &prm, hipStream_t st)
{
    const void *fn = srot::class_kernel(cls);
    const float *C = h->C;
    const double *a = h->a, *b = h->b;
    double *T = h->T, *r = h->r;
    uint32_t *M = h->M;
    int32_t *idx = h->idx;
    const BatchProblem *probs = h->d_probs;
    const int32_t *order = h->d_order + first;
    BatchParams pr = prm;
    BatchResult *res = h->d_res;
    void *args[] = {&C, &a, &b, &T, &r, &M, &idx, &probs, &order, &pr, &res};
    return hipLaunchKernel(fn, dim3(cnt), dim3(srot::class_nt(cls)), args, 0, st);
}

// Tuning cache: the tile chosen for a group, keyed by the group's default
// tile, its widest row and whether its rows allow 16-byte loads (the
// candidates depend on these alone), with the measured time per block step.
// Kept for the process, and in a file of JSON lines when SROT_TUNE_CACHE
// names one: read at the first tuned init, a line appended per new entry.
struct TuneEntry {
    Tile tile;
    float ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Tile &dflt, int64_t nmax, bool vec4)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "gfx950/%dx%dx%d/n%lld/v%d", dflt.nt, dflt.cpt, dflt.vec, (long long)nmax,
             vec4 ? 1 : 0);
    return buf;
}

void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("SROT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        char key[256];
        int nt = 0, cpt = 0, vec = 0;
        float ms = 0.0f;
        if (sscanf(line, "{\"key\": \"%255[^\"]\", \"nt\": %d, \"cpt\": %d, \"vec\": %d, \"ms\": %f}", key, &nt,
                   &cpt, &vec, &ms) == 5) {
            const Tile t{nt, cpt, vec};
            if (srot::tile_id(t) >= 0) g_tune[key] = TuneEntry{t, ms};
        }
    }
    fclose(f);
}

void tune_cache_store(const std::string &key, const TuneEntry &e)
{
    g_tune[key] = e;
    const char *path = getenv("SROT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"nt\": %d, \"cpt\": %d, \"vec\": %d, \"ms\": %.6g}\n", key.c_str(), e.tile.nt,
            e.tile.cpt, e.tile.vec, e.ms);
    fclose(f);
}

// Milliseconds per block step of one tile on the problem at position `pos`
// of the launch order: one pass and a gap sweep from the initial plan,
// timed on the second of two runs.
int time_tile(srot_batch *h, int pos, int32_t p, const Tile &t, float *ms_per_step)
{
    BatchParams prm = params_of(h->opt);
    prm.max_passes = 1;
    prm.gap_every = 1;
    prm.eps = -1.0;
    h->probs[p].tile = srot::tile_id(t);
    SROT_HIP_B(hipMemcpyAsync(h->d_probs + p, &h->probs[p], sizeof(BatchProblem), hipMemcpyHostToDevice,
                              h->stream));
    hipEvent_t e0, e1;
    SROT_HIP_B(hipEventCreate(&e0));
    SROT_HIP_B(hipEventCreate(&e1));
    float best = 0.0f;
    int rc = SROT_OK;
    for (int rep = 0; rep < 2 && rc == SROT_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess) e = launch_class(h, srot::tile_class(t), pos, 1, prm, h->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = fail(SROT_EHIP, "autotune: %s", hipGetErrorString(e));
        best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_step = best / (float)h->probs[p].m;
    return rc;
}

}  // namespace

extern "C" {

size_t srot_workspace_size_batched(int32_t count, const int64_t *m, const int64_t *n,
                                   const srot_options *opt)
{
    (void)opt;
    if (!batch_sizes_ok(count, m, n)) return 0;
    return batch_layout(count, m, n).total;
}

int srot_init_batched(srot_batch **out, int32_t count, const int64_t *m, const int64_t *n,
                      const int64_t *c_off, const float *C, const double *a, const double *b,
                      void *workspace, size_t ws_bytes, const srot_options *opt, int32_t tune,
                      void *stream)
{
    if (!out) return fail(SROT_EINVAL, "srot_init_batched: out is NULL");
    *out = nullptr;
    if (!batch_sizes_ok(count, m, n))
        return fail(SROT_EINVAL, "srot_init_batched: need count >= 1 and 1 <= m, 1 <= n <= 4096 per problem");
    if (!opt || !(opt->w >= 0.0) || !isfinite(opt->w) || !(opt->eps >= 0.0) ||
        opt->max_passes < 0 || opt->gap_every < 1 ||
        (opt->step_rule != SROT_ELS && opt->step_rule != SROT_DEC))
        return fail(SROT_EINVAL, "srot_init_batched: invalid options");
    if (opt->cost != SROT_COST_F32 || opt->sampling != SROT_UNIFORM)
        return fail(SROT_EINVAL, "srot_init_batched: supports SROT_COST_F32 with SROT_UNIFORM sampling");
    if (!C || !a || !b || !workspace) return fail(SROT_EINVAL, "srot_init_batched: NULL pointer");
    if (((uintptr_t)workspace) % 256 != 0)
        return fail(SROT_EINVAL, "srot_init_batched: workspace must be 256-byte aligned");
    const BatchLayout L = batch_layout(count, m, n);
    if (ws_bytes < L.total)
        return fail(SROT_ENOMEM, "srot_init_batched: workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    srot_batch *h = new srot_batch();
    h->count = count;
    h->opt = *opt;
    h->stream = (hipStream_t)stream;
    h->C = C; h->a = a; h->b = b;
    char *base = (char *)workspace;
    h->d_probs = (BatchProblem *)(base + L.probs);
    h->d_order = (int32_t *)(base + L.order);
    h->d_res = (BatchResult *)(base + L.res);
    h->r = (double *)(base + L.r);
    h->idx = (int32_t *)(base + L.idx);
    h->M = (uint32_t *)(base + L.M);
    h->T = (double *)(base + L.T);
    int64_t ca = 0, cb = 0, cc = 0;
    for (int32_t p = 0; p < count; ++p) {
        BatchProblem bp;
        bp.m = (int32_t)m[p]; bp.n = (int32_t)n[p];
        bp.c_off = c_off ? c_off[p] : cc;
        bp.a_off = ca; bp.b_off = cb;
        bp.T_off = L.T_off[p]; bp.r_off = L.r_off[p]; bp.M_off = L.M_off[p]; bp.idx_off = L.idx_off[p];
        if (bp.c_off < 0) { delete h; return fail(SROT_EINVAL, "srot_init_batched: negative c_off"); }
        cc += m[p] * n[p];
        ca += m[p]; cb += n[p];
        const bool vec4 = (n[p] % 4 == 0) && (bp.c_off % 4 == 0) && (((uintptr_t)C) % 16 == 0);
        const srot::Ownership o = srot::choose_ownership(n[p], SROT_COST_F32, vec4);
        Tile t{o.nt, o.cpt, o.vec};
        if (srot::tile_id(t) < 0) t = Tile{256, 16, 1};  // any n <= 4096 fits
        bp.tile = srot::tile_id(t);
        bp.pad = 0;
        h->probs.push_back(bp);
        h->tile.push_back(t);
    }
    // problems of one default tile form a group; in it the largest go first
    std::vector<int32_t> ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    auto key = [&](int32_t p) { const Tile &t = h->tile[p]; return (t.nt * 64 + t.cpt) * 8 + t.vec; };
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
        if (key(x) != key(y)) return key(x) < key(y);
        return (int64_t)h->probs[x].m * h->probs[x].n > (int64_t)h->probs[y].m * h->probs[y].n;
    });
    for (int q = 0; q < count;) {
        int e = q;
        while (e < count && key(ord[e]) == key(ord[q])) ++e;
        h->groups.push_back({h->tile[ord[q]], {q, e - q}});
        q = e;
    }
    int rc = SROT_OK;
    int32_t flag = 0;
    hipError_t e = hipMemcpyAsync(h->d_probs, h->probs.data(), sizeof(BatchProblem) * count,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->d_order, ord.data(), sizeof(int32_t) * count,
                                            hipMemcpyHostToDevice, h->stream);
    int32_t *d_flag = (int32_t *)h->d_res;  // results are written by every solve; borrow one word
    if (e == hipSuccess) e = hipMemsetAsync(d_flag, 0, sizeof(int32_t), h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(srot::batch_validate_kernel, dim3(64, count), dim3(256), 0, h->stream, C, a, b,
                           (const BatchProblem *)h->d_probs, d_flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = fail(SROT_EHIP, "srot_init_batched: %s", hipGetErrorString(e));
    else if (flag & 1) rc = fail(SROT_ENONFINITE, "srot_init_batched: NaN/Inf in C, a or b, or a negative weight");

    // autotuner: per group, time every candidate tile on the group's widest
    // problem with the fewest rows (the time per block step follows the row
    // width; a pass is m steps), unless the tuning cache holds the group's
    // size class
    h->tune_ms.assign(h->groups.size(), 0.0f);
    h->tune_cached = 0;
    std::unique_lock<std::mutex> lock(g_tune_mu, std::defer_lock);
    if (tune) {
        lock.lock();
        tune_cache_load();
    }
    for (size_t gi = 0; rc == SROT_OK && tune && gi < h->groups.size(); ++gi) {
        const int first = h->groups[gi].second.first, cnt = h->groups[gi].second.second;
        int pos0 = first;
        for (int q = first + 1; q < first + cnt; ++q) {
            const BatchProblem &x = h->probs[ord[q]], &y = h->probs[ord[pos0]];
            if (x.n > y.n || (x.n == y.n && x.m < y.m)) pos0 = q;
        }
        const int p0 = ord[pos0];
        int64_t nmax = 0;
        bool vec4 = h->groups[gi].first.vec == 4;
        for (int q = first; q < first + cnt; ++q) nmax = std::max<int64_t>(nmax, h->probs[ord[q]].n);
        const std::string key = tune_key(h->groups[gi].first, nmax, vec4);
        Tile best = h->groups[gi].first;
        float best_ms = 0.0f;
        auto hit = g_tune.find(key);
        if (hit != g_tune.end()) {
            best = hit->second.tile;
            best_ms = hit->second.ms;
            h->tune_cached += 1;
        } else {
            for (const Tile &t : srot::tile_candidates(nmax, vec4)) {
                float ms = 0.0f;
                rc = time_tile(h, pos0, p0, t, &ms);
                if (rc != SROT_OK) break;
                if (best_ms == 0.0f || ms < best_ms) { best_ms = ms; best = t; }
            }
            if (rc == SROT_OK) tune_cache_store(key, TuneEntry{best, best_ms});
        }
        h->groups[gi].first = best;
        h->tune_ms[gi] = best_ms;
        for (int q = first; q < first + cnt; ++q) {
            h->tile[ord[q]] = best;
            h->probs[ord[q]].tile = srot::tile_id(best);
        }
    }
    if (lock.owns_lock()) lock.unlock();

    // launch order: per class, the largest problems first (each solve then
    // reorders by the measured run times)
    for (int c = 0; c < srot::kClasses; ++c) {
        h->cls_first[c] = (int)h->order.size();
        for (int32_t p : ord)
            if (srot::tile_class(h->tile[p]) == c) h->order.push_back(p);
        h->cls_count[c] = (int)h->order.size() - h->cls_first[c];
        std::stable_sort(h->order.begin() + h->cls_first[c], h->order.end(), [&](int32_t x, int32_t y) {
            return (int64_t)h->probs[x].m * h->probs[x].n > (int64_t)h->probs[y].m * h->probs[y].n;
        });
    }
    if (rc == SROT_OK) {
        e = hipMemcpyAsync(h->d_probs, h->probs.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice,
                           h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_order, h->order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(SROT_EHIP, "srot_init_batched: %s", hipGetErrorString(e));
    }

    // one graph: a kernel node per class, no dependencies between them
    if (rc == SROT_OK) {
        e = hipGraphCreate(&h->graph, 0);
        const BatchParams prm = params_of(h->opt);
        for (int c = 0; e == hipSuccess && c < srot::kClasses; ++c) {
            if (h->cls_count[c] == 0) continue;
            const float *Cp = h->C;
            const double *ap = h->a, *bp = h->b;
            double *Tp = h->T, *rp = h->r;
            uint32_t *Mp = h->M;
            int32_t *ip = h->idx;
            const BatchProblem *pp = h->d_probs;
            const int32_t *op = h->d_order + h->cls_first[c];
            BatchParams pr = prm;
            BatchResult *resp = h->d_res;
            void *args[] = {&Cp, &ap, &bp, &Tp, &rp, &Mp, &ip, &pp, &op, &pr, &resp};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void *>(srot::class_kernel(c));
            kp.gridDim = dim3(h->cls_count[c]);
            kp.blockDim = dim3(srot::class_nt(c));
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            e = hipGraphAddKernelNode(&node, h->graph, nullptr, 0, &kp);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(SROT_EHIP, "srot_init_batched: graph: %s", hipGetErrorString(e));
    }
    if (rc != SROT_OK) {
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        delete h;
        return rc;
    }
    *out = h;
    return SROT_OK;
}

int srot_solve_batched(srot_batch *h, double *out3, int64_t *passes, int32_t *status)
{
    if (!h) return fail(SROT_EINVAL, "srot_solve_batched: NULL handle");
    std::vector<BatchResult> res(h->count);
    SROT_HIP_B(hipGraphLaunch(h->exec, h->stream));
    SROT_HIP_B(hipMemcpyAsync(res.data(), h->d_res, sizeof(BatchResult) * h->count, hipMemcpyDeviceToHost,
                              h->stream));
    SROT_HIP_B(hipStreamSynchronize(h->stream));
    bool all = true;
    int32_t bad = -1;
    for (int32_t p = 0; p < h->count; ++p) {
        if (out3) { out3[3 * p] = res[p].g; out3[3 * p + 1] = res[p].f; out3[3 * p + 2] = res[p].D; }
        if (passes) passes[p] = res[p].passes;
        if (status) status[p] = res[p].status;
        all &= (res[p].status == SROT_OK);
        if (res[p].status < 0 && bad < 0) bad = p;
    }
    if (bad >= 0) return fail(SROT_EINVAL, "srot_solve_batched: problem %d was launched with a tile of another class", bad);
    // the next solve starts each class's longest-running problems first
    // (the results do not depend on the order)
    std::vector<int32_t> next = h->order;
    for (int c = 0; c < srot::kClasses; ++c)
        std::stable_sort(next.begin() + h->cls_first[c], next.begin() + h->cls_first[c] + h->cls_count[c],
                         [&](int32_t x, int32_t y) { return res[x].ticks > res[y].ticks; });
    if (next != h->order) {
        h->order = next;
        SROT_HIP_B(hipMemcpyAsync(h->d_order, h->order.data(), sizeof(int32_t) * h->count, hipMemcpyHostToDevice,
                                  h->stream));
        SROT_HIP_B(hipStreamSynchronize(h->stream));
    }
    return all ? SROT_OK : SROT_NOT_CONVERGED;
}

int srot_get_plan_batched(srot_batch *h, int32_t p, double *T_out, double *r_out)
{
    if (!h || p < 0 || p >= h->count) return fail(SROT_EINVAL, "srot_get_plan_batched: bad handle or index");
    const BatchProblem &bp = h->probs[p];
    if (T_out) {
        srot::Ownership o;
        o.nt = h->tile[p].nt; o.cpt = h->tile[p].cpt; o.vec = h->tile[p].vec; o.words = 1; o.reg = 1;
        hipLaunchKernelGGL(srot::batch_plan_kernel, dim3(std::min(bp.m, 4096)), dim3(256), 0, h->stream,
                           (const double *)(h->T + bp.T_off), (const uint32_t *)(h->M + bp.M_off), bp.m, bp.n,
                           o, T_out);
        SROT_HIP_B(hipGetLastError());
    }
    if (r_out)
        SROT_HIP_B(hipMemcpyAsync(r_out, h->r + bp.r_off, sizeof(double) * bp.n, hipMemcpyDeviceToDevice,
                                  h->stream));
    return SROT_OK;
}

int srot_get_tiles_batched(srot_batch *h, int32_t *tiles, float *ms_per_step)
{
    if (!h || !tiles) return fail(SROT_EINVAL, "srot_get_tiles_batched: NULL argument");
    for (int32_t p = 0; p < h->count; ++p) {
        tiles[3 * p] = h->tile[p].nt;
        tiles[3 * p + 1] = h->tile[p].cpt;
        tiles[3 * p + 2] = h->tile[p].vec;
    }
    if (ms_per_step) {
        for (int32_t p = 0; p < h->count; ++p) ms_per_step[p] = 0.0f;
        // the group's tuning figure, reported for every member
        for (size_t gi = 0; gi < h->groups.size(); ++gi) {
            const Tile &t = h->groups[gi].first;
            for (int32_t p = 0; p < h->count; ++p)
                if (h->tile[p] == t) ms_per_step[p] = h->tune_ms[gi];
        }
    }
    return SROT_OK;
}

void srot_destroy_batched(srot_batch *h)
{
    if (!h) return;
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
}

}  // extern "C"
