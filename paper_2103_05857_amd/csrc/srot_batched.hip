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
// Problems are grouped by tile shape (threads x columns per thread x vector
// width); each group is one launch of batch_solve_kernel, one workgroup per
// problem, largest problems first.  The group launches are independent
// nodes of one hipGraph, instantiated once and replayed by every
// srot_solve_batched call.  The tile shape of each group is either the
// single-problem default or the fastest candidate measured on the group's
// largest problem (srot_init_batched with tune = 1).
//
// Workspace (caller-owned): problem table, launch order, results, then per
// problem r (n), block indices (m), support masks (m x 256 words) and the
// dense FP64 plan (m x n).  The plan is never cleared: every kernel reads
// t_ij only where the support mask has its bit set.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <numeric>
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
};

struct BatchResult {
    double g, f, D;
    int64_t passes;
    int32_t status, pad;
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
// dual of App. D).  Wave `wid` takes rows wid, wid + NW, ...; per row the
// wave streams the cost row (lowest-index argmin of c_ij + w r_j), then sums
// t_ij (v_ij - G_i) and t_ij c_ij over the support.  The waves' row sums are
// added in wave order; the result is the same in every thread.
template <int NT, int VEC>
__device__ void batch_gap(const ProblemView &P, const double *__restrict__ T,
                          const double *__restrict__ rg, const uint32_t *__restrict__ M,
                          double &g_out, double &f_out, double &D_out)
{
    constexpr int NW = NT / 64;
    __shared__ double s_w[NW][3];
    __shared__ double s_rb[NW][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = P.m, n = P.n;
    const double w = P.w;
    const float *__restrict__ C = (const float *)P.C;
    double aG = 0.0, lin = 0.0, gs = 0.0;
    for (int i = wid; i < m; i += NW) {
        const float *__restrict__ crow = C + (size_t)i * (size_t)n;
        double best = INFINITY;
        int bj = 0x7fffffff;
        if constexpr (VEC == 4) {
            const float4 *__restrict__ c4 = reinterpret_cast<const float4 *>(crow);
            const double2 *__restrict__ r2 = reinterpret_cast<const double2 *>(rg);
            const int ng = n / 4;
            for (int q = lane; q < ng; q += 64) {
                const float4 cv = c4[q];
                const double2 ra = r2[2 * q], rb = r2[2 * q + 1];
                const double v0 = (double)cv.x + w * ra.x, v1 = (double)cv.y + w * ra.y;
                const double v2 = (double)cv.z + w * rb.x, v3 = (double)cv.w + w * rb.y;
                if (v0 < best) { best = v0; bj = 4 * q; }
                if (v1 < best) { best = v1; bj = 4 * q + 1; }
                if (v2 < best) { best = v2; bj = 4 * q + 2; }
                if (v3 < best) { best = v3; bj = 4 * q + 3; }
            }
        } else {
            for (int j = lane; j < n; j += 64) {
                const double v = (double)crow[j] + w * rg[j];
                if (v < best) { best = v; bj = j; }
            }
        }
        wave_argmin(best, bj);
        double x[2] = {0.0, 0.0};
        for (int ts = lane; ts < NT; ts += 64) {
            uint32_t mk = M[(size_t)i * NT + ts];
            while (mk) {
                const int u = __ffs(mk) - 1;
                mk &= mk - 1u;
                const int j = owned_col<NT, VEC>(u, ts);
                const double t = T[(size_t)i * (size_t)n + j];
                const double c = (double)crow[j];
                x[0] += t * (c + w * rg[j] - best);
                x[1] += t * c;
            }
        }
        wave_sum<2>(x);
        aG += P.a[i] * best;
        lin += x[1];
        gs += x[0];
    }
    if (lane == 0) { s_w[wid][0] = aG; s_w[wid][1] = lin; s_w[wid][2] = gs; }
    double rb[2] = {0.0, 0.0};
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

template <int NT, int CPT, int VEC>
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
    constexpr int COST = SROT_COST_F32;
    const int tid = threadIdx.x;
    const int p = order[blockIdx.x];
    const BatchProblem bp = probs[p];
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
            batch_gap<NT, VEC>(P, T, rg, M, g, f, D);
            if (g <= prm.eps) { status = SROT_OK; break; }
        }
    }
    if (tid == 0) {
        BatchResult out;
        out.g = g; out.f = f; out.D = D; out.passes = passes; out.status = status; out.pad = 0;
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

// Tile shapes compiled for the batched kernel (one mask word per thread).
#define SROT_BATCH_TILES(X) \
    X(64, 2, 1) X(64, 4, 1) X(128, 4, 1) X(256, 4, 1) X(256, 8, 1) X(256, 16, 1) \
    X(64, 4, 4) X(128, 4, 4) X(256, 4, 4) X(256, 8, 4) X(256, 16, 4)

const void *batch_kernel_for(const Tile &t)
{
#define SROT_BK(NT_, CPT_, VEC_) \
    if (t.nt == NT_ && t.cpt == CPT_ && t.vec == VEC_) return (const void *)&batch_solve_kernel<NT_, CPT_, VEC_>;
    SROT_BATCH_TILES(SROT_BK)
#undef SROT_BK
    return nullptr;
}

std::vector<Tile> tile_candidates(int64_t n, bool vec4)
{
    std::vector<Tile> out;
#define SROT_BC(NT_, CPT_, VEC_) \
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

hipError_t launch_group(srot_batch *h, const Tile &t, int first, int cnt, const BatchParams &prm,
                        hipStream_t st)
{
    const void *fn = srot::batch_kernel_for(t);
    if (!fn) return hipErrorInvalidDeviceFunction;
    const float *C = h->C;
    const double *a = h->a, *b = h->b;
    double *T = h->T, *r = h->r;
    uint32_t *M = h->M;
    int32_t *idx = h->idx;
    const BatchProblem *probs = h->d_probs;
    const int32_t *order = h->d_order + first;
    BatchResult *res = h->d_res;
    BatchParams pr = prm;
    void *args[] = {&C, &a, &b, &T, &r, &M, &idx, &probs, &order, &pr, &res};
    return hipLaunchKernel(fn, dim3(cnt), dim3(t.nt), args, 0, st);
}

// Milliseconds per block step of one tile on the problem at position `pos`
// of the launch order: two passes and a gap sweep from the initial plan (the
// second of two runs).
int time_tile(srot_batch *h, int pos, int32_t p, const Tile &t, float *ms_per_step)
{
    BatchParams prm = params_of(h->opt);
    prm.max_passes = 2;
    prm.gap_every = 2;
    prm.eps = -1.0;
    hipEvent_t e0, e1;
    SROT_HIP_B(hipEventCreate(&e0));
    SROT_HIP_B(hipEventCreate(&e1));
    float best = 0.0f;
    int rc = SROT_OK;
    for (int rep = 0; rep < 2 && rc == SROT_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess) e = launch_group(h, t, pos, 1, prm, h->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = fail(SROT_EHIP, "autotune: %s", hipGetErrorString(e));
        best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_step = best / (float)(2 * h->probs[p].m);
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
        h->probs.push_back(bp);
        const bool vec4 = (n[p] % 4 == 0) && (bp.c_off % 4 == 0) && (((uintptr_t)C) % 16 == 0);
        const srot::Ownership o = srot::choose_ownership(n[p], SROT_COST_F32, vec4);
        Tile t{o.nt, o.cpt, o.vec};
        if (!srot::batch_kernel_for(t)) t = Tile{256, 16, 1};  // any n <= 4096 fits
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

    // autotuner: per group, time every candidate tile on the group's largest problem
    h->tune_ms.assign(h->groups.size(), 0.0f);
    for (size_t gi = 0; rc == SROT_OK && tune && gi < h->groups.size(); ++gi) {
        const int first = h->groups[gi].second.first, cnt = h->groups[gi].second.second;
        const int p0 = ord[first];
        int64_t nmax = 0;
        bool vec4 = h->groups[gi].first.vec == 4;
        for (int q = first; q < first + cnt; ++q) nmax = std::max<int64_t>(nmax, h->probs[ord[q]].n);
        Tile best = h->groups[gi].first;
        float best_ms = 0.0f;
        for (const Tile &t : srot::tile_candidates(nmax, vec4)) {
            float ms = 0.0f;
            rc = time_tile(h, first, p0, t, &ms);
            if (rc != SROT_OK) break;
            if (best_ms == 0.0f || ms < best_ms) { best_ms = ms; best = t; }
        }
        h->groups[gi].first = best;
        h->tune_ms[gi] = best_ms;
        for (int q = first; q < first + cnt; ++q) h->tile[ord[q]] = best;
    }

    // one graph: a kernel node per group, no dependencies between them
    if (rc == SROT_OK) {
        e = hipGraphCreate(&h->graph, 0);
        const BatchParams prm = params_of(h->opt);
        for (size_t gi = 0; e == hipSuccess && gi < h->groups.size(); ++gi) {
            const Tile &t = h->groups[gi].first;
            const int first = h->groups[gi].second.first, cnt = h->groups[gi].second.second;
            const float *Cp = h->C;
            const double *ap = h->a, *bp = h->b;
            double *Tp = h->T, *rp = h->r;
            uint32_t *Mp = h->M;
            int32_t *ip = h->idx;
            const BatchProblem *pp = h->d_probs;
            const int32_t *op = h->d_order + first;
            BatchParams pr = prm;
            BatchResult *resp = h->d_res;
            void *args[] = {&Cp, &ap, &bp, &Tp, &rp, &Mp, &ip, &pp, &op, &pr, &resp};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void *>(srot::batch_kernel_for(t));
            kp.gridDim = dim3(cnt);
            kp.blockDim = dim3(t.nt);
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
    for (int32_t p = 0; p < h->count; ++p) {
        if (out3) { out3[3 * p] = res[p].g; out3[3 * p + 1] = res[p].f; out3[3 * p + 2] = res[p].D; }
        if (passes) passes[p] = res[p].passes;
        if (status) status[p] = res[p].status;
        all &= (res[p].status == SROT_OK);
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
