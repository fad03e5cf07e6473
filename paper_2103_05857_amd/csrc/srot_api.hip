// C ABI of libsrot (declared in include/srot.h): argument checking, workspace
// layout, and the pass loop around the kernels in srot_kernels.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/srot.h"
#include "srot_internal.h"

struct srot_handle {
    srot::ProblemView P;
    srot::DeviceState S;
    srot_options opt;
    hipStream_t stream;
    int64_t k;     // global block-step counter (decay rule, sampler position)
    int64_t fw_k;  // full Frank-Wolfe iteration counter (decay rule of Alg. A.1)
    void *scratch;            // this device's copy of `scratch` (below), or null
    hipError_t scratch_err;   // why `scratch` is null
    // What a solve loop reads back per batch, in pinned host memory (two
    // slots, so the next batch is queued before the last one is read) with
    // an event per slot; made by srot_init, freed by srot_destroy.
    struct Readback {
        int32_t words[4];  // the stop word and its pass and the team error (or the FW run state)
        double sums[3];    // g, f, D of the last measurement
    } *rb;
    hipEvent_t rb_ev[2];
};

// Scratch of srot_backward_noalloc: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never a device
// address: host code uses only the address hipGetSymbolAddress returns for
// the current device (kept per device below, and per handle).
static __device__ __align__(256) unsigned char scratch[SROT_NOALLOC_SCRATCH_BYTES];

namespace {
// Zeroes the control words of the static scratch (no word an earlier call
// left is read as a flag): a kernel, so the call stays capturable.
__global__ void noalloc_clear_kernel(int32_t *words)
{
    if (threadIdx.x < 64) words[threadIdx.x] = 0;
}

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
hipError_t scratch_address(void **out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace srot {
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
}  // namespace srot

namespace {
using srot::fail;

#define SROT_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(SROT_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t T, r, mask, idx, G, j, g, partials, scalars, meas, flags, slow, Y4, adj, ga_w, team, total;
    int64_t idx_cap;
    int32_t gap_blocks;
};

// Mask words per row for any ownership the kernels may choose for n columns
// (at most 512 threads with one word each, or the wide-row layout).
size_t mask_words_per_row(int64_t n)
{
    const int64_t cpt_glb = (n + 511) / 512;
    const int64_t words_glb = (cpt_glb + 31) / 32;
    return (size_t)std::max<int64_t>(512, words_glb * 512);
}

bool sizes_ok(int64_t m, int64_t n)
{
    return m >= 1 && n >= 1 && m <= 0x7fffffff && n <= 0x7fffffff;
}

Layout make_layout(int64_t m, int64_t n)
{
    Layout L;
    // whole passes of indices, at least 65536 steps
    int64_t passes = std::max<int64_t>(1, (65536 + m - 1) / m);
    L.idx_cap = passes * m;
    L.gap_blocks = srot::gap_blocks_for(m);
    size_t off = 0;
    L.T = off; off = align_up(off + sizeof(double) * (size_t)m * (size_t)n);
    L.r = off; off = align_up(off + sizeof(double) * (size_t)n);
    L.mask = off; off = align_up(off + sizeof(uint32_t) * (size_t)m * mask_words_per_row(n));
    L.idx = off; off = align_up(off + sizeof(int32_t) * (size_t)L.idx_cap);
    L.G = off; off = align_up(off + sizeof(double) * (size_t)m);
    L.j = off; off = align_up(off + sizeof(int32_t) * (size_t)m);
    L.g = off; off = align_up(off + sizeof(double) * (size_t)m);
    L.partials = off;
    off = align_up(off + sizeof(double) * 8 * (size_t)L.gap_blocks);
    L.scalars = off; off = align_up(off + sizeof(double) * 8);
    L.meas = off; off = align_up(off + sizeof(double) * 8);
    L.flags = off; off = align_up(off + sizeof(int32_t) * 8);
    L.slow = off; off = align_up(off + 4 * sizeof(int64_t));
    L.Y4 = off; off = align_up(off + 16 * (size_t)srot::y4_entries(n));
    L.adj = off; off = align_up(off + sizeof(double) * 3 * (size_t)n * (size_t)srot::adjoint_slices_cap(m));
    L.ga_w = off; off = align_up(off + sizeof(double) * (size_t)m);
    L.team = off;
    off = align_up(off + sizeof(unsigned long long) * 2 * srot::TEAM_MAX_MEMBERS * srot::TEAM_REC_STRIDE);
    L.total = off;
    return L;
}

bool options_ok(const srot_options *o)
{
    if (!o) return false;
    if (!(o->w >= 0.0) || !isfinite(o->w)) return false;
    if (o->step_rule != SROT_ELS && o->step_rule != SROT_DEC) return false;
    if (o->sampling != SROT_UNIFORM && o->sampling != SROT_PERMUTE) return false;
    if (!(o->eps >= 0.0)) return false;
    if (o->max_passes < 0 || o->gap_every < 1) return false;
    if (o->cost != SROT_COST_F32 && o->cost != SROT_COST_F64 && o->cost != SROT_COST_SQEUCLID)
        return false;
    return true;
}

// Draws `count` indices for steps k .. k+count-1 into the index buffer and
// returns a pointer to the first; count is reduced to what fits.
int draw_indices(srot_handle *h, int64_t k, int64_t *count, const int32_t **out)
{
    const int32_t m = h->P.m;
    if (h->opt.sampling == SROT_UNIFORM) {
        *count = std::min(*count, h->S.idx_cap);
        SROT_HIP(srot::launch_sample_uniform(h->opt.seed, k, *count, m, h->S.idx, h->stream));
        *out = h->S.idx;
    } else {
        const int64_t p0 = k / m, off = k - p0 * m;
        const int64_t cap_passes = h->S.idx_cap / m;
        const int64_t need = (off + *count + m - 1) / m;
        const int64_t np = std::min(need, cap_passes);
        *count = std::min(*count, np * m - off);
        SROT_HIP(srot::launch_sample_permute(h->opt.seed, p0, np, m, h->S.idx, h->stream));
        *out = h->S.idx + off;
    }
    return SROT_OK;
}

int run_steps(srot_handle *h, int64_t nsteps, int32_t *trace_j, double *trace_gamma,
              const srot::ProblemView *Pv = nullptr)
{
    const srot::ProblemView &P = Pv ? *Pv : h->P;
    int64_t done = 0;
    while (done < nsteps) {
        int64_t cnt = nsteps - done;
        const int32_t *idx = nullptr;
        int rc = draw_indices(h, h->k, &cnt, &idx);
        if (rc != SROT_OK) return rc;
        SROT_HIP(srot::launch_chain(P, h->S, idx, h->k, cnt, h->opt.step_rule,
                                    trace_j ? trace_j + done : nullptr,
                                    trace_gamma ? trace_gamma + done : nullptr, h->stream));
        h->k += cnt;
        done += cnt;
    }
    return SROT_OK;
}

int run_variant_steps(srot_handle *h, int pairwise, int64_t nsteps, int32_t *trace_j, int32_t *trace_away,
                      double *trace_gamma, const srot::ProblemView *Pv = nullptr)
{
    const srot::ProblemView &P = Pv ? *Pv : h->P;
    int64_t done = 0;
    while (done < nsteps) {
        int64_t cnt = nsteps - done;
        const int32_t *idx = nullptr;
        int rc = draw_indices(h, h->k, &cnt, &idx);
        if (rc != SROT_OK) return rc;
        SROT_HIP(srot::launch_active_steps(P, h->S, pairwise, idx, cnt, trace_j ? trace_j + done : nullptr,
                                           trace_away ? trace_away + done : nullptr,
                                           trace_gamma ? trace_gamma + done : nullptr, h->stream));
        h->k += cnt;
        done += cnt;
    }
    return SROT_OK;
}

int variant_ok(srot_handle *h, int variant, const char *who)
{
    if (!h) return fail(SROT_EINVAL, "%s: NULL handle", who);
    if (variant != SROT_STEP_AWAY && variant != SROT_STEP_PAIRWISE)
        return fail(SROT_EINVAL, "%s: variant must be SROT_STEP_AWAY or SROT_STEP_PAIRWISE", who);
    if (h->opt.step_rule != SROT_ELS)
        return fail(SROT_EINVAL, "%s: away and pairwise steps use the exact line search (SROT_ELS)", who);
    if (!srot::active_steps_supported(h->S))
        return fail(SROT_EINVAL, "%s: away and pairwise steps support rows of at most 8192 columns", who);
    return SROT_OK;
}

int ga_ok(srot_handle *h, const char *who)
{
    if (!h) return fail(SROT_EINVAL, "%s: NULL handle", who);
    if (!srot::ga_supported(h->P, h->S))
        return fail(SROT_EINVAL, "%s: gap-adaptive sampling supports at most %d rows of at most 8192 columns", who,
                    (int)srot::GA_MAX_ROWS);
    return SROT_OK;
}

int measure_gap(srot_handle *h, double *out3)
{
    SROT_HIP(srot::launch_gap(h->P, h->S, h->stream));
    double host[3];
    int32_t team_err = 0;
    SROT_HIP(hipMemcpyAsync(host, h->S.scalars, sizeof(host), hipMemcpyDeviceToHost, h->stream));
    if (h->S.team)
        SROT_HIP(hipMemcpyAsync(&team_err, h->S.flags + 6, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    SROT_HIP(hipStreamSynchronize(h->stream));
    if (team_err)
        return fail(SROT_EHIP, "team chain: a member waited too long for the others' records; "
                               "the plan and residual are inconsistent");
    out3[0] = host[0]; out3[1] = host[1]; out3[2] = host[2];
    return SROT_OK;
}

}  // namespace

// Pinned readback slots and their events, made once per handle.
int ensure_readback(srot_handle *h)
{
    if (h->rb) return SROT_OK;
    void *p = nullptr;
    SROT_HIP(hipHostMalloc(&p, 2 * sizeof(srot_handle::Readback), hipHostMallocDefault));
    for (int q = 0; q < 2; ++q) {
        hipError_t e = hipEventCreateWithFlags(&h->rb_ev[q], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int k = 0; k < q; ++k) (void)hipEventDestroy(h->rb_ev[k]);
            (void)hipHostFree(p);
            return fail(SROT_EHIP, "hipEventCreateWithFlags failed: %s", hipGetErrorString(e));
        }
    }
    h->rb = (srot_handle::Readback *)p;
    return SROT_OK;
}

// Passes are queued in batches of kSolveBatch.  The final sum of each
// measuring sweep takes the stop test on the device; once g <= eps every
// later kernel returns at its start, so the state is that of the stopping
// pass.  The host queues batch b + 1 before it reads batch b's stop word
// (copied to pinned memory behind the batch), so the GPU does not wait for
// the host between batches; a batch queued after the stop does nothing.
// steps(p, Ps) queues pass p's block steps, after(p, Ps, measured) what
// follows the pass's sweep (the gap-adaptive sampler's global update).
constexpr int64_t kSolveBatch = 4;

template <class Steps, class After>
int solve_on_device(srot_handle *h, double *out3, int64_t *passes, Steps steps, After after)
{
    *passes = 0;
    out3[0] = INFINITY; out3[1] = NAN; out3[2] = NAN;
    int rc = ensure_readback(h);
    if (rc != SROT_OK) return rc;
    const int64_t m = h->P.m, maxp = h->opt.max_passes;
    int32_t *stop_w = h->S.flags + 4;  // [0] stopped, [1] its pass (low 32 bits), [2] team error
    srot::ProblemView Ps = h->P;
    Ps.stop = stop_w;
    SROT_HIP(hipMemsetAsync(stop_w, 0, 2 * sizeof(int32_t), h->stream));
    const int64_t k0 = h->k;
    // queue passes [p0, p1) and the readback of their outcome into slot q
    auto queue = [&](int64_t p0, int64_t p1, int q) -> int {
        for (int64_t p = p0; p < p1; ++p) {
            int r = steps(p, Ps);
            if (r != SROT_OK) return r;
            const bool measure = (p + 1) % h->opt.gap_every == 0 || p + 1 == maxp;
            if (measure)
                SROT_HIP(srot::launch_gap_stop(Ps, h->S, h->stream, stop_w, h->opt.eps, (int32_t)(uint32_t)p));
            r = after(p, Ps, measure);
            if (r != SROT_OK) return r;
        }
        SROT_HIP(hipMemcpyAsync(h->rb[q].words, stop_w, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        SROT_HIP(hipMemcpyAsync(h->rb[q].sums, h->S.meas, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        SROT_HIP(hipEventRecord(h->rb_ev[q], h->stream));
        return SROT_OK;
    };
    if (maxp <= 0) return SROT_NOT_CONVERGED;
    int64_t p0 = 0, p1 = std::min(maxp, kSolveBatch);
    rc = queue(p0, p1, 0);
    if (rc != SROT_OK) return rc;
    bool measured_any = false;
    for (int64_t b = 0;; ++b) {
        const int q = (int)(b & 1);
        // the next batch goes in before this one is read
        const int64_t n0 = p1, n1 = std::min(maxp, p1 + kSolveBatch);
        if (n0 < maxp) {
            rc = queue(n0, n1, 1 - q);
            if (rc != SROT_OK) return rc;
        }
        SROT_HIP(hipEventSynchronize(h->rb_ev[q]));
        const srot_handle::Readback &R = h->rb[q];
        if (h->S.team && R.words[2])
            return fail(SROT_EHIP, "team chain: a member waited too long for the others' records; "
                                   "the plan and residual are inconsistent");
        for (int64_t p = p0; p < p1; ++p)
            measured_any |= (p + 1) % h->opt.gap_every == 0 || p + 1 == maxp;
        if (measured_any) { out3[0] = R.sums[0]; out3[1] = R.sums[1]; out3[2] = R.sums[2]; }
        if (R.words[0]) {
            // a batch holds fewer than 2^32 passes: the low bits name the pass
            const int64_t p = p0 + (int64_t)(uint32_t)((uint32_t)R.words[1] - (uint32_t)p0);
            *passes = p + 1;
            h->k = k0 + (p + 1) * m;  // the passes queued after it did nothing
            return SROT_OK;
        }
        *passes = p1;
        if (n0 >= maxp) return SROT_NOT_CONVERGED;
        p0 = n0;
        p1 = n1;
    }
}

extern "C" {

void srot_default_options(srot_options *opt)
{
    if (!opt) return;
    opt->w = 1.0;
    opt->step_rule = SROT_ELS;
    opt->sampling = SROT_UNIFORM;
    opt->seed = 0;
    opt->eps = 1e-6;
    opt->max_passes = 1000;
    opt->gap_every = 1;
    opt->cost = SROT_COST_F32;
}

size_t srot_workspace_size(int64_t m, int64_t n, const srot_options *opt)
{
    (void)opt;
    if (!sizes_ok(m, n)) return 0;
    return make_layout(m, n).total;
}

int srot_init(srot_handle **out, int64_t m, int64_t n, const void *C, const float *X,
              const float *Y, const double *a, const double *b, void *workspace, size_t ws_bytes,
              const srot_options *opt, void *stream)
{
    if (!out) return fail(SROT_EINVAL, "srot_init: out is NULL");
    *out = nullptr;
    if (!sizes_ok(m, n)) return fail(SROT_EINVAL, "srot_init: need 1 <= m, n <= 2^31-1 (m=%lld n=%lld)",
                                     (long long)m, (long long)n);
    if (!options_ok(opt)) return fail(SROT_EINVAL, "srot_init: invalid options");
    if (!a || !b) return fail(SROT_EINVAL, "srot_init: a and b are required");
    if (opt->cost == SROT_COST_SQEUCLID) {
        if (!X || !Y) return fail(SROT_EINVAL, "srot_init: X and Y are required for SROT_COST_SQEUCLID");
    } else if (!C) {
        return fail(SROT_EINVAL, "srot_init: C is required for a stored cost");
    }
    if (!workspace) return fail(SROT_EINVAL, "srot_init: workspace is NULL");
    if (((uintptr_t)workspace) % kAlign != 0)
        return fail(SROT_EINVAL, "srot_init: workspace must be 256-byte aligned");
    const Layout L = make_layout(m, n);
    if (ws_bytes < L.total)
        return fail(SROT_ENOMEM, "srot_init: workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    srot_handle *h = (srot_handle *)calloc(1, sizeof(srot_handle));
    if (!h) return fail(SROT_ENOMEM, "srot_init: out of host memory");
    h->opt = *opt;
    h->stream = (hipStream_t)stream;
    h->k = 0;
    h->fw_k = 0;
    h->P.m = (int32_t)m;
    h->P.n = (int32_t)n;
    h->P.cost = opt->cost;
    h->P.C = (opt->cost == SROT_COST_SQEUCLID) ? nullptr : C;
    h->P.X = X;
    h->P.Y = Y;
    h->P.a = a;
    h->P.b = b;
    h->P.w = opt->w;
    char *base = (char *)workspace;
    h->P.Y4 = Y ? (const float4 *)(base + L.Y4) : nullptr;
    h->P.y4n = (int32_t)srot::y4_entries(n);
    h->S.T = (double *)(base + L.T);
    h->S.r = (double *)(base + L.r);
    h->S.mask = (uint32_t *)(base + L.mask);
    h->S.own = srot::choose_ownership(n, opt->cost, ((uintptr_t)C % 16u) == 0u);
    h->S.idx = (int32_t *)(base + L.idx);
    h->S.idx_cap = L.idx_cap;
    h->S.row_G = (double *)(base + L.G);
    h->S.row_j = (int32_t *)(base + L.j);
    h->S.row_g = (double *)(base + L.g);
    h->S.partials = (double *)(base + L.partials);
    h->S.gap_blocks = L.gap_blocks;
    h->S.scalars = (double *)(base + L.scalars);
    h->S.meas = (double *)(base + L.meas);
    h->S.flags = (int32_t *)(base + L.flags);
    h->S.slow_steps = (int64_t *)(base + L.slow);
    h->S.adj_part = (double *)(base + L.adj);
    h->S.ga_w = (double *)(base + L.ga_w);
    h->S.team_rec = (unsigned long long *)(base + L.team);
    h->S.team = srot::team_chain_supported(h->P) ? 1 : 0;

    int rc = SROT_OK;
    int32_t flag = 0;
    hipError_t e = hipMemsetAsync(h->S.flags, 0, sizeof(int32_t) * 8, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->S.slow_steps, 0, sizeof(int64_t) * 4, h->stream);
    if (e == hipSuccess) e = srot::launch_validate(h->P, h->S, h->stream);
    if (e == hipSuccess) e = srot::launch_pad_points(h->P, h->stream);
    if (e == hipSuccess) e = srot::launch_init_plan(h->P, h->S, h->stream);
    if (e == hipSuccess) e = srot::launch_residual(h->P, h->S, h->stream);
    if (e == hipSuccess) e = srot::launch_mask_build(h->P, h->S, h->stream);
    if (e == hipSuccess) e = srot::launch_ga_fill(h->P, h->S, nullptr, SROT_GA_INIT, h->stream);
    // the FP32 LMO screen of wide fused rows needs an error bound (see the
    // wide-row chain kernel): 8 u (Cmax + |w| Rmax), doubled, u = 2^-24
    const bool wide = opt->cost == SROT_COST_SQEUCLID && !h->S.own.reg;
    // the screened chain's FP32 LMO screen needs the same kind of bound on
    // the stored cost: max |c_ij| and max(sum a, max b)
    const bool screened = srot::screened_chain_supported(h->P, h->S) && srot::screened_chain_enabled();
    double bounds[2] = {0.0, 0.0};
    if (e == hipSuccess && wide) e = srot::launch_screen_bounds(h->P, h->S.scalars + 5, h->stream);
    if (e == hipSuccess && screened) e = srot::launch_cost_bounds(h->P, h->S, h->S.scalars + 5, h->stream);
    if (e == hipSuccess && (wide || screened))
        e = hipMemcpyAsync(bounds, h->S.scalars + 5, sizeof(bounds), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, h->S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = fail(SROT_EHIP, "srot_init: %s", hipGetErrorString(e));
    else if (flag & 1) rc = fail(SROT_ENONFINITE, "srot_init: NaN/Inf in C, X, Y, a or b, or a negative weight");
    h->S.screen_delta2 = 0.0;
    h->S.screen_err = 0.0;
    // the allocation-free backward's scratch on this device (its absence
    // only disables srot_backward_noalloc)
    if (rc == SROT_OK) h->scratch_err = scratch_address(&h->scratch);
    // the solve loops' pinned readback words (host memory), made here so
    // that no solve pays for the allocation
    if (rc == SROT_OK) rc = ensure_readback(h);
    if (rc == SROT_OK && screened) {
        // FP32 screen value fma(w, r, c) against c + w r: at most 2^-22
        // (|c| + |w| |r|) off (rounding of r, w and the fma); doubled
        const double scale = bounds[0] + fabs(opt->w) * bounds[1];
        h->S.screen_err = 0x1.0p-21 * scale * (1.0 + 1e-6) + 1e-300;
    }
    if (rc == SROT_OK && wide) {
        const double u = 0x1.0p-24;
        const double scale = bounds[0] + fabs(opt->w) * bounds[1];
        h->S.screen_delta2 = 2.0 * (8.0 * u * scale) * (1.0 + 1e-6) + 1e-300;
    }
    if (rc != SROT_OK) {
        free(h);
        return rc;
    }
    *out = h;
    return SROT_OK;
}

int srot_step(srot_handle *h, int64_t nsteps, const int32_t *idx, int32_t *trace_j,
              double *trace_gamma)
{
    if (!h) return fail(SROT_EINVAL, "srot_step: NULL handle");
    if (nsteps < 0) return fail(SROT_EINVAL, "srot_step: nsteps < 0");
    if (nsteps == 0) return SROT_OK;
    if (!idx) return run_steps(h, nsteps, trace_j, trace_gamma);
    // caller-supplied indices: check them on the device before any update
    int32_t flag = 0;
    SROT_HIP(hipMemsetAsync(h->S.flags, 0, sizeof(int32_t), h->stream));
    SROT_HIP(srot::launch_check_indices(idx, nsteps, h->P.m, h->S.flags, h->stream));
    SROT_HIP(hipMemcpyAsync(&flag, h->S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    SROT_HIP(hipStreamSynchronize(h->stream));
    if (flag & 2) return fail(SROT_EINVAL, "srot_step: block index outside [0, m)");
    SROT_HIP(srot::launch_chain(h->P, h->S, idx, h->k, nsteps, h->opt.step_rule, trace_j,
                                trace_gamma, h->stream));
    h->k += nsteps;
    return SROT_OK;
}

int srot_gap(srot_handle *h, double *out3, double *row_gap, int32_t *row_argmin)
{
    if (!h || !out3) return fail(SROT_EINVAL, "srot_gap: NULL argument");
    int rc = measure_gap(h, out3);
    if (rc != SROT_OK) return rc;
    if (row_gap)
        SROT_HIP(hipMemcpyAsync(row_gap, h->S.row_g, sizeof(double) * h->P.m, hipMemcpyDeviceToDevice, h->stream));
    if (row_argmin)
        SROT_HIP(hipMemcpyAsync(row_argmin, h->S.row_j, sizeof(int32_t) * h->P.m, hipMemcpyDeviceToDevice, h->stream));
    if (row_gap || row_argmin) SROT_HIP(hipStreamSynchronize(h->stream));
    return SROT_OK;
}

int srot_gap_async(srot_handle *h, double *out5)
{
    if (!h || !out5) return fail(SROT_EINVAL, "srot_gap_async: NULL argument");
    // device memory is written by the final-sum kernel itself; host memory
    // gets a copy
    hipPointerAttribute_t at{};
    int dev = -1;
    const bool on_device = hipPointerGetAttributes(&at, out5) == hipSuccess && at.type == hipMemoryTypeDevice &&
                           hipGetDevice(&dev) == hipSuccess && at.device == dev;
    (void)hipGetLastError();  // a host pointer unknown to HIP is not an error here
    SROT_HIP(srot::launch_gap(h->P, h->S, h->stream, on_device ? out5 : nullptr));
    if (!on_device)
        SROT_HIP(hipMemcpyAsync(out5, h->S.scalars, sizeof(double) * 5, hipMemcpyDefault, h->stream));
    return SROT_OK;
}

int srot_solve(srot_handle *h, double *out3, int64_t *passes)
{
    if (!h || !out3 || !passes) return fail(SROT_EINVAL, "srot_solve: NULL argument");
    const int64_t m = h->P.m;
    return solve_on_device(
        h, out3, passes, [&](int64_t, const srot::ProblemView &Ps) { return run_steps(h, m, nullptr, nullptr, &Ps); },
        [](int64_t, const srot::ProblemView &, bool) { return (int)SROT_OK; });
}

int srot_get_plan(srot_handle *h, double *T_out, double *r_out)
{
    if (!h) return fail(SROT_EINVAL, "srot_get_plan: NULL handle");
    if (T_out)
        SROT_HIP(hipMemcpyAsync(T_out, h->S.T, sizeof(double) * (size_t)h->P.m * (size_t)h->P.n,
                                hipMemcpyDeviceToDevice, h->stream));
    if (r_out)
        SROT_HIP(hipMemcpyAsync(r_out, h->S.r, sizeof(double) * (size_t)h->P.n, hipMemcpyDeviceToDevice, h->stream));
    return SROT_OK;
}

int srot_get_plan_csr(srot_handle *h, int32_t *row_ptr, int32_t *col, double *val, int64_t cap, int64_t *nnz)
{
    if (!h || !row_ptr || !nnz) return fail(SROT_EINVAL, "srot_get_plan_csr: NULL argument");
    if (cap < 0) return fail(SROT_EINVAL, "srot_get_plan_csr: cap < 0");
    if (cap > 0 && (!col || !val)) return fail(SROT_EINVAL, "srot_get_plan_csr: col or val NULL with cap > 0");
    *nnz = 0;
    SROT_HIP(srot::launch_plan_count(h->P, h->S, row_ptr, h->stream));
    int32_t total = 0;
    SROT_HIP(hipMemcpyAsync(&total, row_ptr + h->P.m, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    SROT_HIP(hipStreamSynchronize(h->stream));
    if (total < 0) return fail(SROT_EINVAL, "srot_get_plan_csr: more than 2^31 - 1 plan entries");
    *nnz = total;
    if (total > cap)
        return fail(SROT_ECAPACITY, "srot_get_plan_csr: %d entries, the buffers hold %lld", total, (long long)cap);
    if (total > 0) SROT_HIP(srot::launch_plan_fill(h->P, h->S, row_ptr, col, val, h->stream));
    return SROT_OK;
}

int srot_get_state(srot_handle *h, int64_t *k)
{
    if (!h || !k) return fail(SROT_EINVAL, "srot_get_state: NULL argument");
    *k = h->k;
    return SROT_OK;
}

int srot_chain_stats(srot_handle *h, int64_t *out4)
{
    if (!h || !out4) return fail(SROT_EINVAL, "srot_chain_stats: NULL argument");
    SROT_HIP(hipMemcpyAsync(out4, h->S.slow_steps, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, h->stream));
    SROT_HIP(hipStreamSynchronize(h->stream));
    return SROT_OK;
}

int srot_set_state(srot_handle *h, const double *T_in, const double *r_in, int64_t k)
{
    if (!h || !T_in || k < 0) return fail(SROT_EINVAL, "srot_set_state: bad argument");
    SROT_HIP(hipMemcpyAsync(h->S.T, T_in, sizeof(double) * (size_t)h->P.m * (size_t)h->P.n,
                            hipMemcpyDeviceToDevice, h->stream));
    if (r_in)
        SROT_HIP(hipMemcpyAsync(h->S.r, r_in, sizeof(double) * (size_t)h->P.n,
                                hipMemcpyDeviceToDevice, h->stream));
    else
        SROT_HIP(srot::launch_residual(h->P, h->S, h->stream));
    SROT_HIP(srot::launch_mask_build(h->P, h->S, h->stream));
    // a consistent state again: a team-chain failure recorded before is over
    SROT_HIP(hipMemsetAsync(h->S.flags + 6, 0, sizeof(int32_t), h->stream));
    h->k = k;
    return SROT_OK;
}

int srot_backward(srot_handle *h, double grad_out, void *dC, float *dX, float *dY, double *da,
                  double *db)
{
    if (!h) return fail(SROT_EINVAL, "srot_backward: NULL handle");
    if (!isfinite(grad_out)) return fail(SROT_EINVAL, "srot_backward: grad_out is not finite");
    if (dC && h->P.cost == SROT_COST_SQEUCLID)
        return fail(SROT_EINVAL, "srot_backward: dC needs a stored cost (the fused cost has no C)");
    if ((dX || dY) && (!h->P.X || !h->P.Y))
        return fail(SROT_EINVAL, "srot_backward: dX and dY need the points X and Y given to srot_init");
    if (da) SROT_HIP(srot::launch_gap(h->P, h->S, h->stream));  // row minima of the gradient
    SROT_HIP(srot::launch_adjoint(h->P, h->S, grad_out, dC, dX, dY, da, db, h->stream));
    return SROT_OK;
}

int srot_backward_noalloc(srot_handle *h, double grad_out, void *dC, float *dX, float *dY, double *da,
                          double *db)
{
    if (!h) return fail(SROT_EINVAL, "srot_backward_noalloc: NULL handle");
    if (!isfinite(grad_out)) return fail(SROT_EINVAL, "srot_backward_noalloc: grad_out is not finite");
    if (dC && h->P.cost == SROT_COST_SQEUCLID)
        return fail(SROT_EINVAL, "srot_backward_noalloc: dC needs a stored cost (the fused cost has no C)");
    if ((dX || dY) && (!h->P.X || !h->P.Y))
        return fail(SROT_EINVAL, "srot_backward_noalloc: dX and dY need the points X and Y given to srot_init");
    if (!h->scratch)
        return fail(SROT_EHIP, "srot_backward_noalloc: no static scratch on this device: %s",
                    hipGetErrorString(h->scratch_err));
    // layout: 64 control words (the gap sweep's arrival counter at [4]),
    // 8 final sums, the gap sweep's per-workgroup partial sums (da), the
    // per-row-slice column sums of dY
    constexpr size_t kCtl = 0, kSums = 256, kPart = 512;
    const size_t part_bytes = da ? sizeof(double) * 8 * (size_t)h->S.gap_blocks : 0;
    const size_t adj_off = align_up(kPart + part_bytes);
    const size_t adj_bytes = dY ? sizeof(double) * srot::adjoint_part_doubles(h->P, h->S.own) : 0;
    if (adj_off + adj_bytes > (size_t)SROT_NOALLOC_SCRATCH_BYTES)
        return fail(SROT_EINVAL,
                    "srot_backward_noalloc: needs %zu bytes of scratch (m=%d, n=%d), above its static %zu; "
                    "use srot_backward", adj_off + adj_bytes, h->P.m, h->P.n, (size_t)SROT_NOALLOC_SCRATCH_BYTES);
    srot::DeviceState S = h->S;
    char *base = (char *)h->scratch;
    S.flags = (int32_t *)(base + kCtl);
    S.scalars = (double *)(base + kSums);
    S.partials = (double *)(base + kPart);
    S.adj_part = (double *)(base + adj_off);
    if (da) {
        // the row minima of the gradient, as srot_backward
        hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1), dim3(64), 0, h->stream, S.flags);
        SROT_HIP(hipGetLastError());
        SROT_HIP(srot::launch_gap(h->P, S, h->stream));
    }
    SROT_HIP(srot::launch_adjoint(h->P, S, grad_out, dC, dX, dY, da, db, h->stream));
    return SROT_OK;
}

int srot_fw_steps(srot_handle *h, int64_t iters, double *trace_gamma)
{
    if (!h) return fail(SROT_EINVAL, "srot_fw_steps: NULL handle");
    if (iters < 0) return fail(SROT_EINVAL, "srot_fw_steps: iters < 0");
    if (iters == 0) return SROT_OK;
    SROT_HIP(srot::launch_fw_reset(h->P, h->S, h->stream));
    for (int64_t it = 0; it < iters; ++it) {
        const srot::FwSweep f = srot::fw_sweep_args(h->S, -1.0, h->opt.step_rule, 1, h->fw_k + it,
                                                    trace_gamma ? trace_gamma + it : nullptr);
        SROT_HIP(srot::launch_fw_iteration(h->P, h->S, f, h->stream));
    }
    SROT_HIP(srot::launch_fw_flush(h->P, h->S, h->stream));
    h->fw_k += iters;
    return SROT_OK;
}

// Iterations are queued in batches; each sweep checks the device's done
// flag, and the host reads the run state of batch b (written to pinned
// memory by the batch's last step kernel) only after batch b + 1 is queued,
// so the GPU does not wait for the host between batches.
constexpr int64_t kFwBatch = 4;

int srot_fw_solve(srot_handle *h, double *out3, int64_t *iters)
{
    if (!h || !out3 || !iters) return fail(SROT_EINVAL, "srot_fw_solve: NULL argument");
    *iters = 0;
    int rc = ensure_readback(h);
    if (rc != SROT_OK) return rc;
    const int64_t maxit = h->opt.max_passes;
    SROT_HIP(srot::launch_fw_reset(h->P, h->S, h->stream));
    // sweeps i0 .. i1 - 1 and the readback of the run state into slot q; the
    // sweep numbered maxit only measures
    // (the batch's last step kernel writes the run state and the sums into
    // the pinned slot itself: no copy per batch)
    auto queue = [&](int64_t i0, int64_t i1, int q) -> int {
        for (int64_t it = i0; it < i1; ++it) {
            srot::FwSweep f = srot::fw_sweep_args(h->S, h->opt.eps, h->opt.step_rule, it < maxit ? 1 : 0,
                                                  h->fw_k + it, nullptr);
            if (it == i1 - 1) {
                f.rb_words = h->rb[q].words;
                f.rb_sums = h->rb[q].sums;
            }
            SROT_HIP(srot::launch_fw_iteration(h->P, h->S, f, h->stream));
        }
        SROT_HIP(hipEventRecord(h->rb_ev[q], h->stream));
        return SROT_OK;
    };
    const int64_t last = maxit + 1;  // sweeps 0 .. maxit
    int64_t i1 = std::min(last, kFwBatch);
    rc = queue(0, i1, 0);
    if (rc != SROT_OK) return rc;
    const srot_handle::Readback *R = nullptr;
    for (int64_t b = 0;; ++b) {
        const int q = (int)(b & 1);
        const int64_t n0 = i1, n1 = std::min(last, i1 + kFwBatch);
        if (n0 < last) {
            rc = queue(n0, n1, 1 - q);
            if (rc != SROT_OK) return rc;
        }
        SROT_HIP(hipEventSynchronize(h->rb_ev[q]));
        R = &h->rb[q];
        if (R->words[0] || n0 >= last) break;  // done, or every sweep queued and read
        i1 = n1;
    }
    SROT_HIP(srot::launch_fw_flush(h->P, h->S, h->stream));
    // [0] done, [1] step pending, [2] steps taken
    *iters = R->words[2];
    h->fw_k += R->words[2];
    out3[0] = R->sums[0]; out3[1] = R->sums[1]; out3[2] = R->sums[2];
    return R->words[0] ? SROT_OK : SROT_NOT_CONVERGED;
}

int srot_step_variant(srot_handle *h, int variant, int64_t nsteps, const int32_t *idx, int32_t *trace_j,
                      int32_t *trace_away, double *trace_gamma)
{
    int rc = variant_ok(h, variant, "srot_step_variant");
    if (rc != SROT_OK) return rc;
    if (nsteps < 0) return fail(SROT_EINVAL, "srot_step_variant: nsteps < 0");
    if (nsteps == 0) return SROT_OK;
    const int pairwise = variant == SROT_STEP_PAIRWISE;
    if (!idx) return run_variant_steps(h, pairwise, nsteps, trace_j, trace_away, trace_gamma);
    int32_t flag = 0;
    SROT_HIP(hipMemsetAsync(h->S.flags, 0, sizeof(int32_t), h->stream));
    SROT_HIP(srot::launch_check_indices(idx, nsteps, h->P.m, h->S.flags, h->stream));
    SROT_HIP(hipMemcpyAsync(&flag, h->S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    SROT_HIP(hipStreamSynchronize(h->stream));
    if (flag & 2) return fail(SROT_EINVAL, "srot_step_variant: block index outside [0, m)");
    SROT_HIP(srot::launch_active_steps(h->P, h->S, pairwise, idx, nsteps, trace_j, trace_away, trace_gamma,
                                       h->stream));
    h->k += nsteps;
    return SROT_OK;
}

int srot_solve_variant(srot_handle *h, int variant, double *out3, int64_t *passes)
{
    int rc = variant_ok(h, variant, "srot_solve_variant");
    if (rc != SROT_OK) return rc;
    if (!out3 || !passes) return fail(SROT_EINVAL, "srot_solve_variant: NULL argument");
    const int64_t m = h->P.m;
    const int pairwise = variant == SROT_STEP_PAIRWISE;
    return solve_on_device(
        h, out3, passes,
        [&](int64_t, const srot::ProblemView &Ps) {
            return run_variant_steps(h, pairwise, m, nullptr, nullptr, nullptr, &Ps);
        },
        [](int64_t, const srot::ProblemView &, bool) { return (int)SROT_OK; });
}

int srot_ga_reset(srot_handle *h, double init)
{
    int rc = ga_ok(h, "srot_ga_reset");
    if (rc != SROT_OK) return rc;
    if (!(init > 0.0) || !isfinite(init * (double)h->P.m))
        return fail(SROT_EINVAL, "srot_ga_reset: init must be positive with m * init finite");
    SROT_HIP(srot::launch_ga_fill(h->P, h->S, nullptr, init, h->stream));
    return SROT_OK;
}

int srot_ga_refresh(srot_handle *h)
{
    int rc = ga_ok(h, "srot_ga_refresh");
    if (rc != SROT_OK) return rc;
    SROT_HIP(srot::launch_gap(h->P, h->S, h->stream));
    SROT_HIP(srot::launch_ga_fill(h->P, h->S, h->S.row_g, 0.0, h->stream));
    return SROT_OK;
}

int srot_ga_weights(srot_handle *h, double *W_out)
{
    if (!h || !W_out) return fail(SROT_EINVAL, "srot_ga_weights: NULL argument");
    SROT_HIP(hipMemcpyAsync(W_out, h->S.ga_w, sizeof(double) * (size_t)h->P.m, hipMemcpyDeviceToDevice, h->stream));
    return SROT_OK;
}

int srot_step_ga(srot_handle *h, int64_t nsteps, const double *u, int32_t *trace_i, int32_t *trace_j,
                 double *trace_gamma, double *trace_g)
{
    int rc = ga_ok(h, "srot_step_ga");
    if (rc != SROT_OK) return rc;
    if (nsteps < 0) return fail(SROT_EINVAL, "srot_step_ga: nsteps < 0");
    if (nsteps == 0) return SROT_OK;
    SROT_HIP(srot::launch_ga_steps(h->P, h->S, u, h->opt.seed, h->k, nsteps, h->opt.step_rule, trace_i, trace_j,
                                   trace_gamma, trace_g, h->stream));
    h->k += nsteps;
    return SROT_OK;
}

int srot_solve_ga(srot_handle *h, double init, int64_t period, double *out3, int64_t *passes)
{
    int rc = ga_ok(h, "srot_solve_ga");
    if (rc != SROT_OK) return rc;
    if (!out3 || !passes) return fail(SROT_EINVAL, "srot_solve_ga: NULL argument");
    if (period < 1) return fail(SROT_EINVAL, "srot_solve_ga: period must be >= 1");
    rc = srot_ga_reset(h, init > 0.0 ? init : SROT_GA_INIT);
    if (rc != SROT_OK) return rc;
    const int64_t m = h->P.m;
    return solve_on_device(
        h, out3, passes,
        [&](int64_t, const srot::ProblemView &Ps) {
            SROT_HIP(srot::launch_ga_steps(Ps, h->S, nullptr, h->opt.seed, h->k, m, h->opt.step_rule, nullptr,
                                           nullptr, nullptr, nullptr, h->stream));
            h->k += m;
            return (int)SROT_OK;
        },
        [&](int64_t p, const srot::ProblemView &Ps, bool swept) {
            // global update of the stored block gaps from a sweep (Alg. A.4)
            if ((p + 1) % period == 0) {
                if (!swept) SROT_HIP(srot::launch_gap(Ps, h->S, h->stream));
                SROT_HIP(srot::launch_ga_fill(Ps, h->S, h->S.row_g, 0.0, h->stream));
            }
            return (int)SROT_OK;
        });
}

int srot_barycentric(srot_handle *h, float *Xhat)
{
    if (!h || !Xhat) return fail(SROT_EINVAL, "srot_barycentric: NULL argument");
    if (!h->P.X || !h->P.Y) return fail(SROT_EINVAL, "srot_barycentric: needs the points X and Y given to srot_init");
    SROT_HIP(srot::launch_barycentric(h->P, h->S, Xhat, h->stream));
    return SROT_OK;
}

void srot_destroy(srot_handle *h)
{
    if (!h) return;
    if (h->rb) {
        (void)hipStreamSynchronize(h->stream);  // no readback copy still on its way
        (void)hipHostFree(h->rb);
        for (hipEvent_t e : h->rb_ev) (void)hipEventDestroy(e);
    }
    free(h);
}

const char *srot_strerror(int status)
{
    switch (status) {
    case SROT_OK: return "ok";
    case SROT_NOT_CONVERGED: return "not converged within max_passes";
    case SROT_EINVAL: return "invalid argument";
    case SROT_ENOMEM: return "workspace too small";
    case SROT_ENONFINITE: return "non-finite or negative input";
    case SROT_EHIP: return "HIP runtime error";
    case SROT_ECAPACITY: return "output buffer too small";
    default: return "unknown status";
    }
}

const char *srot_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
