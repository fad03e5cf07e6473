// Device-side building blocks shared by the single-problem kernels
// (srot_kernels.hip) and the batched solver (srot_batched.hip): wave and
// workgroup reductions, raw buffer access, the column ownership, the BCFW
// block-step chain (Alg. 1) as device functions, and the Philox4x64-10
// block-index stream.  The design of the chain is described above RowSlot.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/srot.h"
#include "srot_internal.h"

namespace srot {

__device__ __forceinline__ double sqdist(float x0, float x1, float x2, float y0, float y1, float y2)
{
    const double d0 = (double)x0 - (double)y0;
    const double d1 = (double)x1 - (double)y1;
    const double d2 = (double)x2 - (double)y2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

// ---------------------------------------------------------------------------
// Wave and workgroup reductions.
//
// Inside a wave: four DPP exchanges (quad xor 1, quad xor 2, half-row mirror,
// row mirror) give every lane of a 16-lane row the row's result, then the
// four row results are read with v_readlane and combined in row order.  No
// LDS traffic, so these never wait behind outstanding LDS or scalar loads.
// Across waves: one LDS slot per wave, one barrier, partials combined in wave
// order.  Every thread ends with the same bits.  Callers pass a two-slot LDS
// buffer indexed by step parity, so a slot is rewritten only after a later
// barrier.  All lanes of the workgroup must be active.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const int lo = dpp_i32<CTRL>((int)(unsigned)u);
    const int hi = dpp_i32<CTRL>((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

constexpr int DPP_QUAD_XOR1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within 16

// LMO: smallest gradient value, ties to the lowest column index
// (eq. SemiRelaxedSubproblemImplement).
__device__ __forceinline__ void argmin_merge(double &v, int &j, double ov, int oj)
{
    const bool take = (ov < v) || (ov == v && oj < j);
    v = take ? ov : v;
    j = take ? oj : j;
}

template <int CTRL>
__device__ __forceinline__ void argmin_dpp(double &v, int &j)
{
    argmin_merge(v, j, dpp_f64<CTRL>(v), dpp_i32<CTRL>(j));
}

__device__ __forceinline__ void wave_argmin(double &v, int &j)
{
    argmin_dpp<DPP_QUAD_XOR1>(v, j);
    argmin_dpp<DPP_QUAD_XOR2>(v, j);
    argmin_dpp<DPP_HALF_MIRROR>(v, j);
    argmin_dpp<DPP_MIRROR>(v, j);
    double rv = readlane_f64(v, 0);
    int rj = __builtin_amdgcn_readlane(j, 0);
#pragma unroll
    for (int row = 1; row < 4; ++row)
        argmin_merge(rv, rj, readlane_f64(v, 16 * row), __builtin_amdgcn_readlane(j, 16 * row));
    v = rv;
    j = rj;
}

template <int NW>
__device__ __forceinline__ void block_argmin(double &v, int &j, double *sv, int *sj)
{
    wave_argmin(v, j);
    if (NW == 1) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sv[wid] = v; sj[wid] = j; }
    __syncthreads();
    v = sv[0]; j = sj[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) argmin_merge(v, j, sv[k], sj[k]);
}

template <int K>
__device__ __forceinline__ void wave_sum(double (&x)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_f64<DPP_QUAD_XOR1>(x[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_f64<DPP_QUAD_XOR2>(x[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_f64<DPP_HALF_MIRROR>(x[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_f64<DPP_MIRROR>(x[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = readlane_f64(x[k], 0);
        s += readlane_f64(x[k], 16);
        s += readlane_f64(x[k], 32);
        s += readlane_f64(x[k], 48);
        x[k] = s;
    }
}

// Sum of K doubles.  Waves in which every lane holds zeros skip the exchange
// (their partial is exactly zero either way).
template <int NW, int K>
__device__ __forceinline__ void block_sum(double (&x)[K], double (*sh)[K])
{
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) any |= (x[k] != 0.0);
    if (__any(any)) wave_sum<K>(x);
    if (NW == 1) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[wid][k] = x[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = sh[0][k];
#pragma unroll
        for (int q = 1; q < NW; ++q) s += sh[q][k];
        x[k] = s;
    }
}

// Waits for every outstanding vector-memory operation of the wave.  Ending a
// rarely taken branch that touches memory this way lets the compiler keep
// exact wait counts for the prefetched data on the common path.
__device__ __forceinline__ void drain_memory()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15) on gfx9
}

// Copies a wave-uniform value into a vector register, so that loads addressed
// by it are vector loads (counted by vmcnt).  Scalar loads share their wait
// counter with LDS traffic, and a scalar miss on a random row's metadata
// would stall every reduction behind it.
__device__ __forceinline__ int in_vgpr(int x)
{
    int y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// Step size of Alg. 1: decay 2m/(k+2m), or the exact line search
// (eq. SemiRelaxedBCFWStep) restricted to [0, 1].  With s_i = a_i e_j*:
//   num = <t_i - s_i, grad_i f> = sum_j t_j (v_j - G)   (row sums = a_i)
//   den = w ||t_i - s_i||^2     = w (sum_{j != j*} t_j^2 + (t_j* - a_i)^2)
// both free of cancellation; with a vanishing denominator the objective is
// linear along the segment.
__device__ __forceinline__ double step_size(int rule, int64_t k, int32_t m, double w, double num,
                                            double q_off, double tstar, double ai)
{
    if (rule == SROT_DEC) return (2.0 * (double)m) / ((double)k + 2.0 * (double)m);
    const double dt = tstar - ai;
    const double den = w * (q_off + dt * dt);
    if (!(num > 0.0)) return 0.0;
    if (den == 0.0 || num >= den) return 1.0;
    return num / den;
}

// ---------------------------------------------------------------------------
// Raw buffer access.  A row of T (or a mask row) is addressed through a
// buffer resource whose range is that row; an offset of 0x80000000 lies
// outside every range, so a load there returns 0 and a store there is
// dropped without touching memory.  This lets each step issue a fixed,
// branch-free sequence of loads and stores (predication by offset), which
// keeps the compiler's count of outstanding memory operations exact: the
// prefetched rows are then waited on individually instead of by a full
// drain of the memory queue.
// ---------------------------------------------------------------------------
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9-family raw buffer

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kRawBufferWord3);
}
__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_store_f64(double v, __amdgpu_buffer_rsrc_t rs, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store_u32(unsigned v, __amdgpu_buffer_rsrc_t rs, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, (int)off, 0, 0);
}

// ---------------------------------------------------------------------------
// Column ownership (also used by the gap sweep and the mask builder): thread
// tid owns the columns j = ((u / VEC) * NT + tid) * VEC + u % VEC, u < CPT:
// groups of VEC adjacent columns, strided by NT groups.  A wave then reads a
// cost row with fully coalesced 16-byte loads, and bit u of the thread's mask
// word marks column j in the support of the row.
// ---------------------------------------------------------------------------
template <int NT, int VEC>
__device__ __forceinline__ int owned_col(int u, int tid)
{
    return ((u / VEC) * NT + tid) * VEC + (u % VEC);
}

// Loads this thread's CPT entries of a cost row (clamped to valid memory;
// entries beyond column n - 1 are garbage and must be masked by the caller).
template <int NT, int CPT, int VEC, typename CT>
__device__ __forceinline__ void load_cost_row(const CT *__restrict__ row, int n, int tid, CT (&c)[CPT])
{
    if constexpr (VEC == 1) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = u * NT + tid;
            c[u] = row[j < n ? j : n - 1];
        }
    } else {
        // 16-byte vectors: VEC = 16 / sizeof(CT); n % VEC == 0, rows 16-byte aligned
        constexpr int G = CPT / VEC;
        const int ng = n / VEC;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int gi = g * NT + tid;
            const int gc = gi < ng ? gi : ng - 1;
            if constexpr (sizeof(CT) == 4) {
                const float4 v = reinterpret_cast<const float4 *>(row)[gc];
                c[g * 4 + 0] = v.x; c[g * 4 + 1] = v.y; c[g * 4 + 2] = v.z; c[g * 4 + 3] = v.w;
            } else {
                const double2 v = reinterpret_cast<const double2 *>(row)[gc];
                c[g * 2 + 0] = v.x; c[g * 2 + 1] = v.y;
            }
        }
    }
}

// Full FW's step on one row (Alg. A.1): t_ij <- (1 - gamma) t_ij +
// gamma a_i [j == js] on the row's support and at its vertex js, with the
// support masks kept; lanes lane0, lane0 + nl, ... of the caller take the
// row's mask slots.  Used lazily by the sweep that follows the step and by
// the flush at the end of a run.
__device__ __forceinline__ void fw_apply_row(int i, int n, double gamma, double ai, int js, const Ownership &own,
                                             double *__restrict__ T, uint32_t *__restrict__ M, int lane0, int nl)
{
    const int slots = own.words * own.nt;
    const size_t base = (size_t)i * (size_t)n;
    const double gadd = gamma * ai;
    const int jg = js / own.vec;
    const int ts_star = jg % own.nt;
    const int u_star = (jg / own.nt) * own.vec + (js % own.vec);
    constexpr int AW = 8;  // mask words requested at once per lane
    for (int s0 = lane0; s0 < slots; s0 += nl * AW) {
        uint32_t mkv[AW];
#pragma unroll
        for (int q = 0; q < AW; ++q) {
            const int s = s0 + q * nl;
            mkv[q] = (s < slots) ? M[(size_t)i * slots + s] : 0u;
        }
#pragma unroll
        for (int q = 0; q < AW; ++q) {
            const int s = s0 + q * nl;
            if (s >= slots) break;
            const int wd = s / own.nt, ts = s - wd * own.nt;
            const uint32_t mk = mkv[q];
            uint32_t todo = mk, nm = mk;
            if (ts == ts_star && (u_star >> 5) == wd) todo |= 1u << (u_star & 31);
            while (todo) {
                const int bt = __ffs(todo) - 1;
                todo &= todo - 1u;
                const int u = wd * 32 + bt;
                const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                const bool on = (mk >> bt) & 1u;
                const double t = on ? T[base + j] : 0.0;
                const double tn = (1.0 - gamma) * t + ((j == js) ? gadd : 0.0);
                if (tn != t || !on) T[base + j] = tn;
                nm = (tn != 0.0) ? (nm | (1u << bt)) : (nm & ~(1u << bt));
            }
            if (nm != mk) M[(size_t)i * slots + s] = nm;
        }
    }
}

// (1 - gamma) t + gamma * add: the block update of Alg. 1 for one entry, one
// expression shared by every code path so that all paths round alike.
__device__ __forceinline__ double blend(double t, double gamma, double add)
{
    return (1.0 - gamma) * t + add;
}

// ---------------------------------------------------------------------------
// Block-step chain for rows of at most NT * CPT columns (CPT <= 32; VEC > 1
// needs n % VEC == 0 and 16-byte aligned cost rows), in two kernels.
//
// chain_kernel keeps the per-column work of a step to the gradient entry and
// the LMO argmin; everything else touches only the support of the row:
//   * r lives in LDS in ownership-major order (entry (u, tid) for column
//     j(u)); only its owner thread reads or writes an entry, so no barrier
//     guards it, and the few support entries can be indexed dynamically.
//   * the support ("atoms") of row i in a thread's columns: the entries at
//     the (at most) KA lowest bits of its mask word, requested two steps
//     ahead together with their cost entries.
//   * per step one workgroup exchange: each wave reduces its argmin and,
//     relative to its own minimum, its line-search partial sums; the waves'
//     partials are merged in wave order with cancellation-free formulas.
// Every memory operation in the steady-state loop is unconditional (absent
// slots point out of range), which keeps the compiler's count of outstanding
// vector-memory operations exact, so the prefetched rows (DA ahead) and
// atoms (2 ahead) are waited on individually.  A row updated after its data
// was requested is patched from registers.  If a thread's row holds more
// than KA atoms (rare), or once the last full group of DA steps is done,
// chain_fast returns the step it reached.
//
// chain_tail takes steps one at a time with plain loads of every support
// entry (no prefetch, any support size); chain_run alternates the two.
// ---------------------------------------------------------------------------
template <int CPT, typename CT>
struct RowSlot {
    int i;
    double a;
    uint32_t mk;
    CT c[CPT];
    float x[3];
};

constexpr int KA = 2;        // atoms per (row, thread) handled by the prefetching chain
constexpr int CHAIN_DA = 4;  // rows requested ahead (cost row, mask, a_i)

template <typename CT>
struct AtomSlot {
    double t[KA];  // plan entries at the KA lowest mask bits (0 where absent)
    CT c[KA];      // their cost entries (stored cost)
    float y[KA][3];  // their target points (fused cost)
    int q[KA];     // local column indices, -1 where absent
    uint32_t mk;   // the mask the atoms were read with
};

// Local column indices of the KA lowest set bits of mk (-1 where absent).
__device__ __forceinline__ void low_bits(uint32_t mk, int (&q)[KA])
{
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        q[k] = mk ? __ffs(mk) - 1 : -1;
        mk &= mk - 1u;
    }
}

// One wave's share of a step: its LMO candidate (v, j) -- the smallest
// gradient entry of its columns, lowest index on ties -- with, over the
// support entries t of its columns,
//   P = sum t (v_col - v),  Q = sum of t^2 off column j,  tj = t at j,
//   Ts = sum t,  and a flag (some thread has more atoms than the kernel reads).
struct WavePart {
    double v, P, Q, tj, Ts;
    int j, more;
};

// Cancellation-free merge: moving the minimum down from v_A to v adds
// (v_A - v) * Ts_A to P_A; the loser's entry at its own argmin joins Q.
__device__ __forceinline__ WavePart wave_part_merge(const WavePart &A, const WavePart &B)
{
    const bool bw = (B.v < A.v) || (B.v == A.v && B.j < A.j);
    const WavePart &W = bw ? B : A;
    const WavePart &L = bw ? A : B;
    WavePart o;
    o.v = W.v; o.j = W.j; o.tj = W.tj;
    o.Q = (A.Q + B.Q) + L.tj * L.tj;
    const double pa = (A.Ts != 0.0) ? (A.v - W.v) * A.Ts : 0.0;
    const double pb = (B.Ts != 0.0) ? (B.v - W.v) * B.Ts : 0.0;
    o.P = (A.P + B.P) + (pa + pb);
    o.Ts = A.Ts + B.Ts;
    o.more = A.more | B.more;
    return o;
}

// Wave minimum of v (DPP within rows of 16, then the four row results).
__device__ __forceinline__ double wave_min(double v)
{
    v = fmin(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmin(v, dpp_f64<DPP_QUAD_XOR2>(v));
    v = fmin(v, dpp_f64<DPP_HALF_MIRROR>(v));
    v = fmin(v, dpp_f64<DPP_MIRROR>(v));
    double m = readlane_f64(v, 0);
    m = fmin(m, readlane_f64(v, 16));
    m = fmin(m, readlane_f64(v, 32));
    m = fmin(m, readlane_f64(v, 48));
    return m;
}

template <int NT, int CPT, int VEC, int COST, bool TRACE>
__device__ __forceinline__ int64_t chain_fast(const ProblemView &P, double *__restrict__ T,
                                              double *__restrict__ rg, uint32_t *__restrict__ M,
                                              const int32_t *__restrict__ idx, int64_t k0,
                                              int64_t nsteps, int rule,
                                              int32_t *__restrict__ trace_j,
                                              double *__restrict__ trace_gamma)
{
    static_assert(CPT <= 32 && CPT % VEC == 0 && CPT % 2 == 0, "one mask word per thread");
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NW = NT / 64;
    constexpr int DA = CHAIN_DA;
    __shared__ double r_lds[CPT * NT];      // r, entry (u, tid) at ((u/2)*NT + tid)*2 + u%2
    __shared__ WavePart s_part[2][NW];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    const float4 *__restrict__ Y4 = P.Y4;
    const unsigned row_bytes = (unsigned)n * 8u;
    const int64_t nfull = nsteps - nsteps % DA;
    auto r_at = [&](int u) -> int { return ((u >> 1) * NT + tid) * 2 + (u & 1); };

    bool full = true;  // every column this thread owns is a real column
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        r_lds[r_at(u)] = (j < n) ? rg[j] : 0.0;
        full &= (j < n);
    }
    float y0[CPT], y1[CPT], y2[CPT];
    if constexpr (FUSED) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            const float4 yv = Y4[j < n ? j : n - 1];
            y0[u] = yv.x; y1[u] = yv.y; y2[u] = yv.z;
        }
    }

    RowSlot<CPT, CT> ring[DA];
    AtomSlot<CT> at[2];

    // row i's a_i, this thread's mask word and cost entries (vector loads:
    // i is held in a vector register)
    auto issue_row = [&](RowSlot<CPT, CT> &S, int i) {
        S.i = i;
        S.a = P.a[i];
        S.mk = M[(size_t)i * NT + tid];
        if constexpr (FUSED) {
            S.x[0] = P.X[3 * i + 0]; S.x[1] = P.X[3 * i + 1]; S.x[2] = P.X[3 * i + 2];
        } else {
            load_cost_row<NT, CPT, VEC, CT>(C + (size_t)i * (size_t)n, n, tid, S.c);
        }
    };
    // plan and cost entries at the KA lowest bits of mk in row i
    auto issue_atoms = [&](AtomSlot<CT> &A, int i, uint32_t mk) {
        const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + (size_t)i * (size_t)n, row_bytes);
        A.mk = mk;
        low_bits(mk, A.q);
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const unsigned col = A.q[k] >= 0 ? (unsigned)owned_col<NT, VEC>(A.q[k], tid) : 0u;
            A.t[k] = buf_load_f64(rt, A.q[k] >= 0 ? col * 8u : kOOB);
            if constexpr (FUSED) {
                const float4 yv = Y4[col];
                A.y[k][0] = yv.x;
                A.y[k][1] = yv.y;
                A.y[k][2] = yv.z;
            } else {
                const __amdgpu_buffer_rsrc_t rc = buf_rsrc(C + (size_t)i * (size_t)n, (unsigned)(n * sizeof(CT)));
                if constexpr (sizeof(CT) == 4)
                    A.c[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)(col * 4u), 0, 0));
                else
                    A.c[k] = buf_load_f64(rc, col * 8u);
            }
        }
    };

    // block indices are read 2*DA steps ahead, through vector loads
    const int32_t *__restrict__ idxv = idx + in_vgpr(0);
    const int64_t last = nsteps - 1;
    int nidx[DA];
#pragma unroll
    for (int u = 0; u < DA; ++u) {
        issue_row(ring[u], idxv[u < last ? u : last]);
        nidx[u] = idxv[DA + u < last ? DA + u : last];
    }
    issue_atoms(at[0], __builtin_amdgcn_readfirstlane(ring[0].i), ring[0].mk);
    issue_atoms(at[1], __builtin_amdgcn_readfirstlane(ring[1].i), ring[1].mk);

    // the two most recent updates (rows and new masks); F holds the atoms of
    // the latest one when the next step visits the same row
    int f1i = -1, f2i = -1;
    uint32_t f1m = 0u, f2m = 0u;
    AtomSlot<CT> F;

    int64_t done = nfull;
    for (int64_t s0 = 0; s0 < nfull; s0 += DA) {
        bool stop = false;
#pragma unroll
        for (int slot = 0; slot < DA; ++slot) {
            const int64_t s = s0 + slot;
            RowSlot<CPT, CT> &S = ring[slot];
            AtomSlot<CT> &A = (S.i == f1i) ? F : at[slot & 1];
            const int i = __builtin_amdgcn_readfirstlane(S.i);
            const double ai = S.a;
            const size_t base = (size_t)i * (size_t)n;
            const uint32_t mk = A.mk;
            const int more = __popc(mk) > KA;

            // gradient entries c_ij + w r_j (eq. RelaxedGradient) and the
            // thread's smallest one, lowest column on ties
            double vv[CPT];
            double best = INFINITY;
#pragma unroll
            for (int u = 0; u < CPT; u += 2) {
                const double2 rr = *reinterpret_cast<const double2 *>(&r_lds[r_at(u)]);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    double c;
                    if constexpr (FUSED) c = sqdist(S.x[0], S.x[1], S.x[2], y0[u + e], y1[u + e], y2[u + e]);
                    else c = (double)S.c[u + e];
                    vv[u + e] = c + w * (e ? rr.y : rr.x);
                }
            }
            if (!full) {
#pragma unroll
                for (int u = 0; u < CPT; ++u)
                    vv[u] = (owned_col<NT, VEC>(u, tid) < n) ? vv[u] : INFINITY;
            }
            {
                // pairwise tree: the minimum is exact in any order
                double t[CPT];
#pragma unroll
                for (int u = 0; u < CPT; ++u) t[u] = vv[u];
#pragma unroll
                for (int h = CPT / 2; h >= 1; h /= 2) {
#pragma unroll
                    for (int u = 0; u < h; ++u) t[u] = fmin(t[u], t[u + h]);
                }
                best = t[0];
            }
            // lowest owned column holding the minimum (owned_col grows with u)
            int bj;
            {
                unsigned bits = 0u;
#pragma unroll
                for (int u = 0; u < CPT; ++u) bits |= (vv[u] == best) ? (1u << u) : 0u;
                const int us0 = __ffs(bits) - 1;
                bj = ((us0 / VEC) * NT + tid) * VEC + (us0 % VEC);
            }

            // the wave's LMO candidate (eq. SemiRelaxedSubproblemImplement)
            WavePart wp;
            wp.v = wave_min(best);
            {
                unsigned long long hit = __ballot(best == wp.v);
                int jw = 0x7fffffff;
                while (hit) {
                    const int l = __ffsll((long long)hit) - 1;
                    hit &= hit - 1ull;
                    jw = min(jw, __builtin_amdgcn_readlane(bj, l));
                }
                wp.j = jw;
            }
            // the wave's line-search partials over its atoms, relative to wp.v
            double rk[KA], vk[KA], ck[KA];
            {
                double p = 0.0, q2 = 0.0, tj = 0.0, ts = 0.0;
#pragma unroll
                for (int k = 0; k < KA; ++k) {
                    const int qk = A.q[k] >= 0 ? A.q[k] : 0;
                    rk[k] = r_lds[((qk >> 1) * NT + tid) * 2 + (qk & 1)];
                    if constexpr (FUSED) ck[k] = sqdist(S.x[0], S.x[1], S.x[2], A.y[k][0], A.y[k][1], A.y[k][2]);
                    else ck[k] = (double)A.c[k];
                    vk[k] = ck[k] + w * rk[k];
                    const double t = A.t[k];
                    const bool at_j = A.q[k] >= 0 && owned_col<NT, VEC>(A.q[k], tid) == wp.j;
                    p += t * (vk[k] - wp.v);
                    q2 += at_j ? 0.0 : t * t;
                    tj += at_j ? t : 0.0;
                    ts += t;
                }
                unsigned long long act = __ballot((mk != 0u) && (p != 0.0 || q2 != 0.0 || tj != 0.0 || ts != 0.0));
                // each sum over the active lanes in lane order
                double sp = 0.0, sq = 0.0, sj = 0.0, ss = 0.0;
                while (act) {
                    const int l = __ffsll((long long)act) - 1;
                    act &= act - 1ull;
                    sp += readlane_f64(p, l);
                    sq += readlane_f64(q2, l);
                    sj += readlane_f64(tj, l);
                    ss += readlane_f64(ts, l);
                }
                wp.P = sp;
                wp.Q = sq;
                wp.tj = sj;
                wp.Ts = ss;
                wp.more = __any(more) ? 1 : 0;
            }
            // one exchange per step: merge the waves' partials in wave order
            WavePart gp = wp;
            if (NW > 1) {
                if (lane == 0) s_part[s & 1][wid] = wp;
                __syncthreads();
                // pairwise tree over the waves (fixed order)
                WavePart t[NW];
#pragma unroll
                for (int k = 0; k < NW; ++k) t[k] = s_part[s & 1][k];
#pragma unroll
                for (int h = 1; h < NW; h *= 2) {
#pragma unroll
                    for (int k = 0; k + h < NW; k += 2 * h) t[k] = wave_part_merge(t[k], t[k + h]);
                }
                gp = t[0];
            }
            if (gp.more) { stop = true; done = s; break; }
            const int jstar = gp.j;

            // step size of Alg. 1, then t_i <- (1 - gamma) t_i + gamma a_i e_j*
            // and r <- r + (t_i new - t_i old), on the support and at j*
            const double gamma = step_size(rule, k0 + s, m, w, gp.P, gp.Q, gp.tj, ai);
            const double gadd = gamma * ai;
            const int jg = jstar / VEC;
            const int us = ((jg % NT) == tid) ? (jg / NT) * VEC + (jstar % VEC) : -1;
            uint32_t nm = mk;
            const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + base, row_bytes);
            double tn[KA];
            bool star_in = false;
#pragma unroll
            for (int k = 0; k < KA; ++k) {
                const bool st = A.q[k] >= 0 && A.q[k] == us;
                star_in |= st;
                tn[k] = blend(A.t[k], gamma, st ? gadd : 0.0);
                const bool put = A.q[k] >= 0 && tn[k] != A.t[k];
                const int qk = A.q[k] >= 0 ? A.q[k] : 0;
                if (put) r_lds[((qk >> 1) * NT + tid) * 2 + (qk & 1)] = rk[k] + (tn[k] - A.t[k]);
                if (A.q[k] >= 0) nm = (tn[k] != 0.0) ? (nm | (1u << A.q[k])) : (nm & ~(1u << A.q[k]));
                buf_store_f64(tn[k], rt, put ? (unsigned)owned_col<NT, VEC>(qk, tid) * 8u : kOOB);
            }
            const double tsn = blend(0.0, gamma, gadd);
            const bool put_s = us >= 0 && !star_in && tsn != 0.0;
            {
                const int qs = us >= 0 ? us : 0;
                if (put_s) {
                    const int a_ = ((qs >> 1) * NT + tid) * 2 + (qs & 1);
                    r_lds[a_] = r_lds[a_] + tsn;
                    nm |= (1u << qs);
                }
                buf_store_f64(tsn, rt, put_s ? (unsigned)owned_col<NT, VEC>(qs, tid) * 8u : kOOB);
            }
            buf_store_u32(nm, buf_rsrc(M + (size_t)i * NT, NT * 4u), nm != mk ? (unsigned)tid * 4u : kOOB);
            if constexpr (TRACE) {
                // a null trace pointer gets an empty range: its stores are dropped
                const __amdgpu_buffer_rsrc_t rs_tj = buf_rsrc(trace_j, trace_j ? (unsigned)nsteps * 4u : 0u);
                const __amdgpu_buffer_rsrc_t rs_tg = buf_rsrc(trace_gamma, trace_gamma ? (unsigned)nsteps * 8u : 0u);
                buf_store_u32((unsigned)jstar, rs_tj, tid == 0 ? (unsigned)s * 4u : kOOB);
                buf_store_f64(gamma, rs_tg, tid == 0 ? (unsigned)s * 8u : kOOB);
            }

            // the next step visits this row again: hand its new atoms over
            if (ring[(slot + 1) % DA].i == i) {
                F.mk = nm;
                low_bits(nm, F.q);
#pragma unroll
                for (int k = 0; k < KA; ++k) {
                    double tv = 0.0;
                    CT cv = (CT)0;
                    float yv0 = 0.f, yv1 = 0.f, yv2 = 0.f;
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) {
                        const bool hit = A.q[kk] >= 0 && A.q[kk] == F.q[k];
                        tv = hit ? tn[kk] : tv;
                        if constexpr (FUSED) {
                            yv0 = hit ? A.y[kk][0] : yv0; yv1 = hit ? A.y[kk][1] : yv1; yv2 = hit ? A.y[kk][2] : yv2;
                        } else {
                            cv = hit ? A.c[kk] : cv;
                        }
                    }
                    if (put_s && F.q[k] == us) {
                        tv = tsn;
#pragma unroll
                        for (int u = 0; u < CPT; ++u) {
                            if constexpr (FUSED) {
                                yv0 = (u == us) ? y0[u] : yv0; yv1 = (u == us) ? y1[u] : yv1; yv2 = (u == us) ? y2[u] : yv2;
                            } else {
                                cv = (u == us) ? S.c[u] : cv;
                            }
                        }
                    }
                    F.t[k] = tv;
                    if constexpr (FUSED) { F.y[k][0] = yv0; F.y[k][1] = yv1; F.y[k][2] = yv2; }
                    else F.c[k] = cv;
                }
            }
            f2i = f1i; f2m = f1m;
            f1i = i; f1m = nm;

            // atoms of step s + 2, on its mask patched by the last two updates
            {
                RowSlot<CPT, CT> &R = ring[(slot + 2) % DA];
                const int ri = __builtin_amdgcn_readfirstlane(R.i);
                const uint32_t rmk = (ri == f1i) ? f1m : ((ri == f2i) ? f2m : R.mk);
                issue_atoms(at[slot & 1], ri, rmk);
            }
            // row of step s + DA, block index of step s + 2*DA
            issue_row(ring[slot], nidx[slot]);
            nidx[slot] = idxv[s + 2 * DA < last ? s + 2 * DA : last];
        }
        if (stop) break;
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        if (j < n) rg[j] = r_lds[r_at(u)];
    }
    return done;
}

template <int NT, int CPT, int VEC, int COST>
__device__ __forceinline__ void chain_tail(const ProblemView &P, double *__restrict__ T,
                                           double *__restrict__ rg, uint32_t *__restrict__ M,
                                           const int32_t *__restrict__ idx, int64_t k0,
                                           int64_t start, int64_t nsteps, int rule,
                                           int32_t *__restrict__ trace_j,
                                           double *__restrict__ trace_gamma)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NW = NT / 64;
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_sum[2][NW][3];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    if (start >= nsteps) return;

    double r[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        r[u] = (j < n) ? rg[j] : 0.0;
    }
    for (int64_t s = start; s < nsteps; ++s) {
        const int i = idx[s];
        const double ai = P.a[i];
        const size_t base = (size_t)i * (size_t)n;
        const uint32_t mk = M[(size_t)i * NT + tid];
        CT cv[CPT];
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (FUSED) { x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2]; }
        else load_cost_row<NT, CPT, VEC, CT>(C + base, n, tid, cv);
        double t[CPT], vv[CPT];
        double best = INFINITY;
        int bj = 0x7fffffff;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            const int jc = j < n ? j : n - 1;
            t[u] = (mk & (1u << u)) ? T[base + j] : 0.0;
            double c;
            if constexpr (FUSED) c = sqdist(x0, x1, x2, P.Y[3 * jc], P.Y[3 * jc + 1], P.Y[3 * jc + 2]);
            else c = (double)cv[u];
            vv[u] = c + w * r[u];
            const double v = (j < n) ? vv[u] : INFINITY;
            if (v < best) { best = v; bj = j; }
        }
        block_argmin<NW>(best, bj, s_v[s & 1], s_j[s & 1]);
        const double G = best;
        const int jstar = bj;
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const bool st = (owned_col<NT, VEC>(u, tid) == jstar);
            acc[0] += t[u] * (vv[u] - G);
            acc[1] += st ? 0.0 : t[u] * t[u];
            acc[2] = st ? t[u] : acc[2];
        }
        block_sum<NW, 3>(acc, s_sum[s & 1]);
        const double gamma = step_size(rule, k0 + s, m, w, acc[0], acc[1], acc[2], ai);
        const double gadd = gamma * ai;
        const int jg = jstar / VEC;
        const int us = ((jg % NT) == tid) ? (jg / NT) * VEC + (jstar % VEC) : -1;
        uint32_t nm = 0u;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const double tn = blend(t[u], gamma, (u == us) ? gadd : 0.0);
            if (tn != t[u]) T[base + owned_col<NT, VEC>(u, tid)] = tn;
            r[u] += tn - t[u];
            nm |= (tn != 0.0) ? (1u << u) : 0u;
        }
        if (nm != mk) M[(size_t)i * NT + tid] = nm;
        if (tid == 0) {
            if (trace_j) trace_j[s] = jstar;
            if (trace_gamma) trace_gamma[s] = gamma;
        }
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        if (j < n) rg[j] = r[u];
    }
}

// The block-step chain of nsteps steps: chain_fast runs whole groups of
// CHAIN_DA steps; a step it cannot take (a thread holding more than KA
// support entries of the row) and the last nsteps % CHAIN_DA steps go
// through chain_tail one at a time, after which chain_fast resumes with its
// pipeline primed afresh.  Both leave r in global memory between calls, and
// every chain_tail step ends with workgroup barriers, so the LDS of one
// chain_fast call is free before the next one starts.  Returns the number
// of steps taken by chain_tail.
template <int NT, int CPT, int VEC, int COST, bool TRACE>
__device__ __forceinline__ int64_t chain_run(const ProblemView &P, double *__restrict__ T,
                                             double *__restrict__ rg, uint32_t *__restrict__ M,
                                             const int32_t *__restrict__ idx, int64_t k0, int64_t nsteps,
                                             int rule, int32_t *__restrict__ trace_j,
                                             double *__restrict__ trace_gamma)
{
    int64_t start = 0, slow = 0;
    while (start < nsteps) {
        const int64_t rem = nsteps - start;
        int64_t end = nsteps;
        if (rem >= CHAIN_DA) {
            const int64_t done = chain_fast<NT, CPT, VEC, COST, TRACE>(
                P, T, rg, M, idx + start, k0 + start, rem, rule, TRACE ? trace_j + start : nullptr,
                TRACE ? trace_gamma + start : nullptr);
            start += done;
            // a stop: one step without prefetch; else only the remainder is left
            if (done != rem - rem % CHAIN_DA) end = start + 1;
        }
        if (start < end) {
            chain_tail<NT, CPT, VEC, COST>(P, T, rg, M, idx, k0, start, end, rule, trace_j, trace_gamma);
            slow += end - start;
            start = end;
        }
    }
    return slow;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply / xor-swap round with Weyl key schedule.  Output k of the stream
// with key (seed, 0) is lane k mod 4 of the block at counter 1 + floor(k/4)
// (the counter convention of numpy's Philox bit generator).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int rd = 0; rd < 10; ++rd) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ uint64_t philox_output(uint64_t seed, uint64_t k)
{
    uint64_t c[4] = {(k >> 2) + 1ull, 0ull, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    return c[k & 3];
}

// ---------------------------------------------------------------------------
// The final sums of a gap sweep over its nb workgroup partials (component
// c of workgroup k at partials[c * nb + k]), by a workgroup of GAP_FINAL_NT
// threads in a fixed order: thread t adds workgroups t, t + GAP_FINAL_NT,
// ... (all requested at once), then the wave (DPP), then the waves in
// order; thread 0 writes
//   out[0] = g, out[1] = f, out[2] = D, out[3] = <T,C>, out[4] = ||r||^2
// and the same into out2 when given.
// ---------------------------------------------------------------------------
constexpr int GAP_FINAL_NT = 1024;

__device__ __forceinline__ void gap_total(double w, const double *__restrict__ partials, int nb,
                                          double *__restrict__ out, double *__restrict__ out2 = nullptr)
{
    constexpr int PER = GAP_MAX_BLOCKS / GAP_FINAL_NT;  // workgroups per thread
    constexpr int NW = GAP_FINAL_NT / 64;
    __shared__ double s_red[NW * 5];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double v[PER][5];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = tid + q * GAP_FINAL_NT;
#pragma unroll
        for (int c = 0; c < 5; ++c) v[q][c] = (k < nb) ? partials[c * nb + k] : 0.0;
    }
    double f5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // a_i G_i, lin, g, ||r||^2, <b, r>
#pragma unroll
    for (int q = 0; q < PER; ++q) {
#pragma unroll
        for (int c = 0; c < 5; ++c) f5[c] += v[q][c];
    }
    wave_sum<5>(f5);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 5; ++c) s_red[wid * 5 + c] = f5[c];
    }
    __syncthreads();
    if (tid == 0) {
        double t5[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            t5[c] = s_red[c];
#pragma unroll
            for (int q = 1; q < NW; ++q) t5[c] += s_red[q * 5 + c];
        }
        const double pa = t5[0], pl = t5[1], pg = t5[2], rr = t5[3], br = t5[4];
        const double o5[5] = {pg, pl + 0.5 * w * rr, pa - w * br - 0.5 * w * rr, pl, rr};
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c] = o5[c];
        if (out2) {
#pragma unroll
            for (int c = 0; c < 5; ++c) out2[c] = o5[c];
        }
    }
}

}  // namespace srot
