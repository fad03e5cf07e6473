// Block-step chain with a screened LMO (Alg. 1, stored FP32 cost, rows of
// 513..4096 columns in the 256 x {4,8,16} x 4 column ownership).
//
// The block steps stay strictly sequential and exact; what changes is who
// does the per-column work.  One workgroup of eight waves:
//   * wave 0, the stepper, takes every block step alone: LMO over a short
//     candidate list, line-search partials over the support, step size,
//     update of t_i, r and the support masks.  No workgroup exchange.
//   * six screener waves prepare the rows ahead of the stepper: the cost
//     row, the support of the row (plan entries and cost at its nonzeros)
//     and the LMO candidates from an FP32 screen of c_ij + w r_j.
//   * wave 4 shares a SIMD with the stepper and only keeps the barriers.
// All eight waves move in lockstep phases: in phase p the stepper takes step
// p and every screener does one piece of work for a later step, then all
// meet at one barrier.  The row of step s is loaded in phase s - 7, screened
// in phases s - 3 and s - 2 (two halves of its columns) and its support
// gathered in phase s - 1.
//
// LMO screen (eq. SemiRelaxedSubproblemImplement).  Screener lane l covers
// the columns of the four owner threads l + 64 h, h < 4, and keeps its two
// smallest FP32 values u1 <= u2 of fma(w, r_j, c_ij) with the column of u1.
// tau = min over lanes of u2; the candidates are the lanes' u1 columns with
// u1 < tau -- exactly the columns whose FP32 value lies below tau, at most
// one per lane.  Every other column j satisfies, at the time the screen read
// r, c_ij + w r_j >= tau - e with e the FP32 error bound of the screen; until
// the step is taken r_j can only have dropped by the decreases of the steps
// in between: a step scales the row's entries off its vertex by 1 - gamma,
// so no r_j drops by more than gamma times the largest of them.  The stepper
// evaluates the candidates in FP64 at the current r and accepts their minimum only if
// it lies strictly below tau - e - w (sum of those decreases): then every
// other column is strictly larger, and the smallest candidate (lowest column
// on ties) is the exact lowest-index argmin of the full row.  Otherwise the
// stepper scans the whole row itself.
//
// Support.  Rows updated within the last SC_HIST steps may be read stale by
// the screeners; for those, and for rows where a screener lane holds more
// than SC_KS nonzeros, the stepper reads the support from the plan and the
// masks itself.  Global stores of step q are complete before the barrier
// that ends phase q + 1 (the stepper waits for all but its current step's
// stores there), so loads issued in phase s - 7 see every update up to step
// s - 9.
// ---------------------------------------------------------------------------
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/srot.h"
#include "srot_internal.h"
#include "srot_device.h"

namespace srot {

constexpr int SC_NW = 8;
constexpr int SC_NT = SC_NW * 64;
constexpr int SC_SLOTS = 8;    // rows in preparation (steps s .. s + 3 in use)
constexpr int SC_KS = 2;       // nonzeros per screener lane in the prepared support (two slot fields)
constexpr int SC_HIST = 8;     // a row updated within this many steps is re-read by the stepper
constexpr int SC_DECN = 3;     // steps whose residual decreases a screen may have missed
constexpr int LAG_A = 7, LAG_B1 = 3, LAG_B2 = 2, LAG_C = 1;
static_assert((LAG_A - LAG_C) % 6 == 0, "A and C of one screener share a phase");

__device__ __forceinline__ float wave_min_f32(float v)
{
    v = fminf(v, __int_as_float(dpp_i32<DPP_QUAD_XOR1>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_QUAD_XOR2>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_HALF_MIRROR>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_MIRROR>(__float_as_int(v))));
    float m = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16)));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32)));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48)));
    return m;
}

// gfx9 s_waitcnt immediates: lgkmcnt(0) with vmcnt(vm)
constexpr int waitcnt_vm_lgkm0(int vm) { return (vm & 15) | (7 << 4) | ((vm >> 4) << 14); }

// VAR = 1 / 2: the same chain takes away steps (Alg. A.2) or pairwise steps
// (Alg. A.3) instead of BCFW steps (ELS only).  The stepper then also finds
// the away vertex ja, the lowest-index argmax of c_ij + w r_j over the
// support (with the FW vertex, one wave reduction each), adds the four
// further support sums of the away direction, picks the direction and the
// step size clip(-<g, d> / (w ||d||^2), 0, gamma_max), and updates the
// support, emptying atom ja exactly when gamma reaches gamma_max.  A step
// on an away or pairwise direction lowers only t_ija, by at most t_ija: its
// entry in the screen's decrease allowance.
template <int CPT, bool TRACE, int VAR = 0>
__global__ __launch_bounds__(SC_NT) void chain_screened_kernel(ProblemView P, double *__restrict__ T,
                                                               double *__restrict__ rg,
                                                               uint32_t *__restrict__ M,
                                                               const int32_t *__restrict__ idx, int64_t k0,
                                                               int64_t nsteps, int rule,
                                                               int32_t *__restrict__ trace_j,
                                                               double *__restrict__ trace_gamma,
                                                               int32_t *__restrict__ trace_away,
                                                               int64_t *__restrict__ slow_steps, double err_c)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    static_assert(CPT == 4 || CPT == 8 || CPT == 16, "4 owner threads x CPT columns per lane");
    constexpr int NC = 256 * CPT;   // columns of the ownership (n <= NC)
    constexpr int G = CPT / 4;      // 16-byte groups per owner thread
    static_assert(VAR >= 0 && VAR <= 2, "BCFW, away or pairwise steps");
    constexpr int NST = SC_KS + 1 + 1 + (TRACE ? (VAR ? 3 : 2) : 0);  // stores issued by every step
    __shared__ __align__(16) double r64[NC];
    __shared__ __align__(16) float r32[NC];
    // a prepared row: header (row, a_i, tau, overflow flag) and, per lane,
    // 16-byte groups that the stepper reads with one instruction each:
    // {candidate column, its cost, two nonzero columns}, {their plan
    // entries}, {their costs}, {the four support-mask words}
    __shared__ __align__(16) int4 s_hdr[SC_SLOTS][2];       // {i, ovf, tau bits, -}, {a_i bits}
    __shared__ __align__(16) int4 s_g0[SC_SLOTS][64];
    __shared__ __align__(16) double2 s_g1[SC_SLOTS][64];
    __shared__ __align__(16) float2 s_g2[SC_SLOTS][64];
    __shared__ __align__(16) uint4 s_wd[SC_SLOTS][64];
    __shared__ double s_rmax[SC_NW];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const float w32 = (float)w;
    const float *__restrict__ C = (const float *)P.C;
    const unsigned row_bytes = (unsigned)n * 8u;

    double rabs = 0.0;
    for (int j = tid; j < NC; j += SC_NT) {
        const double v = j < n ? rg[j] : 0.0;
        r64[j] = v;
        r32[j] = (float)v;
        rabs = fmax(rabs, fabs(v));
    }
    {
        double x = rabs;
        x = fmax(x, dpp_f64<DPP_QUAD_XOR1>(x));
        x = fmax(x, dpp_f64<DPP_QUAD_XOR2>(x));
        x = fmax(x, dpp_f64<DPP_HALF_MIRROR>(x));
        x = fmax(x, dpp_f64<DPP_MIRROR>(x));
        x = fmax(fmax(readlane_f64(x, 0), readlane_f64(x, 16)), fmax(readlane_f64(x, 32), readlane_f64(x, 48)));
        if (lane == 0) s_rmax[wid] = x;
    }
    __syncthreads();
    // error of the FP32 screen: err_c covers the cost and the residual bound
    // known at init; the residual at launch may exceed it after a state reset
    double err = err_c;
    {
        double rm = 0.0;
#pragma unroll
        for (int k = 0; k < SC_NW; ++k) rm = fmax(rm, s_rmax[k]);
        err += 0x1.0p-20 * fabs(w) * rm;
    }

    const int32_t *__restrict__ idxv = idx + in_vgpr(0);
    const double *__restrict__ av = P.a + in_vgpr(0);

    if (wid == 0) {
        // ---- stepper state
        int hist[SC_HIST];
#pragma unroll
        for (int k = 0; k < SC_HIST; ++k) hist[k] = -1;
        double dec[SC_DECN];
#pragma unroll
        for (int k = 0; k < SC_DECN; ++k) dec[k] = 0.0;
        double wds = 0.0;  // w times the sum of dec, formed at the end of the step before
        int64_t n_fall = 0, n_slow = 0;

        for (int64_t p = -LAG_A; p < nsteps; ++p) {
            if (p >= 0) {
                // =============================== stepper: block step s = p
                const int64_t s = p;
                const int q = (int)(s & (SC_SLOTS - 1));
                const int4 h0 = s_hdr[q][0];
                const int4 h1 = s_hdr[q][1];
                const int4 g0 = s_g0[q][lane];
                const double2 g1 = s_g1[q][lane];
                const float2 g2 = s_g2[q][lane];
                const int i = __builtin_amdgcn_readfirstlane(h0.x);
                const int ovf = h0.y;
                const float tau = __int_as_float(h0.z);
                const double ai = __hiloint2double(h1.y, h1.x);
                const int cj = g0.x;
                const float cc = __int_as_float(g0.y);
                int sq[SC_KS];
                double st[SC_KS];
                float sc[SC_KS];
#pragma unroll
                for (int k = 0; k < SC_KS; ++k) {
                    sq[k] = k == 0 ? g0.z : g0.w;
                    st[k] = k == 0 ? g1.x : g1.y;
                    sc[k] = k == 0 ? g2.x : g2.y;
                }
                const uint4 wdv = s_wd[q][lane];
                bool stale = ovf != 0;
#pragma unroll
                for (int k = 0; k < SC_HIST; ++k) stale |= (hist[k] == i);

                const double rc = r64[cj >= 0 ? cj : 0];
                double sr[SC_KS];
#pragma unroll
                for (int k = 0; k < SC_KS; ++k) sr[k] = r64[sq[k] >= 0 ? sq[k] : 0];

                // away / pairwise: the away vertex over the support (this
                // lane's entries, then the wave; lowest column on ties)
                double vaw = -INFINITY;
                int jaw = 0x7fffffff;
                if constexpr (VAR != 0) {
                    auto away_take = [&](double t, double vk, int col) {
                        const bool take = t > 0.0 && (vk > vaw || (vk == vaw && col < jaw));
                        vaw = take ? vk : vaw;
                        jaw = take ? col : jaw;
                    };
                    if (!stale) {
#pragma unroll
                        for (int k = 0; k < SC_KS; ++k)
                            if (sq[k] >= 0) away_take(st[k], (double)sc[k] + w * sr[k], sq[k]);
                    } else {
                        const uint32_t *__restrict__ mrow = M + (size_t)i * 256;
                        const double *__restrict__ trow = T + (size_t)i * (size_t)n;
                        const float *__restrict__ crow = C + (size_t)i * (size_t)n;
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
                            uint32_t bits = mrow[lane + 64 * h];
                            while (bits) {
                                const int u = __ffs(bits) - 1;
                                bits &= bits - 1u;
                                const int col = owned_col<256, 4>(u, lane + 64 * h);
                                away_take(trow[col], (double)crow[col] + w * r64[col], col);
                            }
                        }
                    }
                    double nv = -vaw;
                    wave_argmin(nv, jaw);
                    vaw = -nv;
                }

                // LMO over the candidates, accepted against the screen's bound
                const double vc = cj >= 0 ? (double)cc + w * rc : INFINITY;
                double vstar = wave_min(vc);
                const double bound = (double)tau - err - wds;
                int jstar;
                bool fell = false;
                if (vstar < bound) {
                    unsigned long long hit = __ballot(vc == vstar);
                    int jw = 0x7fffffff;
                    while (hit) {
                        const int l = __ffsll((long long)hit) - 1;
                        hit &= hit - 1ull;
                        jw = min(jw, __builtin_amdgcn_readlane(cj, l));
                    }
                    jstar = jw;
                } else {
                    fell = true;
                    // full row: the columns of owner threads lane + 64 h
                    ++n_fall;
                    const float4 *__restrict__ crow4 = reinterpret_cast<const float4 *>(C + (size_t)i * (size_t)n);
                    const int ng = n / 4;
                    float4 c4[G][4];
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
                            const int gi = g * 256 + lane + 64 * h;
                            c4[g][h] = crow4[gi < ng ? gi : ng - 1];
                        }
                    // a lane's columns (g*256 + lane + 64h)*4 + e grow with (g, h, e):
                    // a strict comparison keeps the lowest column of equal values
                    double bv = INFINITY;
                    int bj = 0x7fffffff;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
                            const int col0 = (g * 256 + lane + 64 * h) * 4;
                            const bool ok = col0 < n;
                            const double2 ra = *reinterpret_cast<const double2 *>(&r64[col0]);
                            const double2 rb = *reinterpret_cast<const double2 *>(&r64[col0 + 2]);
                            const float cv[4] = {c4[g][h].x, c4[g][h].y, c4[g][h].z, c4[g][h].w};
                            const double rv[4] = {ra.x, ra.y, rb.x, rb.y};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const double v = (double)(ok ? cv[e] : INFINITY) + w * rv[e];
                                const bool take = v < bv;
                                bv = take ? v : bv;
                                bj = take ? col0 + e : bj;
                            }
                        }
                        // keeps the residual reads of one group of columns in flight at a time
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    wave_argmin(bv, bj);
                    vstar = bv;
                    jstar = bj;
                    drain_memory();
                }
                // the owner lane of j* held it as its candidate on the fast path
                const double rstar = fell ? r64[jstar] : rc;

                // line-search partials over the support of row i
                uint32_t wg[4] = {wdv.x, wdv.y, wdv.z, wdv.w};
                double pp = 0.0, q2 = 0.0, tj = 0.0, ts = 0.0;
                double toff_max = 0.0;  // largest entry off the vertex: it drops by gamma times it
                bool star_l = false;
                // away / pairwise: sum t (V - g) over the support, sum of t^2
                // off ja, t_ija and the number of atoms
                double pa = 0.0, qa = 0.0, ta = 0.0, na = 0.0;
                auto away_sums = [&](double t, double vk, int col) {
                    if constexpr (VAR != 0) {
                        const bool on = t > 0.0;
                        pa += on ? t * (vaw - vk) : 0.0;
                        qa += (col == jaw) ? 0.0 : t * t;
                        ta += (col == jaw) ? t : 0.0;
                        na += on ? 1.0 : 0.0;
                    }
                };
                if (!stale) {
#pragma unroll
                    for (int k = 0; k < SC_KS; ++k) {
                        const bool has = sq[k] >= 0;
                        const double t = has ? st[k] : 0.0;
                        const double vk = (double)sc[k] + w * sr[k];
                        const bool atj = has && sq[k] == jstar;
                        pp += has ? t * (vk - vstar) : 0.0;
                        q2 += (has && !atj) ? t * t : 0.0;
                        tj += atj ? t : 0.0;
                        ts += t;
                        toff_max = fmax(toff_max, atj ? 0.0 : t);
                        star_l |= atj;
                        if (has) away_sums(t, vk, sq[k]);
                    }
                } else {
                    ++n_slow;
                    const uint32_t *__restrict__ mrow = M + (size_t)i * 256;
                    const double *__restrict__ trow = T + (size_t)i * (size_t)n;
                    const float *__restrict__ crow = C + (size_t)i * (size_t)n;
#pragma unroll
                    for (int h = 0; h < 4; ++h) wg[h] = mrow[lane + 64 * h];
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        uint32_t bits = wg[h];
                        while (bits) {
                            const int u = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            const int col = owned_col<256, 4>(u, lane + 64 * h);
                            const double t = trow[col];
                            const double vk = (double)crow[col] + w * r64[col];
                            const bool atj = col == jstar;
                            pp += t * (vk - vstar);
                            q2 += atj ? 0.0 : t * t;
                            tj += atj ? t : 0.0;
                            ts += t;
                            toff_max = fmax(toff_max, atj ? 0.0 : t);
                            star_l |= atj;
                            away_sums(t, vk, col);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < SC_KS; ++k) sq[k] = -1;
                }
                // each partial summed over the lanes holding nonzeros, in lane order
                // (rows have few nonzeros: cheaper than a full wave reduction)
                double sp = 0.0, sq2 = 0.0, stj = 0.0, smax = 0.0;
                double spa = 0.0, sqa = 0.0, sta = 0.0, sna = 0.0;
                {
                    unsigned long long act = __ballot(ts != 0.0 || pp != 0.0 || q2 != 0.0 || tj != 0.0);
                    while (act) {
                        const int l = __ffsll((long long)act) - 1;
                        act &= act - 1ull;
                        sp += readlane_f64(pp, l);
                        sq2 += readlane_f64(q2, l);
                        stj += readlane_f64(tj, l);
                        smax = fmax(smax, readlane_f64(toff_max, l));
                        if constexpr (VAR != 0) {
                            spa += readlane_f64(pa, l);
                            sqa += readlane_f64(qa, l);
                            sta += readlane_f64(ta, l);
                            sna += readlane_f64(na, l);
                        }
                    }
                }
                const bool star_in = __any(star_l);
                double gamma;
                bool fw_dir = true, drop = false;
                if constexpr (VAR == 0) {
                    gamma = step_size(rule, k0 + s, m, w, sp, sq2, stj, ai);
                } else {
                    // direction and gamma_max (Alg. A.2 / A.3), then the exact
                    // line search clipped to [0, gamma_max]
                    const double alpha = sta / ai;
                    double num, den, gmax;
                    if constexpr (VAR == 2) {
                        fw_dir = false;
                        num = (jstar != jaw) ? ai * (vaw - vstar) : 0.0;
                        den = (jstar != jaw) ? w * (2.0 * ai * ai) : 0.0;
                        gmax = alpha;
                    } else {
                        fw_dir = sna == 1.0 || jaw == jstar || sp >= spa;
                        if (fw_dir) {
                            num = sp;
                            den = w * (sq2 + (stj - ai) * (stj - ai));
                            gmax = 1.0;
                        } else {
                            num = spa;
                            den = w * (sqa + (sta - ai) * (sta - ai));
                            gmax = alpha / (1.0 - alpha);
                        }
                    }
                    if (!(num > 0.0)) gamma = 0.0;
                    else if (den == 0.0) gamma = gmax;
                    else gamma = num / den < gmax ? num / den : gmax;
                    drop = !fw_dir && gamma > 0.0 && gamma == gmax;
                }
                const double gadd = gamma * ai;
                // the new entry of a support column (ats: the FW vertex, ata: the away vertex)
                auto new_entry = [&](double t, bool ats, bool ata) {
                    if constexpr (VAR == 0) {
                        return blend(t, gamma, ats ? gadd : 0.0);
                    } else {
                        double tn;
                        if (fw_dir) tn = blend(t, gamma, ats ? gadd : 0.0);
                        else if constexpr (VAR == 2) tn = (jstar == jaw) ? t : (ats ? t + gadd : (ata ? t - gadd : t));
                        else tn = (1.0 + gamma) * t - (ata ? gadd : 0.0);
                        return (drop && ata) ? 0.0 : tn;
                    }
                };

                // t_i <- (1 - gamma) t_i + gamma a_i e_j*, r <- r + (t_i new - t_i old)
                double tnv[SC_KS];
                unsigned toff[SC_KS];
                bool zero_l = false;  // a nonzero of this lane became 0 (gamma = 1)
#pragma unroll
                for (int k = 0; k < SC_KS; ++k) {
                    const bool has = sq[k] >= 0;
                    const bool atj = has && sq[k] == jstar;
                    const double tn = new_entry(st[k], atj, has && sq[k] == jaw);
                    const bool put = has && tn != st[k];
                    const int col = has ? sq[k] : 0;
                    const double rn = sr[k] + (tn - st[k]);
                    if (put) {
                        r64[col] = rn;
                        r32[col] = (float)rn;
                    }
                    zero_l |= has && tn == 0.0;
                    tnv[k] = tn;
                    toff[k] = put ? (unsigned)col * 8u : kOOB;
                }
                uint32_t nw[4] = {wg[0], wg[1], wg[2], wg[3]};
                if (stale) {
                    double *__restrict__ trow = T + (size_t)i * (size_t)n;
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        uint32_t bits = wg[h];
                        while (bits) {
                            const int u = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            const int col = owned_col<256, 4>(u, lane + 64 * h);
                            const double t = trow[col];
                            const double tn = new_entry(t, col == jstar, col == jaw);
                            if (tn != t) {
                                const double rn = r64[col] + (tn - t);
                                r64[col] = rn;
                                r32[col] = (float)rn;
                                trow[col] = tn;
                            }
                            if (tn == 0.0) nw[h] &= ~(1u << u);
                        }
                    }
                    drain_memory();
                }
                // the FW vertex when it is not in the support (an away
                // direction leaves it at 0)
                const double tsn = fw_dir ? blend(0.0, gamma, gadd) : ((VAR == 2 && jstar != jaw) ? gadd : 0.0);
                const int oq = (jstar >> 2) & 255;
                const int hs = oq >> 6, us = ((jstar >> 10) << 2) | (jstar & 3);
                const bool put_s = ((oq & 63) == lane) && !star_in && tsn != 0.0;
                const double rns = rstar + tsn;
                if (put_s) {
                    r64[jstar] = rns;
                    r32[jstar] = (float)rns;
                }
                // the step's stores: a fixed sequence (absent ones out of range):
                // the plan entries and the new vertex's mask word
                const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + (size_t)i * (size_t)n, row_bytes);
#pragma unroll
                for (int k = 0; k < SC_KS; ++k) buf_store_f64(tnv[k], rt, toff[k]);
                buf_store_f64(tsn, rt, put_s ? (unsigned)jstar * 8u : kOOB);
                const __amdgpu_buffer_rsrc_t rm = buf_rsrc(M + (size_t)i * 256, 256u * 4u);
                {
                    const uint32_t ws = (hs == 0 ? nw[0] : hs == 1 ? nw[1] : hs == 2 ? nw[2] : nw[3]) | (1u << us);
                    buf_store_u32(ws, rm, (put_s && !stale) ? (unsigned)oq * 4u : kOOB);
                }
                if constexpr (TRACE) {
                    const __amdgpu_buffer_rsrc_t rs_tj = buf_rsrc(trace_j, trace_j ? (unsigned)nsteps * 4u : 0u);
                    const __amdgpu_buffer_rsrc_t rs_tg = buf_rsrc(trace_gamma, trace_gamma ? (unsigned)nsteps * 8u : 0u);
                    buf_store_u32((unsigned)jstar, rs_tj, lane == 0 ? (unsigned)s * 4u : kOOB);
                    buf_store_f64(gamma, rs_tg, lane == 0 ? (unsigned)s * 8u : kOOB);
                    if constexpr (VAR != 0) {
                        const __amdgpu_buffer_rsrc_t rs_ta = buf_rsrc(trace_away, trace_away ? (unsigned)nsteps * 4u : 0u);
                        buf_store_u32((unsigned)(fw_dir ? -1 - jaw : jaw), rs_ta, lane == 0 ? (unsigned)s * 4u : kOOB);
                    }
                }
                // rare: nonzeros that became 0 leave the support (and every word
                // of a row re-read from the plan is rewritten as computed)
                if (stale || __any(zero_l)) {
                    if (!stale) {
#pragma unroll
                        for (int k = 0; k < SC_KS; ++k) {
                            const int col = sq[k] >= 0 ? sq[k] : 0;
                            const int hk = ((col >> 2) & 255) >> 6, uk = ((col >> 10) << 2) | (col & 3);
                            const bool clr = sq[k] >= 0 && tnv[k] == 0.0;
#pragma unroll
                            for (int h = 0; h < 4; ++h) nw[h] = (clr && hk == h) ? (nw[h] & ~(1u << uk)) : nw[h];
                        }
                    }
#pragma unroll
                    for (int h = 0; h < 4; ++h) nw[h] = (put_s && hs == h) ? (nw[h] | (1u << us)) : nw[h];
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        buf_store_u32(nw[h], rm, nw[h] != wg[h] ? (unsigned)(lane + 64 * h) * 4u : kOOB);
                    drain_memory();
                }
#pragma unroll
                for (int k = SC_HIST - 1; k > 0; --k) hist[k] = hist[k - 1];
                hist[0] = i;
#pragma unroll
                for (int k = SC_DECN - 1; k > 0; --k) dec[k] = dec[k - 1];
                // the largest decrease of an r_j in this step: gamma times the
                // largest entry off the FW vertex, or t_ija on an away or
                // pairwise direction
                dec[0] = fw_dir ? gamma * smax : sta;
                {
                    double dsum = 0.0;
#pragma unroll
                    for (int k = 0; k < SC_DECN; ++k) dsum += dec[k];
                    wds = w * dsum;
                }
                // every store of earlier steps is complete before the barrier
                __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(NST));
            }
            __syncthreads();
        }
        if (lane == 0) {
            slow_steps[0] = n_fall;
            slow_steps[1] = n_slow;
            slow_steps[2] = SROT_CHAIN_SCREENED;
        }
    } else if (wid == 4) {
        // shares the stepper's SIMD: keeps the barriers only
        for (int64_t p = -LAG_A; p < nsteps; ++p) __syncthreads();
    } else {
        // ---- screener state (one row in flight per screener)
        const int sk = wid < 4 ? wid - 1 : wid - 2;
        const bool screener = wid != 0 && wid != 4;
        int nexti = 0, ri = 0;
        double ra = 0.0;
        uint32_t wd[4] = {0u, 0u, 0u, 0u};
        float c[4][CPT];
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int u = 0; u < CPT; ++u) c[h][u] = 0.f;
        float m1 = INFINITY, m2 = INFINITY, c1 = 0.f;
        int j1 = -1;
        int aq[SC_KS];
        double atv[SC_KS];
        float acv[SC_KS];
#pragma unroll
        for (int k = 0; k < SC_KS; ++k) { aq[k] = -1; atv[k] = 0.0; acv[k] = 0.f; }
        if (screener && sk < nsteps) nexti = idxv[sk];

        // FP32 screen of the columns of owner thread lane + 64 h
        auto screen_cols = [&](int h) {
            const int th = lane + 64 * h;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int col0 = (g * 256 + th) * 4;
                // Deliberate race: the stepper wave may store to these r32
                // entries in this same phase (plain ds_write_b32 against this
                // ds_read_b128, no barrier between them).  The LDS carries
                // out each dword of a DS access whole, so each value read is
                // the FP32 residual either before or after the step being
                // taken, never a torn word.  Either is covered: the
                // certificate's decrease allowance counts that step among the
                // SC_DECN steps a screen may have missed, and a value that
                // rose since it was read only makes the screened bound
                // smaller than the truth.  Relaxed atomic loads would state
                // the same contract but split this read into four.
                const float4 rr = *reinterpret_cast<const float4 *>(&r32[col0]);
                const float rv[4] = {rr.x, rr.y, rr.z, rr.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float cv = c[h][g * 4 + e];
                    const float v = __builtin_fmaf(w32, rv[e], cv);
                    const bool lt = v < m1;
                    j1 = lt ? h * CPT + g * 4 + e : j1;  // local index: an inline constant
                    c1 = lt ? cv : c1;
                    m2 = __builtin_amdgcn_fmed3f(m1, m2, v);
                    m1 = fminf(m1, v);
                }
            }
        };

        int pm = (LAG_A * 6 - LAG_A) % 6;  // (p mod 6) for p = -LAG_A
        for (int64_t p = -LAG_A; p < nsteps; ++p) {
            // =============================== screeners
            if ((pm + LAG_C) % 6 == sk) {
                // C: the gathered support of the row of step p + LAG_C
                const int64_t s = p + LAG_C;
                if (s >= 0 && s < nsteps) {
                    const int q = (int)(s & (SC_SLOTS - 1));
                    *reinterpret_cast<int2 *>(&s_g0[q][lane].z) = make_int2(aq[0], aq[1]);
                    s_g1[q][lane] = make_double2(atv[0], atv[1]);
                    s_g2[q][lane] = make_float2(acv[0], acv[1]);
                }
                // A: loads for the row of step p + LAG_A
                const int64_t s2 = p + LAG_A;
                if (s2 < nsteps) {
                    ri = __builtin_amdgcn_readfirstlane(nexti);
                    if (s2 + 6 < nsteps) nexti = idxv[s2 + 6];
                    ra = av[ri];
                    const uint32_t *__restrict__ mrow = M + (size_t)ri * 256;
#pragma unroll
                    for (int h = 0; h < 4; ++h) wd[h] = mrow[lane + 64 * h];
                    const float *__restrict__ crow = C + (size_t)ri * (size_t)n;
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        load_cost_row<256, CPT, 4, float>(crow, n, lane + 64 * h, c[h]);
                        // columns past n screen as +inf (r is 0 there)
#pragma unroll
                        for (int u = 0; u < CPT; ++u)
                            c[h][u] = ((u / 4) * 256 + lane + 64 * h) * 4 < n ? c[h][u] : INFINITY;
                    }
                }
            } else if ((pm + LAG_B1) % 6 == sk) {
                // B1: support of the row (requested), screen of the first half
                const int64_t s = p + LAG_B1;
                if (s >= 0 && s < nsteps) {
                    const int q = (int)(s & (SC_SLOTS - 1));
                    m1 = INFINITY; m2 = INFINITY; c1 = 0.f; j1 = -1;
                    screen_cols(0);
                    screen_cols(1);
                    uint64_t bits = 0ull;
                    constexpr uint32_t low = (CPT == 32) ? 0xffffffffu : ((1u << CPT) - 1u);
#pragma unroll
                    for (int h = 0; h < 4; ++h) bits |= (uint64_t)(wd[h] & low) << (h * CPT);
                    const bool over = __popcll(bits) > SC_KS;
                    // the row index is wave-uniform: scalar buffer descriptors (a
                    // descriptor in vector registers costs a loop per load)
                    const int rw = __builtin_amdgcn_readfirstlane(ri);
                    const __amdgpu_buffer_rsrc_t rt = buf_rsrc(T + (size_t)rw * (size_t)n, row_bytes);
                    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(C + (size_t)rw * (size_t)n, (unsigned)n * 4u);
#pragma unroll
                    for (int k = 0; k < SC_KS; ++k) {
                        const int b = bits ? __ffsll((long long)bits) - 1 : -1;
                        bits &= bits - 1ull;
                        const int col = b >= 0 ? owned_col<256, 4>(b % CPT, lane + 64 * (b / CPT)) : 0;
                        aq[k] = b >= 0 ? col : -1;
                        atv[k] = buf_load_f64(rt, b >= 0 ? (unsigned)col * 8u : kOOB);
                        acv[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                               rc, (int)(b >= 0 ? (unsigned)col * 4u : kOOB), 0, 0));
                    }
                    const bool any_over = __any(over);
                    if (lane == 0) {
                        s_hdr[q][0].x = ri;
                        s_hdr[q][0].y = any_over ? 1 : 0;
                        s_hdr[q][1].x = __double2loint(ra);
                        s_hdr[q][1].y = __double2hiint(ra);
                    }
                    s_wd[q][lane] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                }
            } else if ((pm + LAG_B2) % 6 == sk) {
                // B2: screen of the second half, threshold and candidates
                const int64_t s = p + LAG_B2;
                if (s >= 0 && s < nsteps) {
                    const int q = (int)(s & (SC_SLOTS - 1));
                    screen_cols(2);
                    screen_cols(3);
                    const float tau = wave_min_f32(m2);
                    const int jc = j1 >= 0 ? owned_col<256, 4>(j1 % CPT, lane + 64 * (j1 / CPT)) : -1;
                    *reinterpret_cast<int2 *>(&s_g0[q][lane].x) = make_int2((m1 < tau) ? jc : -1, __float_as_int(c1));
                    if (lane == 0) s_hdr[q][0].z = __float_as_int(tau);
                }
            }
            pm = (pm == 5) ? 0 : pm + 1;
            __syncthreads();
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += SC_NT) rg[j] = r64[j];
}

// max |c_ij| per workgroup (grid-stride), then the bound on |c| and |r|
__global__ __launch_bounds__(256) void cost_absmax_kernel(const float *__restrict__ C, size_t count,
                                                          double *__restrict__ part)
{
    __shared__ float sh[256];
    float mx = 0.f;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
        mx = fmaxf(mx, fabsf(C[e]));
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = (double)sh[0];
}

__global__ __launch_bounds__(256) void cost_bound_finish_kernel(ProblemView P, const double *__restrict__ part,
                                                                int nparts, double *__restrict__ out2)
{
    __shared__ double sh[3][256];
    double cm = 0.0, sa = 0.0, mb = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) cm = fmax(cm, part[k]);
    for (int i = threadIdx.x; i < P.m; i += 256) sa += P.a[i];
    for (int j = threadIdx.x; j < P.n; j += 256) mb = fmax(mb, P.b[j]);
    sh[0][threadIdx.x] = cm;
    sh[1][threadIdx.x] = sa;
    sh[2][threadIdx.x] = mb;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + s]);
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = sh[0][0];
        out2[1] = fmax(sh[1][0], sh[2][0]);
    }
}

bool screened_chain_supported(const ProblemView &P, const DeviceState &S)
{
    const Ownership &o = S.own;
    return P.cost == SROT_COST_F32 && o.reg && o.nt == 256 && o.vec == 4 && (o.cpt == 4 || o.cpt == 8 || o.cpt == 16);
}

bool screened_chain_enabled()
{
    const char *env = getenv("SROT_LMO_SCREEN");
    return !(env && strcmp(env, "0") == 0);
}

hipError_t launch_cost_bounds(const ProblemView &P, const DeviceState &S, double *out2, hipStream_t stream)
{
    const size_t count = (size_t)P.m * (size_t)P.n;
    // one partial per workgroup in the gap partial buffer (at least
    // 8 * gap_blocks doubles)
    int blocks = (int)((count + 256 * 64 - 1) / (256 * 64));
    if (blocks > 1024) blocks = 1024;
    if (blocks > 8 * S.gap_blocks) blocks = 8 * S.gap_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(cost_absmax_kernel, dim3(blocks), dim3(256), 0, stream, (const float *)P.C, count,
                       S.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cost_bound_finish_kernel, dim3(1), dim3(256), 0, stream, P, (const double *)S.partials,
                       blocks, out2);
    return hipGetLastError();
}

template <int VAR>
static hipError_t launch_screened_var(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                                      int64_t nsteps, int rule, int32_t *tj, double *tg, int32_t *ta, hipStream_t st)
{
    const bool trace = tj || tg || ta;
#define SROT_SCREENED(CPT_)                                                                          \
    if (S.own.cpt == CPT_) {                                                                         \
        if (trace)                                                                                   \
            hipLaunchKernelGGL((chain_screened_kernel<CPT_, true, VAR>), dim3(1), dim3(SC_NT), 0, st, P, S.T, \
                               S.r, S.mask, idx, k0, nsteps, rule, tj, tg, ta, S.slow_steps, S.screen_err); \
        else                                                                                         \
            hipLaunchKernelGGL((chain_screened_kernel<CPT_, false, VAR>), dim3(1), dim3(SC_NT), 0, st, P, S.T, \
                               S.r, S.mask, idx, k0, nsteps, rule, tj, tg, ta, S.slow_steps, S.screen_err); \
        return hipGetLastError();                                                                    \
    }
    SROT_SCREENED(4)
    SROT_SCREENED(8)
    SROT_SCREENED(16)
#undef SROT_SCREENED
    return hipErrorInvalidConfiguration;
}

hipError_t launch_chain_screened(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                                 int64_t nsteps, int rule, int32_t *tj, double *tg, hipStream_t st)
{
    return launch_screened_var<0>(P, S, idx, k0, nsteps, rule, tj, tg, nullptr, st);
}

hipError_t launch_active_screened(const ProblemView &P, const DeviceState &S, int pairwise, const int32_t *idx,
                                  int64_t nsteps, int32_t *tj, int32_t *ta, double *tg, hipStream_t st)
{
    if (pairwise) return launch_screened_var<2>(P, S, idx, 0, nsteps, SROT_ELS, tj, tg, ta, st);
    return launch_screened_var<1>(P, S, idx, 0, nsteps, SROT_ELS, tj, tg, ta, st);
}

}  // namespace srot
