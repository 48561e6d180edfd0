// The device-side state of a GMRES restart cycle and the serial work that
// closes an Arnoldi step of the delayed reorthogonalisation.  Shared by the
// Krylov kernels and by the first preconditioner pass of the next step,
// which runs that work in one extra workgroup (k_inner, k_first_jr).
#pragma once

#include <cstddef>

#include "gs2_internal.hpp"

namespace gs2 {

constexpr int MAXM = 128; // longest restart supported
constexpr int KT = 256;   // threads per workgroup of the Krylov kernels

struct GState {
    int j, done, kk, status;
    int maxsteps, pad0, pad1, pad2;
    double bnorm, beta, rtol, inv;
    double hA[MAXM + 2], hB[MAXM + 2], nrm[2];
    double g[MAXM + 2], cs[MAXM], sn[MAXM], y[MAXM];
    // delayed CGS2: scalars of the current step and the tentative column
    double bb, dd, wn2, nu, inv_alpha, e;
    double ht[MAXM + 2];
    // scale of the stored preconditioned vector of each step: step j works on
    // the unnormalised tentative vector, z_j = zs[j] * (stored Z column j)
    double zs[MAXM + 2];
    // last, so that everything before it can be staged in LDS (8.5 KB)
    double H[(MAXM + 1) * MAXM]; // H[k * MAXM + col], upper triangle R after rotations
};
constexpr int GSTATE_SMALL_WORDS = (int)(offsetof(GState, H) / 8);
static_assert(offsetof(GState, H) % 8 == 0, "the staged part of the state is whole 8-byte words");

// Sum of p[b] over this thread's b = threadIdx.x, + KT, ... < cnt.  Eight
// loads are in flight at once (a plain strided loop waits for each load
// before the next: one memory latency per partial); the eight running sums
// are added in a fixed order.
__device__ __forceinline__ double strided_sum(const double *__restrict__ p, int cnt)
{
    constexpr int U = 8;
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (int b0 = threadIdx.x; b0 < cnt; b0 += KT * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * KT;
            acc[u] += b < cnt ? p[b] : 0.0;
        }
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += acc[u];
    return s;
}

// Sum of one value per thread over the workgroup (KT threads); result valid
// in thread 0.  Starts and ends with a barrier.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int wv = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < KT / WAVE; ++i) s += red[i];
    return s;
}

// (one lane) Apply rotations 0..jc-1 to col (jc+1 entries used).  The entry
// carried from one rotation to the next stays in a register, so the chain
// is two multiply-adds per rotation; the loads run ahead of it.
__device__ __forceinline__ void apply_rotations(const double *__restrict__ cs, const double *__restrict__ sn,
                                                double *__restrict__ col, int jc)
{
    double carry = col[0];
    for (int k = 0; k < jc; ++k) {
        const double x = col[k + 1];
        col[k] = cs[k] * carry + sn[k] * x;
        carry = -sn[k] * carry + cs[k] * x;
    }
    col[jc] = carry;
}

// (one lane) Apply the committed rotations 0..jc-1 of the state ls (in
// LDS) to col (jc+2 entries), form rotation jc, store column jc of R into H
// (global) and advance the residual recurrence g.
__device__ inline bool commit_column(GState *ls, double *__restrict__ H, double *col, int jc)
{
    apply_rotations(ls->cs, ls->sn, col, jc);
    const double rho = hypot(col[jc], col[jc + 1]);
    if (!isfinite(rho)) {
        ls->status = GS2_ERR_NONFINITE;
        return false;
    }
    if (rho == 0.0) {
        ls->status = GS2_BREAKDOWN_EXACT;
        return false;
    }
    const double c = col[jc] / rho, sn = col[jc + 1] / rho;
    ls->cs[jc] = c;
    ls->sn[jc] = sn;
    col[jc] = rho;
    for (int k = 0; k <= jc; ++k) H[k * MAXM + jc] = col[k];
    const double gj = ls->g[jc];
    ls->g[jc + 1] = -sn * gj;
    ls->g[jc] = c * gj;
    return true;
}

// Reorthogonalisation scalars of u from the reduced sums of pass 1:
// alpha^2 = u.u - |a|^2 and e = (u.w - a.c)/alpha (alpha = 1, e = u.w at
// j = 0).  as/cs_ hold a and c in LDS; the sums run in one wavefront in a
// fixed order, so every workgroup that calls this gets the same bits.
// Returns false when u has fallen into span(Q) (or alpha^2 is not finite).
__device__ inline bool reorth_scalars(const GState *st, int j, const double *as, const double *cs_, double *sc,
                               double *alpha, double *e, double *a2)
{
    const int t = threadIdx.x, ln = t & (WAVE - 1);
    if (t < WAVE) {
        double aa = 0.0, ac = 0.0;
        for (int k = ln; k < j; k += WAVE) {
            aa += as[k] * as[k];
            ac += as[k] * cs_[k];
        }
        aa = wave_sum(aa);
        ac = wave_sum(ac);
        if (ln == 0) {
            sc[0] = aa;
            sc[1] = ac;
        }
    }
    __syncthreads();
    *a2 = st->bb - sc[0];
    const bool ok = j == 0 || (isfinite(*a2) && *a2 > 0.0);
    *alpha = j == 0 ? 1.0 : sqrt(*a2);
    *e = j == 0 ? st->dd : (st->dd - sc[1]) / *alpha;
    return ok;
}

// The step's serial work (one workgroup): correct and commit column j-1
// ([ht + nu a; nu alpha]) now that u's reorthogonalisation is known, store
// the new tentative column [c, e], form ||w'|| from the partials, the
// tentative rotation of column j and the residual estimate, and either stop
// the cycle or advance j (the next tentative vector keeps its scale 1/||w'||
// in zs[j+1]).  When u fell into span(Q) the cycle ends on the tentative
// column j-1.  The work is latency-bound: the whole workgroup (KT threads)
// stages the state (all but H) in LDS together with the partial sums, so one
// round trip to memory precedes the serial work of one lane, and writes it
// back.
__device__ __forceinline__ void dcgs_finish_block(const double *__restrict__ part, int nb, GState *__restrict__ st)
{
    __shared__ unsigned long long sw[GSTATE_SMALL_WORDS];
    __shared__ double col[MAXM + 2], red[KT / WAVE], sc[2];
    GState *ls = reinterpret_cast<GState *>(sw);
    const int t = threadIdx.x;
    const unsigned long long *gw = reinterpret_cast<const unsigned long long *>(st);
    {
        // all of this thread's words in flight at once, then into LDS
        constexpr int SQ = (GSTATE_SMALL_WORDS + KT - 1) / KT;
        unsigned long long v[SQ];
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            const int k = t + q * KT;
            v[q] = k < GSTATE_SMALL_WORDS ? gw[k] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            const int k = t + q * KT;
            if (k < GSTATE_SMALL_WORDS) sw[k] = v[q];
        }
    }
    double tot = strided_sum(part, nb);
    tot = block_sum(tot, red); // ends with a barrier: the staged state is complete
    if (ls->done) return;
    const int j = ls->j;
    double alpha, e, a2;
    const bool ok = reorth_scalars(ls, j, ls->hA, ls->hB, sc, &alpha, &e, &a2);
    if (t == 0) {
        const double nu_prev = ls->nu;
        if (!ok) {
            if (!isfinite(a2)) {
                ls->status = GS2_ERR_NONFINITE;
                ls->kk = j - 1;
            } else {
                for (int k = 0; k < j; ++k) col[k] = ls->ht[k];
                col[j] = nu_prev;
                ls->kk = commit_column(ls, st->H, col, j - 1) ? j : j - 1;
            }
            ls->done = 1;
        } else {
            bool good = true;
            if (j > 0) {
                for (int k = 0; k < j; ++k) col[k] = ls->ht[k] + nu_prev * ls->hA[k];
                col[j] = nu_prev * alpha;
                good = commit_column(ls, st->H, col, j - 1);
            }
            if (!good) {
                ls->kk = j - 1;
                ls->done = 1;
            }
        }
        if (ok && !ls->done) {
            ls->inv_alpha = 1.0 / alpha;
            ls->e = e;
            // tentative column j: [c, e; ||w'||]
            for (int k = 0; k < j; ++k) ls->ht[k] = ls->hB[k];
            ls->ht[j] = e;
            const double nu = sqrt(tot);
            ls->nu = nu;
            for (int k = 0; k <= j; ++k) col[k] = ls->ht[k];
            col[j + 1] = nu;
            apply_rotations(ls->cs, ls->sn, col, j);
            const double rho = hypot(col[j], col[j + 1]);
            if (!isfinite(rho) || !isfinite(nu)) {
                ls->status = GS2_ERR_NONFINITE;
                ls->done = 1;
                ls->kk = j;
            } else {
                const double est = rho > 0.0 ? fabs(col[j + 1] / rho * ls->g[j]) : 0.0;
                const bool breakdown = nu <= 1e-14 * sqrt(ls->wn2);
                ls->kk = j + 1;
                if (est <= ls->rtol * ls->bnorm || breakdown || j + 1 >= ls->maxsteps) {
                    for (int k = 0; k <= j; ++k) col[k] = ls->ht[k];
                    col[j + 1] = nu;
                    if (!commit_column(ls, st->H, col, j)) ls->kk = j;
                    ls->done = 1;
                } else {
                    ls->inv = 1.0 / nu;
                    ls->zs[j + 1] = 1.0 / nu;
                    ls->j = j + 1;
                }
            }
        }
    }
    __syncthreads();
    unsigned long long *gwo = reinterpret_cast<unsigned long long *>(st);
    for (int k = t; k < GSTATE_SMALL_WORDS; k += KT) gwo[k] = sw[k];
}

} // namespace gs2
