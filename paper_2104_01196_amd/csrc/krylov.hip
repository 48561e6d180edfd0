// Restarted flexible GMRES(m) in float64 (the Krylov solver the paper pairs
// with GS2, Sections 1 and 8): right preconditioning with the preconditioned
// vectors Z stored, Arnoldi by classical Gram-Schmidt with one full
// reorthogonalisation (delayed: both passes folded into two sweeps over the
// basis per step; or plain CGS2), Givens rotations applied on the device, and
// the true residual ||b - A x|| at the end of every cycle.  The host
// synchronises once per cycle; within a cycle every kernel reads a
// device-side stop flag and returns at once after the residual estimate has
// met the tolerance.  A cycle is captured once into a HIP graph and replayed.
//
// Reductions are deterministic: each workgroup writes one partial per
// quantity (fixed row range, fixed butterfly), then one workgroup per
// quantity sums the partials in a fixed order.  No floating-point atomics.
#include <algorithm>
#include <atomic>
#include <climits>
#include <chrono>
#include <cmath>
#include <new>

#include "dcgs_state.hpp"
#include "gs2_internal.hpp"
#include "sella.hpp"

namespace gs2 {

constexpr int RB = KRB; // rows per workgroup in the vector kernels (sella.hpp)

static std::atomic<int> g_graphs{1}; // replay restart cycles from HIP graphs

struct GHeader {
    int j, done, kk, status;
    int maxsteps, pad0, pad1, pad2;
    double bnorm, beta, rtol, inv;
};

// Everything a captured restart cycle bakes in.
struct CycleKey {
    const void *rp = nullptr, *ci = nullptr, *va = nullptr, *b = nullptr, *x = nullptr, *P = nullptr;
    const void *sa = nullptr; // values of the sliced-ELL copy (rebuilt with a new pattern)
    int kind = -1, m = 0, steps = 0;
    double rtol = 0.0;
    int orth = 0;
    bool operator==(const CycleKey &o) const
    {
        return rp == o.rp && ci == o.ci && va == o.va && b == o.b && x == o.x && P == o.P && sa == o.sa &&
               kind == o.kind &&
               m == o.m && steps == o.steps && rtol == o.rtol && orth == o.orth;
    }
};

struct GmresWork {
    int64_t n = 0;
    int m = 0;
    int nb = 0; // workgroups of the vector kernels
    double *V = nullptr, *Z = nullptr, *w = nullptr, *w2 = nullptr, *part = nullptr;
    GState *st = nullptr;
    GHeader *hdr = nullptr; // pinned host copy
    // HIP graph of one restart cycle (captured on its own stream, launched on the caller's)
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    CycleKey key;
    SellA A;         // the solver's copy of the system matrix
    int fmt_req = -1; // the layout request it was built for
    // Arnoldi steps from which the delayed passes keep fewer loads in flight
    // (INT_MAX: never), timed once per workspace (tune_basis); basis_tuned 1
    // decided there, 2 forced by the handle's request
    int upd_narrow = INT_MAX, dot_narrow = INT_MAX, basis_tuned = 0;
};

template <typename F>
static int capture_cycle(GmresWork *W, const CycleKey &key, F &&enqueue)
{
    if (W->exec) (void)hipGraphExecDestroy(W->exec);
    if (W->graph) (void)hipGraphDestroy(W->graph);
    W->exec = nullptr;
    W->graph = nullptr;
    if (!W->cap) GS2_TRY_HIP(hipStreamCreateWithFlags(&W->cap, hipStreamNonBlocking));
    GS2_TRY_HIP(hipStreamBeginCapture(W->cap, hipStreamCaptureModeThreadLocal));
    const int st = enqueue(W->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(W->cap, &g);
    if (st != GS2_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != GS2_OK ? st : GS2_ERR_HIP;
    }
    W->graph = g;
    GS2_TRY_HIP(hipGraphInstantiate(&W->exec, g, nullptr, nullptr, 0));
    W->key = key;
    return GS2_OK;
}

void free_gmres_work(GmresWork *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    sella_free(g->A);
    for (void *p : {(void *)g->V, (void *)g->Z, (void *)g->w, (void *)g->w2, (void *)g->part, (void *)g->st})
        if (p) (void)hipFree(p);
    if (g->hdr) (void)hipHostFree(g->hdr);
    delete g;
}

static int alloc_work(GmresWork **out, int64_t n, int m)
{
    GmresWork *g = new (std::nothrow) GmresWork;
    if (!g) return GS2_ERR_NOMEM;
    g->n = n;
    g->m = m;
    g->nb = (int)std::max<int64_t>(1, (n + RB - 1) / RB);
    const size_t N = (size_t)std::max<int64_t>(n, 1);
    int st = GS2_OK;
    auto A = [&](void **p, size_t bytes) {
        if (st == GS2_OK && hipMalloc(p, bytes) != hipSuccess) st = GS2_ERR_NOMEM;
    };
    A((void **)&g->V, sizeof(double) * N * (m + 1));
    A((void **)&g->Z, sizeof(double) * N * m);
    A((void **)&g->w, sizeof(double) * N);
    A((void **)&g->w2, sizeof(double) * N);
    A((void **)&g->part, sizeof(double) * (size_t)g->nb * (2 * MAXM + 3)); // delayed CGS2: 2j+3 per block
    A((void **)&g->st, sizeof(GState));
    if (st == GS2_OK && hipHostMalloc((void **)&g->hdr, sizeof(GHeader), hipHostMallocDefault) != hipSuccess)
        st = GS2_ERR_NOMEM;
    if (st != GS2_OK) {
        free_gmres_work(g);
        return st;
    }
    *out = g;
    return GS2_OK;
}

// ---------------------------------------------------------------- kernels

// Partial dots of the block's rows [r0, r0 + RB) against the basis vectors
// V[0..nk).  The block's values a (and b when TWO) sit in LDS, zero past n.
// The basis is split over the wavefronts (wave w takes k = w, w+4, ...) and
// each lane covers RL = RB/64 rows of a vector, so one cross-lane reduction
// serves RL loaded values and a wavefront keeps RL independent loads in
// flight.  The a/b operands are re-read from LDS for every vector rather
// than held in registers: that keeps the kernels near 60 VGPRs (8 waves per
// SIMD instead of 4), which measured 1.4x faster for the fused SpMV + dots.
// The basis is read once per pass, so it is loaded non-temporally (streaming
// cache policy): it then does not evict the gathered SpMV operand or the
// preconditioner's matrices, which are re-read within a step (measured:
// 120 -> 98 us for the fused SpMV + first pass, 44.7 -> 41.5 ms per solve
// with the same hint in the second pass and the residual kernel).
// Rows past n are clamped to the last row for loading (their factor is
// zero).  Results go to LDS: ra[k] = V_k.a, rb[k] = V_k.b.  With
// with_norms each wavefront first forms a.a, a.b and b.b over its quarter of
// the rows into rn[3 w + 0..2] (norm_part sums them in a fixed order); left
// to one wavefront after its vectors, they held the workgroup about 6 %
// longer (microbenchmark, 24 and 48 columns).
//
// G: loads a wavefront keeps in flight over one vector.  The loads are
// issued in groups of G, and the next group waits for the last (an empty
// asm statement that takes the group's values as operands makes the
// compiler wait for them there).  With all RL = 16 in flight the pass runs
// at 84 % of 8 TB/s over 24 basis columns of the 192^3 problem and at
// 82 % over 48; with two at a time, 88 % and 87 % (fewer requests in
// flight, each wavefront's range of rows more compact in time).  Over the
// first few columns of a cycle the wider groups are faster (1-4 columns:
// 72-87 % against 62-86 %).  The sums run in the same order for every G.
constexpr int RL = RB / WAVE;
constexpr int NWV = KT / WAVE; // wavefronts per workgroup

// norm c (0: a.a, 1: a.b, 2: b.b) of the workgroup from the wavefronts' parts
__device__ __forceinline__ double norm_part(const double *rn, int c)
{
    double o = 0.0;
    for (int q = 0; q < NWV; ++q) o += rn[3 * q + c];
    return o;
}

template <bool TWO, int G = RL>
__device__ __forceinline__ void block_multidot(int64_t n, int64_t r0, const double *al, const double *bl,
                                               const double *__restrict__ V, int64_t ldv, int nk, bool with_norms,
                                               double *ra, double *rb, double *rn)
{
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    const int last = (int)(n - 1 - r0 < RB - 1 ? n - 1 - r0 : RB - 1);
    if (with_norms) {
        constexpr int QR = RL / NWV;
        double aa = 0.0, ab = 0.0, bb = 0.0;
#pragma unroll
        for (int s = 0; s < QR; ++s) {
            const int i = ln + (wv * QR + s) * WAVE;
            const double a = al[i], b = TWO ? bl[i] : 0.0;
            aa += a * a;
            if (TWO) {
                ab += a * b;
                bb += b * b;
            }
        }
        aa = wave_sum(aa);
        if (TWO) {
            ab = wave_sum(ab);
            bb = wave_sum(bb);
        }
        if (ln == 0) {
            rn[3 * wv] = aa;
            rn[3 * wv + 1] = ab;
            rn[3 * wv + 2] = bb;
        }
    }
    for (int k = wv; k < nk; k += KT / WAVE) {
        asm volatile("" ::: "memory"); // keep the LDS operands in LDS (no hoisting into registers)
        const double *__restrict__ vk = V + (int64_t)k * ldv + r0;
        double sa = 0.0, sb = 0.0;
        static_assert(RL % G == 0, "groups of loads divide the rows per lane");
#pragma unroll
        for (int s0 = 0; s0 < RL; s0 += G) {
            double x[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int i = ln + (s0 + g) * WAVE;
                x[g] = __builtin_nontemporal_load(&vk[i < last ? i : last]);
            }
            if constexpr (G < RL) {
#pragma unroll
                for (int g = 0; g < G; ++g) asm volatile("" : "+v"(x[g])::"memory");
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int i = ln + (s0 + g) * WAVE;
                sa += x[g] * al[i];
                if (TWO) sb += x[g] * bl[i];
            }
        }
        sa = wave_sum(sa);
        if (TWO) sb = wave_sum(sb);
        if (ln == 0) {
            ra[k] = sa;
            if (TWO) rb[k] = sb;
        }
    }
}

// w = A z (sliced ELL, K lanes per row) fused with h = V^T w and ||w||^2
// partials, written k-major: part[k*nb + b], the norm at k = nk.
template <int SEL>
__global__ __launch_bounds__(KT) void k_spmv_dot(SellAView A, DiaAView D, int64_t n, const double *__restrict__ z,
                                                 double *__restrict__ w, const double *__restrict__ V, int64_t ldv,
                                                 const GState *__restrict__ st, double *__restrict__ part, int nb,
                                                 int fixed_nk)
{
    __shared__ double wl[RB];
    __shared__ double ra[MAXM + 2], rn[3 * NWV];
    if (st && st->done) return;
    const int nk = st ? st->j + 1 : fixed_nk;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int t = threadIdx.x;
    mat_rows<SEL, KT / WAVE>(A, D, n, r0, z, wl);
    for (int i = t; i < RB; i += KT)
        if (r0 + i < n) w[r0 + i] = wl[i];
    block_multidot<false>(n, r0, wl, nullptr, V, ldv, nk, true, ra, nullptr, rn);
    __syncthreads();
    for (int k = t; k <= nk; k += KT) part[(int64_t)k * nb + blockIdx.x] = k < nk ? ra[k] : norm_part(rn, 0);
}

// r = b - A x written to out, with ||r||^2 partials.
template <int SEL>
__global__ __launch_bounds__(KT) void k_true_resid(SellAView A, DiaAView D, int64_t n, const double *__restrict__ x,
                                                   const double *__restrict__ b, double *__restrict__ out,
                                                   double *__restrict__ part, int nb)
{
    __shared__ double wl[RB];
    __shared__ double red[KT / WAVE];
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int t = threadIdx.x;
    mat_rows<SEL, KT / WAVE>(A, D, n, r0, x, wl);
    double s = 0.0;
    for (int i = t; i < RB; i += KT) {
        const int64_t row = r0 + i;
        if (row < n) {
            const double r = b[row] - wl[i];
            out[row] = r;
            s += r * r;
        }
    }
    s = block_sum(s, red);
    if (t == 0) part[blockIdx.x] = s;
}

// ||b||^2 partials
__global__ __launch_bounds__(KT) void k_norm_part(int64_t n, const double *__restrict__ b, double *__restrict__ part, int nb)
{
    __shared__ double red[4];
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    double s = 0.0;
    for (int u = 0; u < RB / KT; ++u) {
        const int64_t row = r0 + threadIdx.x + u * KT;
        if (row < n) s += b[row] * b[row];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// CGS pass: wout = win - V h (h = first nk entries of hsrc), then partial
// dots V^T wout (and ||wout||^2 if with_norm, at k = nk or 0).  wout may be a
// column of V past the first nk.
__global__ __launch_bounds__(KT) void k_update_dot(int64_t n, const double *__restrict__ V, int64_t ldv,
                                                   const GState *__restrict__ st, int which_h,
                                                   const double *__restrict__ win, double *__restrict__ wout,
                                                   int do_dot, int with_norm, double *__restrict__ part, int nb)
{
    __shared__ double wl[RB];
    __shared__ double ra[MAXM + 2], rn[3 * NWV], hs[MAXM + 2];
    if (st->done) return;
    const int nk = st->j + 1;
    const double *hsrc = which_h == 0 ? st->hA : st->hB;
    for (int k = threadIdx.x; k < nk; k += KT) hs[k] = hsrc[k];
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int t = threadIdx.x;
    const int last = (int)(n - 1 - r0 < RB - 1 ? n - 1 - r0 : RB - 1);
    constexpr int NQ = RB / KT;
    double acc[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int i = t + u * KT;
        acc[u] = win[r0 + (i < last ? i : last)];
    }
    for (int k = 0; k < nk; ++k) { // k outer: NQ independent loads per vector
        const double h = hs[k];
        const double *__restrict__ vk = V + (int64_t)k * ldv + r0;
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int i = t + u * KT;
            acc[u] -= h * vk[i < last ? i : last];
        }
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int i = t + u * KT;
        const bool in = i <= last;
        if (in) wout[r0 + i] = acc[u];
        wl[i] = in ? acc[u] : 0.0;
    }
    __syncthreads();
    if (!do_dot && !with_norm) return;
    const int cnt = do_dot ? nk : 0;
    block_multidot<false>(n, r0, wl, nullptr, V, ldv, cnt, with_norm != 0, ra, nullptr, rn);
    __syncthreads();
    for (int k = t; k < cnt + (with_norm ? 1 : 0); k += KT)
        part[(int64_t)k * nb + blockIdx.x] = k < cnt ? ra[k] : norm_part(rn, 0);
}

// out[k] = sum_b part[k*nb + b] for k < cnt (one workgroup per k).  dst
// selects a GState field; cnt is read from the state when cnt_from_j.
__global__ __launch_bounds__(KT) void k_reduce(const double *__restrict__ part, int nb, GState *__restrict__ st,
                                               int dst, int cnt_extra, int fixed_cnt)
{
    __shared__ double red[4];
    if (dst != 9 && dst != 8 && st->done) return;
    const int cnt = fixed_cnt > 0 ? fixed_cnt : st->j + 1 + cnt_extra;
    const int k = blockIdx.x;
    if (k >= cnt) return;
    double s = strided_sum(part + (int64_t)k * nb, nb);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        switch (dst) {
        case 0: st->hA[k] = s; break;
        case 1: st->hB[k] = s; break;
        case 2: st->nrm[k] = s; break;
        case 3: { // delayed CGS2 pass-1 sums: a[0..j), c[0..j), u.u, u.w, w.w
            const int j = st->j;
            if (k < j) st->hA[k] = s;
            else if (k < 2 * j) st->hB[k - j] = s;
            else if (k == 2 * j) st->bb = s;
            else if (k == 2 * j + 1) st->dd = s;
            else st->wn2 = s;
            break;
        }
        case 8: st->bnorm = sqrt(s); break;
        case 9: st->beta = sqrt(s); break;
        }
    }
}

// Hessenberg column j = hA + hB, h_{j+1,j} = ||w||; apply the previous
// rotations, form a new one, update the residual estimate g, and decide
// whether the cycle stops.  One wavefront stages the state in LDS, one lane
// runs the O(j) serial recurrence on it.
__global__ __launch_bounds__(WAVE) void k_givens(GState *__restrict__ st)
{
    __shared__ double c[MAXM + 2], cs[MAXM], sn[MAXM];
    if (st->done) return;
    const int j = st->j;
    for (int k = threadIdx.x; k <= j; k += WAVE) {
        c[k] = st->hA[k] + st->hB[k];
        if (k < j) {
            cs[k] = st->cs[k];
            sn[k] = st->sn[k];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double hn = sqrt(st->nrm[0]);
    const double wn0 = sqrt(st->hA[j + 1]); // ||A z_j|| (slot j+1 of the first pass)
    for (int k = 0; k < j; ++k) {
        const double a = cs[k] * c[k] + sn[k] * c[k + 1];
        c[k + 1] = -sn[k] * c[k] + cs[k] * c[k + 1];
        c[k] = a;
    }
    const double rho = hypot(c[j], hn);
    if (!isfinite(rho) || !isfinite(hn)) {
        st->status = GS2_ERR_NONFINITE;
        st->done = 1;
        st->kk = j; // discard this column
        return;
    }
    if (rho == 0.0) {
        st->status = GS2_BREAKDOWN_EXACT;
        st->done = 1;
        st->kk = j;
        return;
    }
    st->cs[j] = c[j] / rho;
    st->sn[j] = hn / rho;
    c[j] = rho;
    for (int k = 0; k <= j; ++k) st->H[k * MAXM + j] = c[k];
    st->g[j + 1] = -st->sn[j] * st->g[j];
    st->g[j] = st->cs[j] * st->g[j];
    st->kk = j + 1;
    const bool breakdown = hn <= 1e-14 * wn0;
    st->inv = breakdown ? 0.0 : 1.0 / hn;
    if (fabs(st->g[j + 1]) <= st->rtol * st->bnorm || breakdown || j + 1 >= st->maxsteps) st->done = 1;
    else st->j = j + 1;
}

// v_{j+1} *= 1/h_{j+1,j}  (skipped once the cycle has stopped)
__global__ void k_scale_next(int64_t n, double *__restrict__ V, int64_t ldv, const GState *__restrict__ st)
{
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) V[(int64_t)st->j * ldv + i] *= st->inv;
}

// ------------------------------------------------------------ delayed CGS2
//
// Two passes over V per Arnoldi step instead of four.  Step j starts from the
// tentative vector u = V[j]: the previous step's projected vector, not yet
// reorthogonalised, stored unnormalised with its scale zs[j] = 1/||u_raw||.
// The preconditioner is linear (every apply starts from zero), so it is
// applied to the raw vector and the scale is folded into the consumers: the
// SpMV result and u are scaled when the first pass loads them, and the
// solution update weighs column j of Z by zs[j].  Pass 1, fused with
// w = A z_j, forms a = Q^T u, c = Q^T w, u.u, u.w and w.w (Q = V[0..j)) in
// one read of Q.
// Then q_j = (u - Q a)/alpha with alpha^2 = u.u - |a|^2, the coefficient of
// w on q_j is e = (u.w - a.c)/alpha, and the previous step's tentative
// Hessenberg column is corrected now that its vector's reorthogonalisation
// is known: column j-1 = [ht + nu a; nu alpha].  Pass 2 writes q_j and the
// next tentative vector w' = w - Q c - e q_j in one read of Q.  The
// convergence estimate of step j uses the tentative column [c, e; ||w'||],
// equal to the final column in exact arithmetic; when the cycle stops the
// tentative column is committed as it stands.

template <int SEL>
__global__ __launch_bounds__(KT) void k_spmv_dot2(SellAView A, DiaAView D, int64_t n, const double *__restrict__ z,
                                                  double *__restrict__ w, const double *__restrict__ V, int64_t ldv,
                                                  const GState *__restrict__ st, double *__restrict__ part, int nb)
{
    __shared__ double wl[RB], ul[RB];
    __shared__ double ra[MAXM + 2], rc[MAXM + 2], rn[3 * NWV];
    if (st->done) return;
    const int j = st->j;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int t = threadIdx.x;
    mat_rows<SEL, KT / WAVE>(A, D, n, r0, z, wl);
    const double zsc = st->zs[j];
    const double *__restrict__ u = V + (int64_t)j * ldv;
    for (int i = t; i < RB; i += KT) {
        const int64_t row = r0 + i;
        const double wv = zsc * wl[i];
        wl[i] = wv;
        if (row < n) w[row] = wv;
        ul[i] = row < n ? zsc * u[row] : 0.0;
    }
    __syncthreads();
    // a = Q^T u, c = Q^T w (Q = V[0..j)), then u.u, u.w, w.w
    block_multidot<true>(n, r0, ul, wl, V, ldv, j, true, ra, rc, rn);
    __syncthreads();
    for (int k = t; k < 2 * j + 3; k += KT)
        part[(int64_t)k * nb + blockIdx.x] = k < j ? ra[k] : k < 2 * j ? rc[k - j] : norm_part(rn, k - 2 * j);
}

// The same pass split in two for the diagonal copy of A: k_dia_spmv writes
// w = zs[j] (A z) straight from registers (one block of 64 R rows per
// wavefront), then k_dot2 forms the dot products from w, u and Q.  Staging
// the product in LDS ahead of the dot products, as the fused kernel does,
// held the product to 58 % of the peak on the 192^3 problem (111 us) against
// 77 % written directly (82 us); the split costs one more read of w.
//
// ND > 0: exactly ND diagonals (7 for 7-point stencils), the loop unrolled
// completely so that every diagonal's loads are issued before the first
// wait (issuing them 1, 2 or 4 diagonals at a time measured no faster in the
// solve).  w is stored non-temporally, as are the second basis pass's
// outputs (196.3 against 197.3 ms per 192^3 solve).  Every launched wavefront loads in bounds (the copy is padded to
// 1024-row workgroups and a clamped column only meets a stored zero); rows
// past n are not written.
template <int R, int ND>
__global__ __launch_bounds__(KT) void k_dia_spmv(DiaAView A, int64_t n, const double *__restrict__ z,
                                                 double *__restrict__ w, const GState *__restrict__ st)
{
    using V2 = double __attribute__((ext_vector_type(2)));
    if (st && st->done) return;
    const double zsc = st ? st->zs[st->j] : 1.0;
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    const int64_t base = ((int64_t)blockIdx.x * (KT / WAVE) + wv) * (WAVE * R);
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    const int nd = ND > 0 ? ND : A.ndiag;
    constexpr int UNR = ND > 0 ? ND : 1;
#pragma unroll UNR
    for (int d = 0; d < nd; ++d) {
        const int o = A.off[d];
        const double *__restrict__ vd = A.val + (int64_t)d * A.stride;
        double a[R];
        if constexpr (R == 2) {
            const V2 t = __builtin_nontemporal_load((const V2 *)(vd + base + 2 * ln));
            a[0] = t.x;
            a[1] = t.y;
        } else {
            a[0] = __builtin_nontemporal_load(vd + base + ln);
        }
        const bool inside = base + o >= 0 && base + WAVE * R + o <= n;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int64_t c = base + k * WAVE + ln + o;
            const int64_t cc = c < 0 ? 0 : (c >= n ? n - 1 : c);
            c = inside ? c : cc;
            acc[k] += a[k] * z[c];
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t row = base + k * WAVE + ln;
        if (row < n) __builtin_nontemporal_store(zsc * acc[k], &w[row]);
    }
}

// w = zs[j] (A z) from the 3-row block copy (node-major planes), a lane
// owning NB nodes 64 apart: per node offset it gathers the neighbour node's
// three z entries once and loads the nine values of the block (nine
// coalesced loads), forming its three rows' sums in the order b3_rows uses.
// The planes are padded to whole 1024-node groups, so every load is in
// bounds; nodes past n/3 are not written.
template <int NB>
__global__ __launch_bounds__(KT) void k_b3_spmv(DiaAView A, int64_t n, const double *__restrict__ z,
                                                double *__restrict__ w, const GState *__restrict__ st)
{
    if (st && st->done) return;
    const double zsc = st ? st->zs[st->j] : 1.0;
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    const int64_t nn = n / 3, g0 = ((int64_t)blockIdx.x * (KT / WAVE) + wv) * (WAVE * NB);
    double acc[NB][3];
    int64_t nd[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t i = g0 + b * WAVE + ln;
        acc[b][0] = acc[b][1] = acc[b][2] = 0.0;
        nd[b] = i < nn ? i : nn - 1;
    }
    const int64_t f1 = (g0 + WAVE * NB < nn ? g0 + WAVE * NB : nn) - 1; // the wavefront's last node
    for (int d = 0; d < A.ndiag; ++d) {
        const int64_t o = A.off[d];
        const bool inside = g0 + o >= 0 && f1 + o < nn;
        const double *__restrict__ p0 = A.val + (int64_t)(9 * d) * A.stride;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t i = g0 + b * WAVE + ln;
            int64_t c = nd[b] + o;
            c = inside ? c : (c < 0 ? 0 : (c >= nn ? nn - 1 : c));
            c *= 3;
            const double z0 = z[c], z1 = z[c + 1], z2 = z[c + 2];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double *__restrict__ pv = p0 + (int64_t)(3 * k) * A.stride + i;
                acc[b][k] += __builtin_nontemporal_load(pv) * z0;
                acc[b][k] += __builtin_nontemporal_load(pv + A.stride) * z1;
                acc[b][k] += __builtin_nontemporal_load(pv + 2 * A.stride) * z2;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t i = g0 + b * WAVE + ln;
        if (i < nn)
#pragma unroll
            for (int k = 0; k < 3; ++k) __builtin_nontemporal_store(zsc * acc[b][k], &w[3 * i + k]);
    }
}

template <int G>
__global__ __launch_bounds__(KT) void k_dot2(int64_t n, const double *__restrict__ w, const double *__restrict__ V,
                                             int64_t ldv, const GState *__restrict__ st, double *__restrict__ part,
                                             int nb)
{
    __shared__ double wl[RB], ul[RB];
    __shared__ double ra[MAXM + 2], rc[MAXM + 2], rn[3 * NWV];
    if (st->done) return;
    const int j = st->j;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int t = threadIdx.x;
    const double zsc = st->zs[j];
    const double *__restrict__ u = V + (int64_t)j * ldv;
    // u.u, u.w and w.w from the values as they are staged (every wavefront
    // its own rows; 237.6 -> 225.7 us per launch in the 192^3 solve against
    // the norms formed by one wavefront after its vectors)
    double aa = 0.0, ab = 0.0, bb = 0.0;
    for (int i = t; i < RB; i += KT) {
        const int64_t row = r0 + i;
        const double wv = row < n ? w[row] : 0.0, uv = row < n ? zsc * u[row] : 0.0;
        wl[i] = wv;
        ul[i] = uv;
        aa += uv * uv;
        ab += uv * wv;
        bb += wv * wv;
    }
    aa = wave_sum(aa);
    ab = wave_sum(ab);
    bb = wave_sum(bb);
    if ((t & (WAVE - 1)) == 0) {
        rn[3 * (t / WAVE)] = aa;
        rn[3 * (t / WAVE) + 1] = ab;
        rn[3 * (t / WAVE) + 2] = bb;
    }
    __syncthreads();
    block_multidot<true, G>(n, r0, ul, wl, V, ldv, j, false, ra, rc, nullptr);
    __syncthreads();
    for (int k = t; k < 2 * j + 3; k += KT)
        part[(int64_t)k * nb + blockIdx.x] = k < j ? ra[k] : k < 2 * j ? rc[k - j] : norm_part(rn, k - 2 * j);
}

// Pass 2 of step j: q_j = (u - Q a)/alpha over u's slot, w' = w - Q c - e q_j
// into V[j+1], partial ||w'||^2.  Every workgroup derives alpha and e itself
// (identical bits) and skips the pass when u has fallen into span(Q).
__global__ __launch_bounds__(KT) void k_dcgs_update(int64_t n, double *__restrict__ V, int64_t ldv,
                                                    const GState *__restrict__ st, const double *__restrict__ w,
                                                    double *__restrict__ part)
{
    __shared__ double as[MAXM + 2], cs_[MAXM + 2], red[KT / WAVE], sc[2];
    if (st->done) return;
    const int j = st->j, t = threadIdx.x;
    for (int k = t; k < j; k += KT) {
        as[k] = st->hA[k];
        cs_[k] = st->hB[k];
    }
    __syncthreads();
    double alpha, e, a2;
    if (!reorth_scalars(st, j, as, cs_, sc, &alpha, &e, &a2)) return; // the same in every workgroup
    const double ia = 1.0 / alpha, zsc = st->zs[j];
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    double s = 0.0;
    double *__restrict__ u = V + (int64_t)j * ldv;
    double *__restrict__ wn = V + (int64_t)(j + 1) * ldv;
    constexpr int NQ = RB / KT;
    // rows past n are clamped to n-1 for loads and skipped for stores
    int64_t rows[NQ];
    double aq[NQ], aw[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t row = r0 + t + q * KT;
        rows[q] = row < n ? row : n - 1;
        aq[q] = zsc * u[rows[q]];
        aw[q] = w[rows[q]];
    }
#pragma unroll 2
    for (int k = 0; k < j; ++k) {
        const double *__restrict__ vk = V + (int64_t)k * ldv;
        const double a = as[k], c = cs_[k];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double x = __builtin_nontemporal_load(&vk[rows[q]]);
            aq[q] -= a * x;
            aw[q] -= c * x;
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t row = r0 + t + q * KT;
        if (row >= n) continue;
        const double qv = aq[q] * ia;
        const double wp = aw[q] - e * qv;
        u[row] = qv;
        wn[row] = wp;
        s += wp * wp;
    }
    s = block_sum(s, red);
    if (t == 0) part[blockIdx.x] = s;
}

// The same pass with 16-byte loads for an even n (every column then starts
// 16-byte aligned): each thread owns NP pairs of consecutive rows, so a
// workgroup covers 2 NP KT rows and writes one partial.  Measured on the
// 192^3 problem's basis: 238 us against 273 us for the one-row-per-load
// pass over 1024-row workgroups (microbenchmark, 24 columns); in the solve,
// four pairs per thread and two measured alike (261 / 262 us per launch).
// G: loads in flight per thread over one column, issued in groups as in
// block_multidot; the loop over the columns is not unrolled (unrolled, the
// pass took 118 registers and 4 wavefronts per SIMD).  Over 24 and 48
// columns one load at a time runs at 84 % and 86 % of 8 TB/s against 79 %
// for all four; over 1-8 columns all four are faster (81-84 % against
// 77-80 %).  The updates run in the same order for every G.
template <int NP, int G>
__global__ __launch_bounds__(KT) void k_dcgs_update_pairs(int64_t n, double *__restrict__ V, int64_t ldv,
                                                          const GState *__restrict__ st, const double *__restrict__ w,
                                                          double *__restrict__ part)
{
    using D2 = double __attribute__((ext_vector_type(2)));
    __shared__ double as[MAXM + 2], cs_[MAXM + 2], red[KT / WAVE], sc[2];
    if (st->done) return;
    const int j = st->j, t = threadIdx.x;
    for (int k = t; k < j; k += KT) {
        as[k] = st->hA[k];
        cs_[k] = st->hB[k];
    }
    __syncthreads();
    double alpha, e, a2;
    if (!reorth_scalars(st, j, as, cs_, sc, &alpha, &e, &a2)) return; // the same in every workgroup
    const double ia = 1.0 / alpha, zsc = st->zs[j];
    const int64_t r0 = (int64_t)blockIdx.x * (2 * NP * KT);
    double s = 0.0;
    double *__restrict__ u = V + (int64_t)j * ldv;
    double *__restrict__ wn = V + (int64_t)(j + 1) * ldv;
    // pairs past n are clamped to the last pair for loads and skipped for stores
    int64_t rows[NP];
    D2 aq[NP], aw[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int64_t row = r0 + 2 * (t + q * KT);
        rows[q] = row < n ? row : n - 2;
        aq[q] = zsc * *(const D2 *)&u[rows[q]];
        aw[q] = *(const D2 *)&w[rows[q]];
    }
    static_assert(NP % G == 0, "groups of loads divide the pairs per thread");
#pragma unroll 1
    for (int k = 0; k < j; ++k) {
        const double *__restrict__ vk = V + (int64_t)k * ldv;
        const double a = as[k], c = cs_[k];
#pragma unroll
        for (int q0 = 0; q0 < NP; q0 += G) {
            D2 x[G];
#pragma unroll
            for (int g = 0; g < G; ++g) x[g] = __builtin_nontemporal_load((const D2 *)&vk[rows[q0 + g]]);
            if constexpr (G < NP) {
#pragma unroll
                for (int g = 0; g < G; ++g) asm volatile("" : "+v"(x[g])::"memory");
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                aq[q0 + g] -= a * x[g];
                aw[q0 + g] -= c * x[g];
                // the group's updates before the next group's wait: its loaded values die here
                if constexpr (G < NP) asm volatile("" : "+v"(aq[q0 + g]), "+v"(aw[q0 + g]));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int64_t row = r0 + 2 * (t + q * KT);
        if (row >= n) continue;
        const D2 qv = aq[q] * ia;
        const D2 wp = aw[q] - e * qv;
        __builtin_nontemporal_store(qv, (D2 *)&u[row]);
        __builtin_nontemporal_store(wp, (D2 *)&wn[row]);
        s += wp.x * wp.x;
        s += wp.y * wp.y;
    }
    s = block_sum(s, red);
    if (t == 0) part[blockIdx.x] = s;
}
constexpr int UPD_PAIRS = 4; // pairs of rows per thread in k_dcgs_update_pairs (2048-row workgroups)
// Arnoldi steps from which the basis passes keep fewer loads in flight when
// that is faster on the basis at hand (tune_basis; the crossovers measured
// on the 192^3 problem's basis, where each column is 57 MB: on the 128^3
// one, 17 MB per column and much of the basis in the last-level cache, the
// wide groups are faster at every step)
constexpr int UPD_NARROW_FROM = 12, DOT_NARROW_FROM = 8;

// A state for timing the passes at step j: nothing converged, a = c = 0,
// unit norms (the reorthogonalisation scalars stay finite).
__global__ void k_probe_state(GState *__restrict__ st, int j)
{
    if (threadIdx.x != 0) return;
    st->j = j;
    st->done = 0;
    for (int k = 0; k < MAXM + 2; ++k) {
        st->hA[k] = 0.0;
        st->hB[k] = 0.0;
        st->zs[k] = 1.0;
    }
    st->bb = 1.0;
    st->dd = 0.0;
}

__global__ __launch_bounds__(KT) void k_dcgs_finish(const double *__restrict__ part, int nb, GState *__restrict__ st)
{
    dcgs_finish_block(part, nb, st);
}

__global__ void k_cycle_init(GState *__restrict__ st, int maxsteps, double rtol)
{
    if (threadIdx.x != 0) return;
    st->j = 0;
    st->done = 0;
    st->kk = 0;
    st->status = GS2_OK;
    st->maxsteps = maxsteps;
    st->rtol = rtol;
    st->inv = 1.0 / st->beta;
    for (int k = 0; k < MAXM + 2; ++k) st->g[k] = 0.0;
    st->g[0] = st->beta;
    for (int k = 0; k < MAXM + 2; ++k) st->zs[k] = 1.0; // V[0] is normalised explicitly; CGS2 normalises all
}

__global__ void k_scale0(int64_t n, double *__restrict__ v, const GState *__restrict__ st)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] *= st->inv;
}

// y = R^{-1} g over the kk columns of this cycle (one wavefront).  Row k of
// the triangular solve is a dot product over l > k, split over the lanes; the
// lanes load row k-1 of R while row k is being reduced, so each row costs a
// reduction rather than a memory latency.
__global__ __launch_bounds__(WAVE) void k_backsolve(GState *__restrict__ st)
{
    __shared__ double ys[MAXM];
    const int kk = st->kk, ln = threadIdx.x;
    constexpr int PER = (MAXM + WAVE - 1) / WAVE; // row entries per lane
    double h[PER], hn[PER];
    auto load_row = [&](int k, double (&dst)[PER]) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int l = k + 1 + ln + q * WAVE;
            dst[q] = (k >= 0 && l < kk) ? st->H[k * MAXM + l] : 0.0;
        }
    };
    load_row(kk - 1, h);
    for (int k = kk - 1; k >= 0; --k) {
        load_row(k - 1, hn); // in flight while row k is reduced
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int l = k + 1 + ln + q * WAVE;
            if (l < kk) p += h[q] * ys[l];
        }
        p = wave_sum(p);
        if (ln == 0) ys[k] = (st->g[k] - p) / st->H[k * MAXM + k];
        __syncthreads(); // one wavefront: orders the LDS write before the next row's reads
#pragma unroll
        for (int q = 0; q < PER; ++q) h[q] = hn[q];
    }
    for (int k = ln; k < kk; k += WAVE) st->y[k] = ys[k];
}

// x += Z y (column k of Z weighed by its scale zs[k])
__global__ __launch_bounds__(KT) void k_update_x(int64_t n, const double *__restrict__ Z, int64_t ldz,
                                                 const GState *__restrict__ st, double *__restrict__ x)
{
    __shared__ double ys[MAXM];
    const int kk = st->kk;
    for (int k = threadIdx.x; k < kk; k += KT) ys[k] = st->y[k] * st->zs[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = x[i];
    for (int k = 0; k < kk; ++k) acc += ys[k] * Z[(int64_t)k * ldz + i];
    x[i] = acc;
}

// The same update over pairs of rows for an even n and a 16-byte aligned x
// (16-byte loads), NP pairs per thread, G loads in flight per thread (as in
// the second basis pass); the sums run in the same order.  Over the 50
// columns of a cycle on the 192^3 problem: 439 us with one load in flight
// (84 % of 8 TB/s), 465 us with four, 536 us for the one-row kernel.
constexpr int UPDX_G = 1;
template <int NP, int G>
__global__ __launch_bounds__(KT) void k_update_x_pairs(int64_t n, const double *__restrict__ Z, int64_t ldz,
                                                       const GState *__restrict__ st, double *__restrict__ x)
{
    using D2 = double __attribute__((ext_vector_type(2)));
    __shared__ double ys[MAXM];
    const int kk = st->kk, t = threadIdx.x;
    for (int k = t; k < kk; k += KT) ys[k] = st->y[k] * st->zs[k];
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * (2 * NP * KT);
    int64_t rows[NP];
    D2 acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int64_t row = r0 + 2 * (t + q * KT);
        rows[q] = row < n ? row : n - 2;
        acc[q] = *(const D2 *)&x[rows[q]];
    }
    static_assert(NP % G == 0, "groups of loads divide the pairs per thread");
#pragma unroll 1
    for (int k = 0; k < kk; ++k) {
        const double *__restrict__ zk = Z + (int64_t)k * ldz;
        const double y = ys[k];
#pragma unroll
        for (int q0 = 0; q0 < NP; q0 += G) {
            D2 v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) v[g] = __builtin_nontemporal_load((const D2 *)&zk[rows[q0 + g]]);
            if constexpr (G < NP) {
#pragma unroll
                for (int g = 0; g < G; ++g) asm volatile("" : "+v"(v[g])::"memory");
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                acc[q0 + g] += y * v[g];
                if constexpr (G < NP) asm volatile("" : "+v"(acc[q0 + g]));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int64_t row = r0 + 2 * (t + q * KT);
        if (row < n) *(D2 *)&x[row] = acc[q];
    }
}

__global__ void k_zero64(int64_t n, double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

__global__ void k_copy_stop(int64_t n, const double *__restrict__ a, double *__restrict__ b,
                            const GState *__restrict__ st)
{
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------- host side

// SEL > 0: sliced ELL with SEL lanes per row; -9 <= SEL < 0: the diagonal
// copy with -SEL rows per lane; SEL <= -10: the 3-row block copy (the fused
// kernels form its rows one node per thread whatever -SEL - 10 says)
#define GS2_SPMV_DISPATCH(K, kern, grid, ...)                                \
    do {                                                                     \
        switch (K) {                                                         \
        case -1: kern<-1><<<grid, KT, 0, s>>>(__VA_ARGS__); break;           \
        case -2: kern<-2><<<grid, KT, 0, s>>>(__VA_ARGS__); break;           \
        case -11: kern<-11><<<grid, KT, 0, s>>>(__VA_ARGS__); break;         \
        case -12: kern<-12><<<grid, KT, 0, s>>>(__VA_ARGS__); break;         \
        case 1: kern<1><<<grid, KT, 0, s>>>(__VA_ARGS__); break;             \
        case 2: kern<2><<<grid, KT, 0, s>>>(__VA_ARGS__); break;             \
        case 4: kern<4><<<grid, KT, 0, s>>>(__VA_ARGS__); break;             \
        case 8: kern<8><<<grid, KT, 0, s>>>(__VA_ARGS__); break;             \
        case 16: kern<16><<<grid, KT, 0, s>>>(__VA_ARGS__); break;           \
        case 32: kern<32><<<grid, KT, 0, s>>>(__VA_ARGS__); break;           \
        default: kern<64><<<grid, KT, 0, s>>>(__VA_ARGS__); break;           \
        }                                                                    \
    } while (0)

static int precondition(int kind, gs2_handle *P, const double *v, double *z, int64_t n, const GState *st,
                        hipStream_t s)
{
    switch (kind) {
    case GS2_PREC_GS2: return apply_gs2(P->h, v, z, s);
    case GS2_PREC_JR: return apply_jr(P->h, P->h.sweeps, P->h.omega, v, z, s);
    case GS2_PREC_GS_TRISOLVE: return apply_trisolve(P->h, P->h.variant, P->h.omega, v, z, s);
    case GS2_PREC_MTGS: return apply_mtgs(P->h, P->h.variant, P->h.omega, v, z, s);
    default:
        k_copy_stop<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, v, z, st);
        return GS2_OK;
    }
}

// Below this many rows the product's layout is not timed (sliced ELL at the
// rule's lanes per row, unless forced): launch overhead would dominate.
constexpr int64_t SPMV_TUNE_MIN_ROWS = 65536;

// Loads in flight of the two delayed basis passes (all groups of one width:
// block_multidot's and k_dcgs_update_pairs' G), decided once per workspace
// by timing both widths of each pass at step min(m - 1, 24) on the zeroed
// basis (best of three batches of three launches after a warm-up batch; a
// narrow variant must win by 3 %).  The narrow width then runs from the
// crossover step.  Small bases (fewer than BASIS_TUNE_MIN_ROWS rows, or a
// restart below 16) keep the wide groups.  The probe's writes (two columns,
// the partial sums, the state) are all set again by the solve.
constexpr int64_t BASIS_TUNE_MIN_ROWS = 1 << 20;
static int tune_basis(GmresWork *W, int req, hipStream_t s)
{
    if (W->basis_tuned) return GS2_OK;
    W->upd_narrow = W->dot_narrow = INT_MAX;
    const int64_t n = W->n;
    if (req == 2 && n % 2 == 0) { // forced narrow (from the crossover steps)
        W->upd_narrow = UPD_NARROW_FROM;
        W->dot_narrow = DOT_NARROW_FROM;
    }
    if (req != 0 || n < BASIS_TUNE_MIN_ROWS || W->m < 16 || n % 2) {
        W->basis_tuned = req != 0 ? 2 : 1;
        return GS2_OK;
    }
    const int jt = std::min(W->m - 1, 24), nb = W->nb;
    const unsigned nbu = (unsigned)((n + 2 * UPD_PAIRS * KT - 1) / (2 * UPD_PAIRS * KT));
    GS2_TRY_HIP(hipMemsetAsync(W->V, 0, sizeof(double) * (size_t)n * (jt + 2), s));
    GS2_TRY_HIP(hipMemsetAsync(W->w, 0, sizeof(double) * (size_t)n, s));
    k_probe_state<<<1, 64, 0, s>>>(W->st, jt);
    GS2_TRY_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    GS2_TRY_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    GS2_TRY_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    int st = GS2_OK;
    auto timed = [&](auto launch) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < 4 && st == GS2_OK; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) st = GS2_ERR_HIP;
            for (int b = 0; b < 3; ++b) launch();
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = GS2_ERR_HIP;
            float t = 0.f;
            if (st == GS2_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = GS2_ERR_HIP;
            if (rep > 0) best = std::min(best, t);
        }
        return best;
    };
    GState *gs = W->st;
    const float dw = timed([&] { k_dot2<8><<<(unsigned)nb, KT, 0, s>>>(n, W->w, W->V, n, gs, W->part, nb); });
    const float dn = timed([&] { k_dot2<2><<<(unsigned)nb, KT, 0, s>>>(n, W->w, W->V, n, gs, W->part, nb); });
    const float uw = timed([&] {
        k_dcgs_update_pairs<UPD_PAIRS, UPD_PAIRS><<<nbu, KT, 0, s>>>(n, W->V, n, gs, W->w, W->part);
    });
    const float un = timed([&] { k_dcgs_update_pairs<UPD_PAIRS, 1><<<nbu, KT, 0, s>>>(n, W->V, n, gs, W->w, W->part); });
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    GS2_TRY(st);
    GS2_TRY_HIP(hipGetLastError());
    if (dn < 0.97f * dw) W->dot_narrow = DOT_NARROW_FROM;
    if (un < 0.97f * uw) W->upd_narrow = UPD_NARROW_FROM;
    W->basis_tuned = 1;
    return GS2_OK;
}

// Time of one product in the layout sel (best of three batches of five
// launches after a warm-up batch; timing-only events): w2 = b - A w, or for
// the block copy the kernel the solver's steps use, w2 = A w.
static int time_product(GmresWork *W, int sel, hipStream_t s, float *ms)
{
    const int64_t n = W->n;
    const int nb = W->nb;
    const SellAView AS = view(W->A);
    const DiaAView AD = dview(W->A);
    hipEvent_t e0, e1;
    GS2_TRY_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    GS2_TRY_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    k_zero64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, W->w);
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
        GS2_TRY_HIP(hipEventRecord(e0, s));
        for (int b = 0; b < 5; ++b) {
            if (sel <= -10) {
                const int R = -sel - 10;
                const unsigned gD = (unsigned)((n / 3 + (int64_t)KT * R - 1) / ((int64_t)KT * R));
                if (R == 2) k_b3_spmv<2><<<gD, KT, 0, s>>>(AD, n, W->w, W->w2, nullptr);
                else k_b3_spmv<1><<<gD, KT, 0, s>>>(AD, n, W->w, W->w2, nullptr);
            } else {
                GS2_SPMV_DISPATCH(sel, k_true_resid, (unsigned)nb, AS, AD, n, W->w, W->w, W->w2, W->part, nb);
            }
        }
        GS2_TRY_HIP(hipEventRecord(e1, s));
        GS2_TRY_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        GS2_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
        if (rep > 0) best = std::min(best, t / 5);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return GS2_OK;
}

static int build_layout(SellA &S, const gs2_csr &A, int sel, const std::vector<int> &offs, hipStream_t s)
{
    if (sel > 0) return sella_build_sell(S, A, sel, s);
    if (sel <= -10) GS2_TRY(sella_build_b3(S, A, -sel - 10, offs, s));
    else GS2_TRY(sella_build_dia(S, A, -sel, offs, s));
    return sella_fill_values(S, A, false, s);
}

// The layout of the solver's copy of A, chosen once per CSR pattern (keyed
// by its row-pointer and column arrays and sizes) and kept with the
// workspace; the values are copied again at every solve, so values changed
// in place between solves are honoured.  Candidates: sliced ELL at the
// lanes per row the mean row length suggests and at twice that, and, when
// A qualifies, the diagonal copy at one and two rows per lane (8- and
// 16-byte value loads) or, failing that, the 3-row block copy at one and
// two nodes per lane.  fmt GS2_FORMAT_AUTO times them (one product each;
// a later candidate must win by 3 %) on matrices of at least
// SPMV_TUNE_MIN_ROWS rows; GS2_FORMAT_SELL / _DIA / _BLOCK3 force a layout
// (the diagonal one at two rows per lane, the block one at two nodes per
// lane, falling back to sliced ELL when A does not qualify).
static int prepare_matrix(GmresWork *W, const gs2_csr &A, int fmt, hipStream_t s)
{
    SellA &S = W->A;
    if (S.rp == A.rowptr && S.ci == A.colind && S.n == A.n && S.nnz == A.nnz && (S.val || S.dval) &&
        W->fmt_req == fmt)
        return sella_fill_values(S, A, false, s);
    sella_free(S);
    std::vector<int> offs;
    int hst = GS2_OK;
    const bool dia_ok = fmt != GS2_FORMAT_SELL && fmt != GS2_FORMAT_BLOCK3 && sella_dia_offsets(A, offs, s, &hst);
    GS2_TRY(hst);
    const bool b3_ok = !dia_ok && fmt != GS2_FORMAT_SELL && fmt != GS2_FORMAT_DIA && sella_b3_offsets(A, offs, s, &hst);
    GS2_TRY(hst);
    const int K0 = sella_rule_lanes(A);
    int sel = K0, tuned = 0;
    if (fmt == GS2_FORMAT_DIA && dia_ok) {
        sel = -2;
    } else if (fmt == GS2_FORMAT_BLOCK3 && b3_ok) {
        sel = -12;
    } else if (fmt == GS2_FORMAT_AUTO && A.n >= SPMV_TUNE_MIN_ROWS) {
        std::vector<int> cands{K0};
        if (K0 < WAVE) cands.push_back(2 * K0);
        if (dia_ok) {
            cands.push_back(-1);
            cands.push_back(-2);
        }
        if (b3_ok) {
            cands.push_back(-11);
            cands.push_back(-12);
        }
        float best = 1e30f;
        std::vector<int> timed;
        for (int c : cands) {
            GS2_TRY(build_layout(S, A, c, offs, s));
            // the padding rule may widen a sliced-ELL candidate to one already timed
            if (std::find(timed.begin(), timed.end(), S.sel) != timed.end()) continue;
            timed.push_back(S.sel);
            float ms = 0.f;
            GS2_TRY(time_product(W, S.sel, s, &ms));
            if (ms < 0.97f * best) {
                best = ms;
                sel = S.sel;
            }
        }
        tuned = 1;
    }
    if (S.sel != sel || !(S.val || S.dval)) GS2_TRY(build_layout(S, A, sel, offs, s));
    S.tuned = tuned;
    S.rp = A.rowptr; // complete: key it
    S.ci = A.colind;
    W->fmt_req = fmt;
    return GS2_OK;
}

static int gmres_impl(const gs2_csr &A, const double *b, double *x, int m, double rtol, int maxit, int kind,
                      gs2_handle *P, gs2_solve_info *info, hipStream_t s)
{
    const int64_t n = A.n;
    GmresWork *own = nullptr;
    GmresWork *W = nullptr;
    if (P) {
        if (!P->h.gw || P->h.gw->n != n || P->h.gw->m < m) {
            if (P->h.gw) free_gmres_work(P->h.gw);
            P->h.gw = nullptr;
            GS2_TRY(alloc_work(&P->h.gw, n, m));
        }
        W = P->h.gw;
    } else {
        GS2_TRY(alloc_work(&own, n, m));
        W = own;
    }
    struct Guard {
        GmresWork *g;
        ~Guard() { if (g) free_gmres_work(g); }
    } guard{own};

    const int nb = W->nb;
    const unsigned gN = (unsigned)nb;
    const unsigned gE = (unsigned)((n + 255) / 256);
    GS2_TRY(prepare_matrix(W, A, P ? P->h.spmv_fmt : GS2_FORMAT_AUTO, s));
    GS2_TRY(tune_basis(W, P ? P->h.basis_req : 0, s));
    const SellAView AS = view(W->A);
    const DiaAView AD = dview(W->A);
    const int K = W->A.sel;
    GState *st = W->st;
    GHeader *hdr = W->hdr;
    if (P) P->h.stop = &st->done;
    struct StopReset {
        gs2_handle *P;
        ~StopReset() { if (P) P->h.stop = nullptr; }
    } stop_reset{P};

    auto read_hdr = [&]() -> int {
        GS2_TRY_HIP(hipMemcpyAsync(hdr, st, sizeof(GHeader), hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        return GS2_OK;
    };

    info->iterations = 0;
    info->restarts = 0;
    info->converged = 0;
    info->relres = 0.0;
    k_norm_part<<<gN, KT, 0, s>>>(n, b, W->part, nb);
    k_reduce<<<1, KT, 0, s>>>(W->part, nb, st, 8, 0, 1);
    GS2_TRY_HIP(hipGetLastError());
    GS2_TRY(read_hdr());
    const double bnorm = hdr->bnorm;
    if (!std::isfinite(bnorm)) return GS2_ERR_NONFINITE;
    if (bnorm == 0.0) {
        k_zero64<<<gE, 256, 0, s>>>(n, x);
        GS2_TRY_HIP(hipStreamSynchronize(s));
        info->converged = 1;
        return GS2_OK;
    }
    // orthogonalisation: 0 = delayed CGS2 (default), 1 = CGS2
    const int orth = P ? P->h.orth : 0;
    // z_j is always a copy: the delayed variant rewrites v_j after z_j was formed
    double *Zb = W->Z;
    int total = 0, cycles = 0, status = GS2_OK;
    bool have_prev = false;
    // stagnation: the true residual at the end of a cycle has not halved for
    // `stag` consecutive cycles (0 = default 50; < 0 = no test)
    const int stag = P ? (P->h.stag_cycles == 0 ? 50 : P->h.stag_cycles) : 50;
    double ref_res = -1.0;
    int ref_cycle = 0;
    // algorithmic bytes: SpMV with A (entries, slice pointers, z gathered once,
    // w written), and one pass over nk Krylov vectors
    const double spmv_b = sella_bytes(W->A);
    const double red_b = 8.0 * nb;
    for (;;) {
        prof_set_step(cycles, -1);
        {
            Prof pr(s, PK_TRUE_RESID, spmv_b + 8.0 * n);
            GS2_SPMV_DISPATCH(K, k_true_resid, gN, AS, AD, n, x, b, W->V, W->part, nb);
        }
        {
            Prof pr(s, PK_REDUCE, red_b);
            k_reduce<<<1, KT, 0, s>>>(W->part, nb, st, 9, 0, 1);
        }
        GS2_TRY_HIP(hipGetLastError());
        GS2_TRY(read_hdr());
        if (have_prev) {
            total += hdr->kk;
            prof_drop_from_step(cycles - 1, hdr->kk);
            if (hdr->status != GS2_OK) { status = hdr->status; break; }
        }
        const double beta = hdr->beta;
        info->relres = beta / bnorm;
        if (!std::isfinite(beta)) { status = GS2_ERR_NONFINITE; break; }
        if (info->relres <= rtol) { info->converged = 1; break; }
        if (total >= maxit) { status = GS2_NOT_CONVERGED; break; }
        if (ref_res < 0.0 || info->relres < 0.5 * ref_res) {
            ref_res = info->relres;
            ref_cycle = cycles;
        } else if (stag > 0 && cycles - ref_cycle >= stag) {
            status = GS2_STAGNATED;
            break;
        }
        if (cycles > 0) info->restarts++;
        cycles++;
        const int steps = std::min(m, maxit - total);
        // one restart cycle, enqueued on stream `cs`
        // The serial work closing step j (k_dcgs_finish) runs as one extra
        // workgroup of the next step's first preconditioner pass when that is
        // a GS2 or JR pass: it needs only step j's partial sums and the state,
        // and the pass needs neither.  The last step's runs alone.
        const bool fuse_fin = orth == 0 && P && (kind == GS2_PREC_GS2 || kind == GS2_PREC_JR);
        // the second basis pass loads pairs of rows when every column is 16-byte aligned
        const bool pairs = n % 2 == 0;
        const int nbu = pairs ? (int)((n + 2 * UPD_PAIRS * KT - 1) / (2 * UPD_PAIRS * KT)) : nb;
        auto enqueue_cycle = [&](hipStream_t cs) -> int {
            k_cycle_init<<<1, 64, 0, cs>>>(st, steps, rtol);
            k_scale0<<<gE, 256, 0, cs>>>(n, W->V, st);
            for (int j = 0; j < steps; ++j) {
                prof_set_step(cycles - 1, j);
                const double *vj = W->V + (int64_t)j * n;
                double *zj = Zb + (int64_t)j * n;
                const double vb = 8.0 * n * (j + 1);
                if (orth == 0) { // delayed CGS2
                    if (fuse_fin && j > 0) P->h.fin = Handle::FinJob{W->part, nbu, st}; // closes step j-1
                    GS2_TRY(precondition(kind, P, vj, zj, n, st, cs));
                    if (K < 0) { // diagonal or block copy: the product, then the dot products
                        {
                            Prof pr(cs, PK_SPMV, spmv_b);
                            const int R = K <= -10 ? -K - 10 : -K;
                            const int64_t units = K <= -10 ? n / 3 : n; // nodes or rows
                            const unsigned gD = (unsigned)((units + (int64_t)KT * R - 1) / ((int64_t)KT * R));
                            if (K <= -10) {
                                if (K == -12) k_b3_spmv<2><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                                else k_b3_spmv<1><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                            } else if (AD.ndiag == 7) {
                                if (K == -2) k_dia_spmv<2, 7><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                                else k_dia_spmv<1, 7><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                            } else {
                                if (K == -2) k_dia_spmv<2, 0><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                                else k_dia_spmv<1, 0><<<gD, KT, 0, cs>>>(AD, n, zj, W->w, st);
                            }
                        }
                        Prof pr(cs, PK_SPMV_DOT, vb + 8.0 * n);
                        if (j < W->dot_narrow) k_dot2<8><<<gN, KT, 0, cs>>>(n, W->w, W->V, n, st, W->part, nb);
                        else k_dot2<2><<<gN, KT, 0, cs>>>(n, W->w, W->V, n, st, W->part, nb);
                    } else {
                        Prof pr(cs, PK_SPMV_DOT, spmv_b + vb);
                        hipStream_t s = cs;
                        GS2_SPMV_DISPATCH(K, k_spmv_dot2, gN, AS, AD, n, zj, W->w, W->V, n, st, W->part, nb);
                    }
                    {
                        Prof pr(cs, PK_REDUCE, red_b * (2 * j + 3));
                        k_reduce<<<2 * j + 3, KT, 0, cs>>>(W->part, nb, st, 3, 0, 2 * j + 3);
                    }
                    {
                        Prof pr(cs, PK_CGS, 8.0 * n * (j + 4));
                        if (!pairs)
                            k_dcgs_update<<<gN, KT, 0, cs>>>(n, W->V, n, st, W->w, W->part);
                        else if (j < W->upd_narrow)
                            k_dcgs_update_pairs<UPD_PAIRS, UPD_PAIRS>
                                <<<(unsigned)nbu, KT, 0, cs>>>(n, W->V, n, st, W->w, W->part);
                        else
                            k_dcgs_update_pairs<UPD_PAIRS, 1><<<(unsigned)nbu, KT, 0, cs>>>(n, W->V, n, st, W->w, W->part);
                    }
                    if (!fuse_fin || j == steps - 1) {
                        Prof pr(cs, PK_GIVENS, red_b);
                        k_dcgs_finish<<<1, KT, 0, cs>>>(W->part, nbu, st);
                    }
                    GS2_TRY_HIP(hipGetLastError());
                    continue;
                }
                GS2_TRY(precondition(kind, P, vj, zj, n, st, cs));
                {   // w = A z_j, hA = V^T w, ||w||^2
                    Prof pr(cs, PK_SPMV_DOT, spmv_b + vb);
                    hipStream_t s = cs;
                    GS2_SPMV_DISPATCH(K, k_spmv_dot, gN, AS, AD, n, zj, W->w, W->V, n, st, W->part, nb, 0);
                }
                {
                    Prof pr(cs, PK_REDUCE, red_b * (j + 2));
                    k_reduce<<<j + 2, KT, 0, cs>>>(W->part, nb, st, 0, 1, 0);
                }
                {   // w2 = w - V hA ; hB = V^T w2
                    Prof pr(cs, PK_CGS, vb + 16.0 * n);
                    k_update_dot<<<gN, KT, 0, cs>>>(n, W->V, n, st, 0, W->w, W->w2, 1, 0, W->part, nb);
                }
                {
                    Prof pr(cs, PK_REDUCE, red_b * (j + 1));
                    k_reduce<<<j + 1, KT, 0, cs>>>(W->part, nb, st, 1, 0, 0);
                }
                {   // v_{j+1} = w2 - V hB ; ||v_{j+1}||^2
                    Prof pr(cs, PK_CGS, vb + 16.0 * n);
                    k_update_dot<<<gN, KT, 0, cs>>>(n, W->V, n, st, 1, W->w2, W->V + (int64_t)(j + 1) * n, 0, 1,
                                                    W->part, nb);
                }
                {
                    Prof pr(cs, PK_REDUCE, red_b);
                    k_reduce<<<1, KT, 0, cs>>>(W->part, nb, st, 2, 0, 1);
                }
                {
                    Prof pr(cs, PK_GIVENS, 0.0);
                    k_givens<<<1, 64, 0, cs>>>(st);
                }
                {
                    Prof pr(cs, PK_SCALE, 16.0 * n);
                    k_scale_next<<<gE, 256, 0, cs>>>(n, W->V, n, st);
                }
                GS2_TRY_HIP(hipGetLastError());
            }
            prof_set_step(cycles - 1, -1);
            k_backsolve<<<1, WAVE, 0, cs>>>(st);
            {
                Prof pr(cs, PK_UPDATE_X, 8.0 * n * steps + 16.0 * n);
                if (n % 2 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0)
                    k_update_x_pairs<4, UPDX_G>
                        <<<(unsigned)((n + 8 * KT - 1) / (8 * KT)), KT, 0, cs>>>(n, Zb, n, st, x);
                else
                    k_update_x<<<gE, KT, 0, cs>>>(n, Zb, n, st, x);
            }
            GS2_TRY_HIP(hipGetLastError());
            return GS2_OK;
        };
        // Replay the cycle from a HIP graph, captured once per set of pointers
        // and parameters (with a handle: its work space outlives the call).
        // Per-kernel event profiling needs the launches one by one.
        if (P && g_graphs.load() && !prof_on()) {
            const CycleKey key{A.rowptr, A.colind, A.val, b, x, P, W->A.sel < 0 ? (const void *)W->A.dval : W->A.val,
                               kind, m, steps, rtol, orth};
            if (!(W->exec && W->key == key)) GS2_TRY(capture_cycle(W, key, enqueue_cycle));
            GS2_TRY_HIP(hipGraphLaunch(W->exec, s));
        } else {
            GS2_TRY(enqueue_cycle(s));
        }
        have_prev = true;
    }
    prof_set_step(0, -1);
    info->iterations = total;
    return status;
}

} // namespace gs2

using namespace gs2;

extern "C" int gs2_graphs(int enable) { return g_graphs.exchange(enable != 0 ? 1 : 0); }

extern "C" int gs2_gmres_schedule(const gs2_handle *H, int *format, int *lanes_per_row, int *rows_per_lane,
                                  int *ndiag, int *tuned)
{
    if (!H) return GS2_ERR_ARG;
    const GmresWork *W = H->h.gw;
    const bool built = W && (W->A.val || W->A.dval);
    const int sel = built ? W->A.sel : 0;
    if (format) *format = !built ? 0 : sel <= -10 ? GS2_FORMAT_BLOCK3 : sel < 0 ? GS2_FORMAT_DIA : GS2_FORMAT_SELL;
    if (lanes_per_row) *lanes_per_row = sel > 0 ? sel : 0;
    if (rows_per_lane) *rows_per_lane = sel <= -10 ? -sel - 10 : sel < 0 ? -sel : 0;
    if (ndiag) *ndiag = sel < 0 ? W->A.ndiag : 0;
    if (tuned) *tuned = built ? W->A.tuned : 0;
    return GS2_OK;
}

extern "C" int gs2_gmres_basis_schedule(const gs2_handle *H, int *dot_narrow_from, int *update_narrow_from, int *tuned)
{
    if (!H) return GS2_ERR_ARG;
    const GmresWork *W = H->h.gw;
    const bool done = W && W->basis_tuned;
    if (dot_narrow_from) *dot_narrow_from = !done ? 0 : W->dot_narrow == INT_MAX ? -1 : W->dot_narrow;
    if (update_narrow_from) *update_narrow_from = !done ? 0 : W->upd_narrow == INT_MAX ? -1 : W->upd_narrow;
    if (tuned) *tuned = !done || W->basis_tuned == 2 ? 0 : (W->n >= BASIS_TUNE_MIN_ROWS && W->m >= 16 && W->n % 2 == 0) ? 1 : 0;
    return GS2_OK;
}

extern "C" int gmres_solve(const gs2_csr *A, const double *b, double *x, int restart, double rtol, int maxit,
                           int prec_kind, gs2_handle *prec, gs2_solve_info *info, void *stream)
{
    gs2_solve_info local;
    gs2_solve_info *inf = info ? info : &local;
    std::memset(inf, 0, sizeof(*inf));
    int st = GS2_ERR_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    if (!A || A->n <= 0 || A->n >= (int64_t(1) << 31) - 1 || !A->rowptr || !A->colind || !A->val || !b || !x ||
        restart < 1 || restart > MAXM || !(rtol >= 0.0) || maxit < 0 || prec_kind < GS2_PREC_NONE ||
        prec_kind > GS2_PREC_MTGS || (prec_kind != GS2_PREC_NONE && !prec) || (prec && prec->h.n != A->n)) {
        st = GS2_ERR_ARG;
    } else if ((prec_kind == GS2_PREC_GS_TRISOLVE && prec->h.nlev_l == 0) ||
               (prec_kind == GS2_PREC_MTGS && prec->h.ncolors == 0)) {
        st = GS2_ERR_NO_LEVELS;
    } else {
        try {
            st = gmres_impl(*A, b, x, restart, rtol, maxit, prec_kind, prec, inf, (hipStream_t)stream);
        } catch (const std::bad_alloc &) {
            st = GS2_ERR_NOMEM;
        } catch (...) {
            st = GS2_ERR_HIP;
        }
    }
    inf->status = st;
    inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}
