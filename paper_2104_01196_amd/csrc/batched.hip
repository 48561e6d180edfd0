// Batched GS2-preconditioned GMRES for many independent systems of uneven
// sizes, each with several right-hand sides (the segregated multiple-RHS
// systems of Section 11 motivate it).
//
// One persistent kernel launch solves everything.  A work item is one system
// together with a group of R right-hand sides, solved start to finish by a
// team of G workgroups: G = 1 for most items, so that every reduction and
// every ordering point is a workgroup barrier, and up to 8 for the largest,
// whose single-workgroup time (rows x iterations, and the iteration count
// grows with the system) would otherwise outlast everything else.  Workgroups
// pop (item, member) slots from an atomic counter, largest systems first
// (longest processing time first), and leave when the queue is empty.  A
// team's rows are split among its members; its passes are separated by a
// barrier on a per-item arrival counter (agent-scope release / acquire), and
// its reductions sum the members' partials in member order, so every member
// holds bit-identical scalars and repeats the small serial work itself.  The
// R right-hand sides of an item are stored interleaved (row-major n x R), so
// each matrix entry is loaded once per group and applied to R vectors (an
// SpMM-like access).
// Each right-hand side keeps its own Hessenberg matrix, rotations and
// convergence flag; a right-hand side that has converged stops contributing
// while the others continue.  The Arnoldi process is classical Gram-Schmidt
// with delayed reorthogonalisation (two passes over the basis per step, as in
// the single-system solver).  The launch is captured in a HIP graph at setup
// and replayed by every solve; its arguments live in device memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <numeric>

#include "gs2_internal.hpp"

namespace gs2 {

constexpr int BT = 512;        // threads per workgroup of the persistent solver
constexpr int BNW = BT / WAVE; // wavefronts per workgroup
constexpr int BMAXM = 32;      // longest restart of the batched solver
// Krylov vectors per chunk of a multi-dot: 16 accumulators per thread
template <int R>
constexpr int kc_of()
{
    return 8 / R;
}
constexpr int RED_STRIDE = 20; // >= (16/R + 1) * R for R in {1, 2, 4}

struct BSys {
    int64_t n, nslices;
    const int64_t *Lsp, *Usp;
    const int32_t *Lcol, *Ucol;
    const void *Lval, *Uval;
    const double *sl, *sr;
    const int32_t *rp, *ci;
    const double *va;
    int64_t row0; // rows of all earlier systems
};

struct BItem {
    int sys, r0;
    int64_t base; // scalar offset (row x rhs units) of this item's vectors
    int G;        // workgroups in the item's team
    int pad;
    int64_t xoff; // offset of the team's exchange area (2 x G x XS doubles)
};

struct BSlot {
    int item, member;
};

struct BParams {
    const double *B;
    double *X;
    double rtol;
    int maxit, pad;
};

struct BConst {
    const BSys *sys;
    const BItem *items;
    int nitems, m, nrhs;
    int sweeps, inner, variant, compact;
    double omega, gamma;
    double *V, *Z, *W; // float64 work: (m+1), m, 2 vectors per item
    void *P;           // preconditioner vectors, 5 per item
    unsigned *queue;
    gs2_solve_info *info;
    const BParams *prm;
    const BSlot *slots;
    int nslots, pad;
    unsigned *tbar;   // per item: team barrier arrivals
    double *xch;      // team reduction exchange areas
    int *abort;       // set when a team barrier times out
    long long spin_ticks; // wall-clock ticks a team barrier may wait
};

// Exchange slots per member and buffer: the largest team reduction is pass 1
// of the delayed reorthogonalisation, (2m + 3) R values.
constexpr int XS = (2 * BMAXM + 3) * 4 + 4;

// A team of G workgroups solving one item; member me.  ep (in LDS) counts
// the team barriers passed (the same in every member), ab (in LDS) is set
// once the team has aborted.  With G = 1 every team operation is a plain
// workgroup barrier.
struct BTeam {
    int G, me;
    unsigned *bar;
    double *xch;
    int *abort;
    long long spin;
    unsigned *ep;
    int *ab;
};

// this workgroup's share of an item's rows: thread / wavefront index within
// the team and the team's totals
__device__ __forceinline__ int64_t tthread(const BTeam &T) { return (int64_t)T.me * BT + threadIdx.x; }
__device__ __forceinline__ int64_t tthreads(const BTeam &T) { return (int64_t)T.G * BT; }
__device__ __forceinline__ int64_t twave(const BTeam &T) { return (int64_t)T.me * BNW + threadIdx.x / WAVE; }
__device__ __forceinline__ int64_t twaves(const BTeam &T) { return (int64_t)T.G * BNW; }

// Team barrier: every member's global writes before it are visible to every
// member after it.  Each wavefront first waits for its own stores to reach
// the L2 (a workgroup barrier alone does not), then one thread per workgroup
// arrives with a release at agent scope (the L2 is written back, which makes
// the writes visible to workgroups on other XCDs) and waits for
// G * (epoch + 1) arrivals; every thread then acquires at agent scope.  The
// wait is bounded: past spin ticks of the wall clock the abort flag is
// raised, every waiting member leaves, and the item ends with an error
// instead of a hang.  Returns false once aborted.  Out of line, so that
// single-workgroup items (G = 1, a plain workgroup barrier) do not carry its
// registers.
__device__ __noinline__ bool team_wait(const BTeam T)
{
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(T.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (unsigned)T.G * (*T.ep + 1);
        const long long t0 = wall_clock64();
        int ab = 0;
        while (__hip_atomic_load(T.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(T.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ab = 1;
                break;
            }
            if (wall_clock64() - t0 > T.spin) {
                __hip_atomic_store(T.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (ab) *T.ab = 1;
        *T.ep += 1;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *T.ab == 0;
}

__device__ __forceinline__ bool team_sync(const BTeam &T)
{
    __syncthreads();
    if (T.G == 1) return true;
    return team_wait(T);
}

// Sum the members' partials of up to three LDS arrays (lengths c0, c1, c2,
// c0 + c1 + c2 <= XS) in member order; every member gets the same bits.
// Buffers alternate with the barrier count, so a member that runs ahead into
// the next reduction never overwrites partials still being read.
__device__ __noinline__ void team_sum_wait(const BTeam T, double *a0, int c0, double *a1, int c1, double *a2, int c2)
{
    const int tot = c0 + c1 + c2;
    double *buf = T.xch + (size_t)(*T.ep & 1u) * T.G * XS;
    for (int i = threadIdx.x; i < tot; i += BT)
        buf[(size_t)T.me * XS + i] = i < c0 ? a0[i] : i < c0 + c1 ? a1[i - c0] : a2[i - c0 - c1];
    __syncthreads();
    if (!team_wait(T)) return;
    for (int i = threadIdx.x; i < tot; i += BT) {
        double s = 0.0;
        for (int q = 0; q < T.G; ++q) s += buf[(size_t)q * XS + i];
        if (i < c0) a0[i] = s;
        else if (i < c0 + c1) a1[i - c0] = s;
        else a2[i - c0 - c1] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ void team_sum(const BTeam &T, double *a0, int c0, double *a1 = nullptr, int c1 = 0,
                                         double *a2 = nullptr, int c2 = 0)
{
    if (T.G == 1) return;
    team_sum_wait(T, a0, c0, a1, c1, a2, c2);
}

enum : int { BD_G = 0, BD_XADD = 1, BD_XSET = 2, BD_ZADD = 3, BD_ZSET = 4 };

template <typename AT, int R>
__device__ __forceinline__ void bfinish(int dst, int64_t row, const AT (&g)[R], AT w, AT *gout, AT *xh, AT *xout,
                                        double *z, const double *sr)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row * R + r;
        switch (dst) {
        case BD_G: gout[i] = g[r]; break;
        case BD_XADD: xout[i] = xh[i] + w * g[r]; break;
        case BD_XSET: xout[i] = w * g[r]; break;
        case BD_ZADD: z[i] = sr[row] * (double)(xh[i] + w * g[r]); break;
        default: z[i] = sr[row] * (double)(w * g[r]); break;
        }
    }
}

// A workgroup has only BNW wavefronts for a whole system, so each wavefront
// works on BU slices at once: their (slice pointer -> column -> gathered
// value) chains are in flight together instead of one after the other.
template <typename AT, int R>
constexpr int bu_of()
{
    return (sizeof(AT) == 8 ? 2 : 4) / R > 0 ? (sizeof(AT) == 8 ? 2 : 4) / R : 1;
}

// acc[u][r] += sum over the stored entries of slice s0 + u of val * src(col, r)
template <typename VT, typename AT, int R, int BU, typename Src>
__device__ __forceinline__ void bslice_dots(const int64_t *sp, const int32_t *col, const VT *val, int64_t s0,
                                            int64_t nslices, int lane, Src src, AT (&acc)[BU][R])
{
    int64_t beg[BU];
    int steps[BU];
    int tmax = 0;
#pragma unroll
    for (int u = 0; u < BU; ++u) {
        const int64_t s = s0 + u;
        const bool ok = s < nslices;
        beg[u] = ok ? sp[s] : 0;
        steps[u] = ok ? (int)((sp[s + 1] - beg[u]) / WAVE) : 0;
        tmax = steps[u] > tmax ? steps[u] : tmax;
    }
    // TS steps at a time: first every (column, value) load of the chunk, then
    // the gathers they feed, so one chunk costs two memory latencies
    constexpr int TS = 4;
    for (int t0 = 0; t0 < tmax; t0 += TS) {
        int cc[BU][TS];
        AT av[BU][TS];
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
            for (int q = 0; q < TS; ++q) {
                const bool in = t0 + q < steps[u];
                const int64_t p = beg[u] + (int64_t)(in ? t0 + q : 0) * WAVE + lane;
                cc[u][q] = in ? col[p] : -1;
                av[u][q] = in ? (AT)val[p] : AT(0);
            }
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
            for (int q = 0; q < TS; ++q)
                if (cc[u][q] >= 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[u][r] += av[u][q] * src(cc[u][q], r);
                }
    }
}

// inner JR pass g = rh - w T g_old for R interleaved right-hand sides
template <typename VT, typename AT, int R, int K>
__device__ void bp_inner(const BTeam T, const BSys &S, int lower, const AT *rh, const AT *gin, const double *v, int rv,
                         int gv, int damp, AT w, AT gamma, int dst, AT *gout, AT *xh, double *z)
{
    constexpr int BU = bu_of<AT, R>();
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t *sp = lower ? S.Lsp : S.Usp;
    const int32_t *col = lower ? S.Lcol : S.Ucol;
    const VT *val = (const VT *)(lower ? S.Lval : S.Uval);
    for (int64_t s0 = twave(T) * BU; s0 < S.nslices; s0 += twaves(T) * BU) {
        AT acc[BU][R];
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[u][r] = AT(0);
        if (gv)
            bslice_dots<VT, AT, R, BU>(sp, col, val, s0, S.nslices, lane,
                                       [&](int c, int r) { return (AT)(v[(int64_t)c * R + r] * S.sl[c]); }, acc);
        else
            bslice_dots<VT, AT, R, BU>(sp, col, val, s0, S.nslices, lane,
                                       [&](int c, int r) { return gin[(int64_t)c * R + r]; }, acc);
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            if (K > 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) acc[u][r] = group_sum<K>(acc[u][r]);
            }
            const int64_t row = (s0 + u) * (WAVE / K) + lane / K;
            if ((K > 1 && (lane & (K - 1))) || row >= S.n) continue;
            AT g[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row * R + r;
                const AT rr = rv ? (AT)(v[i] * S.sl[row]) : rh[i];
                g[r] = rr - w * acc[u][r];
                if (damp) {
                    const AT go = gv ? (AT)(v[i] * S.sl[row]) : gin[i];
                    g[r] = (AT(1) - gamma) * go + gamma * g[r];
                }
            }
            bfinish<AT, R>(dst, row, g, w, gout, xh, xh, z, S.sr);
        }
    }
}

// outer residual (non-compact: both triangles; compact: the opposite one)
template <typename VT, typename AT, int R, int K>
__device__ __forceinline__ void bp_resid(const BTeam T, const BSys &S, int lower, int compact, const AT *xh, const double *v, AT cdiag,
                         AT w, int dst, AT *rh, AT *xout, double *z)
{
    constexpr int BU = bu_of<AT, R>();
    const int lane = threadIdx.x & (WAVE - 1);
    auto gx = [&](int c, int r) { return xh[(int64_t)c * R + r]; };
    for (int64_t s0 = twave(T) * BU; s0 < S.nslices; s0 += twaves(T) * BU) {
        AT acc[BU][R];
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[u][r] = AT(0);
        if (!(compact && lower)) // compact: only the triangle opposite to the inner one
            bslice_dots<VT, AT, R, BU>(S.Lsp, S.Lcol, (const VT *)S.Lval, s0, S.nslices, lane, gx, acc);
        if (!(compact && !lower))
            bslice_dots<VT, AT, R, BU>(S.Usp, S.Ucol, (const VT *)S.Uval, s0, S.nslices, lane, gx, acc);
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            if (K > 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) acc[u][r] = group_sum<K>(acc[u][r]);
            }
            const int64_t row = (s0 + u) * (WAVE / K) + lane / K;
            if ((K > 1 && (lane & (K - 1))) || row >= S.n) continue;
            AT g[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row * R + r;
                g[r] = ((AT)(v[i] * S.sl[row]) - cdiag * xh[i]) - acc[u][r];
            }
            bfinish<AT, R>(dst, row, g, w, rh, const_cast<AT *>(xh), xout, z, S.sr);
        }
    }
}

template <typename AT, int R>
__device__ void bp_first_jr(const BTeam T, const BSys &S, const double *v, AT w, int fin, AT *xh, double *z)
{
    for (int64_t i = tthread(T); i < S.n * R; i += tthreads(T)) {
        const int64_t row = i / R;
        const AT r = (AT)(v[i] * S.sl[row]);
        if (fin) z[i] = S.sr[row] * (double)(w * r);
        else xh[i] = w * r;
    }
}

// z = Mhat^{-1} v for the R right-hand sides of one system (the same pass
// sequence as the single-system apply, with a team barrier between passes).
template <typename VT, typename AT, int R, int K>
__device__ void b_precond(const BTeam &T, const BConst &c, const BSys &S, const double *v, double *z, AT *P)
{
    const int64_t nR = S.n * R;
    AT *xa = P, *xb = P + nR, *rh = P + 2 * nR, *ga = P + 3 * nR, *gb = P + 4 * nR;
    AT *xc = xa, *xo = xb;
    const int per = c.variant == GS2_SYMMETRIC ? 2 : 1;
    const int H = c.sweeps * per;
    const AT w = (AT)c.omega, gamma = (AT)c.gamma;
    const int damp = c.gamma != 1.0;
    const AT cdiag = c.compact ? (AT)(1.0 - 1.0 / c.omega) : AT(1);
    bool xzero = true;
    for (int t = 0; t < H; ++t) {
        const int lower = (c.variant == GS2_FORWARD || (c.variant == GS2_SYMMETRIC && (t % 2) == 0)) ? 1 : 0;
        const bool fin = t == H - 1;
        const bool set = xzero || c.compact;
        if (c.inner == 0) {
            if (xzero) {
                bp_first_jr<AT, R>(T, S, v, w, fin ? 1 : 0, xc, z);
            } else {
                const int dst = fin ? (set ? BD_ZSET : BD_ZADD) : (set ? BD_XSET : BD_XADD);
                bp_resid<VT, AT, R, K>(T, S, lower, c.compact, xc, v, cdiag, w, dst, nullptr, xo, z);
                AT *tmp = xc;
                xc = xo;
                xo = tmp;
            }
            team_sync(T);
        } else {
            int rv = 1;
            if (!xzero) {
                bp_resid<VT, AT, R, K>(T, S, lower, c.compact, xc, v, cdiag, w, BD_G, rh, nullptr, nullptr);
                rv = 0;
                team_sync(T);
            }
            const AT *gin = rh;
            for (int j = 1; j <= c.inner; ++j) {
                const bool last = j == c.inner;
                const int gv = (j == 1 && xzero) ? 1 : 0;
                AT *gout = (j & 1) ? ga : gb;
                const int dst = !last ? BD_G : fin ? (set ? BD_ZSET : BD_ZADD) : (set ? BD_XSET : BD_XADD);
                bp_inner<VT, AT, R, K>(T, S, lower, rh, gin, v, rv, gv, damp, w, gamma, dst, gout, xc, z);
                gin = gout;
                team_sync(T);
            }
        }
        xzero = false;
    }
}

// ------------------------------------------------- block-level Krylov pieces

// w = A z (w = b - A z with bstride > 0, w = scl[r] (A z) with scl) for R
// interleaved vectors; a
// thread works on RU rows (RU*BT apart) at once so that their CSR chains
// (row pointer -> column -> z) are in flight together.
template <int R>
__device__ void b_spmv(const BTeam T, const BSys &S, const double *z, double *w, const double *b, int64_t bstride,
                       const double *scl = nullptr)
{
    constexpr int RU = 4 / R;
    const int64_t NT = tthreads(T);
    for (int64_t r0 = tthread(T); r0 < S.n; r0 += NT * RU) {
        int pb[RU], pe[RU];
        int len = 0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + (int64_t)u * NT;
            pb[u] = row < S.n ? S.rp[row] : 0;
            pe[u] = row < S.n ? S.rp[row + 1] : 0;
            len = pe[u] - pb[u] > len ? pe[u] - pb[u] : len;
        }
        double acc[RU][R];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[u][r] = 0.0;
        constexpr int TS = 4; // entries per row and chunk: loads first, then the gathers
        for (int t0 = 0; t0 < len; t0 += TS) {
            int cc[RU][TS];
            double av[RU][TS];
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int q = 0; q < TS; ++q) {
                    const int p = pb[u] + t0 + q;
                    const bool in = p < pe[u];
                    cc[u][q] = in ? S.ci[p] : -1;
                    av[u][q] = in ? S.va[p] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int q = 0; q < TS; ++q)
                    if (cc[u][q] >= 0) {
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[u][r] += av[u][q] * z[(int64_t)cc[u][q] * R + r];
                    }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + (int64_t)u * NT;
            if (row >= S.n) continue;
#pragma unroll
            for (int r = 0; r < R; ++r)
                w[row * R + r] = b ? b[row * bstride + r] - acc[u][r] : scl ? scl[r] * acc[u][r] : acc[u][r];
        }
    }
}

// out[k*R + r] = <V_k(:,r), w(:,r)> for k < nk, then (with_norm) out[nk*R + r]
// = ||w(:,r)||^2.  Chunks of KC vectors; fixed-order reductions.
template <int R>
__device__ __forceinline__ void b_multidot(const BTeam &T, int64_t n, const double *V, int64_t ldv, int nk, const double *w,
                           int with_norm, double *out, double *red)
{
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t NT = tthreads(T);
    constexpr int KC = kc_of<R>();
    const int stride_red = RED_STRIDE;
    for (int k0 = 0; k0 < nk || (k0 == 0 && with_norm); k0 += KC) {
        const int kc = min(KC, nk - k0);
        const bool nrm = with_norm && k0 == 0;
        double acc[KC][R];
        double nacc[R];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[kk][r] = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) nacc[r] = 0.0;
        // RU rows per thread at once: all their loads are issued before use, since
        // a workgroup's few wavefronts cannot hide one memory latency per row
        constexpr int RU = 2;
        for (int64_t r0 = tthread(T); r0 < n; r0 += NT * RU) {
            double wr[RU][R];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t row = r0 + (int64_t)u * NT;
                const int64_t rr = row < n ? row : n - 1; // clamped; its factor is zero
#pragma unroll
                for (int r = 0; r < R; ++r) wr[u][r] = row < n ? w[rr * R + r] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                if (kk < kc) {
                    const double *vk = V + (int64_t)(k0 + kk) * ldv;
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const int64_t row = r0 + (int64_t)u * NT;
                        const int64_t rr = row < n ? row : n - 1;
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[kk][r] += vk[rr * R + r] * wr[u][r];
                    }
                }
            }
            if (nrm) {
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) nacc[r] += wr[u][r] * wr[u][r];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            if (kk < kc) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double s = wave_sum(acc[kk][r]);
                    if (lane == 0) red[wv * stride_red + kk * R + r] = s;
                }
            }
        }
        if (nrm) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double s = wave_sum(nacc[r]);
                if (lane == 0) red[wv * stride_red + KC * R + r] = s;
            }
        }
        __syncthreads();
        const int cnt = max(kc, 0) * R;
        for (int t = threadIdx.x; t < cnt + (nrm ? R : 0); t += BT) {
            const int slot = t < cnt ? t : KC * R + (t - cnt);
            double s = 0.0;
            for (int q = 0; q < BNW; ++q) s += red[q * stride_red + slot];
            if (t < cnt) out[k0 * R + t] = s;
            else out[nk * R + (t - cnt)] = s;
        }
        __syncthreads();
        if (nk <= 0) break;
    }
    team_sum(T, out, (nk > 0 ? nk : 0) * R + (with_norm ? R : 0));
}

// Pass 1 of the delayed reorthogonalisation for R interleaved right-hand
// sides: outA[k*R + r] = <V_k, u>, outC[k*R + r] = <V_k, w> for k < nk, with
// u = us[r] * uraw (the unnormalised tentative vector and its scale), and
// outN[r], outN[R + r], outN[2R + r] = u.u, u.w, w.w.  Chunks of KC2 vectors
// (2*KC2*R + 3R <= RED_STRIDE reduction slots); fixed-order reductions.
template <int R>
__device__ __forceinline__ void b_multidot2(const BTeam &T, int64_t n, const double *V, int64_t ldv, int nk, const double *uraw,
                            const double *us, const double *w, double *outA, double *outC, double *outN, double *red)
{
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    constexpr int KC2 = 4 / R;
    constexpr int RU = 2;
    const int64_t NT = tthreads(T);
    for (int k0 = 0; k0 < nk || k0 == 0; k0 += KC2) {
        const int kc = min(KC2, nk - k0);
        const bool nrm = k0 == 0;
        double aa[KC2][R], cc[KC2][R], nn[3][R];
#pragma unroll
        for (int kk = 0; kk < KC2; ++kk)
#pragma unroll
            for (int r = 0; r < R; ++r) aa[kk][r] = cc[kk][r] = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) nn[q][r] = 0.0;
        for (int64_t r0 = tthread(T); r0 < n; r0 += NT * RU) {
            double ur[RU][R], wr[RU][R];
            int64_t rr[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t row = r0 + (int64_t)u * NT;
                rr[u] = row < n ? row : n - 1; // clamped; its factors are zero
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    ur[u][r] = row < n ? us[r] * uraw[rr[u] * R + r] : 0.0;
                    wr[u][r] = row < n ? w[rr[u] * R + r] : 0.0;
                }
            }
#pragma unroll
            for (int kk = 0; kk < KC2; ++kk) {
                if (kk < kc) {
                    const double *vk = V + (int64_t)(k0 + kk) * ldv;
#pragma unroll
                    for (int u = 0; u < RU; ++u)
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const double x = vk[rr[u] * R + r];
                            aa[kk][r] += x * ur[u][r];
                            cc[kk][r] += x * wr[u][r];
                        }
                }
            }
            if (nrm) {
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        nn[0][r] += ur[u][r] * ur[u][r];
                        nn[1][r] += ur[u][r] * wr[u][r];
                        nn[2][r] += wr[u][r] * wr[u][r];
                    }
            }
        }
        // slots: [a: KC2*R][c: KC2*R][norms: 3R]
#pragma unroll
        for (int kk = 0; kk < KC2; ++kk) {
            if (kk < kc) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double sa = wave_sum(aa[kk][r]);
                    const double sc = wave_sum(cc[kk][r]);
                    if (lane == 0) {
                        red[wv * RED_STRIDE + kk * R + r] = sa;
                        red[wv * RED_STRIDE + (KC2 + kk) * R + r] = sc;
                    }
                }
            }
        }
        if (nrm) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double sn = wave_sum(nn[q][r]);
                    if (lane == 0) red[wv * RED_STRIDE + 2 * KC2 * R + q * R + r] = sn;
                }
        }
        __syncthreads();
        const int cnt = max(kc, 0) * R;
        for (int t = threadIdx.x; t < 2 * cnt + (nrm ? 3 * R : 0); t += BT) {
            int slot;
            double *dst;
            if (t < cnt) {
                slot = t;
                dst = outA + k0 * R + t;
            } else if (t < 2 * cnt) {
                slot = KC2 * R + (t - cnt);
                dst = outC + k0 * R + (t - cnt);
            } else {
                slot = 2 * KC2 * R + (t - 2 * cnt);
                dst = outN + (t - 2 * cnt);
            }
            double sum = 0.0;
            for (int q = 0; q < BNW; ++q) sum += red[q * RED_STRIDE + slot];
            *dst = sum;
        }
        __syncthreads();
        if (nk <= 0) break;
    }
    const int cnt = (nk > 0 ? nk : 0) * R;
    team_sum(T, outA, cnt, outC, cnt, outN, 3 * R);
}

// Pass 2 for R interleaved right-hand sides: q = (us[r] uraw - sum_k a_k V_k)
// * ia[r] over uraw's slot, w' = w - sum_k c_k V_k - e[r] q into wn, and
// nrm[r] = ||w'||^2.  Vectors outer, RU rows per thread inner.
template <int R>
__device__ __forceinline__ void b_update2(const BTeam &T, int64_t n, const double *V, int64_t ldv, int nk, const double *a,
                          const double *cvec, double *uraw, const double *us, const double *ia, const double *e,
                          const double *w, double *wn, double *nrm, double *red)
{
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    constexpr int RU = 4 / R;
    const int64_t NT = tthreads(T);
    double nacc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) nacc[r] = 0.0;
    for (int64_t r0 = tthread(T); r0 < n; r0 += NT * RU) {
        double aq[RU][R], aw[RU][R];
        int64_t rr[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + (int64_t)u * NT;
            rr[u] = row < n ? row : n - 1; // clamped for loads, skipped for stores
#pragma unroll
            for (int r = 0; r < R; ++r) {
                aq[u][r] = us[r] * uraw[rr[u] * R + r];
                aw[u][r] = w[rr[u] * R + r];
            }
        }
        for (int k = 0; k < nk; ++k) {
            const double *vk = V + (int64_t)k * ldv;
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double x = vk[rr[u] * R + r];
                    aq[u][r] -= a[k * R + r] * x;
                    aw[u][r] -= cvec[k * R + r] * x;
                }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + (int64_t)u * NT;
            if (row >= n) continue;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double qv = aq[u][r] * ia[r];
                const double wp = aw[u][r] - e[r] * qv;
                uraw[row * R + r] = qv;
                wn[row * R + r] = wp;
                nacc[r] += wp * wp;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sn = wave_sum(nacc[r]);
        if (lane == 0) red[wv * RED_STRIDE + r] = sn;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < R; t += BT) {
        double sum = 0.0;
        for (int q = 0; q < BNW; ++q) sum += red[q * RED_STRIDE + t];
        nrm[t] = sum;
    }
    __syncthreads();
    team_sum(T, nrm, R); // also the barrier after the writes of q and w'
}

struct BLds {
    double *red, *hA, *hB, *H, *cs, *sn, *g, *y, *bnorm, *beta, *inv, *wn2, *nrm, *col;
    // delayed reorthogonalisation: tentative column, scale of each stored Z
    // column, ||w'|| of the last step, pass-1 norms (u.u, u.w, w.w), the scale
    // of the current tentative vector, 1/alpha and e of the current step
    double *ht, *zs, *nu, *nrm3, *us, *ia, *ev;
    int *done, *kk, *iters, *restarts, *status, *conv, *flag, *abort;
    unsigned *epoch;
};

__host__ __device__ inline size_t blds_bytes(int m, int R)
{
    const size_t d = (size_t)BNW * RED_STRIDE + 5 * (size_t)(m + 2) * R + (size_t)(m + 1) * m * R +
                     3 * (size_t)m * R + (size_t)(m + 2) * R + 12 * (size_t)R;
    return d * sizeof(double) + (6 * (size_t)R + 4) * sizeof(int) + 64;
}

__device__ inline BLds blds_carve(double *base, int m, int R)
{
    BLds L;
    double *p = base;
    L.red = p; p += BNW * RED_STRIDE;
    L.col = p; p += (m + 2) * R; // Givens work column per right-hand side
    L.hA = p; p += (m + 2) * R;
    L.hB = p; p += (m + 2) * R;
    L.H = p; p += (m + 1) * m * R;
    L.cs = p; p += m * R;
    L.sn = p; p += m * R;
    L.y = p; p += m * R;
    L.g = p; p += (m + 2) * R;
    L.bnorm = p; p += R;
    L.beta = p; p += R;
    L.inv = p; p += R;
    L.wn2 = p; p += R;
    L.nrm = p; p += R;
    L.ht = p; p += (m + 2) * R;
    L.zs = p; p += (m + 2) * R;
    L.nu = p; p += R;
    L.nrm3 = p; p += 3 * R;
    L.us = p; p += R;
    L.ia = p; p += R;
    L.ev = p; p += R;
    int *q = (int *)p;
    L.done = q; q += R;
    L.kk = q; q += R;
    L.iters = q; q += R;
    L.restarts = q; q += R;
    L.status = q; q += R;
    L.conv = q; q += R;
    L.flag = q;
    L.abort = q + 1;
    L.epoch = (unsigned *)(q + 2);
    return L;
}

// (one thread per right-hand side) apply the committed rotations 0..jc-1 of
// right-hand side r to col (jc+2 entries), form rotation jc, store column jc
// of R and advance the residual recurrence g.  False on a zero or
// non-finite rotation radius (status set).
__device__ __forceinline__ bool bcommit(BLds &L, int R, int m, int r, double *col, int jc)
{
    for (int k = 0; k < jc; ++k) {
        const double a = L.cs[k * R + r] * col[k] + L.sn[k * R + r] * col[k + 1];
        col[k + 1] = -L.sn[k * R + r] * col[k] + L.cs[k * R + r] * col[k + 1];
        col[k] = a;
    }
    const double rho = hypot(col[jc], col[jc + 1]);
    if (!isfinite(rho)) {
        L.status[r] = GS2_ERR_NONFINITE;
        return false;
    }
    if (rho == 0.0) {
        L.status[r] = GS2_BREAKDOWN_EXACT;
        return false;
    }
    const double cs = col[jc] / rho, sn = col[jc + 1] / rho;
    L.cs[jc * R + r] = cs;
    L.sn[jc * R + r] = sn;
    col[jc] = rho;
    for (int k = 0; k <= jc; ++k) L.H[(k * m + jc) * R + r] = col[k];
    const double gj = L.g[jc * R + r];
    L.g[(jc + 1) * R + r] = -sn * gj;
    L.g[jc * R + r] = cs * gj;
    return true;
}

template <typename VT, typename AT, int R, int K>
__device__ __forceinline__ void b_solve_item(const BConst &c, const BItem &it, const BTeam &T, BLds &L)
{
    const BSys S = c.sys[it.sys];
    const BParams prm = *c.prm;
    const int m = c.m, nrhs = c.nrhs;
    const int64_t n = S.n, nR = n * R;
    const double *Bb = prm.B + S.row0 * nrhs + it.r0;
    double *Xb = prm.X + S.row0 * nrhs + it.r0;
    double *V = c.V + it.base * (m + 1);
    double *Z = c.Z + it.base * m;
    double *w = c.W + it.base * 2, *w2 = w + nR;
    AT *P = (AT *)c.P + it.base * 5;
    const int t = threadIdx.x;
    const int64_t tt = tthread(T), NT = tthreads(T);
    int *ab = T.ab;
    const double rtol = prm.rtol;
    const int maxit = prm.maxit;
    if (t == 0) {
        *ab = 0;
        *T.ep = 0u;
    }

    // ||b|| per right-hand side: gather b into w (interleaved), then a norm pass
    for (int64_t i = tt; i < nR; i += NT) w[i] = Bb[(i / R) * nrhs + (i % R)];
    team_sync(T);
    b_multidot<R>(T, n, nullptr, 0, 0, w, 1, L.bnorm, L.red); // writes L.bnorm[0..R) = ||b||^2
    if (t < R) {
        L.bnorm[t] = sqrt(L.bnorm[t]);
        L.iters[t] = 0;
        L.restarts[t] = 0;
        L.status[t] = GS2_OK;
        L.conv[t] = 0;
        L.done[t] = 0;
        if (!isfinite(L.bnorm[t])) L.status[t] = GS2_ERR_NONFINITE;
        else if (L.bnorm[t] == 0.0) L.conv[t] = 1;
        L.beta[t] = 0.0;
    }
    __syncthreads();
    // b = 0 -> x = 0
    for (int64_t i = tt; i < nR; i += NT)
        if (L.conv[i % R]) Xb[(i / R) * nrhs + (i % R)] = 0.0;
    // working copy of x in w2 (interleaved)
    for (int64_t i = tt; i < nR; i += NT) w2[i] = Xb[(i / R) * nrhs + (i % R)];
    team_sync(T);

    int cycle = 0;
    while (!*ab) {
        // true residual r = b - A x into V_0, ||r||^2
        b_spmv<R>(T, S, w2, V, Bb, nrhs);
        team_sync(T);
        b_multidot<R>(T, n, nullptr, 0, 0, V, 1, L.beta, L.red);
        if (t == 0) L.flag[0] = 0;
        __syncthreads();
        if (t < R) {
            const double beta = sqrt(L.beta[t]);
            L.beta[t] = beta;
            bool act = false;
            if (L.status[t] == GS2_OK && !L.conv[t]) {
                const double rel = beta / L.bnorm[t];
                if (!isfinite(beta)) L.status[t] = GS2_ERR_NONFINITE;
                else if (rel <= rtol) L.conv[t] = 1;
                else if (L.iters[t] >= maxit) L.status[t] = GS2_NOT_CONVERGED;
                else act = true;
            }
            L.done[t] = act ? 0 : 1;
            L.kk[t] = 0;
            L.inv[t] = act ? 1.0 / beta : 0.0;
            if (act) {
                if (cycle > 0) L.restarts[t]++;
                for (int k = 0; k < m + 2; ++k) L.g[k * R + t] = 0.0;
                L.g[t] = beta;
                atomicOr(L.flag, 1);
            }
        }
        __syncthreads();
        if (!L.flag[0] || *ab) break;
        ++cycle;
        for (int64_t i = tt; i < nR; i += NT) V[i] = L.inv[i % R] == 0.0 ? 0.0 : V[i] * L.inv[i % R];
        if (t < R) L.zs[t] = 1.0; // V_0 is normalised explicitly
        team_sync(T);
        // Arnoldi steps with delayed reorthogonalisation (two passes over the
        // basis per step; the tentative vector V_j stays unnormalised, its
        // scale in zs, and is reorthogonalised one step late)
        for (int j = 0; j < m; ++j) {
            double *vj = V + (int64_t)j * nR;
            double *zj = Z + (int64_t)j * nR;
            b_precond<VT, AT, R, K>(T, c, S, vj, zj, P); // on the raw vector: the apply is linear
            if (t < R) L.us[t] = L.done[t] ? 0.0 : L.zs[j * R + t];
            __syncthreads();
            b_spmv<R>(T, S, zj, w, nullptr, 0, L.us); // w = A z_j, z_j = us * stored column
            team_sync(T);
            // pass 1: a = Q^T u, c = Q^T w, u.u, u.w, w.w (Q = V_0..V_{j-1})
            b_multidot2<R>(T, n, V, nR, j, vj, L.us, w, L.hA, L.hB, L.nrm3, L.red);
            if (t < R) {
                const int r = t;
                L.ia[r] = 0.0;
                L.ev[r] = 0.0;
                if (!L.done[r]) {
                    double *col = L.col + r * (m + 2);
                    double aa = 0.0, ac = 0.0;
                    for (int k = 0; k < j; ++k) {
                        aa += L.hA[k * R + r] * L.hA[k * R + r];
                        ac += L.hA[k * R + r] * L.hB[k * R + r];
                    }
                    const double a2 = L.nrm3[r] - aa;
                    const bool ok = j == 0 || (isfinite(a2) && a2 > 0.0);
                    const double alpha = j == 0 ? 1.0 : sqrt(ok ? a2 : 1.0);
                    if (j > 0 && !isfinite(a2)) {
                        L.status[r] = GS2_ERR_NONFINITE;
                        L.done[r] = 1;
                    } else if (!ok) { // u fell into span(Q): end on the tentative column j-1
                        for (int k = 0; k < j; ++k) col[k] = L.ht[k * R + r];
                        col[j] = L.nu[r];
                        if (bcommit(L, R, m, r, col, j - 1)) L.kk[r] = j;
                        L.done[r] = 1;
                    } else {
                        bool good = true;
                        if (j > 0) { // column j-1 corrected: [ht + nu a; nu alpha]
                            for (int k = 0; k < j; ++k) col[k] = L.ht[k * R + r] + L.nu[r] * L.hA[k * R + r];
                            col[j] = L.nu[r] * alpha;
                            good = bcommit(L, R, m, r, col, j - 1);
                            if (good) L.kk[r] = j;
                        }
                        if (!good) {
                            L.done[r] = 1;
                        } else {
                            const double e = j == 0 ? L.nrm3[R + r] : (L.nrm3[R + r] - ac) / alpha;
                            for (int k = 0; k < j; ++k) L.ht[k * R + r] = L.hB[k * R + r];
                            L.ht[j * R + r] = e;
                            L.wn2[r] = L.nrm3[2 * R + r];
                            L.ia[r] = 1.0 / alpha;
                            L.ev[r] = e;
                        }
                    }
                    if (L.done[r]) {
                        L.us[r] = 0.0;
                        L.ia[r] = 0.0;
                    }
                }
            }
            __syncthreads();
            // pass 2: q_j over V_j, w' = w - Q c - e q_j into V_{j+1}, ||w'||^2
            double *vn = V + (int64_t)(j + 1) * nR;
            b_update2<R>(T, n, V, nR, j, L.hA, L.hB, vj, L.us, L.ia, L.ev, w, vn, L.nrm, L.red);
            if (t == 0) L.flag[0] = 0;
            __syncthreads();
            if (t < R && !L.done[t]) { // tentative rotation of column j, residual estimate, stop test
                const int r = t;
                double *col = L.col + r * (m + 2);
                const double nu = sqrt(L.nrm[r]);
                L.nu[r] = nu;
                for (int k = 0; k <= j; ++k) col[k] = L.ht[k * R + r];
                col[j + 1] = nu;
                for (int k = 0; k < j; ++k) {
                    const double a = L.cs[k * R + r] * col[k] + L.sn[k * R + r] * col[k + 1];
                    col[k + 1] = -L.sn[k * R + r] * col[k] + L.cs[k * R + r] * col[k + 1];
                    col[k] = a;
                }
                const double rho = hypot(col[j], col[j + 1]);
                if (!isfinite(rho) || !isfinite(nu)) {
                    L.status[r] = GS2_ERR_NONFINITE;
                    L.done[r] = 1;
                } else {
                    L.iters[r]++;
                    const double est = rho > 0.0 ? fabs(col[j + 1] / rho * L.g[j * R + r]) : 0.0;
                    const bool bd = nu <= 1e-14 * sqrt(L.wn2[r]);
                    if (est <= rtol * L.bnorm[r] || bd || j + 1 >= m || L.iters[r] >= maxit) {
                        for (int k = 0; k <= j; ++k) col[k] = L.ht[k * R + r];
                        col[j + 1] = nu;
                        if (bcommit(L, R, m, r, col, j)) L.kk[r] = j + 1;
                        else L.iters[r]--;
                        L.done[r] = 1;
                    } else {
                        L.zs[(j + 1) * R + r] = 1.0 / nu;
                        atomicOr(L.flag, 1);
                    }
                }
            }
            __syncthreads();
            if (!L.flag[0] || *ab) break;
        }
        // y = R^{-1} g, x += Z y  (per right-hand side)
        if (t < R) {
            const int r = t, kk = L.kk[r];
            for (int k = kk - 1; k >= 0; --k) {
                double s = L.g[k * R + r];
                for (int l = k + 1; l < kk; ++l) s -= L.H[(k * m + l) * R + r] * L.y[l * R + r];
                L.y[k * R + r] = s / L.H[(k * m + k) * R + r];
            }
        }
        __syncthreads();
        for (int64_t i = tt; i < nR; i += NT) {
            const int r = (int)(i % R);
            double acc = w2[i];
            for (int k = 0; k < L.kk[r]; ++k) acc += L.y[k * R + r] * L.zs[k * R + r] * Z[(int64_t)k * nR + i];
            w2[i] = acc;
        }
        team_sync(T);
    }
    // write back x and the per-right-hand-side records (member 0)
    for (int64_t i = tt; i < nR; i += NT) Xb[(i / R) * nrhs + (i % R)] = w2[i];
    if (t < R && T.me == 0) {
        gs2_solve_info f;
        f.iterations = L.iters[t];
        f.restarts = L.restarts[t];
        f.relres = L.bnorm[t] > 0.0 ? L.beta[t] / L.bnorm[t] : 0.0;
        f.converged = *ab ? 0 : L.conv[t];
        f.status = *ab ? GS2_ERR_HIP
                       : L.conv[t] ? GS2_OK : (L.status[t] != GS2_OK ? L.status[t] : GS2_NOT_CONVERGED);
        f.seconds = 0.0;
        c.info[(int64_t)it.sys * nrhs + it.r0 + t] = f;
    }
    __syncthreads();
}

template <typename VT, typename AT, int R, int K>
__global__ __launch_bounds__(BT) void k_batched(BConst c)
{
    extern __shared__ double lds[];
    __shared__ int s_slot;
    BLds L = blds_carve(lds, c.m, R);
    for (;;) {
        if (threadIdx.x == 0) s_slot = (int)atomicAdd(c.queue, 1u);
        __syncthreads();
        const int slot = __builtin_amdgcn_readfirstlane(s_slot); // uniform: the item's fields load into SGPRs
        __syncthreads();
        if (slot >= c.nslots) break;
        const BSlot sl = c.slots[slot];
        const BItem it = c.items[sl.item];
        const BTeam T{it.G, sl.member, c.tbar + sl.item, c.xch + it.xoff, c.abort, c.spin_ticks, L.epoch, L.abort};
        b_solve_item<VT, AT, R, K>(c, it, T, L);
    }
}

// a new solve: empty queue, team arrival counters and abort flag at zero
__global__ void k_reset_queue(unsigned *q, unsigned *tbar, int nitems, int *abort)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        q[0] = 0u;
        abort[0] = 0;
    }
    for (int k = i; k < nitems; k += gridDim.x * blockDim.x) tbar[k] = 0u;
}

// ---------------------------------------------------------------- host side

typedef void (*BatchedKernel)(BConst);

template <typename VT, typename AT>
static BatchedKernel pick_kernel_t(int R, int K)
{
    if (K == 1) {
        if (R == 1) return k_batched<VT, AT, 1, 1>;
        if (R == 2) return k_batched<VT, AT, 2, 1>;
        return k_batched<VT, AT, 4, 1>;
    }
    if (R == 1) return k_batched<VT, AT, 1, 4>;
    if (R == 2) return k_batched<VT, AT, 2, 4>;
    return k_batched<VT, AT, 4, 4>;
}

static BatchedKernel pick_kernel(int prec, int R, int K)
{
    if (prec == GS2_FP64) return pick_kernel_t<double, double>(R, K);
    if (prec == GS2_FP32) return pick_kernel_t<float, float>(R, K);
    return pick_kernel_t<_Float16, float>(R, K);
}

struct Batch {
    int nsys = 0, m = 0, nrhs = 0, R = 1, K = 1, precision = GS2_FP32;
    int tuned = 0; // lanes per row and right-hand sides per item chosen by timing
    std::vector<Handle *> hs;
    std::vector<int64_t> sizes;
    int32_t *rp = nullptr, *ci = nullptr;
    double *va = nullptr;
    BSys *d_sys = nullptr;
    BItem *d_items = nullptr;
    int nitems = 0;
    int team_rows = 0; // rows x right-hand sides per team member (0 = default, < 0 = no teams)
    BSlot *d_slots = nullptr;
    int nslots = 0;
    unsigned *tbar = nullptr;
    double *xch = nullptr;
    int *abort = nullptr;
    double *V = nullptr, *Z = nullptr, *W = nullptr;
    void *P = nullptr;
    unsigned *queue = nullptr;
    gs2_solve_info *d_info = nullptr;
    BParams *d_prm = nullptr, *h_prm = nullptr;
    BConst cst{};
    int grid = 1;
    size_t lds = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (Handle *h : hs) delete h;
        for (void *p : {(void *)rp, (void *)ci, (void *)va, (void *)d_sys, (void *)d_items, (void *)V, (void *)Z,
                        (void *)W, P, (void *)queue, (void *)d_info, (void *)d_prm, (void *)d_slots, (void *)tbar,
                        (void *)xch, (void *)abort})
            if (p) (void)hipFree(p);
        if (h_prm) (void)hipHostFree(h_prm);
    }
};

// Rows x right-hand sides per team member: an item of n rows and R
// right-hand sides is solved by G = n R / team_rows workgroups (rounded,
// 1..8).  Smaller shares pay more in team barriers than they gain (measured
// on the 512-system convection-diffusion batch: 8192, 16384, 32768 and 65536
// gave 3.50, 2.77, 2.72 and 3.03 s with R = 4, one workgroup per item 6.13
// s; at most 16 members instead of 8 did not help).
constexpr int64_t TEAM_ROWS_DEFAULT = 32768;
constexpr int TEAM_MAX = 8;

static int team_size(const Batch &b, int64_t n, int R)
{
    if (b.team_rows < 0) return 1;
    const int64_t tr = b.team_rows > 0 ? b.team_rows : TEAM_ROWS_DEFAULT;
    const int64_t g = (n * R + tr / 2) / tr;
    return (int)std::max<int64_t>(1, std::min<int64_t>(TEAM_MAX, g));
}

static int build_items(Batch &b, int R)
{
    for (void *p : {(void *)b.d_items, (void *)b.d_slots, (void *)b.tbar, (void *)b.xch})
        if (p) (void)hipFree(p);
    b.d_items = nullptr;
    b.d_slots = nullptr;
    b.tbar = nullptr;
    b.xch = nullptr;
    std::vector<int> order(b.nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b.sizes[a] > b.sizes[c]; });
    std::vector<int64_t> row0(b.nsys + 1, 0);
    for (int i = 0; i < b.nsys; ++i) row0[i + 1] = row0[i] + b.sizes[i];
    std::vector<BItem> items;
    std::vector<BSlot> slots;
    int64_t xoff = 0;
    for (int i : order)
        for (int r0 = 0; r0 < b.nrhs; r0 += R) {
            const int G = team_size(b, b.sizes[i], R);
            for (int q = 0; q < G; ++q) slots.push_back(BSlot{(int)items.size(), q});
            items.push_back(BItem{i, r0, row0[i] * b.nrhs + (int64_t)r0 * b.sizes[i], G, 0, xoff});
            if (G > 1) xoff += 2 * (int64_t)G * XS;
        }
    b.nitems = (int)items.size();
    b.nslots = (int)slots.size();
    GS2_TRY_HIP(hipMalloc(&b.d_items, sizeof(BItem) * items.size()));
    GS2_TRY_HIP(hipMemcpy(b.d_items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice));
    GS2_TRY_HIP(hipMalloc(&b.d_slots, sizeof(BSlot) * slots.size()));
    GS2_TRY_HIP(hipMemcpy(b.d_slots, slots.data(), sizeof(BSlot) * slots.size(), hipMemcpyHostToDevice));
    GS2_TRY_HIP(hipMalloc(&b.tbar, sizeof(unsigned) * items.size()));
    GS2_TRY_HIP(hipMalloc(&b.xch, sizeof(double) * (size_t)std::max<int64_t>(xoff, 1)));
    return GS2_OK;
}

static int configure(Batch &b, int R)
{
    b.R = R;
    GS2_TRY(build_items(b, R));
    b.lds = blds_bytes(b.m, R);
    BatchedKernel kern = pick_kernel(b.precision, R, b.K);
    if (b.lds > 48 * 1024)
        GS2_TRY_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds));
    int per_cu = 0;
    GS2_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BT, b.lds));
    int dev = 0, cus = 0;
    GS2_TRY_HIP(hipGetDevice(&dev));
    GS2_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // every workgroup can be resident at once, and a team (at most TEAM_MAX
    // members) waits only for slots that running workgroups pop
    b.grid = std::max(1, std::min(b.nslots, std::max(1, per_cu) * cus));
    if (b.grid < std::min(b.nslots, TEAM_MAX)) return GS2_ERR_HIP;
    b.cst.items = b.d_items;
    b.cst.nitems = b.nitems;
    b.cst.slots = b.d_slots;
    b.cst.nslots = b.nslots;
    b.cst.tbar = b.tbar;
    b.cst.xch = b.xch;
    // (re)capture: queue reset + one persistent launch
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    GS2_TRY_HIP(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    k_reset_queue<<<(unsigned)std::min(1024, (b.nitems + 255) / 256), 256, 0, b.cap>>>(b.queue, b.tbar, b.nitems,
                                                                                   b.abort);
    kern<<<b.grid, BT, b.lds, b.cap>>>(b.cst);
    GS2_TRY_HIP(hipStreamEndCapture(b.cap, &b.graph));
    GS2_TRY_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    return GS2_OK;
}

static int run(Batch &b, const double *B, double *X, double rtol, int maxit, hipStream_t s)
{
    b.h_prm->B = B;
    b.h_prm->X = X;
    b.h_prm->rtol = rtol;
    b.h_prm->maxit = maxit;
    GS2_TRY_HIP(hipMemcpyAsync(b.d_prm, b.h_prm, sizeof(BParams), hipMemcpyHostToDevice, s));
    Prof pr(s, PK_BATCHED, 0.0);
    GS2_TRY_HIP(hipGraphLaunch(b.exec, s));
    return GS2_OK;
}

static int setup_batched_impl(Batch &b, const gs2_csr *As, int nsys, int sweeps, int inner, double damping,
                              int variant, const gs2_options &o, int restart, int nrhs, hipStream_t s)
{
    b.nsys = nsys;
    b.m = restart;
    b.nrhs = nrhs;
    b.precision = o.precision;
    int64_t rows = 0, nnz = 0, maxslices_rows = 0;
    double maxavg = 0.0;
    for (int i = 0; i < nsys; ++i) {
        rows += As[i].n;
        nnz += As[i].nnz;
        maxslices_rows = std::max<int64_t>(maxslices_rows, As[i].n);
        if (As[i].n) maxavg = std::max(maxavg, (double)(As[i].nnz - As[i].n) / (2.0 * As[i].n));
    }
    // lanes per row of the systems' triangles: 1 or 4 (timed below unless forced)
    std::vector<int> kcands;
    if (o.lanes_per_row == 1 || o.lanes_per_row == 4) kcands = {o.lanes_per_row};
    else if (o.lanes_per_row != 0) return GS2_ERR_ARG;
    else if (!o.autotune) kcands = {maxavg > 12.0 ? 4 : 1};
    else {
        kcands = {1};
        if (4 <= 2.0 * std::max(1.0, maxavg)) kcands.push_back(4); // as the single-system tuner: K <= 2 x mean row
    }
    GS2_TRY_HIP(hipMalloc(&b.rp, sizeof(int32_t) * (rows + nsys)));
    GS2_TRY_HIP(hipMalloc(&b.ci, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
    GS2_TRY_HIP(hipMalloc(&b.va, sizeof(double) * std::max<int64_t>(nnz, 1)));
    {
        int64_t roff = 0, noff = 0;
        for (int i = 0; i < nsys; ++i) {
            GS2_TRY_HIP(hipMemcpyAsync(b.rp + roff, As[i].rowptr, sizeof(int32_t) * (As[i].n + 1),
                                       hipMemcpyDeviceToDevice, s));
            GS2_TRY_HIP(hipMemcpyAsync(b.ci + noff, As[i].colind, sizeof(int32_t) * As[i].nnz, hipMemcpyDeviceToDevice,
                                       s));
            GS2_TRY_HIP(hipMemcpyAsync(b.va + noff, As[i].val, sizeof(double) * As[i].nnz, hipMemcpyDeviceToDevice, s));
            b.sizes.push_back(As[i].n);
            roff += As[i].n + 1;
            noff += As[i].nnz;
        }
    }
    // the systems' triangles with K lanes per row (replacing any built before)
    auto build_systems = [&](int K) -> int {
        b.K = K;
        for (Handle *h : b.hs) delete h;
        b.hs.clear();
        gs2_options so = o;
        so.autotune = 0;
        so.build_levels = 0;
        so.lanes_per_row = K;
        so.format = GS2_FORMAT_SELL;
        std::vector<BSys> sys(nsys);
        int64_t roff = 0, noff = 0, row0 = 0;
        for (int i = 0; i < nsys; ++i) {
            Handle *h = new (std::nothrow) Handle;
            if (!h) return GS2_ERR_NOMEM;
            b.hs.push_back(h);
            h->n = As[i].n;
            h->sweeps = sweeps;
            h->inner = inner;
            h->variant = variant;
            h->omega = damping;
            h->gamma = o.inner_damping;
            h->precision = o.precision;
            GS2_TRY(setup_handle(*h, As[i], so, s, false));
            BSys &d = sys[i];
            d.n = h->n;
            d.nslices = h->L.nslices;
            d.Lsp = h->L.slice_ptr;
            d.Usp = h->U.slice_ptr;
            d.Lcol = h->L.col;
            d.Ucol = h->U.col;
            d.Lval = h->L.val;
            d.Uval = h->U.val;
            d.sl = h->sl;
            d.sr = h->sr;
            d.rp = b.rp + roff;
            d.ci = b.ci + noff;
            d.va = b.va + noff;
            d.row0 = row0;
            roff += As[i].n + 1;
            noff += As[i].nnz;
            row0 += As[i].n;
        }
        if (!b.d_sys) GS2_TRY_HIP(hipMalloc(&b.d_sys, sizeof(BSys) * nsys));
        GS2_TRY_HIP(hipMemcpyAsync(b.d_sys, sys.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        return GS2_OK;
    };
    GS2_TRY(build_systems(kcands.front()));
    // the copied row pointers index the copied arrays from 0: rowptr is relative per system, as given
    const size_t tot = (size_t)std::max<int64_t>(rows, 1) * nrhs;
    GS2_TRY_HIP(hipMalloc(&b.V, sizeof(double) * tot * (restart + 1)));
    GS2_TRY_HIP(hipMalloc(&b.Z, sizeof(double) * tot * restart));
    GS2_TRY_HIP(hipMalloc(&b.W, sizeof(double) * tot * 2));
    GS2_TRY_HIP(hipMalloc(&b.P, prec_bytes(o.precision) * tot * 5));
    GS2_TRY_HIP(hipMalloc(&b.queue, sizeof(unsigned) * 64));
    GS2_TRY_HIP(hipMalloc(&b.abort, sizeof(int) * 64));
    GS2_TRY_HIP(hipMalloc(&b.d_info, sizeof(gs2_solve_info) * (size_t)nsys * nrhs));
    GS2_TRY_HIP(hipMalloc(&b.d_prm, sizeof(BParams)));
    GS2_TRY_HIP(hipHostMalloc((void **)&b.h_prm, sizeof(BParams), hipHostMallocDefault));
    GS2_TRY_HIP(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    b.cst.sys = b.d_sys;
    b.cst.m = restart;
    b.cst.nrhs = nrhs;
    b.cst.sweeps = sweeps;
    b.cst.inner = inner;
    b.cst.variant = variant;
    b.cst.compact = o.compact ? 1 : 0;
    b.cst.omega = damping;
    b.cst.gamma = o.inner_damping;
    b.cst.V = b.V;
    b.cst.Z = b.Z;
    b.cst.W = b.W;
    b.cst.P = b.P;
    b.cst.queue = b.queue;
    b.cst.abort = b.abort;
    {
        int dev = 0, khz = 0;
        GS2_TRY_HIP(hipGetDevice(&dev));
        GS2_TRY_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const long long ms = o.team_wait_ms > 0 ? o.team_wait_ms : 30000;
        // a negative limit ends every wait at once: the abandon path, for tests
        b.cst.spin_ticks = o.team_wait_ms < 0 ? -1 : (long long)std::max(khz, 1000) * ms;
    }
    b.team_rows = o.team_rows;
    b.cst.info = b.d_info;
    b.cst.prm = b.d_prm;

    // right-hand sides per work item: autotuned over the divisors of nrhs in {1, 2, 4}
    std::vector<int> cands;
    if (o.rhs_per_item) {
        if ((o.rhs_per_item != 1 && o.rhs_per_item != 2 && o.rhs_per_item != 4) || nrhs % o.rhs_per_item)
            return GS2_ERR_ARG;
        cands.push_back(o.rhs_per_item);
    } else {
        for (int R : {4, 2, 1})
            if (nrhs % R == 0) cands.push_back(R);
    }
    int bestR = cands.front(), bestK = kcands.front();
    b.tuned = o.autotune && (cands.size() > 1 || kcands.size() > 1);
    if (b.tuned) {
        double *Bt = nullptr, *Xt = nullptr;
        GS2_TRY_HIP(hipMalloc(&Bt, sizeof(double) * tot));
        GS2_TRY_HIP(hipMalloc(&Xt, sizeof(double) * tot));
        std::vector<double> ones(tot, 1.0);
        GS2_TRY_HIP(hipMemcpy(Bt, ones.data(), sizeof(double) * tot, hipMemcpyHostToDevice));
        hipEvent_t e0, e1;
        GS2_TRY_HIP(hipEventCreate(&e0));
        GS2_TRY_HIP(hipEventCreate(&e1));
        // One restart cycle per item, every right-hand side doing the same
        // work, measures throughput only.  In a real solve the right-hand
        // sides of an item converge at different steps and the item runs until
        // its slowest one has.  With one workgroup per item the largest items
        // form the critical path, so the smallest R within 25% of the best
        // tuning time is taken; with teams the largest items are split and the
        // fastest R is taken.  Each lanes-per-row candidate is timed with its
        // own choice of R; a wider one must win by 3 % (the timing noise).
        float bestAll = 1e30f;
        for (size_t kc = 0; kc < kcands.size(); ++kc) {
            if (kcands[kc] != b.K) GS2_TRY(build_systems(kcands[kc]));
            std::vector<float> ms_of(cands.size(), 0.f);
            float best = 1e30f;
            for (size_t c = 0; c < cands.size(); ++c) {
                GS2_TRY(configure(b, cands[c]));
                GS2_TRY_HIP(hipMemsetAsync(Xt, 0, sizeof(double) * tot, s));
                GS2_TRY_HIP(hipEventRecord(e0, s));
                GS2_TRY(run(b, Bt, Xt, 0.0, restart, s));
                GS2_TRY_HIP(hipEventRecord(e1, s));
                GS2_TRY_HIP(hipEventSynchronize(e1));
                GS2_TRY_HIP(hipEventElapsedTime(&ms_of[c], e0, e1));
                best = std::min(best, ms_of[c]);
            }
            const float slack = b.team_rows < 0 ? 1.25f : 1.0f;
            size_t pick = 0;
            for (size_t c = 0; c < cands.size(); ++c) // cands is in decreasing R
                if (ms_of[c] <= slack * best) pick = c;
            if (ms_of[pick] < (kc == 0 ? 1.0f : 0.97f) * bestAll) {
                bestAll = ms_of[pick];
                bestK = kcands[kc];
                bestR = cands[pick];
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(Bt);
        (void)hipFree(Xt);
    }
    if (b.K != bestK) GS2_TRY(build_systems(bestK));
    GS2_TRY(configure(b, bestR));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    return GS2_OK;
}

} // namespace gs2

using namespace gs2;

struct gs2_batch {
    Batch b;
};

extern "C" {

int gs2_setup_batched(const gs2_csr *As, int nsys, int sweeps, int inner, double damping, int variant,
                      const gs2_options *opt, int restart, int nrhs, void *stream, gs2_batch **out)
{
    if (!out) return GS2_ERR_ARG;
    *out = nullptr;
    if (!As || nsys < 1 || sweeps < 1 || inner < 0 || variant < GS2_FORWARD || variant > GS2_SYMMETRIC ||
        !(damping > 0.0 && damping < 2.0) || restart < 1 || restart > BMAXM || nrhs < 1)
        return GS2_ERR_ARG;
    for (int i = 0; i < nsys; ++i)
        if (As[i].n < 1 || As[i].n >= (int64_t(1) << 31) - 1 || !As[i].rowptr || !As[i].colind || !As[i].val ||
            As[i].nnz < As[i].n)
            return GS2_ERR_ARG;
    gs2_options o;
    gs2_default_options(&o);
    if (opt) o = *opt;
    if (o.precision < GS2_FP64 || o.precision > GS2_FP16_SCALED || !(o.inner_damping > 0.0 && o.inner_damping <= 2.0))
        return GS2_ERR_ARG;
    gs2_batch *B = new (std::nothrow) gs2_batch;
    if (!B) return GS2_ERR_NOMEM;
    int st = GS2_ERR_HIP;
    try {
        st = setup_batched_impl(B->b, As, nsys, sweeps, inner, damping, variant, o, restart, nrhs, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        st = GS2_ERR_NOMEM;
    } catch (...) {
        st = GS2_ERR_HIP;
    }
    if (st != GS2_OK) {
        (void)hipDeviceSynchronize();
        delete B;
        return st;
    }
    *out = B;
    return GS2_OK;
}

int gmres_solve_batched(gs2_batch *B, int nrhs, const double *Bv, double *X, double rtol, int maxit,
                        gs2_solve_info *infos, void *stream)
{
    if (!B || nrhs != B->b.nrhs || !Bv || !X || !(rtol >= 0.0) || maxit < 0) return GS2_ERR_ARG;
    Batch &b = B->b;
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    GS2_TRY(run(b, Bv, X, rtol, maxit, s));
    std::vector<gs2_solve_info> h((size_t)b.nsys * nrhs);
    GS2_TRY_HIP(hipMemcpyAsync(h.data(), b.d_info, sizeof(gs2_solve_info) * h.size(), hipMemcpyDeviceToHost, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int st = GS2_OK;
    for (auto &f : h) {
        f.seconds = sec;
        if (st == GS2_OK && f.status != GS2_OK) st = f.status;
    }
    if (infos) std::memcpy(infos, h.data(), sizeof(gs2_solve_info) * h.size());
    return st;
}

int gs2_batched_schedule(const gs2_batch *B, int *lanes_per_row, int *rhs_per_item, int *tuned)
{
    if (!B) return GS2_ERR_ARG;
    if (lanes_per_row) *lanes_per_row = B->b.K;
    if (rhs_per_item) *rhs_per_item = B->b.R;
    if (tuned) *tuned = B->b.tuned;
    return GS2_OK;
}

void gs2_destroy_batched(gs2_batch *B)
{
    if (!B) return;
    (void)hipDeviceSynchronize();
    delete B;
}

} // extern "C"
