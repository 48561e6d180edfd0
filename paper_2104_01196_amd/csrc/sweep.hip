// GS2 / JR / exact-GS preconditioner applies (Section 4, eqs. (two-stage),
// (jr-initial-guess), (jacobi); damping factors; compact form eq.
// (two-stage-3); level-set scheduled Gauss-Seidel of Section 3).
//
// All vectors inside the preconditioner live in scaled space (see
// gs2_internal.hpp): xh = S_r^{-1} x, rh = S_l r.  A half sweep is
//   rh = S_l v - xh - Lh xh - Uh xh          (outer residual, k_resid)
//   g  = rh                                  (eq. (jr-initial-guess): D = I)
//   g  = rh - w T g   (n_j times)            (eq. (jacobi), k_inner)
//   xh = xh + w g                            (fused into the last k_inner)
// and the last pass of an apply writes z = S_r xh in float64.  The first
// half of an apply starts from xh = 0, so its residual is S_l v exactly and
// needs no SpMV.  Every pass reads its triangle exactly once.
#include <algorithm>
#include <cmath>

#include "dcgs_state.hpp"
#include "gs2_internal.hpp"

namespace gs2 {

// destinations of the fused passes
enum : int { DST_G = 0, DST_XADD = 1, DST_XSET = 2, DST_ZADD = 3, DST_ZSET = 4 };

struct SellView {
    const int64_t *sp;
    const int32_t *col;
    const uint16_t *off; // col - row - off_min per entry, when the triangle has them
    int off_min;
    int nt; // load values and offsets with the non-temporal policy
    const void *val;
};

static SellView view(const Sell &S) { return SellView{S.slice_ptr, S.col, S.off, S.off_min, S.nt, S.val}; }

template <typename AT>
__device__ __forceinline__ void finish(int dst, int64_t row, AT g, AT w, AT *gout, AT *xh, AT *xout, double *z,
                                       const double *sr)
{
    switch (dst) {
    case DST_G: gout[row] = g; break;
    case DST_XADD: xout[row] = xh[row] + w * g; break;
    case DST_XSET: xout[row] = w * g; break;
    case DST_ZADD: z[row] = sr[row] * (double)(xh[row] + w * g); break;
    default: z[row] = sr[row] * (double)(w * g); break;
    }
}

// Slices per wavefront in the sweep kernels.  A slice of a 32-bit form
// carries half the bytes of a float64 one, so its wavefront spends
// proportionally more time on the fixed per-slice chain (slice pointer ->
// columns -> gathered values); two slices per wavefront keep their loads in
// flight together.  Measured on the 128^3 solve: float32 / scaled-float16
// 38.2 / 37.9 -> 36.9 / 36.4 ms; for float64 one slice per wavefront stays
// best (two or four were measured slower).
template <typename AT>
constexpr int su_of()
{
    return sizeof(AT) == 8 ? 1 : 2;
}

// acc[u] += sum over the stored entries of slice s0 + u of val * src(col);
// the column is row + off_min + off (2 index bytes per entry) when the
// triangle has 16-bit offsets, else read in full.  A large triangle's values
// and offsets are streamed with the non-temporal policy.
template <typename VT, typename AT, int SUN, int K, typename Src>
__device__ __forceinline__ void slice_dots(const SellView T, int64_t s0, int64_t nslices, int lane, Src src,
                                           AT (&acc)[SUN])
{
    int64_t beg[SUN];
    int steps[SUN];
    int tmax = 0;
#pragma unroll
    for (int u = 0; u < SUN; ++u) {
        const int64_t s = s0 + u;
        const bool ok = s < nslices;
        beg[u] = ok ? T.sp[s] : 0;
        steps[u] = ok ? (int)((T.sp[s + 1] - beg[u]) / WAVE) : 0;
        tmax = steps[u] > tmax ? steps[u] : tmax;
    }
    const VT *__restrict__ val = (const VT *)T.val;
    if (T.off) {
        const uint16_t *__restrict__ off = T.off;
        int rw[SUN];
#pragma unroll
        for (int u = 0; u < SUN; ++u) rw[u] = (int)((s0 + u) * (WAVE / K) + lane / K) + T.off_min;
        if (T.nt) {
#pragma unroll 4
            for (int t = 0; t < tmax; ++t) {
#pragma unroll
                for (int u = 0; u < SUN; ++u) {
                    if (t < steps[u]) {
                        const int64_t p = beg[u] + (int64_t)t * WAVE + lane;
                        acc[u] += (AT)__builtin_nontemporal_load(&val[p]) *
                                  src(rw[u] + (int)__builtin_nontemporal_load(&off[p]));
                    }
                }
            }
            return;
        }
#pragma unroll 4
        for (int t = 0; t < tmax; ++t) {
#pragma unroll
            for (int u = 0; u < SUN; ++u) {
                if (t < steps[u]) {
                    const int64_t p = beg[u] + (int64_t)t * WAVE + lane;
                    acc[u] += (AT)val[p] * src(rw[u] + (int)off[p]);
                }
            }
        }
        return;
    }
    const int32_t *__restrict__ col = T.col;
#pragma unroll 4
    for (int t = 0; t < tmax; ++t) {
#pragma unroll
        for (int u = 0; u < SUN; ++u) {
            if (t < steps[u]) {
                const int64_t p = beg[u] + (int64_t)t * WAVE + lane;
                acc[u] += (AT)val[p] * src(col[p]);
            }
        }
    }
}

// Inner JR pass: g_new = rh - w T g_old (optionally damped with gamma), one
// or two slices of T per wavefront.  rv: rh_i = AT(v_i s_l[i]) (first half
// of an apply); gv: g_old_j = AT(v_j s_l[j]) (its first inner pass).  With
// fst, the first workgroup instead runs the serial work that closes the
// previous GMRES step (dcgs_finish_block): it reads only that step's partial
// sums and the solver state, nothing this pass touches, so the two overlap
// (it is dispatched first, before the pass fills the machine) and the step
// saves a launch.
template <typename VT, typename AT, int K, bool FIN>
__global__ __launch_bounds__(KT) void k_inner(const int *__restrict__ stop, int64_t n, int64_t nslices, SellView T,
                                              const AT *__restrict__ rh, const AT *__restrict__ gin,
                                              const double *__restrict__ v, const double *__restrict__ sl, int rv,
                                              int gv, int damp, AT w, AT gamma, int dst, AT *__restrict__ gout,
                                              AT *__restrict__ xh, double *__restrict__ z,
                                              const double *__restrict__ sr, const double *__restrict__ fpart,
                                              int fnb, void *fst)
{
    constexpr int SUN = su_of<AT>();
    if constexpr (FIN) {
        if (blockIdx.x == 0) {
            dcgs_finish_block(fpart, fnb, static_cast<GState *>(fst));
            return;
        }
    }
    // In a FIN launch the first workgroup may set the stop flag while the
    // others read it; either value is correct: a pass that runs after the
    // cycle has converged only writes vectors the cycle no longer reads.
    if (stop && *stop) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned sh = FIN ? 1u : 0u;
    const int64_t s0 =
        (xcd_remap(blockIdx.x - sh, gridDim.x - sh) * (blockDim.x / WAVE) + threadIdx.x / WAVE) * SUN;
    if (s0 >= nslices) return;
    AT acc[SUN];
#pragma unroll
    for (int u = 0; u < SUN; ++u) acc[u] = AT(0);
    if (gv) slice_dots<VT, AT, SUN, K>(T, s0, nslices, lane, [&](int c) { return (AT)(v[c] * sl[c]); }, acc);
    else slice_dots<VT, AT, SUN, K>(T, s0, nslices, lane, [&](int c) { return gin[c]; }, acc);
#pragma unroll
    for (int u = 0; u < SUN; ++u) {
        const AT a = K > 1 ? group_sum<K>(acc[u]) : acc[u];
        const int64_t row = (s0 + u) * (WAVE / K) + lane / K;
        if ((K > 1 && (lane & (K - 1))) || row >= n) continue;
        const AT r = rv ? (AT)(v[row] * sl[row]) : rh[row];
        AT g = r - w * a;
        if (damp) {
            const AT go = gv ? (AT)(v[row] * sl[row]) : gin[row];
            g = (AT(1) - gamma) * go + gamma * g;
        }
        finish<AT>(dst, row, g, w, gout, xh, xh, z, sr);
    }
}

// Outer residual pass.  compact = 0: rh = S_l v - xh - A xh (both triangles,
// unit diagonal).  compact = 1: rh = S_l v - O xh - (1 - 1/w) xh with O the
// triangle opposite to the inner one (eq. (two-stage-3) with damping).
// The result goes to rh (DST_G) or is fused into a Jacobi-type update of xh
// written to xout (double-buffered: xh is gathered here).  The couplings to
// other blocks (hybrid relaxation) multiply the values frozen at the last
// exchange.  The triangles' cache policy is the size-based one of
// slice_dots.
template <typename VT, typename AT, int K>
__global__ __launch_bounds__(256) void k_resid(const int *__restrict__ stop, int64_t n, int64_t nslices, SellView P,
                                               SellView Q, int two, const AT *__restrict__ xh,
                                               const double *__restrict__ v, const double *__restrict__ sl, AT cdiag,
                                               AT w, int dst, AT *__restrict__ rh, AT *__restrict__ xout,
                                               double *__restrict__ z, const double *__restrict__ sr, SellView Ev,
                                               const AT *__restrict__ ye)
{
    constexpr int SUN = su_of<AT>();
    if (stop && *stop) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t s0 = (xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x / WAVE) + threadIdx.x / WAVE) * SUN;
    if (s0 >= nslices) return;
    AT acc[SUN];
#pragma unroll
    for (int u = 0; u < SUN; ++u) acc[u] = AT(0);
    auto gx = [&](int c) { return xh[c]; };
    slice_dots<VT, AT, SUN, K>(P, s0, nslices, lane, gx, acc);
    if (two) slice_dots<VT, AT, SUN, K>(Q, s0, nslices, lane, gx, acc);
    if (ye) slice_dots<VT, AT, SUN, K>(Ev, s0, nslices, lane, [&](int c) { return ye[c]; }, acc);
#pragma unroll
    for (int u = 0; u < SUN; ++u) {
        const AT a = K > 1 ? group_sum<K>(acc[u]) : acc[u];
        const int64_t row = (s0 + u) * (WAVE / K) + lane / K;
        if ((K > 1 && (lane & (K - 1))) || row >= n) continue;
        const AT r = ((AT)(v[row] * sl[row]) - cdiag * xh[row]) - a;
        finish<AT>(dst, row, r, w, rh, const_cast<AT *>(xh), xout, z, sr);
    }
}

// First half of JR from xh = 0: xh = w S_l v, or z = S_r w S_l v if final.
// With fst, the first workgroup closes the previous GMRES step (as in
// k_inner).
template <typename AT, bool FIN>
__global__ __launch_bounds__(KT) void k_first_jr(const int *__restrict__ stop, int64_t n,
                                                 const double *__restrict__ v, const double *__restrict__ sl,
                                                 const double *__restrict__ sr, AT w, int final_, AT *__restrict__ xh,
                                                 double *__restrict__ z, const double *__restrict__ fpart, int fnb,
                                                 void *fst)
{
    if constexpr (FIN) {
        if (blockIdx.x == 0) {
            dcgs_finish_block(fpart, fnb, static_cast<GState *>(fst));
            return;
        }
    }
    if (stop && *stop) return; // may race with a FIN workgroup's write, harmlessly (as in k_inner)
    const int64_t i = (int64_t)(blockIdx.x - (FIN ? 1u : 0u)) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const AT r = (AT)(v[i] * sl[i]);
    if (final_) z[i] = sr[i] * (double)(w * r);
    else xh[i] = w * r;
}

template <typename AT>
__global__ void k_copy_at(const int *__restrict__ stop, int64_t n, const AT *__restrict__ a, AT *__restrict__ b)
{
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <typename AT>
__global__ void k_fill_zero(const int *__restrict__ stop, int64_t n, AT *__restrict__ x)
{
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = AT(0);
}

template <typename AT>
__global__ void k_unscale(const int *__restrict__ stop, int64_t n, const AT *__restrict__ xh, const double *__restrict__ sr,
                          double *__restrict__ z)
{
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = sr[i] * (double)xh[i];
}

// One level of a level-scheduled Gauss-Seidel / SOR sweep (compact row
// update of the sequential loop of Section 6):
//   x_i = (1 - w) xold_i + w (S_l v_i - sum_main ah_ij xnew_j - sum_other ah_ij xold_j)
// main = the triangle solved in this sweep (entries already updated),
// other = the opposite triangle (previous iterate; xold == NULL means 0).
template <typename VT, typename AT>
__global__ void k_tri_level(const int *__restrict__ stop, const int32_t *__restrict__ rows, int64_t cnt, int K, SellView M, SellView O,
                            const AT *__restrict__ xold, AT *__restrict__ xnew, const double *__restrict__ v,
                            const double *__restrict__ sl, AT w)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int i = rows[t];
    const int C = WAVE / K;
    const int64_t s = i / C;
    const int lb = (i % C) * K;
    AT acc = AT(0);
    {
        const int64_t beg = M.sp[s], steps = (M.sp[s + 1] - beg) / WAVE;
        for (int64_t st = 0; st < steps; ++st)
            for (int q = 0; q < K; ++q) {
                const int64_t p = beg + st * WAVE + lb + q;
                acc += (AT)((const VT *)M.val)[p] * xnew[M.col[p]];
            }
    }
    AT xo = AT(0);
    if (xold) {
        const int64_t beg = O.sp[s], steps = (O.sp[s + 1] - beg) / WAVE;
        for (int64_t st = 0; st < steps; ++st)
            for (int q = 0; q < K; ++q) {
                const int64_t p = beg + st * WAVE + lb + q;
                acc += (AT)((const VT *)O.val)[p] * xold[O.col[p]];
            }
        xo = xold[i];
    }
    xnew[i] = (AT(1) - w) * xo + w * ((AT)(v[i] * sl[i]) - acc);
}

// One color of a multicolor Gauss-Seidel / SOR sweep: rows of one color are
// never coupled, so they update in place from the current iterate,
//   x_i = (1 - w) x_i + w (S_l v_i - sum_{j != i} ah_ij x_j)   (scaled space).
template <typename VT, typename AT>
__global__ void k_color(const int *__restrict__ stop, const int32_t *__restrict__ rows, int64_t cnt, int K,
                        SellView L, SellView U, AT *x, const double *__restrict__ v, const double *__restrict__ sl,
                        AT w)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int i = rows[t];
    const int C = WAVE / K;
    const int64_t s = i / C;
    const int lb = (i % C) * K;
    AT acc = AT(0);
    for (int part = 0; part < 2; ++part) {
        const SellView &M = part ? U : L;
        const int64_t beg = M.sp[s], steps = (M.sp[s + 1] - beg) / WAVE;
        for (int64_t st = 0; st < steps; ++st)
            for (int q = 0; q < K; ++q) {
                const int64_t p = beg + st * WAVE + lb + q;
                acc += (AT)((const VT *)M.val)[p] * x[M.col[p]];
            }
    }
    x[i] = (AT(1) - w) * x[i] + w * ((AT)(v[i] * sl[i]) - acc);
}

// ------------------------------------------------ diagonal-interleaved passes
//
// The same passes on the diagonal-interleaved copies of the triangles (Dia in
// gs2_internal.hpp).  A lane owns R rows, 64 apart, so every gather and every
// per-row load or store of a wavefront covers 64 consecutive elements, and
// the lane's R values of one diagonal arrive in a single R * sizeof(VT) byte
// load.  No column index is loaded: the column of diagonal d is row + off[d],
// clamped into [0, n) (a clamped column only ever meets a stored zero).
// With LDS staging the workgroup first copies the source vector over its rows
// plus DIA_HALO elements on each side into LDS, and the diagonals with
// |off| <= DIA_HALO (the neighbours in the fastest grid direction) read from
// there.

// the FIN variants run the Krylov step's finish, written for KT threads
static_assert(DIA_THREADS == KT, "one workgroup size for the diagonal passes and the step finish");

struct DiaView {
    int ndiag;
    int nt;
    int b3;
    int64_t stride;
    const void *val;
    int off[DIA_MAX];
};

// compile-time flags of the diagonal passes: LDS staging of the source, and
// the non-temporal cache policy for the values
// and 3-row blocks (never staged in LDS)
enum : int { DIA_FL_LDS = 1, DIA_FL_NT = 2, DIA_FL_B3 = 4 };
static int dia_flags(const Handle &h, const Dia &D)
{
    if (D.b3) return DIA_FL_B3 | (D.nt ? DIA_FL_NT : 0);
    return (h.lds ? DIA_FL_LDS : 0) | (D.nt ? DIA_FL_NT : 0);
}

static DiaView dview(const Dia &D)
{
    DiaView v;
    v.ndiag = D.ndiag;
    v.nt = D.nt;
    v.b3 = D.b3;
    v.stride = D.stride;
    v.val = D.val;
    for (int d = 0; d < DIA_MAX; ++d) v.off[d] = D.off[d];
    return v;
}

template <int BYTES>
struct RawVec;
template <>
struct RawVec<16> {
    typedef unsigned int T __attribute__((ext_vector_type(4)));
};
template <>
struct RawVec<8> {
    typedef unsigned int T __attribute__((ext_vector_type(2)));
};
template <>
struct RawVec<4> {
    typedef unsigned int T;
};
template <>
struct RawVec<2> {
    typedef unsigned short T;
};

// The R values a lane holds on one diagonal, in one load.
template <typename VT, typename AT, int R, bool NT>
__device__ __forceinline__ void dia_vals(const VT *__restrict__ p, AT (&a)[R])
{
    static_assert(R * sizeof(VT) >= 2 && R * sizeof(VT) <= 16, "one load of 2 to 16 bytes per lane");
    using RV = typename RawVec<R * (int)sizeof(VT)>::T;
    RV raw;
    if constexpr (NT) raw = __builtin_nontemporal_load((const RV *)p);
    else raw = *(const RV *)p;
    VT t[R];
    __builtin_memcpy(t, &raw, sizeof(t));
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = (AT)t[k];
}

__device__ __forceinline__ int clamp_col(int c, int n) { return c < 0 ? 0 : (c >= n ? n - 1 : c); }

// acc[k] += sum_d T_d(row_k) * x(row_k + off_d) for row_k = rb + 64k; pos is
// the lane's first value of diagonal 0.  src(c) loads the source at a column
// c in [0, n); with LDS, xs holds the source over [base, base + span).
// Columns need clamping only in the workgroups whose rows [w0, w0 + RB),
// shifted by the offset, leave [0, n) (a uniform test per diagonal).  The
// clamp is a select, not a branch, and the values' cache policy (NT) is a
// compile-time choice, so the loop body is straight-line code and the
// compiler issues every diagonal's loads before the first wait: with a branch
// per diagonal it waited on each diagonal in turn (24 against 64 registers,
// the float64 residual pass 107 against 83 us on the 192^3 problem).
//
// ND > 0: the triangle has exactly ND diagonals and the loop over them is
// unrolled completely, so every diagonal's loads are in flight together
// (measured for three diagonals in scaled float16, rows-per-lane 8: 24.9
// against 29.9 us per inner pass over the 192^3 problem); ND = 0: any count.
template <typename VT, typename AT, int R, bool LDS, bool NT, int ND, typename Src>
__device__ __forceinline__ void dia_dots(const DiaView &T, int64_t pos, int w0, int rb, int n, Src src, const AT *xs,
                                         int base, AT (&acc)[R])
{
    constexpr int RB = DIA_THREADS * R;
    const VT *__restrict__ val = (const VT *)T.val;
    const int nd = ND > 0 ? ND : T.ndiag;
    constexpr int UNR = ND > 0 ? ND : 2;
#pragma unroll UNR
    for (int d = 0; d < nd; ++d) {
        AT a[R];
        dia_vals<VT, AT, R, NT>(val + (int64_t)d * T.stride + pos, a);
        const int o = T.off[d];
        if (LDS && o >= -DIA_HALO && o <= DIA_HALO) {
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] += a[k] * xs[rb + k * WAVE + o - base];
        } else {
            const bool inside = w0 + o >= 0 && w0 + RB + o <= n;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                int c = rb + k * WAVE + o;
                c = inside ? c : clamp_col(c, n);
                acc[k] += a[k] * src(c);
            }
        }
    }
}

// The sums on a 3-row block triangle, one node per lane slot:
// acc[k][j] += sum over the node offsets o of the block row j of node
// nb + 64 k against the source at the neighbour node's three unknowns
// 3(node + o) .. 3(node + o) + 2.  Per offset a lane gathers those three
// source entries once for its node's three rows and loads the block's nine
// planes (the lane's R nodes' values of one plane sit side by side: one
// R-value load per plane; pos is the lane's first value in a plane).  Each
// row's sum runs over o, then the three columns of the block, in order.
// Node indices are clamped into [0, n/3) only in workgroups whose nodes,
// shifted by o, leave that range (a uniform test per offset; a clamped node
// meets stored zeros).  Nodes past n/3 read in-bounds padding.
template <typename VT, typename AT, int R, bool NT, typename Src>
__device__ __forceinline__ void b3_node_dots(const DiaView &T, int64_t pos, int g0, int nb, int nn, Src src,
                                             AT (&acc)[R][3])
{
    constexpr int NBW = DIA_THREADS * R; // nodes per workgroup
    const VT *__restrict__ val = (const VT *)T.val;
    const int f1 = (g0 + NBW < nn ? g0 + NBW : nn) - 1;
    int node[R];
#pragma unroll
    for (int k = 0; k < R; ++k) node[k] = nb + k * WAVE < nn ? nb + k * WAVE : nn - 1;
    // one offset per iteration: the nine value loads and three gathers of an
    // offset already fill the wavefront's loads in flight, and unrolling by
    // two took the float64 inner pass from 50 to 78 registers at one node per
    // lane
#pragma unroll 1
    for (int d = 0; d < T.ndiag; ++d) {
        const int o = T.off[d];
        const bool inside = g0 + o >= 0 && f1 + o < nn;
        AT zs[R][3];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int c = node[k] + o;
            c = 3 * (inside ? c : (c < 0 ? 0 : (c >= nn ? nn - 1 : c)));
#pragma unroll
            for (int b = 0; b < 3; ++b) zs[k][b] = src(c + b);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                AT a[R];
                dia_vals<VT, AT, R, NT>(val + (int64_t)(9 * d + 3 * j + b) * T.stride + pos, a);
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k][j] += a[k] * zs[k][b];
            }
    }
}

// Copy src over [base, base + span) into xs (columns clamped into [0, n));
// thread 0 also reads the stop flag, so that every wavefront of the workgroup
// takes the same early exit after the barrier.  Returns the flag.
template <typename AT, int SPAN, typename Src>
__device__ __forceinline__ int dia_stage(AT *xs, int base, int n, Src src, const int *stop, int *sflag)
{
    for (int e = threadIdx.x; e < SPAN; e += DIA_THREADS) xs[e] = src(clamp_col(base + e, n));
    if (threadIdx.x == 0) *sflag = stop ? *stop : 0;
    __syncthreads();
    return *sflag;
}

// Inner JR pass on a diagonal-interleaved triangle (as k_inner).  FIN: the
// first workgroup closes the previous GMRES step instead (as in k_inner);
// the other workgroups may then read the stop flag while that workgroup sets
// it, and either value is correct: a pass that runs after the cycle has
// converged only writes vectors the cycle no longer reads.
template <typename VT, typename AT, int R, int FL, bool FIN, int ND>
__global__ __launch_bounds__(DIA_THREADS) void k_dia_inner(const int *__restrict__ stop, int remap, int n, DiaView T,
                                                  const AT *__restrict__ rh, const AT *__restrict__ gin,
                                                  const double *__restrict__ v, const double *__restrict__ sl, int rv,
                                                  int gv, int damp, AT w, AT gamma, int dst, AT *__restrict__ gout,
                                                  AT *__restrict__ xh, double *__restrict__ z,
                                                  const double *__restrict__ sr, const double *__restrict__ fpart,
                                                  int fnb, void *fst)
{
    constexpr bool LDS = FL & DIA_FL_LDS, NT = FL & DIA_FL_NT;
    static_assert(!(FL & DIA_FL_B3), "3-row block triangles take k_b3_inner");
    constexpr int RB = DIA_THREADS * R; // rows per workgroup
    constexpr int SPAN = LDS ? RB + 2 * DIA_HALO : 1;
    if constexpr (FIN) {
        if (blockIdx.x == 0) {
            dcgs_finish_block(fpart, fnb, static_cast<GState *>(fst));
            return;
        }
    }
    const int sh = FIN ? 1 : 0;
    const int wg = remap ? (int)xcd_remap(blockIdx.x - sh, gridDim.x - sh) : (int)(blockIdx.x - sh);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int w0 = wg * RB;
    const int rb = w0 + wv * (WAVE * R) + lane;
    const int64_t pos = (int64_t)w0 + wv * (WAVE * R) + lane * R;
    auto sv = [&](int c) { return (AT)(v[c] * sl[c]); };
    auto sg = [&](int c) { return gin[c]; };
    AT acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = AT(0);
    if constexpr (LDS) {
        __shared__ AT xs[SPAN];
        __shared__ int sflag;
        const int base = w0 - DIA_HALO;
        if (gv) {
            if (dia_stage<AT, SPAN>(xs, base, n, sv, stop, &sflag)) return;
            dia_dots<VT, AT, R, true, NT, ND>(T, pos, w0, rb, n, sv, xs, base, acc);
        } else {
            if (dia_stage<AT, SPAN>(xs, base, n, sg, stop, &sflag)) return;
            dia_dots<VT, AT, R, true, NT, ND>(T, pos, w0, rb, n, sg, xs, base, acc);
        }
    } else {
        if (stop && *stop) return;
        if (gv) dia_dots<VT, AT, R, false, NT, ND>(T, pos, w0, rb, n, sv, nullptr, 0, acc);
        else dia_dots<VT, AT, R, false, NT, ND>(T, pos, w0, rb, n, sg, nullptr, 0, acc);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = rb + k * WAVE;
        if (row >= n) break;
        const AT r = rv ? (AT)(v[row] * sl[row]) : rh[row];
        AT g = r - w * acc[k];
        if (damp) {
            const AT go = gv ? (AT)(v[row] * sl[row]) : gin[row];
            g = (AT(1) - gamma) * go + gamma * g;
        }
        finish<AT>(dst, row, g, w, gout, xh, xh, z, sr);
    }
}

// Outer residual pass on diagonal-interleaved triangles (as k_resid without
// the hybrid term): rh = S_l v - cdiag xh - P xh [- Q xh].  ND > 0 kernels
// always add Q.  svp, when given, holds S_l v already rounded to AT (the
// same value this pass would form from v and s_l).

// S_l v rounded to the working precision, formed once per apply by the 32-
// and 16-bit forms on the diagonal layout (both work in float32): the first
// inner pass then gathers one float value per neighbour instead of two
// float64 values (v and s_l), and every residual pass reads 4 bytes per row
// instead of 16.  FIN: the
// first workgroup closes the previous GMRES step instead (as in k_dia_inner).
// Q: rows per thread, consecutive, for 16-byte loads of v and s_l (Q = 4
// needs n % 4 == 0 and v, s_l, sv aligned to 16 and 4 sizeof(AT) bytes);
// Q = 1 any.
template <typename AT, bool FIN, int Q>
__global__ __launch_bounds__(KT) void k_dia_prep(const int *__restrict__ stop, int n, const double *__restrict__ v,
                                                 const double *__restrict__ sl, AT *__restrict__ sv,
                                                 const double *__restrict__ fpart, int fnb, void *fst)
{
    if constexpr (FIN) {
        if (blockIdx.x == 0) {
            dcgs_finish_block(fpart, fnb, static_cast<GState *>(fst));
            return;
        }
    }
    if (stop && *stop) return;
    const int i = ((int)(blockIdx.x - (FIN ? 1 : 0)) * KT + (int)threadIdx.x) * Q;
    if (i >= n) return;
    if constexpr (Q == 1) {
        sv[i] = (AT)(v[i] * sl[i]);
    } else {
        static_assert(Q == 4, "one or four rows per thread");
        using D2 = double __attribute__((ext_vector_type(2)));
        using A4 = AT __attribute__((ext_vector_type(4)));
        const D2 v0 = __builtin_nontemporal_load((const D2 *)&v[i]), v1 = __builtin_nontemporal_load((const D2 *)&v[i + 2]);
        const D2 s0 = *(const D2 *)&sl[i], s1 = *(const D2 *)&sl[i + 2];
        A4 o;
        o.x = (AT)(v0.x * s0.x);
        o.y = (AT)(v0.y * s0.y);
        o.z = (AT)(v1.x * s1.x);
        o.w = (AT)(v1.y * s1.y);
        *(A4 *)&sv[i] = o;
    }
}
template <typename VT, typename AT, int R, int FL, int ND>
__global__ __launch_bounds__(DIA_THREADS) void k_dia_resid(const int *__restrict__ stop, int remap, int n, DiaView P, DiaView Q, int two,
                                                  const AT *__restrict__ xh, const double *__restrict__ v,
                                                  const double *__restrict__ sl, const AT *__restrict__ svp, AT cdiag, AT w, int dst,
                                                  AT *__restrict__ rh, AT *__restrict__ xout, double *__restrict__ z,
                                                  const double *__restrict__ sr)
{
    constexpr bool LDS = FL & DIA_FL_LDS, NT = FL & DIA_FL_NT;
    static_assert(!(FL & DIA_FL_B3), "3-row block triangles take k_b3_resid");
    constexpr int RB = DIA_THREADS * R;
    constexpr int SPAN = LDS ? RB + 2 * DIA_HALO : 1;
    const int wg = remap ? (int)xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int w0 = wg * RB;
    const int rb = w0 + wv * (WAVE * R) + lane;
    const int64_t pos = (int64_t)w0 + wv * (WAVE * R) + lane * R;
    auto sx = [&](int c) { return xh[c]; };
    AT acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = AT(0);
    AT own[R];
    if constexpr (LDS) {
        __shared__ AT xs[SPAN];
        __shared__ int sflag;
        const int base = w0 - DIA_HALO;
        if (dia_stage<AT, SPAN>(xs, base, n, sx, stop, &sflag)) return;
        dia_dots<VT, AT, R, true, NT, ND>(P, pos, w0, rb, n, sx, xs, base, acc);
        if (ND > 0 || two) dia_dots<VT, AT, R, true, NT, ND>(Q, pos, w0, rb, n, sx, xs, base, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) own[k] = xs[rb + k * WAVE - base];
    } else {
        if (stop && *stop) return;
        dia_dots<VT, AT, R, false, NT, ND>(P, pos, w0, rb, n, sx, nullptr, 0, acc);
        if (ND > 0 || two) dia_dots<VT, AT, R, false, NT, ND>(Q, pos, w0, rb, n, sx, nullptr, 0, acc);
#pragma unroll
        for (int k = 0; k < R; ++k) own[k] = xh[clamp_col(rb + k * WAVE, n)];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = rb + k * WAVE;
        if (row >= n) break;
        const AT s0 = svp ? svp[row] : (AT)(v[row] * sl[row]);
        const AT r = (s0 - cdiag * own[k]) - acc[k];
        finish<AT>(dst, row, r, w, rh, const_cast<AT *>(xh), xout, z, sr);
    }
}

// Inner JR pass on a 3-row block triangle (as k_dia_inner), a lane owning
// the R nodes nb + 64 k and their three rows each.  FIN as in k_dia_inner.
template <typename VT, typename AT, int R, bool NT, bool FIN>
__global__ __launch_bounds__(DIA_THREADS) void k_b3_inner(const int *__restrict__ stop, int remap, int n, DiaView T,
                                                          const AT *__restrict__ rh, const AT *__restrict__ gin,
                                                          const double *__restrict__ v, const double *__restrict__ sl,
                                                          int rv, int gv, int damp, AT w, AT gamma, int dst,
                                                          AT *__restrict__ gout, AT *__restrict__ xh,
                                                          double *__restrict__ z, const double *__restrict__ sr,
                                                          const double *__restrict__ fpart, int fnb, void *fst)
{
    constexpr int NBW = DIA_THREADS * R; // nodes per workgroup
    if constexpr (FIN) {
        if (blockIdx.x == 0) {
            dcgs_finish_block(fpart, fnb, static_cast<GState *>(fst));
            return;
        }
    }
    const int sh = FIN ? 1 : 0;
    const int wg = remap ? (int)xcd_remap(blockIdx.x - sh, gridDim.x - sh) : (int)(blockIdx.x - sh);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int nn = n / 3, g0 = wg * NBW;
    const int nb = g0 + wv * (WAVE * R) + lane;
    const int64_t pos = (int64_t)g0 + wv * (WAVE * R) + lane * R;
    if (stop && *stop) return;
    auto sv = [&](int c) { return (AT)(v[c] * sl[c]); };
    auto sg = [&](int c) { return gin[c]; };
    AT acc[R][3];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k][0] = acc[k][1] = acc[k][2] = AT(0);
    if (gv) b3_node_dots<VT, AT, R, NT>(T, pos, g0, nb, nn, sv, acc);
    else b3_node_dots<VT, AT, R, NT>(T, pos, g0, nb, nn, sg, acc);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int node = nb + k * WAVE;
        if (node >= nn) break;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int row = 3 * node + j;
            const AT r = rv ? (AT)(v[row] * sl[row]) : rh[row];
            AT g = r - w * acc[k][j];
            if (damp) {
                const AT go = gv ? (AT)(v[row] * sl[row]) : gin[row];
                g = (AT(1) - gamma) * go + gamma * g;
            }
            finish<AT>(dst, row, g, w, gout, xh, xh, z, sr);
        }
    }
}

// Outer residual pass on 3-row block triangles (as k_dia_resid), a lane
// owning the R nodes nb + 64 k and their three rows each.
template <typename VT, typename AT, int R, bool NT>
__global__ __launch_bounds__(DIA_THREADS) void k_b3_resid(const int *__restrict__ stop, int remap, int n, DiaView P,
                                                          DiaView Q, int two, const AT *__restrict__ xh,
                                                          const double *__restrict__ v, const double *__restrict__ sl,
                                                          const AT *__restrict__ svp, AT cdiag, AT w, int dst,
                                                          AT *__restrict__ rh, AT *__restrict__ xout,
                                                          double *__restrict__ z, const double *__restrict__ sr)
{
    constexpr int NBW = DIA_THREADS * R;
    const int wg = remap ? (int)xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int nn = n / 3, g0 = wg * NBW;
    const int nb = g0 + wv * (WAVE * R) + lane;
    const int64_t pos = (int64_t)g0 + wv * (WAVE * R) + lane * R;
    if (stop && *stop) return;
    auto sx = [&](int c) { return xh[c]; };
    AT acc[R][3];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k][0] = acc[k][1] = acc[k][2] = AT(0);
    b3_node_dots<VT, AT, R, NT>(P, pos, g0, nb, nn, sx, acc);
    if (two) b3_node_dots<VT, AT, R, NT>(Q, pos, g0, nb, nn, sx, acc);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int node = nb + k * WAVE;
        if (node >= nn) break;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int row = 3 * node + j;
            const AT s0 = svp ? svp[row] : (AT)(v[row] * sl[row]);
            const AT r = (s0 - cdiag * xh[row]) - acc[k][j];
            finish<AT>(dst, row, r, w, rh, const_cast<AT *>(xh), xout, z, sr);
        }
    }
}

// ---------------------------------------- inner-iteration diagnostic (f1)
//
// Section 8 follows the inner JR iteration on its own: for a fixed r, the
// relative residual ||r - (wL + D) g_j|| / ||r|| of the lower triangular
// system after j inner steps.  In scaled space S_l (r - (wL + D) g) =
// rh - (I + w Lh) gh = gh_{j+1} - gh_j, since gh_{j+1} = rh - w Lh gh_j: the
// residual of step j is the change made by step j + 1, unscaled by 1/s_l.

// part[blockIdx] = sum over the workgroup's rows of ((gnew - gold) / s_l)^2,
// gold = AT(r s_l) when gold is null (step 0); with gnew null, the sum of
// r^2 instead.  One partial per workgroup, summed later in a fixed order.
template <typename AT>
__global__ __launch_bounds__(KT) void k_diff_sums(int64_t n, const AT *__restrict__ gnew, const AT *__restrict__ gold,
                                                  const double *__restrict__ r, const double *__restrict__ sl,
                                                  double *__restrict__ part)
{
    __shared__ double red[KT / WAVE];
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    double t = 0.0;
    if (i < n) {
        if (!gnew) {
            t = r[i] * r[i];
        } else {
            const double go = gold ? (double)gold[i] : (double)(AT)(r[i] * sl[i]);
            const double d = ((double)gnew[i] - go) / sl[i];
            t = d * d;
        }
    }
    const double sblk = block_sum(t, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sblk;
}

// out[q] = sum of part[q * nb .. q * nb + nb) in a fixed order, q < nq.
__global__ __launch_bounds__(KT) void k_sum_parts(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double red[KT / WAVE];
    const double t = strided_sum(part + (int64_t)blockIdx.x * nb, nb);
    const double sblk = block_sum(t, red);
    if (threadIdx.x == 0) out[blockIdx.x] = sblk;
}

// out[j] = sqrt(sums[j]) / sqrt(sums[nq - 1]) for j < nq - 1.
__global__ void k_ratios(const double *__restrict__ sums, int nq, double *__restrict__ out)
{
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j < nq - 1) out[j] = sqrt(sums[j]) / sqrt(sums[nq - 1]);
}

// Reads p[0 .. m) (zeros) so that the caches hold none of the data a timed
// pass is about to read; the sum is stored only if nonzero, which keeps the
// loads.
__global__ __launch_bounds__(KT) void k_flush(double *__restrict__ p, int64_t m)
{
    double t = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < m; i += (int64_t)gridDim.x * KT) t += p[i];
    if (t != 0.0) p[0] = t;
}

// ------------------------------------------------------------ host drivers

constexpr int TB = KT; // 4 wavefronts per workgroup, one or two slices each

static inline unsigned grid_for(int64_t nslices, int su)
{
    const int64_t per = 4 * su;
    return (unsigned)std::max<int64_t>(1, (nslices + per - 1) / per);
}
static inline unsigned grid_rows(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TB - 1) / TB); }

template <typename VT, typename AT>
struct Launch {
    // rows per lane of the diagonal-interleaved layout: one load of 2..16 bytes
    template <int R>
    static constexpr bool r_ok()
    {
        return R * sizeof(VT) >= 2 && R * sizeof(VT) <= 16;
    }
    static double dia_bytes(const Dia &D) { return (double)D.nnz * sizeof(VT); }
    static const Dia &dia_of(const Handle &h, const Sell &T) { return &T == &h.L ? h.DL : h.DU; }

    template <int R, int FL>
    static void dia_inner_r(const Handle &h, const Dia &T, const AT *rh, const AT *gin, const double *v, int rv,
                            int gv, int dst, AT *gout, AT *xh, double *z, hipStream_t s, const Handle::FinJob &fj)
    {
        const int damp = h.gamma != 1.0;
        const int64_t units = (FL & DIA_FL_B3) ? h.n / 3 : h.n; // nodes or rows
        const unsigned grid = (unsigned)((units + (int64_t)DIA_THREADS * R - 1) / ((int64_t)DIA_THREADS * R)) + (fj.st ? 1u : 0u);
        const DiaView dv = dview(T);
        const int n = (int)h.n;
        if constexpr ((FL & DIA_FL_B3) != 0) {
            constexpr bool NT = FL & DIA_FL_NT;
            if (fj.st)
                k_b3_inner<VT, AT, R, NT, true><<<grid, DIA_THREADS, 0, s>>>(
                    h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh,
                    z, h.sr, fj.part, fj.nb, fj.st);
            else
                k_b3_inner<VT, AT, R, NT, false><<<grid, DIA_THREADS, 0, s>>>(
                    h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh,
                    z, h.sr, nullptr, 0, nullptr);
        } else {
            // three diagonals per triangle (7-point stencils): the loop over them unrolled
            if (T.ndiag == 3) {
                if (fj.st)
                    k_dia_inner<VT, AT, R, FL, true, 3><<<grid, DIA_THREADS, 0, s>>>(
                        h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout,
                        xh, z, h.sr, fj.part, fj.nb, fj.st);
                else
                    k_dia_inner<VT, AT, R, FL, false, 3><<<grid, DIA_THREADS, 0, s>>>(
                        h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout,
                        xh, z, h.sr, nullptr, 0, nullptr);
                return;
            }
            if (fj.st)
                k_dia_inner<VT, AT, R, FL, true, 0><<<grid, DIA_THREADS, 0, s>>>(
                    h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh,
                    z, h.sr, fj.part, fj.nb, fj.st);
            else
                k_dia_inner<VT, AT, R, FL, false, 0><<<grid, DIA_THREADS, 0, s>>>(
                    h.stop, h.remap, n, dv, rh, gin, v, h.sl, rv, gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh,
                    z, h.sr, nullptr, 0, nullptr);
        }
    }
    template <int R>
    static void dia_inner_f(const Handle &h, const Dia &T, const AT *rh, const AT *gin, const double *v, int rv,
                            int gv, int dst, AT *gout, AT *xh, double *z, hipStream_t s, const Handle::FinJob &fj)
    {
        switch (dia_flags(h, T)) {
        case 0: dia_inner_r<R, 0>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 1: dia_inner_r<R, 1>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 2: dia_inner_r<R, 2>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 3: dia_inner_r<R, 3>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 4: dia_inner_r<R, 4>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        default: dia_inner_r<R, 6>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        }
    }
    static void dia_inner_l(const Handle &h, const Dia &T, const AT *rh, const AT *gin, const double *v, int rv,
                            int gv, int dst, AT *gout, AT *xh, double *z, hipStream_t s, const Handle::FinJob &fj)
    {
        switch (T.R) {
        case 1:
            if constexpr (r_ok<1>()) dia_inner_f<1>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj);
            break;
        case 2:
            if constexpr (r_ok<2>()) dia_inner_f<2>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj);
            break;
        case 4:
            if constexpr (r_ok<4>()) dia_inner_f<4>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj);
            break;
        default:
            if constexpr (r_ok<8>()) dia_inner_f<8>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj);
            break;
        }
    }
    template <int R, int FL>
    static void dia_resid_r(const Handle &h, const Dia &P, const Dia *Q, const AT *xh, const double *v, const AT *svp, AT cdiag,
                            AT w, int dst, AT *rh, AT *xout, double *z, hipStream_t s)
    {
        const int64_t units = (FL & DIA_FL_B3) ? h.n / 3 : h.n; // nodes or rows
        const unsigned grid = (unsigned)((units + (int64_t)DIA_THREADS * R - 1) / ((int64_t)DIA_THREADS * R));
        const int n = (int)h.n;
        if constexpr ((FL & DIA_FL_B3) != 0) {
            k_b3_resid<VT, AT, R, (FL & DIA_FL_NT) != 0><<<grid, DIA_THREADS, 0, s>>>(
                h.stop, h.remap, n, dview(P), Q ? dview(*Q) : dview(P), Q ? 1 : 0, xh, v, h.sl, svp, cdiag, w, dst, rh,
                xout, z, h.sr);
        } else {
            // ND = 3 kernels always add both triangles (no branch on `two`, so the
            // loads of all six diagonals are issued together); one triangle (the
            // compact form's residual) takes the general kernel
            if (P.ndiag == 3 && Q && Q->ndiag == 3) {
                k_dia_resid<VT, AT, R, FL, 3><<<grid, DIA_THREADS, 0, s>>>(h.stop, h.remap, n, dview(P), dview(*Q), 1,
                                                                           xh, v, h.sl, svp, cdiag, w, dst, rh, xout,
                                                                           z, h.sr);
                return;
            }
            k_dia_resid<VT, AT, R, FL, 0><<<grid, DIA_THREADS, 0, s>>>(h.stop, h.remap, n, dview(P),
                                                                       Q ? dview(*Q) : dview(P), Q ? 1 : 0, xh, v,
                                                                       h.sl, svp, cdiag, w, dst, rh, xout, z, h.sr);
        }
    }
    template <int R>
    static void dia_resid_f(const Handle &h, const Dia &P, const Dia *Q, const AT *xh, const double *v, const AT *svp, AT cdiag,
                            AT w, int dst, AT *rh, AT *xout, double *z, hipStream_t s)
    {
        switch (dia_flags(h, P)) {
        case 0: dia_resid_r<R, 0>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        case 1: dia_resid_r<R, 1>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        case 2: dia_resid_r<R, 2>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        case 3: dia_resid_r<R, 3>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        case 4: dia_resid_r<R, 4>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        default: dia_resid_r<R, 6>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s); break;
        }
    }
    static void dia_resid_l(const Handle &h, const Dia &P, const Dia *Q, const AT *xh, const double *v, const AT *svp, AT cdiag,
                            AT w, int dst, AT *rh, AT *xout, double *z, hipStream_t s)
    {
        switch (P.R) {
        case 1:
            if constexpr (r_ok<1>()) dia_resid_f<1>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s);
            break;
        case 2:
            if constexpr (r_ok<2>()) dia_resid_f<2>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s);
            break;
        case 4:
            if constexpr (r_ok<4>()) dia_resid_f<4>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s);
            break;
        default:
            if constexpr (r_ok<8>()) dia_resid_f<8>(h, P, Q, xh, v, svp, cdiag, w, dst, rh, xout, z, s);
            break;
        }
    }

    template <int K>
    static void inner_k(const Handle &h, const Sell &T, const AT *rh, const AT *gin, const double *v, int rv, int gv,
                        int dst, AT *gout, AT *xh, double *z, hipStream_t s, const Handle::FinJob &fj)
    {
        const int damp = h.gamma != 1.0;
        const unsigned grid = grid_for(T.nslices, su_of<AT>()) + (fj.st ? 1u : 0u);
        if (fj.st)
            k_inner<VT, AT, K, true><<<grid, TB, 0, s>>>(h.stop, h.n, T.nslices, view(T), rh, gin, v, h.sl, rv, gv,
                                                         damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh, z, h.sr,
                                                         fj.part, fj.nb, fj.st);
        else
            k_inner<VT, AT, K, false><<<grid, TB, 0, s>>>(h.stop, h.n, T.nslices, view(T), rh, gin, v, h.sl, rv,
                                                          gv, damp, (AT)h.omega, (AT)h.gamma, dst, gout, xh, z,
                                                          h.sr, nullptr, 0, nullptr);
    }
    // algorithmic bytes of one pass: each stored entry (value + column) and
    // each vector element read or written once; padding is not counted
    static double tri_bytes(const Sell &T)
    {
        return (double)T.nnz * (sizeof(VT) + T.idx_bytes()) + 8.0 * (T.nslices + 1);
    }
    static double dst_bytes(int dst)
    {
        const double bx = sizeof(AT);
        switch (dst) {
        case DST_G: return bx;
        case DST_XADD: return 2 * bx;
        case DST_XSET: return bx;
        case DST_ZADD: return bx + 16;
        default: return 16;
        }
    }
    static void inner(const Handle &h, const Sell &T, const AT *rh, const AT *gin, const double *v, int rv, int gv,
                      int dst, AT *gout, AT *xh, double *z, hipStream_t s,
                      const Handle::FinJob &fj = Handle::FinJob{})
    {
        const double bx = sizeof(AT);
        const double src = gv ? 16.0 : rv ? 16.0 + bx : 2 * bx;
        if (h.fmt == FMT_DIA) {
            const Dia &D = dia_of(h, T);
            Prof pr(s, PK_INNER, dia_bytes(D) + (double)h.n * (src + dst_bytes(dst)));
            dia_inner_l(h, D, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj);
            return;
        }
        Prof pr(s, PK_INNER, tri_bytes(T) + (double)h.n * (src + dst_bytes(dst)));
        switch (T.K) {
        case 1: inner_k<1>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 2: inner_k<2>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 4: inner_k<4>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 8: inner_k<8>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 16: inner_k<16>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        case 32: inner_k<32>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        default: inner_k<64>(h, T, rh, gin, v, rv, gv, dst, gout, xh, z, s, fj); break;
        }
    }
    template <int K>
    static void resid_k(const Handle &h, const Sell &P, const Sell *Q, const AT *xh, const double *v, AT cdiag, AT w,
                        int dst, AT *rh, AT *xout, double *z, hipStream_t s, const AT *ye)
    {
        k_resid<VT, AT, K><<<grid_for(P.nslices, su_of<AT>()), TB, 0, s>>>(h.stop, h.n, P.nslices, view(P), Q ? view(*Q) : view(P),
                                                              Q ? 1 : 0, xh, v, h.sl, cdiag, w, dst, rh, xout, z, h.sr,
                                                              ye ? view(h.E) : view(P), ye);
    }
    // ye: values the off-block part E multiplies (NULL: no E term); svp:
    // S_l v in AT from this apply's prep pass (diagonal layout only), or NULL
    static void resid(const Handle &h, const Sell &P, const Sell *Q, const AT *xh, const double *v, AT cdiag, AT w,
                      int dst, AT *rh, AT *xout, double *z, hipStream_t s, const AT *ye = nullptr,
                      const AT *svp = nullptr)
    {
        const double out = (dst == DST_ZADD || dst == DST_ZSET) ? 16.0 : (double)sizeof(AT);
        if (h.fmt == FMT_DIA && !ye) {
            const Dia &DP = dia_of(h, P);
            const Dia *DQ = Q ? &dia_of(h, *Q) : nullptr;
            const double src = svp ? (double)sizeof(AT) : 16.0;
            Prof pr(s, PK_RESID, dia_bytes(DP) + (DQ ? dia_bytes(*DQ) : 0.0) + (double)h.n * (src + sizeof(AT) + out));
            dia_resid_l(h, DP, DQ, xh, v, svp, cdiag, w, dst, rh, xout, z, s);
            return;
        }
        Prof pr(s, PK_RESID,
                tri_bytes(P) + (Q ? tri_bytes(*Q) : 0.0) + (ye ? tri_bytes(h.E) + (double)h.n * sizeof(AT) : 0.0) +
                    (double)h.n * (16.0 + sizeof(AT) + out));
        switch (P.K) {
        case 1: resid_k<1>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        case 2: resid_k<2>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        case 4: resid_k<4>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        case 8: resid_k<8>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        case 16: resid_k<16>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        case 32: resid_k<32>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        default: resid_k<64>(h, P, Q, xh, v, cdiag, w, dst, rh, xout, z, s, ye); break;
        }
    }

    // z = Mhat^{-1} v (Fig. code:two-stage on one process: `sweeps` outer
    // sweeps, each a forward and/or backward half with n_j inner sweeps).
    // sv = AT(S_l v), carrying the previous GMRES step's closing work when fj is set
    static void prep(const Handle &h, const double *v, AT *sv, hipStream_t s, const Handle::FinJob &fj)
    {
        Prof pr(s, PK_PREP, (double)h.n * (16.0 + sizeof(AT)));
        const bool q4 = h.n % 4 == 0 && reinterpret_cast<uintptr_t>(v) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(h.sl) % 16 == 0 && reinterpret_cast<uintptr_t>(sv) % (4 * sizeof(AT)) == 0;
        const unsigned grid = q4 ? (unsigned)((h.n / 4 + KT - 1) / KT) : grid_rows(h.n);
        const int n = (int)h.n;
        if (q4) {
            if (fj.st) k_dia_prep<AT, true, 4><<<grid + 1u, KT, 0, s>>>(h.stop, n, v, h.sl, sv, fj.part, fj.nb, fj.st);
            else k_dia_prep<AT, false, 4><<<grid, KT, 0, s>>>(h.stop, n, v, h.sl, sv, nullptr, 0, nullptr);
        } else {
            if (fj.st) k_dia_prep<AT, true, 1><<<grid + 1u, KT, 0, s>>>(h.stop, n, v, h.sl, sv, fj.part, fj.nb, fj.st);
            else k_dia_prep<AT, false, 1><<<grid, KT, 0, s>>>(h.stop, n, v, h.sl, sv, nullptr, 0, nullptr);
        }
    }
    static int gs2(Handle &h, const double *v, double *z, hipStream_t s)
    {
        AT *xc = (AT *)h.xh, *xo = (AT *)h.xh2, *rh = (AT *)h.rh, *ga = (AT *)h.ga, *gb = (AT *)h.gb;
        AT *y = (AT *)h.yh;
        // a GMRES step's closing work rides on this apply's first pass
        Handle::FinJob fj = h.fin;
        h.fin = Handle::FinJob{};
        const int per = h.variant == GS2_SYMMETRIC ? 2 : 1;
        const bool hyb = h.blocks > 1;
        const int nk = hyb ? h.local_sweeps : 1;
        const int H = h.sweeps * nk * per;
        const AT w = (AT)h.omega;
        const AT cdiag = h.compact ? (AT)(1.0 - 1.0 / h.omega) : AT(1);
        bool xzero = true, yzero = true;
        // the interface is exchanged once per global sweep (Fig. code:two-stage), so every
        // half of it sees the same off-block values; with a single half that is the live iterate
        const bool freeze = hyb && nk * per > 1;
        // 32- and 16-bit forms on the diagonal layout: S_l v formed once in AT
        // (prep), read by the first inner pass and every residual pass
        AT *svb = (sizeof(AT) < sizeof(double) && h.fmt == FMT_DIA && h.sv && h.inner >= 1 && !hyb) ? (AT *)h.sv
                                                                                                     : nullptr;
        int t = 0;
        for (int ts = 0; ts < h.sweeps; ++ts) {
            if (freeze) { // exchange: freeze the off-block values for this global sweep
                yzero = xzero;
                if (!xzero) k_copy_at<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, xc, y);
            }
            for (int k = 0; k < nk; ++k)
                for (int hf = 0; hf < per; ++hf, ++t) {
                    const bool lower = h.variant == GS2_FORWARD || (h.variant == GS2_SYMMETRIC && hf == 0);
                    const Sell &T = lower ? h.L : h.U;
                    const Sell &O = lower ? h.U : h.L;
                    const bool fin = t == H - 1;
                    const bool set = xzero || h.compact; // x <- w g replaces x
                    // off-block term: frozen copy, or the live iterate when the global sweep has one half
                    const AT *ye = !hyb ? nullptr : freeze ? (yzero ? nullptr : y) : xc;
                    if (h.inner == 0) {
                        if (xzero) {
                            Prof pr(s, PK_FIRST_JR, (double)h.n * (16.0 + (fin ? 16.0 : sizeof(AT))));
                            if (fj.st)
                                k_first_jr<AT, true><<<grid_rows(h.n) + 1u, TB, 0, s>>>(
                                    h.stop, h.n, v, h.sl, h.sr, w, fin ? 1 : 0, xc, z, fj.part, fj.nb, fj.st);
                            else
                                k_first_jr<AT, false><<<grid_rows(h.n), TB, 0, s>>>(
                                    h.stop, h.n, v, h.sl, h.sr, w, fin ? 1 : 0, xc, z, nullptr, 0, nullptr);
                            fj = Handle::FinJob{};
                        } else {
                            const int dst = fin ? (set ? DST_ZSET : DST_ZADD) : (set ? DST_XSET : DST_XADD);
                            if (h.compact) resid(h, O, nullptr, xc, v, cdiag, w, dst, nullptr, xo, z, s);
                            else resid(h, T, &O, xc, v, cdiag, w, dst, nullptr, xo, z, s, ye);
                            std::swap(xc, xo);
                        }
                    } else {
                        int rv = 1;
                        const AT *rsrc = rh; // this half's r (scaled), when not formed from v
                        if (!xzero) {
                            if (h.compact) resid(h, O, nullptr, xc, v, cdiag, w, DST_G, rh, nullptr, nullptr, s, nullptr, svb);
                            else resid(h, T, &O, xc, v, cdiag, w, DST_G, rh, nullptr, nullptr, s, ye, svb);
                            rv = 0;
                        } else if (svb) { // r = S_l v and g_0 = r, both read from sv
                            prep(h, v, svb, s, fj);
                            fj = Handle::FinJob{};
                            rsrc = svb;
                            rv = 0;
                        }
                        const AT *gin = rsrc;
                        for (int j = 1; j <= h.inner; ++j) {
                            const bool last = j == h.inner;
                            const int gv = (j == 1 && xzero && !svb) ? 1 : 0;
                            AT *gout = (j & 1) ? ga : gb;
                            const int dst =
                                !last ? DST_G : fin ? (set ? DST_ZSET : DST_ZADD) : (set ? DST_XSET : DST_XADD);
                            inner(h, T, rsrc, gin, v, rv, gv, dst, gout, xc, z, s, fj);
                            fj = Handle::FinJob{};
                            gin = gout;
                        }
                    }
                    xzero = false;
                }
        }
        // keep the handle's notion of the current iterate buffer stable
        if (xc != (AT *)h.xh) std::swap(h.xh, h.xh2);
        return GS2_OK;
    }

    // JR(n_t, n_k): `sweeps` global sweeps of n_k local sweeps each (one local
    // sweep without blocks)
    static int jr(Handle &h, int sweeps, double omega, const double *v, double *z, hipStream_t s)
    {
        AT *xc = (AT *)h.xh, *xo = (AT *)h.xh2, *y = (AT *)h.yh;
        const AT w = (AT)omega;
        const bool hyb = h.blocks > 1;
        const int nk = hyb ? h.local_sweeps : 1;
        const int total = sweeps * nk;
        {
            // a GMRES step's closing work rides on this first pass
            const Handle::FinJob fj = h.fin;
            h.fin = Handle::FinJob{};
            Prof pr(s, PK_FIRST_JR, (double)h.n * (16.0 + (total == 1 ? 16.0 : sizeof(AT))));
            if (fj.st)
                k_first_jr<AT, true><<<grid_rows(h.n) + 1u, TB, 0, s>>>(
                    h.stop, h.n, v, h.sl, h.sr, w, total == 1 ? 1 : 0, xc, z, fj.part, fj.nb, fj.st);
            else
                k_first_jr<AT, false><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, v, h.sl, h.sr, w,
                                                                    total == 1 ? 1 : 0, xc, z, nullptr, 0, nullptr);
        }
        bool yzero = true;
        for (int step = 1; step < total; ++step) {
            if (hyb && nk > 1 && step % nk == 0) {
                k_copy_at<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, xc, y);
                yzero = false;
            }
            const AT *ye = !hyb ? nullptr : nk > 1 ? (yzero ? nullptr : y) : xc;
            resid(h, h.L, &h.U, xc, v, AT(1), w, step == total - 1 ? DST_ZADD : DST_XADD, nullptr, xo, z, s, ye);
            std::swap(xc, xo);
        }
        if (xc != (AT *)h.xh) std::swap(h.xh, h.xh2);
        return GS2_OK;
    }

    static int tri(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s)
    {
        AT *xa = (AT *)h.xh, *xb = (AT *)h.xh2;
        const AT w = (AT)omega;
        const AT *xold = nullptr;
        AT *xnew = xa;
        for (int t = 0; t < h.sweeps; ++t) {
            for (int half = 0; half < 2; ++half) {
                const bool fwd = half == 0;
                if (fwd && variant == GS2_BACKWARD) continue;
                if (!fwd && variant == GS2_FORWARD) continue;
                k_fill_zero<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, xnew);
                const Sell &Mt = fwd ? h.L : h.U;
                const Sell &Ot = fwd ? h.U : h.L;
                const std::vector<int64_t> &ptr = fwd ? h.lev_ptr_l : h.lev_ptr_u;
                const int32_t *rows = fwd ? h.lev_rows_l : h.lev_rows_u;
                const int nlev = fwd ? h.nlev_l : h.nlev_u;
                for (int l = 0; l < nlev; ++l) {
                    const int64_t cnt = ptr[l + 1] - ptr[l];
                    if (cnt <= 0) continue;
                    Prof pr(s, PK_TRI, (double)cnt * (16.0 + 2 * sizeof(AT)));
                    k_tri_level<VT, AT><<<(unsigned)((cnt + TB - 1) / TB), TB, 0, s>>>(
                        h.stop, rows + ptr[l], cnt, Mt.K, view(Mt), view(Ot), xold, xnew, v, h.sl, w);
                }
                xold = xnew;
                xnew = (xnew == xa) ? xb : xa;
            }
        }
        k_unscale<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, xold, h.sr, z);
        return GS2_OK;
    }

    // multicolor GS/SOR: `sweeps` sweeps from x = 0, colors ascending
    // (forward), descending (backward) or both (symmetric)
    static int mtgs(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s)
    {
        AT *x = (AT *)h.xh;
        const AT w = (AT)omega;
        k_fill_zero<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, x);
        for (int t = 0; t < h.sweeps; ++t)
            for (int half = 0; half < 2; ++half) {
                const bool fwd = half == 0;
                if (fwd && variant == GS2_BACKWARD) continue;
                if (!fwd && variant == GS2_FORWARD) continue;
                for (int q = 0; q < h.ncolors; ++q) {
                    const int c = fwd ? q : h.ncolors - 1 - q;
                    const int64_t cnt = h.color_ptr[c + 1] - h.color_ptr[c];
                    if (cnt <= 0) continue;
                    Prof pr(s, PK_TRI, (double)cnt * (16.0 + 2 * sizeof(AT)));
                    k_color<VT, AT><<<(unsigned)((cnt + TB - 1) / TB), TB, 0, s>>>(
                        h.stop, h.color_rows + h.color_ptr[c], cnt, h.L.K, view(h.L), view(h.U), x, v, h.sl, w);
                }
            }
        k_unscale<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, x, h.sr, z);
        return GS2_OK;
    }

    // The diagnostic of Section 8 for j = 0 .. inner with the handle's L,
    // damping and precision, enqueued on s: per-workgroup partial sums in
    // part (nb * (inner + 2) doubles, nb = ceil(n / KT)), their totals in sums
    // (inner + 2), the ratios in out (device, inner + 1).  Every slot of part
    // and sums is written before it is read, so neither needs clearing.
    static int inner_residuals_enqueue(Handle &h, const double *r, int nj, double *part, double *sums,
                                       double *out, hipStream_t s)
    {
        const int nb = (int)((h.n + KT - 1) / KT);
        const int nq = nj + 2; // quantities: steps 0..inner, then ||r||^2
        AT *ga = (AT *)h.ga, *gb = (AT *)h.gb;
        const AT *gold = nullptr;
        for (int j = 0; j <= nj; ++j) {
            AT *gnew = (j & 1) ? gb : ga; // gh_{j+1}
            inner(h, h.L, nullptr, gold, r, 1, j == 0 ? 1 : 0, DST_G, gnew, nullptr, nullptr, s);
            k_diff_sums<AT><<<nb, KT, 0, s>>>(h.n, gnew, gold, r, h.sl, part + (size_t)j * nb);
            gold = gnew;
        }
        k_diff_sums<AT><<<nb, KT, 0, s>>>(h.n, nullptr, nullptr, r, h.sl, part + (size_t)(nj + 1) * nb);
        k_sum_parts<<<nq, KT, 0, s>>>(part, nb, sums);
        k_ratios<<<(unsigned)((nq + KT - 1) / KT), KT, 0, s>>>(sums, nq, out);
        GS2_TRY_HIP(hipGetLastError());
        return GS2_OK;
    }

    // The same with its own temporaries (allocated and freed here); out is a
    // host array.  Synchronises the stream.
    static int inner_residuals(Handle &h, const double *r, int nj, double *out, hipStream_t s)
    {
        const int nb = (int)((h.n + KT - 1) / KT);
        const int nq = nj + 2;
        double *part = nullptr, *sums = nullptr;
        GS2_TRY_HIP(hipMalloc(&part, sizeof(double) * (size_t)nb * nq));
        if (hipMalloc(&sums, sizeof(double) * (2 * nq - 1)) != hipSuccess) {
            (void)hipFree(part);
            return GS2_ERR_NOMEM;
        }
        int st = inner_residuals_enqueue(h, r, nj, part, sums, sums + nq, s);
        if (st == GS2_OK && (hipMemcpyAsync(out, sums + nq, sizeof(double) * (nj + 1), hipMemcpyDeviceToHost, s) !=
                                 hipSuccess ||
                             hipStreamSynchronize(s) != hipSuccess))
            st = GS2_ERR_HIP;
        (void)hipFree(part);
        (void)hipFree(sums);
        return st;
    }

    // Time of one inner pass over L (and, with resid, one residual pass over
    // both triangles): batches of back-to-back passes between one pair of
    // events (timing-only events, no cache writeback), best of three batches
    // after a warm-up batch.
    static int time_inner(Handle &h, hipStream_t s, float *ms, bool with_resid)
    {
        // with the flush buffer: one pair of passes per timing, each after a
        // read of the buffer; without it, batches of five back to back
        const int batch = h.flush ? 1 : 5, reps = h.flush ? 6 : 4;
        hipEvent_t e0, e1;
        GS2_TRY_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
        GS2_TRY_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
        k_fill_zero<AT><<<grid_rows(h.n), TB, 0, s>>>(h.stop, h.n, (AT *)h.ga);
        float best = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            if (h.flush) k_flush<<<2048, TB, 0, s>>>(h.flush, (int64_t)(FLUSH_BYTES / sizeof(double)));
            GS2_TRY_HIP(hipEventRecord(e0, s));
            for (int b = 0; b < batch; ++b) {
                inner(h, h.L, (const AT *)h.ga, (const AT *)h.ga, nullptr, 0, 0, DST_G, (AT *)h.gb, nullptr, nullptr,
                      s);
                if (with_resid)
                    resid(h, h.L, &h.U, (const AT *)h.ga, h.sl, AT(1), AT(1), DST_G, (AT *)h.rh, nullptr,
                          nullptr, s);
            }
            GS2_TRY_HIP(hipEventRecord(e1, s));
            GS2_TRY_HIP(hipEventSynchronize(e1));
            float t = 0.f;
            GS2_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) best = std::min(best, t / batch);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = best;
        return GS2_OK;
    }
};

#define GS2_DISPATCH(h, call)                                                        \
    ((h).precision == GS2_FP64   ? Launch<double, double>::call                      \
     : (h).precision == GS2_FP32 ? Launch<float, float>::call                        \
                                 : Launch<_Float16, float>::call)

int apply_gs2(Handle &h, const double *v, double *z, hipStream_t s)
{
    int st = GS2_DISPATCH(h, gs2(h, v, z, s));
    GS2_TRY_HIP(hipGetLastError());
    return st;
}

int apply_jr(Handle &h, int sweeps, double omega, const double *v, double *z, hipStream_t s)
{
    int st = GS2_DISPATCH(h, jr(h, sweeps, omega, v, z, s));
    GS2_TRY_HIP(hipGetLastError());
    return st;
}

int apply_trisolve(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s)
{
    int st = GS2_DISPATCH(h, tri(h, variant, omega, v, z, s));
    GS2_TRY_HIP(hipGetLastError());
    return st;
}

int apply_mtgs(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s)
{
    int st = GS2_DISPATCH(h, mtgs(h, variant, omega, v, z, s));
    GS2_TRY_HIP(hipGetLastError());
    return st;
}

int inner_residuals(Handle &h, const double *r, int inner, double *out, hipStream_t s)
{
    return GS2_DISPATCH(h, inner_residuals(h, r, inner, out, s));
}

// --------------------------------- fixed scratch of the allocation-free entry
//
// The allocation-free diagnostic keeps its partial sums in this array: one
// copy per device, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address resolved once per device by
// noalloc_scratch().
static __device__ __align__(256) double scratch[GS2_NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (resolved on the first
// call per device, with that device current).
int noalloc_scratch(double **ptr)
{
    int dev = 0;
    GS2_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return GS2_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        GS2_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return GS2_ERR_HIP;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    if (ptr) *ptr = g_scratch_ptr[dev];
    return GS2_OK;
}

int time_inner_pass(Handle &h, hipStream_t s, float *ms, bool with_resid)
{
    int st = GS2_DISPATCH(h, time_inner(h, s, ms, with_resid));
    GS2_TRY_HIP(hipGetLastError());
    return st;
}

} // namespace gs2

using namespace gs2;

extern "C" {

int gs2_apply(gs2_handle *H, const double *v, double *z, void *stream)
{
    if (!H || (H->h.n > 0 && (!v || !z)) || v == z) return GS2_ERR_ARG;
    if (H->h.n == 0) return GS2_OK;
    return apply_gs2(H->h, v, z, (hipStream_t)stream);
}

int jr_apply(gs2_handle *H, int sweeps, double damping, const double *v, double *z, void *stream)
{
    if (!H || sweeps < 1 || !(damping > 0.0 && damping < 2.0) || (H->h.n > 0 && (!v || !z)) || v == z)
        return GS2_ERR_ARG;
    if (H->h.n == 0) return GS2_OK;
    return apply_jr(H->h, sweeps, damping, v, z, (hipStream_t)stream);
}

int gs_trisolve_apply(gs2_handle *H, int variant, double damping, const double *v, double *z, void *stream)
{
    if (!H || variant < GS2_FORWARD || variant > GS2_SYMMETRIC || !(damping > 0.0 && damping < 2.0) ||
        (H->h.n > 0 && (!v || !z)) || v == z)
        return GS2_ERR_ARG;
    if (H->h.n == 0) return GS2_OK;
    if (H->h.nlev_l == 0) return GS2_ERR_NO_LEVELS;
    return apply_trisolve(H->h, variant, damping, v, z, (hipStream_t)stream);
}

int mtgs_apply(gs2_handle *H, int variant, double damping, const double *v, double *z, void *stream)
{
    if (!H || variant < GS2_FORWARD || variant > GS2_SYMMETRIC || !(damping > 0.0 && damping < 2.0) ||
        (H->h.n > 0 && (!v || !z)) || v == z)
        return GS2_ERR_ARG;
    if (H->h.n == 0) return GS2_OK;
    if (H->h.ncolors == 0) return GS2_ERR_NO_LEVELS;
    return apply_mtgs(H->h, variant, damping, v, z, (hipStream_t)stream);
}

int gs2_inner_residuals(gs2_handle *H, const double *r, int inner, double *out, void *stream)
{
    if (!H || inner < 0 || !out || (H->h.n > 0 && !r)) return GS2_ERR_ARG;
    if (H->h.n == 0 || H->h.blocks > 1) return H->h.n == 0 ? GS2_OK : GS2_ERR_ARG;
    return inner_residuals(H->h, r, inner, out, (hipStream_t)stream);
}

int gs2_inner_residuals_noalloc(gs2_handle *H, const double *r, int inner, double *out, void *stream)
{
    if (!H || inner < 0 || !out || (H->h.n > 0 && !r)) return GS2_ERR_ARG;
    if (H->h.n == 0 || H->h.blocks > 1) return H->h.n == 0 ? GS2_OK : GS2_ERR_ARG;
    const int64_t nb = (H->h.n + KT - 1) / KT, nq = (int64_t)inner + 2;
    if (nb * nq + nq > GS2_NOALLOC_SCRATCH_DOUBLES) return GS2_ERR_SCRATCH;
    double *part = nullptr;
    GS2_TRY(noalloc_scratch(&part));
    ProfPause quiet; // the profiler's event records would allocate
    Handle &h = H->h;
    const hipStream_t s = (hipStream_t)stream;
    return GS2_DISPATCH(h, inner_residuals_enqueue(h, r, inner, part, part + nb * nq, out, s));
}

} // extern "C"
