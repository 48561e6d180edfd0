// A float64 sliced-ELL copy of the system matrix for the Krylov solvers'
// products w = A z (the same layout as the preconditioner's triangles: K
// lanes per row, C = 64/K rows per slice, one wavefront per slice, 64
// contiguous entries per step, padding (own column, 0)).  The CSR input's
// per-row pointer chain rowptr -> colind -> z becomes one independent load
// of (value, column) per step plus the gather of z.
//
// Columns stay 32-bit here: 16-bit column offsets (as the preconditioner's
// triangles use) made this copy's product slower on the 128^3 Laplacian
// (110.6 against 108.0 us per fused product and first Gram-Schmidt pass),
// with either cache policy for the offsets.
//
// The structure (slice pointers, columns) is built once per CSR pattern
// (keyed by the rowptr / colind pointers and sizes) and kept with the solver
// workspace; the values are copied again at the start of every solve, so a
// matrix whose values change in place between solves is honoured (its
// pattern must not change while the same arrays are passed).
#pragma once

#include "gs2_internal.hpp"

namespace gs2 {

// Rows per workgroup of the Krylov kernels that form w = A z (and of the
// padding of the diagonal copy below).
constexpr int KRB = 1024;

struct SellA {
    const void *rp = nullptr, *ci = nullptr;
    int64_t n = 0, nnz = 0;
    int K = 1, C = WAVE;
    int64_t nslices = 0, padded = 0;
    int64_t *sp = nullptr; // nslices + 1 offsets (multiples of 64)
    int32_t *col = nullptr;
    double *val = nullptr;
    // Diagonal-interleaved alternative for matrices with at most DIA_MAX
    // distinct offsets col - row (stencils in natural order): diagonal d holds
    // a_{i, i + off[d]} for every row i (0 where absent), rows in blocks of
    // 64 R, lane l of a block owning rows k*64 + l (k < R) with its R values
    // of one diagonal contiguous (one 8R-byte load), rows padded to whole
    // workgroups (KRB).  No column indices.  dR = 0: not built.
    int dR = 0, ndiag = 0;
    int64_t dstride = 0;
    double *dval = nullptr;
    int doff[DIA_MAX] = {};
    // Block-diagonal alternative for matrices of 3-row blocks (3 unknowns
    // per grid node, node-major, e.g. elasticity) with at most DIA_MAX
    // distinct node offsets c/3 - r/3: the same arrays (ndiag node offsets
    // in doff, dval, dstride), indexed by node, where plane 9 d + 3 k + b
    // holds a_{3i + k, 3(i + off[d]) + b} for every node i (0 where absent),
    // nodes contiguous and padded to whole KRB-node groups (dstride).  The
    // nine values of one node's block sit in nine planes at the same
    // position, so a lane that owns a node loads them with nine coalesced
    // loads and gathers the neighbour node's three x entries once for its
    // three rows.  No column indices.
    // the product's layout: sel > 0 sliced ELL with K = sel lanes per row,
    // -9 <= sel < 0 the diagonal copy with R = -sel rows per lane, sel <= -10
    // the 3-row block copy with -sel - 10 nodes per lane
    int sel = 1;
    int tuned = 0; // 1 if sel was chosen by timing the candidates
};

struct SellAView {
    int64_t nslices;
    const int64_t *sp;
    const int32_t *col;
    const double *val;
};

struct DiaAView {
    int ndiag;
    int64_t stride;
    const double *val;
    int off[DIA_MAX];
};

inline SellAView view(const SellA &S) { return SellAView{S.nslices, S.sp, S.col, S.val}; }
inline DiaAView dview(const SellA &S)
{
    DiaAView v;
    v.ndiag = S.ndiag;
    v.stride = S.dstride;
    v.val = S.dval;
    for (int d = 0; d < DIA_MAX; ++d) v.off[d] = S.doff[d];
    return v;
}

// Algorithmic bytes of one product w = A z in the chosen layout: every
// stored entry (value, plus the column for sliced ELL; padding not counted),
// the slice pointers, z gathered once and w written once.
inline double sella_bytes(const SellA &S)
{
    if (S.sel < 0) return 8.0 * (double)S.nnz + 16.0 * (double)S.n;
    return 12.0 * (double)S.nnz + 8.0 * (double)(S.nslices + 1) + 16.0 * (double)S.n;
}

// Building blocks of the copy (sella.hip); the Krylov solver picks among
// them (krylov.hip: prepare_matrix).
void sella_free(SellA &S);
// lanes per row the mean row length suggests
int sella_rule_lanes(const gs2_csr &A);
// sliced ELL with at least K0 lanes per row, values filled
int sella_build_sell(SellA &S, const gs2_csr &A, int K0, hipStream_t s);
// A's distinct offsets when it qualifies for the diagonal copy (<= DIA_MAX
// offsets, stored diagonals <= 1.5x the entries); *st reports HIP failures
bool sella_dia_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st);
// diagonal copy with R rows per lane (zeroed; fill with sella_fill_values)
int sella_build_dia(SellA &S, const gs2_csr &A, int R, const std::vector<int> &offs, hipStream_t s);
// A's distinct node offsets c/3 - r/3 when it qualifies for the 3-row
// block copy (n divisible by 3, <= DIA_MAX offsets, the blocks storing <=
// 1.5x the entries); *st reports HIP failures
bool sella_b3_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st);
// 3-row block copy for the product kernel with R nodes per lane (zeroed;
// fill with sella_fill_values)
int sella_build_b3(SellA &S, const gs2_csr &A, int R, const std::vector<int> &offs, hipStream_t s);
// copy A's values (and columns, for a new sliced-ELL structure) into S
int sella_fill_values(SellA &S, const gs2_csr &A, bool with_col, hipStream_t s);

// ybuf[i] = (A z)[r0 + i] for the RB rows of the workgroup starting at r0
// (0 past n), into LDS.  The workgroup's NW wavefronts take consecutive
// groups of RB / C / NW slices; each wavefront works on four slices at once
// so that their loads are in flight together.  The matrix is streamed with
// non-temporal loads, which leaves the caches to the gathered z.  Ends with
// a barrier.
template <int K, int RB, int NW>
__device__ __forceinline__ void sella_rows(const SellAView A, int64_t n, int64_t r0, const double *__restrict__ z,
                                           double *ybuf)
{
    constexpr int C = WAVE / K;
    constexpr int SPW = RB / C / NW; // slices per wavefront
    static_assert(RB % (C * NW) == 0, "rows per workgroup must split into whole slices per wavefront");
    constexpr int U = SPW < 4 ? SPW : 4;
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    const int64_t s0 = r0 / C + (int64_t)wv * SPW;
    for (int i0 = 0; i0 < SPW; i0 += U) {
        int64_t beg[U];
        int steps[U];
        int tmax = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t s = s0 + i0 + u;
            const bool ok = s < A.nslices;
            beg[u] = ok ? A.sp[s] : 0;
            steps[u] = ok ? (int)((A.sp[s + 1] - beg[u]) / WAVE) : 0;
            tmax = steps[u] > tmax ? steps[u] : tmax;
        }
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = 0.0;
        for (int t = 0; t < tmax; ++t) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t < steps[u]) {
                    const int64_t p = beg[u] + (int64_t)t * WAVE + ln;
                    acc[u] += __builtin_nontemporal_load(&A.val[p]) * z[__builtin_nontemporal_load(&A.col[p])];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double a = group_sum<K>(acc[u]);
            const int64_t row = (s0 + i0 + u) * C + ln / K;
            if ((ln & (K - 1)) == 0) ybuf[row - r0] = row < n ? a : 0.0;
        }
    }
    __syncthreads();
}

// ybuf[i] = (A z)[r0 + i] for the KRB rows of the workgroup starting at r0
// (0 past n), from the diagonal copy with R rows per lane.  Wavefront w of
// the NW takes the KRB / NW consecutive rows r0 + w KRB/NW, i.e. KRB / NW /
// (64 R) blocks; per diagonal a lane loads its R values of a block in one
// 8R-byte load (non-temporal: the copy is streamed once per product) and
// gathers z at row + off, 64 consecutive elements per wavefront load.
// Columns are clamped into [0, n) only in blocks whose shifted rows leave it
// (a clamped column meets a stored zero).  Ends with a barrier.
template <int R, int NW>
__device__ __forceinline__ void dia_rows(const DiaAView A, int64_t n, int64_t r0, const double *__restrict__ z,
                                         double *ybuf)
{
    constexpr int RW = KRB / NW;          // rows per wavefront
    constexpr int NBLK = RW / (WAVE * R); // blocks per wavefront
    static_assert(RW % (WAVE * R) == 0, "a wavefront's rows split into whole blocks");
    using V2 = double __attribute__((ext_vector_type(2)));
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    const int64_t w0 = r0 + (int64_t)wv * RW;
    double acc[NBLK][R];
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int k = 0; k < R; ++k) acc[b][k] = 0.0;
    for (int d = 0; d < A.ndiag; ++d) {
        const int o = A.off[d];
        const double *__restrict__ vd = A.val + (int64_t)d * A.stride;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            const int64_t base = w0 + (int64_t)b * (WAVE * R);
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
                if (!inside) c = c < 0 ? 0 : (c >= n ? n - 1 : c);
                acc[b][k] += a[k] * z[c];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int64_t row = w0 + (int64_t)b * (WAVE * R) + k * WAVE + ln;
            ybuf[row - r0] = row < n ? acc[b][k] : 0.0;
        }
    __syncthreads();
}

// ybuf[i] = (A z)[r0 + i] from the 3-row block copy (layout in SellA): the
// workgroup's threads take the nodes whose rows meet [r0, r0 + KRB), one
// node each in turn (the boundary nodes shared with the neighbouring
// workgroups are formed by both), and per node offset gather the neighbour
// node's three z entries once and load the block's nine values, in the
// order k_b3_spmv uses, so the two give the same sums.  Neighbour nodes are
// clamped into [0, n/3) (a clamped node meets stored zeros).  Rows past n
// get 0.  Ends with a barrier.
template <int NW>
__device__ __forceinline__ void b3_rows(const DiaAView A, int64_t n, int64_t r0, const double *__restrict__ z,
                                        double *ybuf)
{
    constexpr int NT = NW * WAVE; // threads of the workgroup
    const int64_t nn = n / 3, a0 = r0 / 3, a1 = (r0 + KRB - 1) / 3 < nn ? (r0 + KRB - 1) / 3 : nn - 1;
    for (int i = threadIdx.x; i < KRB; i += NT)
        if (r0 + i >= n) ybuf[i] = 0.0;
    for (int64_t i = a0 + threadIdx.x; i <= a1; i += NT) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < A.ndiag; ++d) {
            int64_t c = i + A.off[d];
            c = 3 * (c < 0 ? 0 : (c >= nn ? nn - 1 : c));
            const double z0 = z[c], z1 = z[c + 1], z2 = z[c + 2];
            const double *__restrict__ p0 = A.val + (int64_t)(9 * d) * A.stride + i;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double *__restrict__ pv = p0 + (int64_t)(3 * k) * A.stride;
                acc[k] += __builtin_nontemporal_load(pv) * z0;
                acc[k] += __builtin_nontemporal_load(pv + A.stride) * z1;
                acc[k] += __builtin_nontemporal_load(pv + 2 * A.stride) * z2;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t row = 3 * i + k;
            if (row >= r0 && row < r0 + KRB) ybuf[row - r0] = acc[k];
        }
    }
    __syncthreads();
}

// The product in the layout sel encodes (> 0 sliced ELL, K lanes per row;
// -9..-1 the diagonal copy, -sel rows per lane; <= -10 the 3-row block copy).
template <int SEL, int NW>
__device__ __forceinline__ void mat_rows(const SellAView A, const DiaAView D, int64_t n, int64_t r0,
                                         const double *__restrict__ z, double *ybuf)
{
    if constexpr (SEL > 0) sella_rows<SEL, KRB, NW>(A, n, r0, z, ybuf);
    else if constexpr (SEL <= -10) b3_rows<NW>(D, n, r0, z, ybuf);
    else dia_rows<-SEL, NW>(D, n, r0, z, ybuf);
}

} // namespace gs2
