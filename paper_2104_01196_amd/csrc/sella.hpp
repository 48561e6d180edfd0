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

struct SellA {
    const void *rp = nullptr, *ci = nullptr;
    int64_t n = 0, nnz = 0;
    int K = 1, C = WAVE;
    int64_t nslices = 0, padded = 0;
    int64_t *sp = nullptr; // nslices + 1 offsets (multiples of 64)
    int32_t *col = nullptr;
    double *val = nullptr;
};

struct SellAView {
    int64_t nslices;
    const int64_t *sp;
    const int32_t *col;
    const double *val;
};

inline SellAView view(const SellA &S) { return SellAView{S.nslices, S.sp, S.col, S.val}; }

// (Re)build the structure when the pattern is new, then copy the values.
int sella_prepare(SellA &S, const gs2_csr &A, hipStream_t s);
void sella_free(SellA &S);

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

} // namespace gs2
