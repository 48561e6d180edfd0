// Sliced-ELL copy of the system matrix for the Krylov solvers' SpMV.
#include <algorithm>
#include <vector>

#include "sella.hpp"

namespace gs2 {

// entries stored per slice: 64 * ceil(longest row of the slice / K); the
// element at index nslices is zero so that an exclusive scan ends the list
__global__ void k_sella_len(int64_t n, int64_t nslices, int K, const int32_t *__restrict__ rp,
                            int64_t *__restrict__ len)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nslices) return;
    if (s == nslices) {
        len[s] = 0;
        return;
    }
    const int C = WAVE / K;
    int m = 0;
    for (int r = 0; r < C; ++r) {
        const int64_t row = s * C + r;
        if (row < n) m = max(m, rp[row + 1] - rp[row]);
    }
    len[s] = (int64_t)WAVE * ((m + K - 1) / K);
}

// One thread per (slice, lane): lane l = r*K + q holds entries t*K + q of
// row r at step t; padding is (own column, 0).  Columns only when with_col.
__global__ void k_sella_fill(int64_t n, int64_t nslices, int K, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, const double *__restrict__ va,
                             const int64_t *__restrict__ sp, int with_col, int32_t *__restrict__ col,
                             double *__restrict__ val)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = gid / WAVE;
    if (s >= nslices) return;
    const int l = (int)(gid % WAVE), C = WAVE / K, r = l / K, q = l % K;
    const int64_t row = s * C + r;
    const int64_t beg = sp[s];
    const int steps = (int)((sp[s + 1] - beg) / WAVE);
    const int64_t b = row < n ? rp[row] : 0;
    const int len = row < n ? rp[row + 1] - rp[row] : 0;
    const int32_t pad = (int32_t)(row < n ? row : n - 1);
    for (int t = 0; t < steps; ++t) {
        const int e = t * K + q;
        const int64_t pos = beg + (int64_t)t * WAVE + l;
        const bool real = e < len;
        if (with_col) col[pos] = real ? ci[b + e] : pad;
        val[pos] = real ? va[b + e] : 0.0;
    }
}

void sella_free(SellA &S)
{
    for (void *p : {(void *)S.sp, (void *)S.col, (void *)S.val, (void *)S.dval})
        if (p) (void)hipFree(p);
    S = SellA{};
}

struct DiaOffsA {
    int nd;
    int off[DIA_MAX];
};

// Values of the diagonal (B3 = false) or 3-row block (B3 = true) copy, LANES
// threads per row, each taking every LANES-th entry of the row: entry (i, c)
// goes to diagonal t (the index of c - i among the offsets) at row i's
// position (interleaved by R rows per lane), or to plane
// 9 t + 3 (i mod 3) + (c mod 3) (t the index of the node offset c/3 - i/3)
// at node i/3's position.  The offsets are found by binary search in
// an LDS copy.  Entries of rows past n and absent entries keep the zeros
// written at allocation.  This runs at every solve (the values may have
// changed in place): one thread per row walking its entries took 2.3 ms per
// solve on the 64^3 elasticity matrix.
template <int LANES, bool B3>
__global__ __launch_bounds__(256) void k_copy_fill(int64_t n, int R, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ va,
                                                   DiaOffsA o, int64_t stride, double *__restrict__ val)
{
    __shared__ int soff[DIA_MAX];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < DIA_MAX; ++d) soff[d] = o.off[d];
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = g / LANES;
    if (i >= n) return;
    int64_t pos = i / 3;
    if constexpr (!B3) {
        const int64_t blk = (int64_t)WAVE * R;
        pos = (i / blk) * blk + (i % WAVE) * R + (i % blk) / WAVE;
    }
    for (int32_t k = rp[i] + (int32_t)(g % LANES); k < rp[i + 1]; k += LANES) {
        const int64_t c = ci[k];
        const int d = B3 ? (int)(c / 3 - i / 3) : (int)(c - i);
        int lo = 0, hi = o.nd - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (soff[mid] < d) lo = mid + 1;
            else hi = mid;
        }
        if (soff[lo] == d)
            val[(int64_t)(B3 ? 9 * lo + 3 * (int)(i - 3 * (i / 3)) + (int)(c - 3 * (c / 3)) : lo) * stride + pos] = va[k];
    }
}

// Distinct node offsets c/3 - r/3, ascending (host copy of the pattern);
// false unless n is a multiple of 3, there are at most DIA_MAX of them and
// the blocks store at most 1.5x the entries.
static bool b3A_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st)
{
    *st = GS2_OK;
    offs.clear();
    const int64_t n = A.n;
    if (n % 3 != 0) return false;
    std::vector<int32_t> rp(n + 1), ci(std::max<int64_t>(A.nnz, 1));
    if (hipMemcpyAsync(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        (A.nnz && hipMemcpyAsync(ci.data(), A.colind, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, s) !=
                      hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
        *st = GS2_ERR_HIP;
        return false;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = (int)((int64_t)ci[k] / 3 - i / 3);
            auto it = std::lower_bound(offs.begin(), offs.end(), d);
            if (it == offs.end() || *it != d) {
                if ((int)offs.size() == DIA_MAX) return false;
                offs.insert(it, d);
            }
        }
    return 3.0 * (double)offs.size() * (double)n <= 1.5 * (double)A.nnz + 3.0 * (double)KRB * offs.size();
}

// Distinct offsets col - row of the whole pattern, ascending (host copy of
// the pattern); false when there are more than DIA_MAX or the diagonals
// would store more than 1.5x the entries.
static bool diaA_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st)
{
    *st = GS2_OK;
    offs.clear();
    const int64_t n = A.n;
    std::vector<int32_t> rp(n + 1), ci(std::max<int64_t>(A.nnz, 1));
    if (hipMemcpyAsync(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        (A.nnz && hipMemcpyAsync(ci.data(), A.colind, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, s) !=
                      hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
        *st = GS2_ERR_HIP;
        return false;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = (int)((int64_t)ci[k] - i);
            auto it = std::lower_bound(offs.begin(), offs.end(), d);
            if (it == offs.end() || *it != d) {
                if ((int)offs.size() == DIA_MAX) return false;
                offs.insert(it, d);
            }
        }
    return (double)offs.size() * (double)n <= 1.5 * (double)A.nnz + (double)KRB * offs.size();
}

int sella_build_dia(SellA &S, const gs2_csr &A, int R, const std::vector<int> &offs, hipStream_t s)
{
    sella_free(S);
    S.n = A.n;
    S.nnz = A.nnz;
    S.dR = R;
    S.ndiag = (int)offs.size();
    S.dstride = std::max<int64_t>(1, (A.n + KRB - 1) / KRB) * KRB;
    for (int d = 0; d < DIA_MAX; ++d) S.doff[d] = d < S.ndiag ? offs[d] : 0;
    const size_t bytes = sizeof(double) * (size_t)std::max(S.ndiag, 1) * (size_t)S.dstride;
    GS2_TRY_HIP(hipMalloc(&S.dval, bytes));
    GS2_TRY_HIP(hipMemsetAsync(S.dval, 0, bytes, s));
    S.sel = -R;
    return GS2_OK;
}

int sella_build_b3(SellA &S, const gs2_csr &A, int R, const std::vector<int> &offs, hipStream_t s)
{
    sella_free(S);
    S.n = A.n;
    S.nnz = A.nnz;
    S.dR = R;
    S.ndiag = (int)offs.size();
    S.dstride = std::max<int64_t>(1, (A.n / 3 + KRB - 1) / KRB) * KRB; // nodes
    for (int d = 0; d < DIA_MAX; ++d) S.doff[d] = d < S.ndiag ? offs[d] : 0;
    const size_t bytes = sizeof(double) * 9 * (size_t)std::max(S.ndiag, 1) * (size_t)S.dstride;
    GS2_TRY_HIP(hipMalloc(&S.dval, bytes));
    GS2_TRY_HIP(hipMemsetAsync(S.dval, 0, bytes, s));
    S.sel = -10 - R;
    return GS2_OK;
}

// copy A's values into the built layout
int sella_fill_values(SellA &S, const gs2_csr &A, bool with_col, hipStream_t s)
{
    const int tb = 256;
    if (S.sel <= -10) {
        if (A.n > 0) {
            DiaOffsA o;
            o.nd = S.ndiag;
            for (int d = 0; d < DIA_MAX; ++d) o.off[d] = S.doff[d];
            constexpr int LN = 32; // 81 entries per row for 27-point 3-dof stencils
            k_copy_fill<LN, true><<<(unsigned)((A.n * LN + tb - 1) / tb), tb, 0, s>>>(A.n, 1, A.rowptr, A.colind,
                                                                                      A.val, o, S.dstride, S.dval);
        }
    } else if (S.sel < 0) {
        if (A.n > 0) {
            DiaOffsA o;
            o.nd = S.ndiag;
            for (int d = 0; d < DIA_MAX; ++d) o.off[d] = S.doff[d];
            constexpr int LN = 8; // 7-point stencils: one entry per lane
            k_copy_fill<LN, false><<<(unsigned)((A.n * LN + tb - 1) / tb), tb, 0, s>>>(A.n, S.dR, A.rowptr, A.colind,
                                                                                       A.val, o, S.dstride, S.dval);
        }
    } else if (S.nslices > 0) {
        const int64_t threads = S.nslices * WAVE;
        k_sella_fill<<<(unsigned)((threads + tb - 1) / tb), tb, 0, s>>>(A.n, S.nslices, S.K, A.rowptr, A.colind,
                                                                       A.val, S.sp, with_col ? 1 : 0, S.col, S.val);
    }
    GS2_TRY_HIP(hipGetLastError());
    return GS2_OK;
}

// Lanes per row: from K0 (the rule: the mean row length, as for the
// triangles), K grows while a few long rows would pad the copy beyond twice
// the entries.
static int sella_structure(SellA &S, const gs2_csr &A, int K0, int64_t *len, hipStream_t s)
{
    const int tb = 256;
    for (int K = K0;; K *= 2) {
        S.K = K;
        S.C = WAVE / K;
        S.nslices = (A.n + S.C - 1) / S.C;
        k_sella_len<<<(unsigned)((S.nslices + 1 + tb - 1) / tb), tb, 0, s>>>(A.n, S.nslices, K, A.rowptr, len);
        GS2_TRY(exclusive_scan_i64(len, S.sp, S.nslices + 1, s));
        GS2_TRY_HIP(hipMemcpyAsync(&S.padded, S.sp + S.nslices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        if (K == WAVE || S.padded <= 2 * A.nnz + WAVE * S.nslices) break;
    }
    const int64_t alloc = std::max<int64_t>(S.padded, WAVE);
    GS2_TRY_HIP(hipMalloc(&S.col, sizeof(int32_t) * alloc));
    GS2_TRY_HIP(hipMalloc(&S.val, sizeof(double) * alloc));
    return GS2_OK;
}

int sella_rule_lanes(const gs2_csr &A) { return choose_lanes((double)A.nnz / (double)std::max<int64_t>(A.n, 1), 0); }

// Sliced-ELL structure with at least K0 lanes per row (columns and values
// filled), replacing whatever S held.
int sella_build_sell(SellA &S, const gs2_csr &A, int K0, hipStream_t s)
{
    sella_free(S);
    S.n = A.n;
    S.nnz = A.nnz;
    int64_t *len = nullptr;
    int st = GS2_OK;
    const int64_t max_slices = A.n; // K = 64: one row per slice
    if (hipMalloc(&S.sp, sizeof(int64_t) * (max_slices + 1)) != hipSuccess ||
        hipMalloc(&len, sizeof(int64_t) * (max_slices + 1)) != hipSuccess)
        st = GS2_ERR_NOMEM;
    if (st == GS2_OK) st = sella_structure(S, A, K0, len, s);
    if (len) (void)hipFree(len);
    if (st == GS2_OK) {
        S.sel = S.K;
        st = sella_fill_values(S, A, true, s);
    }
    if (st != GS2_OK) sella_free(S);
    return st;
}

bool sella_dia_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st)
{
    return A.n > 0 && A.n <= (int64_t(1) << 30) && diaA_offsets(A, offs, s, st);
}

bool sella_b3_offsets(const gs2_csr &A, std::vector<int> &offs, hipStream_t s, int *st)
{
    return A.n > 0 && A.n <= (int64_t(1) << 30) && b3A_offsets(A, offs, s, st);
}

} // namespace gs2

