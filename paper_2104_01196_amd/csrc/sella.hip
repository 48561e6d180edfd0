// Sliced-ELL copy of the system matrix for the Krylov solvers' SpMV.
#include <hipcub/hipcub.hpp>

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
    for (void *p : {(void *)S.sp, (void *)S.col, (void *)S.val})
        if (p) (void)hipFree(p);
    S = SellA{};
}

// Lanes per row: the mean row length picks K (as for the triangles), and K
// grows while a few long rows would pad the copy beyond twice the entries.
static int sella_structure(SellA &S, const gs2_csr &A, int64_t *len, void *tmp, size_t tmp_bytes, hipStream_t s)
{
    const int tb = 256;
    for (int K = choose_lanes((double)A.nnz / (double)std::max<int64_t>(A.n, 1), 0);; K *= 2) {
        S.K = K;
        S.C = WAVE / K;
        S.nslices = (A.n + S.C - 1) / S.C;
        k_sella_len<<<(unsigned)((S.nslices + 1 + tb - 1) / tb), tb, 0, s>>>(A.n, S.nslices, K, A.rowptr, len);
        GS2_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, len, S.sp, (int)(S.nslices + 1), s));
        GS2_TRY_HIP(hipMemcpyAsync(&S.padded, S.sp + S.nslices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        if (K == WAVE || S.padded <= 2 * A.nnz + WAVE * S.nslices) break;
    }
    const int64_t alloc = std::max<int64_t>(S.padded, WAVE);
    GS2_TRY_HIP(hipMalloc(&S.col, sizeof(int32_t) * alloc));
    GS2_TRY_HIP(hipMalloc(&S.val, sizeof(double) * alloc));
    return GS2_OK;
}

int sella_prepare(SellA &S, const gs2_csr &A, hipStream_t s)
{
    const bool same = S.val && S.rp == A.rowptr && S.ci == A.colind && S.n == A.n && S.nnz == A.nnz;
    if (!same) {
        sella_free(S);
        S.n = A.n;
        S.nnz = A.nnz;
        int64_t *len = nullptr;
        void *tmp = nullptr;
        size_t tmp_bytes = 0;
        int st = GS2_OK;
        const int64_t max_slices = A.n; // K = 64: one row per slice
        if (hipMalloc(&S.sp, sizeof(int64_t) * (max_slices + 1)) != hipSuccess ||
            hipMalloc(&len, sizeof(int64_t) * (max_slices + 1)) != hipSuccess ||
            hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, len, S.sp, (int)(max_slices + 1), s) != hipSuccess ||
            hipMalloc(&tmp, tmp_bytes + 16) != hipSuccess)
            st = GS2_ERR_NOMEM;
        if (st == GS2_OK) st = sella_structure(S, A, len, tmp, tmp_bytes, s);
        if (tmp) (void)hipFree(tmp);
        if (len) (void)hipFree(len);
        if (st != GS2_OK) {
            sella_free(S);
            return st;
        }
        S.rp = A.rowptr; // the structure is complete: key it
        S.ci = A.colind;
    }
    if (S.nslices > 0) {
        const int tb = 256;
        const int64_t threads = S.nslices * WAVE;
        k_sella_fill<<<(unsigned)((threads + tb - 1) / tb), tb, 0, s>>>(A.n, S.nslices, S.K, A.rowptr, A.colind,
                                                                       A.val, S.sp, same ? 0 : 1, S.col, S.val);
        GS2_TRY_HIP(hipGetLastError());
    }
    return GS2_OK;
}

} // namespace gs2
