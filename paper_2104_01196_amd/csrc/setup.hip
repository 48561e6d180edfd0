// GS2 setup (Sections 3 and 6): validate the CSR input, extract D, build the
// scaling vectors, split the scaled matrix into its strictly lower and upper
// triangles in sliced-ELL layout and the requested precision, optionally
// build level sets, and pick a lane-per-row schedule.  The paper notes that
// GS2 needs no eigenvalue estimate and only this cheap setup (Section 12).

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>

#include "gs2_internal.hpp"

namespace gs2 {

enum : int { ERRF_BAD_CSR = 1, ERRF_ZERO_DIAG = 2, ERRF_NONFINITE = 4, ERRF_FP16 = 8 };

static int flags_to_status(int f)
{
    if (f & ERRF_BAD_CSR) return GS2_ERR_BAD_CSR;
    if (f & ERRF_ZERO_DIAG) return GS2_ERR_ZERO_DIAG;
    if (f & ERRF_NONFINITE) return GS2_ERR_NONFINITE;
    if (f & ERRF_FP16) return GS2_ERR_FP16_RANGE;
    return GS2_OK;
}

// One thread per row: structural checks, triangle counts, diagonal.
__global__ void k_validate(int64_t n, int64_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ va, int32_t *__restrict__ lcnt, int32_t *__restrict__ ucnt,
                           double *__restrict__ d, int *__restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(err, ERRF_BAD_CSR);
    if (i >= n) return;
    const int64_t b = rp[i], e = rp[i + 1];
    if (b < 0 || e < b || e > nnz) {
        atomicOr(err, ERRF_BAD_CSR);
        return;
    }
    int prev = -1, nl = 0, nu = 0, found = 0, f = 0;
    double dv = 0.0;
    for (int64_t k = b; k < e; ++k) {
        const int c = ci[k];
        if (c <= prev || c >= n) f |= ERRF_BAD_CSR;
        prev = c;
        const double v = va[k];
        if (!isfinite(v)) f |= ERRF_NONFINITE;
        if (c < i) ++nl;
        else if (c == i) { found = 1; dv = v; }
        else ++nu;
    }
    if (!found || dv == 0.0) f |= ERRF_ZERO_DIAG;
    if (f) atomicOr(err, f);
    lcnt[i] = nl;
    ucnt[i] = nu;
    d[i] = dv;
}

__global__ void k_scaling(int64_t n, const double *__restrict__ d, double *__restrict__ sl, double *__restrict__ sr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = 1.0 / sqrt(fabs(d[i]));
    sr[i] = s;
    sl[i] = d[i] < 0.0 ? -s : s;
}

// Stored entries of each slice: 64 * ceil(longest row / K).  The extra
// element at index nslices is zero so that an exclusive scan yields the end.
__global__ void k_slice_len(int64_t n, int64_t nslices, int K, const int32_t *__restrict__ cnt,
                            int64_t *__restrict__ len)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nslices) return;
    if (s == nslices) { len[s] = 0; return; }
    const int C = WAVE / K;
    int m = 0;
    for (int r = 0; r < C; ++r) {
        const int64_t row = s * C + r;
        if (row < n) m = max(m, cnt[row]);
    }
    len[s] = (int64_t)WAVE * ((m + K - 1) / K);
}

// IEEE binary16 round-to-nearest-even of a float64, by integer manipulation of
// the binary64 encoding.  Returns the 16-bit pattern; sets *ovf if the
// result is infinite or NaN.
__device__ __forceinline__ uint16_t f64_to_f16_bits(double x, int *ovf)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const int ex = (int)((b >> 52) & 0x7ff);
    const uint64_t man = b & ((1ull << 52) - 1);
    if (ex == 0x7ff) { *ovf = 1; return sign | 0x7e00u; }
    if (ex == 0) return sign; // binary64 zero / subnormal: far below half's range
    const int e = ex - 1023;
    if (e > 15) { *ovf = 1; return sign | 0x7c00u; }
    const int E = e < -14 ? -14 : e;
    const int shift = 42 + (E - e); // bits of the 53-bit significand below half's quantum
    if (shift >= 54) return sign;
    const uint64_t m = man | (1ull << 52);
    uint64_t N = m >> shift;
    const uint64_t rem = m & ((1ull << shift) - 1), halfq = 1ull << (shift - 1);
    if (rem > halfq || (rem == halfq && (N & 1))) ++N;
    const uint32_t bits = ((uint32_t)(E + 14) << 10) + (uint32_t)N;
    if (bits >= 0x7c00u) { *ovf = 1; return sign | 0x7c00u; }
    return sign | (uint16_t)bits;
}

template <typename VT>
__device__ __forceinline__ VT convert_scaled(double v, int *ovf);
template <>
__device__ __forceinline__ double convert_scaled<double>(double v, int *) { return v; }
template <>
__device__ __forceinline__ float convert_scaled<float>(double v, int *ovf)
{
    const float f = (float)v;
    if (!isfinite(f)) *ovf = 1;
    return f;
}
template <>
__device__ __forceinline__ _Float16 convert_scaled<_Float16>(double v, int *ovf)
{
    const uint16_t bits = f64_to_f16_bits(v, ovf);
    _Float16 h;
    __builtin_memcpy(&h, &bits, 2);
    return h;
}

// Which entries of a row a stored part holds, as up to two ranges of the
// row's sorted CSR entries.  Parts: 0 = strictly lower inside the row's
// block, 1 = strictly upper inside the block, 2 = outside the block (the
// couplings of the hybrid relaxation).  Blocks are contiguous ranges of bs
// rows; with one block (bs >= n) part 2 is empty.  Sorted columns put the
// off-block lower entries first and the off-block upper entries last.
enum : int { PART_L = 0, PART_U = 1, PART_E = 2 };

struct Ranges {
    int32_t *off1 = nullptr, *cnt1 = nullptr, *off2 = nullptr, *cnt2 = nullptr, *tot = nullptr;
};

__global__ void k_ranges(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const int32_t *__restrict__ lcnt, const int32_t *__restrict__ ucnt, int64_t bs, int part,
                         Ranges R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t b0 = (i / bs) * bs, b1 = b0 + bs < n ? b0 + bs : n;
    const int lc = lcnt[i], uc = ucnt[i];
    const int64_t r = rp[i];
    int lo = 0, hi = 0;
    while (lo < lc && ci[r + lo] < b0) ++lo;
    while (hi < uc && ci[r + lc + uc - hi] >= b1) ++hi;
    int o1 = 0, c1 = 0, o2 = 0, c2 = 0;
    if (part == PART_L) {
        o1 = lo;
        c1 = lc - lo;
    } else if (part == PART_U) {
        o1 = lc + 1;
        c1 = uc - hi;
    } else {
        o1 = 0;
        c1 = lo;
        o2 = lc + 1 + uc - hi;
        c2 = hi;
    }
    R.off1[i] = o1;
    R.cnt1[i] = c1;
    R.off2[i] = o2;
    R.cnt2[i] = c2;
    R.tot[i] = c1 + c2;
}

// One thread per (slice, lane): writes the lane's entries of its row, the
// value (s_l[i] * a_ij) * s_r[j] rounded once to VT, padding with
// (own column, 0).
template <typename VT>
__global__ void k_fill(int64_t n, int64_t nslices, int K, const int32_t *__restrict__ rp,
                       const int32_t *__restrict__ ci, const double *__restrict__ va, Ranges R,
                       const double *__restrict__ sl, const double *__restrict__ sr,
                       const int64_t *__restrict__ sp, int32_t *__restrict__ col, VT *__restrict__ val,
                       int *__restrict__ err)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = gid / WAVE;
    if (s >= nslices) return;
    const int l = (int)(gid % WAVE);
    const int C = WAVE / K;
    const int r = l / K, q = l % K;
    const int64_t row = s * C + r;
    const int64_t beg = sp[s];
    const int steps = (int)((sp[s + 1] - beg) / WAVE);
    const int c_row = row < n ? R.tot[row] : 0;
    const int c1 = row < n ? R.cnt1[row] : 0;
    const int64_t base = row < n ? (int64_t)rp[row] : 0;
    const int o1 = row < n ? R.off1[row] : 0, o2 = row < n ? R.off2[row] : 0;
    const int32_t pad_col = (int32_t)(row < n ? row : n - 1);
    const double srow = row < n ? sl[row] : 0.0;
    int ovf = 0;
    for (int t = 0; t < steps; ++t) {
        const int e = t * K + q;
        const int64_t pos = beg + (int64_t)t * WAVE + l;
        if (e < c_row) {
            const int64_t idx = base + (e < c1 ? o1 + e : o2 + (e - c1));
            const int32_t c = ci[idx];
            const double sc = (srow * va[idx]) * sr[c];
            col[pos] = c;
            val[pos] = convert_scaled<VT>(sc, &ovf);
        } else {
            col[pos] = pad_col;
            val[pos] = VT(0);
        }
    }
    if (ovf) atomicOr(err, ERRF_FP16);
}

void free_sell(Sell &S)
{
    if (S.slice_ptr) (void)hipFree(S.slice_ptr);
    if (S.col) (void)hipFree(S.col);
    if (S.off) (void)hipFree(S.off);
    if (S.val) (void)hipFree(S.val);
    S.slice_ptr = nullptr;
    S.col = nullptr;
    S.off = nullptr;
    S.val = nullptr;
}

// One thread per (slice, lane): d = col - row for each of its entries.
// Pass 0 folds the smallest and largest d into mm[0], mm[1]; pass 1 writes
// d - dmin.
__global__ void k_col_offsets(int64_t nslices, int K, const int64_t *__restrict__ sp, const int32_t *__restrict__ col,
                              int pass, int dmin, uint16_t *__restrict__ off, int *__restrict__ mm)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = gid / WAVE;
    if (s >= nslices) return;
    const int l = (int)(gid % WAVE);
    const int64_t row = s * (WAVE / K) + l / K;
    const int64_t beg = sp[s];
    const int steps = (int)((sp[s + 1] - beg) / WAVE);
    int lo = 0x7fffffff, hi = -0x7fffffff;
    for (int t = 0; t < steps; ++t) {
        const int64_t pos = beg + (int64_t)t * WAVE + l;
        const int d = (int)((int64_t)col[pos] - row);
        if (pass == 0) {
            lo = d < lo ? d : lo;
            hi = d > hi ? d : hi;
        } else {
            off[pos] = (uint16_t)(d - dmin);
        }
    }
    if (pass == 0 && steps > 0) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

int build_col_offsets(int64_t nslices, int K, const int64_t *sp, const int32_t *col, int64_t padded, uint16_t **off,
                      int *off_min, hipStream_t s)
{
    *off = nullptr;
    *off_min = 0;
    if (nslices <= 0) return GS2_OK;
    int *mm = nullptr;
    GS2_TRY_HIP(hipMalloc(&mm, 2 * sizeof(int)));
    const int init[2] = {0x7fffffff, -0x7fffffff};
    int h[2] = {0, 0};
    const int tb = 256;
    const unsigned grid = (unsigned)((nslices * WAVE + tb - 1) / tb);
    int st = GS2_OK;
    // a blocking copy: init lives on this stack frame
    if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(mm, init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess)
        st = GS2_ERR_HIP;
    if (st == GS2_OK) {
        k_col_offsets<<<grid, tb, 0, s>>>(nslices, K, sp, col, 0, 0, nullptr, mm);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = GS2_ERR_HIP;
    }
    (void)hipFree(mm);
    if (st != GS2_OK) return st;
    if (h[0] > h[1] || (int64_t)h[1] - (int64_t)h[0] > 65535) return GS2_OK; // no entries, or too wide: 32 bits
    uint16_t *o = nullptr;
    GS2_TRY_HIP(hipMalloc(&o, sizeof(uint16_t) * std::max<int64_t>(padded, WAVE)));
    k_col_offsets<<<grid, tb, 0, s>>>(nslices, K, sp, col, 1, h[0], o, nullptr);
    if (hipGetLastError() != hipSuccess) {
        (void)hipFree(o);
        return GS2_ERR_HIP;
    }
    *off = o;
    *off_min = h[0];
    return GS2_OK;
}

// ------------------------------------------- diagonal-interleaved triangles

void free_dia(Dia &D)
{
    if (D.val) (void)hipFree(D.val);
    D.val = nullptr;
}

struct DiaOffs {
    int nd;
    int off[DIA_MAX];
};

// Distinct offsets col - row of the strictly lower and upper parts, ascending,
// and their entry counts, from a host copy of the pattern.  False when either
// part has more than DIA_MAX offsets.  Columns are sorted within a row, so a
// row's offsets ascend; each is looked up by binary search.
static bool dia_offsets(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int64_t n,
                        std::vector<int> &offL, std::vector<int> &offU, int64_t &nnzL, int64_t &nnzU)
{
    offL.clear();
    offU.clear();
    nnzL = nnzU = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = (int)((int64_t)ci[k] - i);
            if (d == 0) continue;
            std::vector<int> &o = d < 0 ? offL : offU;
            (d < 0 ? nnzL : nnzU)++;
            auto it = std::lower_bound(o.begin(), o.end(), d);
            if (it == o.end() || *it != d) {
                if ((int)o.size() == DIA_MAX) return false;
                o.insert(it, d);
            }
        }
    }
    return true;
}

// The same for 3-row blocks (n a multiple of 3): distinct node offsets c/3 -
// r/3 of the strictly lower entries (c < r, node offsets <= 0) and of the
// strictly upper ones (node offsets >= 0).  False when n is not a multiple
// of 3 or either part has more than DIA_MAX node offsets.
static bool b3_offsets(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int64_t n,
                       std::vector<int> &offL, std::vector<int> &offU)
{
    offL.clear();
    offU.clear();
    if (n % 3 != 0) return false;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if ((int64_t)ci[k] == i) continue;
            const int d = (int)((int64_t)ci[k] / 3 - i / 3);
            std::vector<int> &o = (int64_t)ci[k] < i ? offL : offU;
            auto it = std::lower_bound(o.begin(), o.end(), d);
            if (it == o.end() || *it != d) {
                if ((int)o.size() == DIA_MAX) return false;
                o.insert(it, d);
            }
        }
    }
    return true;
}

// One thread per row: the row's entries of one part go to their diagonal at
// the row's interleaved position, value (s_l[i] * a_ij) * s_r[j] rounded once
// to VT.  The array is zeroed beforehand (rows past n and absent entries).
template <typename VT>
__global__ void k_dia_fill(int64_t n, int R, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ va, const int32_t *__restrict__ lcnt, int lower, DiaOffs o,
                           const double *__restrict__ sl, const double *__restrict__ sr, int64_t stride,
                           VT *__restrict__ val, int *__restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t blk = (int64_t)WAVE * R;
    const int64_t pos = (i / blk) * blk + (i % WAVE) * R + (i % blk) / WAVE;
    const int64_t b = lower ? rp[i] : rp[i] + lcnt[i] + 1, e = lower ? rp[i] + lcnt[i] : rp[i + 1];
    const double srow = sl[i];
    int t = 0, ovf = 0;
    for (int64_t k = b; k < e; ++k) {
        const int c = ci[k];
        const int d = (int)((int64_t)c - i);
        while (t < o.nd - 1 && o.off[t] < d) ++t; // offsets ascend within a row
        if (o.off[t] != d) {
            atomicOr(err, ERRF_BAD_CSR); // cannot happen for a pattern the offsets came from
            return;
        }
        val[(int64_t)t * stride + pos] = convert_scaled<VT>((srow * va[k]) * sr[c], &ovf);
    }
    if (ovf) atomicOr(err, ERRF_FP16);
}

// The 3-row block layout: entry (i, c) of the part goes to plane
// 9 t + 3 (i mod 3) + (c mod 3), t the index of its node offset c/3 - i/3,
// at node i/3's interleaved position (R nodes per lane); scaled and rounded
// as in k_dia_fill.
template <typename VT>
__global__ void k_b3_fill(int64_t n, int R, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const double *__restrict__ va, const int32_t *__restrict__ lcnt, int lower, DiaOffs o,
                          const double *__restrict__ sl, const double *__restrict__ sr, int64_t stride,
                          VT *__restrict__ val, int *__restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t blk = (int64_t)WAVE * R, node = i / 3, j = i - 3 * node;
    const int64_t pos = (node / blk) * blk + (node % WAVE) * R + (node % blk) / WAVE;
    const int64_t b = lower ? rp[i] : rp[i] + lcnt[i] + 1, e = lower ? rp[i] + lcnt[i] : rp[i + 1];
    const double srow = sl[i];
    int t = 0, ovf = 0;
    for (int64_t k = b; k < e; ++k) {
        const int c = ci[k];
        const int cn = c / 3;
        const int d = (int)((int64_t)cn - node);
        while (t < o.nd - 1 && o.off[t] < d) ++t; // node offsets ascend within a row
        if (o.off[t] != d) {
            atomicOr(err, ERRF_BAD_CSR); // cannot happen for a pattern the offsets came from
            return;
        }
        val[(int64_t)(9 * t + 3 * j + (c - 3 * cn)) * stride + pos] = convert_scaled<VT>((srow * va[k]) * sr[c], &ovf);
    }
    if (ovf) atomicOr(err, ERRF_FP16);
}

// Build one triangle (lower or upper) in the diagonal-interleaved layout
// with R rows per lane, or in the 3-row block layout with R nodes per lane;
// rows (nodes) are padded to whole workgroups of the sweep kernels
// (DIA_THREADS * R of them) so that every launched lane has a slot.
static int build_dia(Dia &D, int64_t n, int precision, int lower, int R, const std::vector<int> &offs, int64_t nnz,
                     const gs2_csr &A, const int32_t *lcnt, const double *sl, const double *sr, int *err,
                     hipStream_t s, int b3 = 0)
{
    free_dia(D);
    D.ndiag = (int)offs.size();
    D.R = R;
    D.nnz = nnz;
    D.b3 = b3;
    D.val_bytes = precision == GS2_FP64 ? 8 : precision == GS2_FP32 ? 4 : 2;
    const int64_t wg = (int64_t)DIA_THREADS * R, units = b3 ? n / 3 : n;
    D.stride = std::max<int64_t>(1, (units + wg - 1) / wg) * wg;
    DiaOffs o;
    o.nd = D.ndiag;
    for (int d = 0; d < DIA_MAX; ++d) {
        D.off[d] = d < D.ndiag ? offs[d] : 0;
        o.off[d] = D.off[d];
    }
    const size_t bytes = (size_t)std::max(1, D.ndiag) * (b3 ? 9 : 1) * (size_t)D.stride * D.val_bytes;
    GS2_TRY_HIP(hipMalloc(&D.val, bytes));
    GS2_TRY_HIP(hipMemsetAsync(D.val, 0, bytes, s));
    if (D.ndiag == 0 || n == 0) return GS2_OK;
    const int tb = 256;
    const unsigned g = (unsigned)((n + tb - 1) / tb);
    if (b3) {
        if (precision == GS2_FP64)
            k_b3_fill<double><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                               (double *)D.val, err);
        else if (precision == GS2_FP32)
            k_b3_fill<float><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                              (float *)D.val, err);
        else
            k_b3_fill<_Float16><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                                 (_Float16 *)D.val, err);
    } else if (precision == GS2_FP64)
        k_dia_fill<double><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                            (double *)D.val, err);
    else if (precision == GS2_FP32)
        k_dia_fill<float><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                           (float *)D.val, err);
    else
        k_dia_fill<_Float16><<<g, tb, 0, s>>>(n, R, A.rowptr, A.colind, A.val, lcnt, lower, o, sl, sr, D.stride,
                                              (_Float16 *)D.val, err);
    GS2_TRY_HIP(hipGetLastError());
    return GS2_OK;
}

// ------------------------------------------------------- exclusive scan
//
// out[i] = sum of in[0..i), for the slice pointers of the sliced-ELL arrays.
// Three passes: each workgroup scans its 1024 elements (four per thread, the
// thread totals combined by a Hillis-Steele scan in LDS) and writes its
// total; one workgroup scans the totals in chunks of 256 with a running
// carry; every element then adds its workgroup's offset.  Integer sums, so
// the result is exact whatever the order.
constexpr int SCAN_TB = 256, SCAN_PER = 4, SCAN_BLOCK = SCAN_TB * SCAN_PER;

__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_TB; off <<= 1) {
        const int64_t x = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    return sh[t];
}

__global__ __launch_bounds__(SCAN_TB) void k_scan_local(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                        int64_t m, int64_t *__restrict__ bsum)
{
    __shared__ int64_t sh[SCAN_TB];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER;
    int64_t v[SCAN_PER], run = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        v[q] = base + q < m ? in[base + q] : 0;
        run += v[q];
    }
    const int64_t incl = block_incl_scan(run, sh);
    int64_t e = incl - run;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        if (base + q < m) out[base + q] = e;
        e += v[q];
    }
    if (threadIdx.x == SCAN_TB - 1) bsum[blockIdx.x] = incl;
}

__global__ __launch_bounds__(SCAN_TB) void k_scan_sums(int64_t *__restrict__ bsum, int64_t nb)
{
    __shared__ int64_t sh[SCAN_TB];
    int64_t carry = 0; // the same in every thread
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_TB) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        const int64_t incl = block_incl_scan(v, sh);
        if (i < nb) bsum[i] = carry + incl - v;
        carry += sh[SCAN_TB - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(SCAN_TB) void k_scan_add(int64_t *__restrict__ out, int64_t m,
                                                      const int64_t *__restrict__ bsum)
{
    const int64_t i = (int64_t)blockIdx.x * SCAN_TB + threadIdx.x;
    if (i < m) out[i] += bsum[i / SCAN_BLOCK];
}

int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t m, hipStream_t s)
{
    if (m <= 0) return GS2_OK;
    const int64_t nb = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    int64_t *bsum = nullptr;
    GS2_TRY_HIP(hipMalloc(&bsum, sizeof(int64_t) * nb));
    k_scan_local<<<(unsigned)nb, SCAN_TB, 0, s>>>(in, out, m, bsum);
    k_scan_sums<<<1, SCAN_TB, 0, s>>>(bsum, nb);
    k_scan_add<<<(unsigned)((m + SCAN_TB - 1) / SCAN_TB), SCAN_TB, 0, s>>>(out, m, bsum);
    const hipError_t e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(bsum);
    GS2_TRY_HIP(e);
    GS2_TRY_HIP(e2);
    return GS2_OK;
}

int choose_lanes(double avg_len, int max_len)
{
    (void)max_len;
    if (avg_len <= 12.0) return 1;
    if (avg_len <= 24.0) return 2;
    if (avg_len <= 48.0) return 4;
    if (avg_len <= 96.0) return 8;
    return 16;
}

static int build_one(Sell &S, int64_t n, int K, int precision, const gs2_csr &A, const Ranges &R,
                     const double *sl, const double *sr, int *err, hipStream_t s)
{
    const int32_t *cnt = R.tot;
    free_sell(S);
    S.n = n;
    S.K = K;
    S.C = WAVE / K;
    S.nslices = (n + S.C - 1) / S.C;
    S.val_bytes = precision == GS2_FP64 ? 8 : precision == GS2_FP32 ? 4 : 2;
    int64_t *len = nullptr;
    GS2_TRY_HIP(hipMalloc(&S.slice_ptr, sizeof(int64_t) * (S.nslices + 1)));
    GS2_TRY_HIP(hipMalloc(&len, sizeof(int64_t) * (S.nslices + 1)));
    const int tb = 256;
    k_slice_len<<<(unsigned)((S.nslices + 1 + tb - 1) / tb), tb, 0, s>>>(n, S.nslices, K, cnt, len);
    GS2_TRY(exclusive_scan_i64(len, S.slice_ptr, S.nslices + 1, s));
    GS2_TRY_HIP(hipMemcpyAsync(&S.padded, S.slice_ptr + S.nslices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    (void)hipFree(len);
    const int64_t alloc = std::max<int64_t>(S.padded, WAVE);
    GS2_TRY_HIP(hipMalloc(&S.col, sizeof(int32_t) * alloc));
    GS2_TRY_HIP(hipMalloc(&S.val, (size_t)S.val_bytes * alloc));
    const int64_t threads = S.nslices * WAVE;
    const unsigned grid = (unsigned)((threads + tb - 1) / tb);
    if (S.nslices > 0) {
        if (precision == GS2_FP64)
            k_fill<double><<<grid, tb, 0, s>>>(n, S.nslices, K, A.rowptr, A.colind, A.val, R, sl, sr, S.slice_ptr,
                                               S.col, (double *)S.val, err);
        else if (precision == GS2_FP32)
            k_fill<float><<<grid, tb, 0, s>>>(n, S.nslices, K, A.rowptr, A.colind, A.val, R, sl, sr, S.slice_ptr,
                                              S.col, (float *)S.val, err);
        else
            k_fill<_Float16><<<grid, tb, 0, s>>>(n, S.nslices, K, A.rowptr, A.colind, A.val, R, sl, sr, S.slice_ptr,
                                                 S.col, (_Float16 *)S.val, err);
        GS2_TRY_HIP(hipGetLastError());
        GS2_TRY(build_col_offsets(S.nslices, K, S.slice_ptr, S.col, S.padded, &S.off, &S.off_min, s));
    }
    return GS2_OK;
}

// Process-wide cache of autotuned lane counts, keyed by the size bucket,
// rounded mean row length, longest-row bucket and precision.
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_cache;

static std::string tune_key(int64_t n, double avg, int maxlen, int prec)
{
    int nb = 0;
    while ((int64_t(1) << nb) < n) ++nb;
    int mb = 0;
    while ((1 << mb) < maxlen) ++mb;
    char buf[96];
    std::snprintf(buf, sizeof buf, "n%d_a%d_m%d_p%d", nb, (int)std::lround(avg), mb, prec);
    return buf;
}

struct SetupScratch {
    int32_t *lcnt = nullptr, *ucnt = nullptr;
    double *d = nullptr;
    int *err = nullptr;
    Ranges R;
    ~SetupScratch()
    {
        for (void *p : {(void *)lcnt, (void *)ucnt, (void *)d, (void *)err, (void *)R.off1, (void *)R.cnt1,
                        (void *)R.off2, (void *)R.cnt2, (void *)R.tot})
            if (p) (void)hipFree(p);
    }
};

// Ranges of part `part` for every row, then the part itself in sliced-ELL.
static int build_part(Handle &h, Sell &S, int part, int K, const gs2_csr &A, SetupScratch &sc, hipStream_t s)
{
    const int64_t bs = h.blocks > 1 ? (h.n + h.blocks - 1) / h.blocks : std::max<int64_t>(h.n, 1);
    k_ranges<<<(unsigned)((h.n + 255) / 256), 256, 0, s>>>(h.n, A.rowptr, A.colind, sc.lcnt, sc.ucnt, bs, part, sc.R);
    GS2_TRY_HIP(hipGetLastError());
    return build_one(S, h.n, K, h.precision, A, sc.R, h.sl, h.sr, sc.err, s);
}

static int64_t count_total(const int32_t *tot, int64_t n, hipStream_t s, int *st)
{
    std::vector<int32_t> t(n);
    *st = GS2_OK;
    if (n && hipMemcpyAsync(t.data(), tot, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess) *st = GS2_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) *st = GS2_ERR_HIP;
    int64_t c = 0;
    for (int32_t v : t) c += v;
    return c;
}

// The setup's flush buffer (FLUSH_BYTES of zeros, read before each timed
// pass), held for the timing and released when the setup returns.  Without
// memory for it the passes are timed back to back.
struct FlushBuffer {
    Handle &h;
    FlushBuffer(Handle &hh, bool on, hipStream_t s) : h(hh)
    {
        h.flush = nullptr;
        if (!on) return;
        if (hipMalloc(&h.flush, FLUSH_BYTES) != hipSuccess) {
            h.flush = nullptr;
            (void)hipGetLastError();
            return;
        }
        if (hipMemsetAsync(h.flush, 0, FLUSH_BYTES, s) != hipSuccess) {
            (void)hipFree(h.flush);
            h.flush = nullptr;
            (void)hipGetLastError();
        }
    }
    ~FlushBuffer()
    {
        if (h.flush) (void)hipFree(h.flush);
        h.flush = nullptr;
    }
};

// Schedules of the diagonal layout chosen by timing, per (size bucket, mean
// row length, longest-row bucket, precision, diagonal counts).
struct DiaChoice {
    int fmt, R, lds, remap, b3;
};
static std::map<std::string, DiaChoice> g_dia_cache;

// Decide the layout of the GS2 / JR passes: keep the sliced-ELL triangles, or
// build diagonal-interleaved copies (Dia: scalar diagonals, or 3-row blocks
// along node offsets) and time them against sliced ELL.
static int choose_format(Handle &h, const gs2_csr &A, const gs2_options &o, SetupScratch &sc, hipStream_t s,
                         bool can_time, const std::string &key_base)
{
    h.fmt = FMT_SELL;
    h.lds = 0;
    h.tuned = 0;
    if (o.format == GS2_FORMAT_SELL) return GS2_OK;
    // the automatic choice is made by timing only; without it sliced ELL stays
    if (o.format == GS2_FORMAT_AUTO && !(can_time && o.autotune)) return GS2_OK;
    const int64_t n = h.n;
    const bool any = h.blocks == 1 && n > 0 && n <= (int64_t(1) << 30);
    std::vector<int> offL, offU, boffL, boffU;
    int64_t nnzL = 0, nnzU = 0;
    bool dia_ok = false, b3_ok = false;
    if (any) {
        std::vector<int32_t> rp(n + 1), ci(std::max<int64_t>(A.nnz, 1));
        GS2_TRY_HIP(hipMemcpyAsync(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
        if (A.nnz)
            GS2_TRY_HIP(hipMemcpyAsync(ci.data(), A.colind, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        if (o.format != GS2_FORMAT_BLOCK3) {
            dia_ok = dia_offsets(rp, ci, n, offL, offU, nnzL, nnzU);
            // stored diagonal entries (padding included) at most 1.5x the real ones
            dia_ok = dia_ok && (double)offL.size() * n <= 1.5 * nnzL + 64.0 * offL.size() &&
                     (double)offU.size() * n <= 1.5 * nnzU + 64.0 * offU.size();
        }
        if (!dia_ok && o.format != GS2_FORMAT_DIA) {
            nnzL = nnzU = 0; // dia_offsets may have stopped part way
            for (int64_t i = 0; i < n; ++i)
                for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                    if ((int64_t)ci[k] != i) ((int64_t)ci[k] < i ? nnzL : nnzU)++;
            b3_ok = b3_offsets(rp, ci, n, boffL, boffU) &&
                    3.0 * boffL.size() * n <= 1.5 * nnzL + 192.0 * boffL.size() &&
                    3.0 * boffU.size() * n <= 1.5 * nnzU + 192.0 * boffU.size();
        }
    }
    h.DL.ndiag = dia_ok ? (int)offL.size() : b3_ok ? (int)boffL.size() : 0;
    h.DU.ndiag = dia_ok ? (int)offU.size() : b3_ok ? (int)boffU.size() : 0;
    if (!dia_ok && !b3_ok) return o.format == GS2_FORMAT_AUTO ? GS2_OK : GS2_ERR_ARG;
    const int b3 = dia_ok ? 0 : 1; // the one diagonal kind this pattern admits
    const int vb = h.precision == GS2_FP64 ? 8 : h.precision == GS2_FP32 ? 4 : 2;
    std::vector<int> Rs, ldss;
    for (int R = 1; R <= 8; R *= 2)
        if (R * vb >= 2 && R * vb <= 16 && (o.rows_per_lane == 0 || o.rows_per_lane == R)) Rs.push_back(R);
    if (Rs.empty()) return GS2_ERR_ARG; // a forced rows-per-lane whose load is not 2..16 bytes
    // the block passes try the widest load first: a narrower one must then win
    // by the margin below (the float64 elasticity passes at two nodes per lane
    // ran 10 % faster in the solve than at one, while the timed pair of passes
    // often put the two within the margin)
    if (b3) std::reverse(Rs.begin(), Rs.end());
    if (b3) ldss = {0}; // block passes read their source directly
    else if (o.lds_staging == 0) ldss = {0, 1};
    else ldss = {o.lds_staging == 2 ? 1 : 0};
    std::vector<int> rms;
    if (o.xcd_ranges == 0) rms = {1, 0};
    else rms = {o.xcd_ranges == 2 ? 1 : 0};
    auto build = [&](int R) -> int {
        GS2_TRY(build_dia(h.DL, n, h.precision, 1, R, b3 ? boffL : offL, nnzL, A, sc.lcnt, h.sl, h.sr, sc.err, s, b3));
        GS2_TRY(build_dia(h.DU, n, h.precision, 0, R, b3 ? boffU : offU, nnzU, A, sc.lcnt, h.sl, h.sr, sc.err, s, b3));
        h.DL.nt = h.DU.nt = h.DL.stored_bytes() + h.DU.stored_bytes() > NT_TRIANGLES_BYTES ? 1 : 0;
        return GS2_OK;
    };
    const bool timed = can_time && o.autotune &&
                       (o.format == GS2_FORMAT_AUTO || Rs.size() > 1 || ldss.size() > 1 || rms.size() > 1);
    if (!timed) {
        if (o.format == GS2_FORMAT_AUTO) return GS2_OK; // untimed automatic choice: sliced ELL
        GS2_TRY(build(*std::max_element(Rs.begin(), Rs.end()))); // forced: the widest load allowed
        h.fmt = FMT_DIA;
        h.lds = ldss.back();
        h.remap = rms.front();
        return GS2_OK;
    }
    char kb[56];
    std::snprintf(kb, sizeof kb, "_d%d_%d_b%d_f%d_r%d_s%d_x%d", h.DL.ndiag, h.DU.ndiag, b3, o.format, o.rows_per_lane,
                  o.lds_staging, o.xcd_ranges);
    const std::string key = key_base + kb;
    DiaChoice ch{FMT_SELL, 0, 0, 1, 0};
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_dia_cache.find(key);
        if (it != g_dia_cache.end()) {
            ch = it->second;
            cached = true;
        }
    }
    if (!cached) {
        float best = 1e30f;
        if (o.format == GS2_FORMAT_AUTO) {
            h.fmt = FMT_SELL;
            GS2_TRY(time_inner_pass(h, s, &best, true));
        }
        for (int R : Rs) {
            GS2_TRY(build(R));
            for (int l : ldss)
                for (int rm : rms) { // workgroups walked per XCD, or in dispatch order
                    h.fmt = FMT_DIA;
                    h.lds = l;
                    h.remap = rm;
                    float ms = 0.f;
                    GS2_TRY(time_inner_pass(h, s, &ms, true));
                    // a new candidate must win by more than the timing noise
                    if (ms < 0.97f * best) {
                        best = ms;
                        ch = DiaChoice{FMT_DIA, R, l, rm, b3};
                    }
                }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_dia_cache[key] = ch;
    }
    h.tuned = 1;
    if (ch.fmt == FMT_SELL) {
        h.fmt = FMT_SELL;
        h.lds = 0;
        free_dia(h.DL);
        free_dia(h.DU);
        return GS2_OK;
    }
    if (!h.DL.val || h.DL.R != ch.R) GS2_TRY(build(ch.R));
    h.fmt = FMT_DIA;
    h.lds = ch.lds;
    h.remap = ch.remap;
    return GS2_OK;
}

static int read_err(int *err, hipStream_t s)
{
    int f = 0;
    GS2_TRY_HIP(hipMemcpyAsync(&f, err, sizeof(int), hipMemcpyDeviceToHost, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    return flags_to_status(f);
}

// Level sets of the DAGs of L (ascending) and U (descending), computed on the
// host from a copy of the pattern: level_i = 1 + max level over the
// triangle's entries of row i.  Rows are then grouped level by level.
// Multicolor ordering (Section 6, multi-threaded Gauss-Seidel): greedy first
// fit in natural row order on the symmetrised pattern; a row takes the
// smallest color not held by an earlier row it is coupled to (a_ij or a_ji
// nonzero).  Rows are then grouped color by color.
static int build_colors(Handle &h, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, hipStream_t s)
{
    const int64_t n = h.n;
    // transpose pattern (column -> rows), to see couplings a_ji from earlier rows j
    std::vector<int32_t> tp(n + 1, 0), tc(std::max<size_t>(ci.size(), 1));
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) tp[ci[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) tc[fill[ci[k]]++] = (int32_t)i;
    std::vector<int32_t> color(n), seen(n + 2, -1);
    int ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] < i) seen[color[ci[k]]] = (int32_t)i;
        for (int32_t k = tp[i]; k < tp[i + 1]; ++k)
            if (tc[k] < i) seen[color[tc[k]]] = (int32_t)i;
        int c = 0;
        while (seen[c] == i) ++c;
        color[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    std::vector<int64_t> ptr(ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[color[i] + 1]++;
    for (int c = 0; c < ncol; ++c) ptr[c + 1] += ptr[c];
    std::vector<int32_t> rows(std::max<int64_t>(n, 1));
    std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[pos[color[i]]++] = (int32_t)i;
    GS2_TRY_HIP(hipMalloc(&h.color_rows, sizeof(int32_t) * rows.size()));
    GS2_TRY_HIP(hipMemcpyAsync(h.color_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    h.ncolors = ncol;
    h.color_ptr = std::move(ptr);
    return GS2_OK;
}

static int build_levels(Handle &h, const gs2_csr &A, hipStream_t s)
{
    const int64_t n = A.n;
    std::vector<int32_t> rp(n + 1), ci(A.nnz);
    GS2_TRY_HIP(hipMemcpyAsync(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
    if (A.nnz) GS2_TRY_HIP(hipMemcpyAsync(ci.data(), A.colind, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> lev(n);
    for (int lower = 1; lower >= 0; --lower) {
        int nlev = 0;
        for (int64_t q = 0; q < n; ++q) {
            const int64_t i = lower ? q : n - 1 - q;
            int lv = 0;
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t c = ci[k];
                if (lower ? c < i : c > i) lv = std::max(lv, lev[c] + 1);
            }
            lev[i] = lv;
            nlev = std::max(nlev, lv + 1);
        }
        std::vector<int64_t> ptr(nlev + 1, 0);
        for (int64_t i = 0; i < n; ++i) ptr[lev[i] + 1]++;
        for (int l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
        std::vector<int32_t> rows(std::max<int64_t>(n, 1));
        std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < n; ++i) rows[pos[lev[i]]++] = (int32_t)i;
        int32_t *&d_rows = lower ? h.lev_rows_l : h.lev_rows_u; // owned by the handle from here on
        GS2_TRY_HIP(hipMalloc(&d_rows, sizeof(int32_t) * rows.size()));
        GS2_TRY_HIP(hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        if (lower) {
            h.nlev_l = nlev;
            h.lev_ptr_l = std::move(ptr);
        } else {
            h.nlev_u = nlev;
            h.lev_ptr_u = std::move(ptr);
        }
    }
    return build_colors(h, rp, ci, s);
}

static int alloc_vectors(Handle &h)
{
    const size_t vb = prec_bytes(h.precision) * (size_t)std::max<int64_t>(h.n, 1);
    GS2_TRY_HIP(hipMalloc(&h.xh, vb));
    GS2_TRY_HIP(hipMalloc(&h.xh2, vb));
    GS2_TRY_HIP(hipMalloc(&h.rh, vb));
    GS2_TRY_HIP(hipMalloc(&h.ga, vb));
    GS2_TRY_HIP(hipMalloc(&h.gb, vb));
    if (h.precision != GS2_FP64) GS2_TRY_HIP(hipMalloc(&h.sv, vb));
    return GS2_OK;
}

int setup_handle(Handle &h, const gs2_csr &A, const gs2_options &o, hipStream_t s, bool alloc_vecs)
{
    const int64_t n = A.n;
    if (n == 0) return GS2_OK;
    SetupScratch sc;
    const size_t nb = (size_t)std::max<int64_t>(n, 1);
    GS2_TRY_HIP(hipMalloc(&sc.lcnt, sizeof(int32_t) * nb));
    GS2_TRY_HIP(hipMalloc(&sc.ucnt, sizeof(int32_t) * nb));
    GS2_TRY_HIP(hipMalloc(&sc.d, sizeof(double) * nb));
    GS2_TRY_HIP(hipMalloc(&sc.err, sizeof(int)));
    for (int32_t **p : {&sc.R.off1, &sc.R.cnt1, &sc.R.off2, &sc.R.cnt2, &sc.R.tot})
        GS2_TRY_HIP(hipMalloc(p, sizeof(int32_t) * nb));
    GS2_TRY_HIP(hipMalloc(&h.sl, sizeof(double) * nb));
    GS2_TRY_HIP(hipMalloc(&h.sr, sizeof(double) * nb));
    GS2_TRY_HIP(hipMemsetAsync(sc.err, 0, sizeof(int), s));
    const int tb = 256;
    const unsigned g = (unsigned)((n + tb) / tb);
    k_validate<<<g, tb, 0, s>>>(n, A.nnz, A.rowptr, A.colind, A.val, sc.lcnt, sc.ucnt, sc.d, sc.err);
    GS2_TRY_HIP(hipGetLastError());
    GS2_TRY(read_err(sc.err, s));
    k_scaling<<<g, tb, 0, s>>>(n, sc.d, h.sl, h.sr);
    GS2_TRY_HIP(hipGetLastError());

    // row-length statistics of L (U has the same count for symmetric patterns)
    const double avg = n ? (double)(A.nnz - n) / (2.0 * n) : 0.0;
    int maxlen = 0;
    {
        std::vector<int32_t> rp(n + 1);
        GS2_TRY_HIP(hipMemcpyAsync(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i) maxlen = std::max(maxlen, rp[i + 1] - rp[i] - 1);
    }
    if (alloc_vecs) GS2_TRY(alloc_vectors(h));

    int K = o.lanes_per_row;
    if (K != 0 && (K < 1 || K > 64 || (K & (K - 1)))) return GS2_ERR_ARG;
    // the schedule timing below reads the flush buffer before each timed pass
    FlushBuffer flush(h, o.autotune && alloc_vecs && n >= 4096, s);
    if (K == 0) {
        K = choose_lanes(avg, maxlen);
        if (o.autotune && alloc_vecs && n >= 4096) {
            const std::string key = tune_key(n, avg, maxlen, h.precision);
            int cached = 0;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                auto it = g_tune_cache.find(key);
                if (it != g_tune_cache.end()) cached = it->second;
            }
            if (cached) {
                K = cached;
            } else {
                float best = 1e30f;
                int bestK = K;
                // each candidate is timed on one inner pass over L and one residual pass
                // over L and U, with the cache policy its stored size implies
                for (int cand = 1; cand <= 16; cand *= 2) {
                    if (cand > 1 && cand > 2 * std::max(1.0, avg)) break;
                    GS2_TRY(build_part(h, h.L, PART_L, cand, A, sc, s));
                    GS2_TRY(build_part(h, h.U, PART_U, cand, A, sc, s));
                    h.L.nt = h.U.nt = h.L.stored_bytes() + h.U.stored_bytes() > NT_TRIANGLES_BYTES ? 1 : 0;
                    float ms = 0.f;
                    GS2_TRY(time_inner_pass(h, s, &ms, true));
                    // a wider candidate must win by more than the timing noise
                    if (ms < 0.97f * best) { best = ms; bestK = cand; }
                }
                K = bestK;
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune_cache[key] = K;
            }
        }
    }
    int cst = GS2_OK;
    GS2_TRY(build_part(h, h.L, PART_L, K, A, sc, s));
    h.L.nnz = count_total(sc.R.tot, n, s, &cst);
    GS2_TRY(cst);
    GS2_TRY(build_part(h, h.U, PART_U, K, A, sc, s));
    h.U.nnz = count_total(sc.R.tot, n, s, &cst);
    GS2_TRY(cst);
    h.L.nt = h.U.nt = h.L.stored_bytes() + h.U.stored_bytes() > NT_TRIANGLES_BYTES ? 1 : 0;
    GS2_TRY(choose_format(h, A, o, sc, s, alloc_vecs && n >= 4096, tune_key(n, avg, maxlen, h.precision)));
    if (h.blocks > 1) {
        GS2_TRY(build_part(h, h.E, PART_E, K, A, sc, s));
        h.E.nnz = count_total(sc.R.tot, n, s, &cst);
        GS2_TRY(cst);
        if (alloc_vecs) GS2_TRY_HIP(hipMalloc(&h.yh, prec_bytes(h.precision) * nb));
    }
    GS2_TRY(read_err(sc.err, s));
    if (o.build_levels) GS2_TRY(build_levels(h, A, s));
    GS2_TRY_HIP(hipStreamSynchronize(s));
    return GS2_OK;
}

} // namespace gs2

using namespace gs2;

Handle::~Handle()
{
    free_sell(L);
    free_sell(U);
    free_sell(E);
    free_dia(DL);
    free_dia(DU);
    for (void *p : {(void *)sl, (void *)sr, xh, xh2, rh, ga, gb, sv, yh, (void *)lev_rows_l, (void *)lev_rows_u,
                    (void *)color_rows})
        if (p) (void)hipFree(p);
    if (gw) free_gmres_work(gw);
    if (cw) free_cg_work(cw);
}

extern "C" {

void gs2_default_options(gs2_options *opt)
{
    if (!opt) return;
    opt->precision = GS2_FP64;
    opt->inner_damping = 1.0;
    opt->compact = 0;
    opt->build_levels = 0;
    opt->autotune = 1;
    opt->lanes_per_row = 0;
    opt->rhs_per_item = 0;
    opt->orthogonalization = 0;
    opt->blocks = 1;
    opt->local_sweeps = 1;
    opt->team_rows = 0;
    opt->team_wait_ms = 0;
    opt->format = GS2_FORMAT_AUTO;
    opt->rows_per_lane = 0;
    opt->lds_staging = 0;
    opt->stagnation_cycles = 0;
    opt->spmv_format = GS2_FORMAT_AUTO;
    opt->basis_loads = 0;
    opt->xcd_ranges = 0;
}

int gs2_setup(const gs2_csr *A, int sweeps, int inner, double damping, int variant, const gs2_options *opt,
              void *stream, gs2_handle **out)
{
    if (!out) return GS2_ERR_ARG;
    *out = nullptr;
    if (!A || A->n < 0 || A->n >= (int64_t(1) << 31) - 1 || A->nnz < A->n || A->nnz >= (int64_t(1) << 31) - 1)
        return GS2_ERR_ARG;
    if ((A->n > 0) && (!A->rowptr || !A->colind || !A->val)) return GS2_ERR_ARG;
    if (sweeps < 1 || inner < 0 || variant < GS2_FORWARD || variant > GS2_SYMMETRIC) return GS2_ERR_ARG;
    if (!(damping > 0.0 && damping < 2.0)) return GS2_ERR_ARG;
    gs2_options o;
    gs2_default_options(&o);
    if (opt) o = *opt;
    if (o.precision < GS2_FP64 || o.precision > GS2_FP16_SCALED) return GS2_ERR_ARG;
    if (o.orthogonalization < 0 || o.orthogonalization > 1) return GS2_ERR_ARG;
    if (o.blocks < 0 || o.local_sweeps < 0 || (o.blocks > 1 && (o.compact || o.build_levels)) ||
        (int64_t)o.blocks > std::max<int64_t>(A->n, 1))
        return GS2_ERR_ARG;
    if (!(o.inner_damping > 0.0 && o.inner_damping <= 2.0)) return GS2_ERR_ARG;
    if (o.format < GS2_FORMAT_AUTO || o.format > GS2_FORMAT_BLOCK3 || o.rows_per_lane < 0 || o.lds_staging < 0 ||
        o.lds_staging > 2 || o.spmv_format < GS2_FORMAT_AUTO || o.spmv_format > GS2_FORMAT_BLOCK3 || o.xcd_ranges < 0 ||
        o.xcd_ranges > 2 || o.basis_loads < 0 || o.basis_loads > 2)
        return GS2_ERR_ARG;
    gs2_handle *H = new (std::nothrow) gs2_handle;
    if (!H) return GS2_ERR_NOMEM;
    Handle &h = H->h;
    h.n = A->n;
    h.sweeps = sweeps;
    h.inner = inner;
    h.variant = variant;
    h.omega = damping;
    h.gamma = o.inner_damping;
    h.compact = o.compact ? 1 : 0;
    h.orth = o.orthogonalization;
    h.stag_cycles = o.stagnation_cycles;
    h.spmv_fmt = o.spmv_format;
    h.basis_req = o.basis_loads;
    h.blocks = std::max(1, o.blocks);
    h.local_sweeps = std::max(1, o.local_sweeps);
    h.precision = o.precision;
    hipStream_t s = (hipStream_t)stream;
    // resolve the allocation-free entry point's scratch on this device now
    // (cached per device; should it fail, that entry point reports it)
    (void)noalloc_scratch(nullptr);
    int st = GS2_ERR_HIP;
    try {
        st = setup_handle(h, *A, o, s, true);
    } catch (const std::bad_alloc &) {
        st = GS2_ERR_NOMEM;
    } catch (...) {
        st = GS2_ERR_HIP;
    }
    if (st != GS2_OK) {
        (void)hipStreamSynchronize(s);
        delete H;
        return st;
    }
    *out = H;
    return GS2_OK;
}

void gs2_destroy(gs2_handle *H)
{
    if (!H) return;
    (void)hipDeviceSynchronize();
    delete H;
}

const char *gs2_status_string(int status)
{
    switch (status) {
    case GS2_OK: return "success";
    case GS2_ERR_ARG: return "invalid argument";
    case GS2_ERR_BAD_CSR: return "malformed CSR (unsorted, duplicate or out-of-range column, bad row pointer)";
    case GS2_ERR_ZERO_DIAG: return "diagonal entry missing or zero";
    case GS2_ERR_NONFINITE: return "non-finite value (NaN or Inf)";
    case GS2_ERR_NOMEM: return "device allocation failed";
    case GS2_ERR_HIP: return "HIP runtime error";
    case GS2_ERR_FP16_RANGE: return "scaled matrix value outside binary16 range";
    case GS2_ERR_NO_LEVELS: return "handle was built without level sets";
    case GS2_ERR_SCRATCH: return "input exceeds the fixed scratch of the allocation-free entry point";
    case GS2_NOT_CONVERGED: return "not converged within maxit iterations";
    case GS2_BREAKDOWN_EXACT: return "GMRES exact breakdown (singular Hessenberg)";
    case GS2_STAGNATED: return "GMRES stagnated (true residual not halved over the stagnation window)";
    default: return "unknown status";
    }
}

int gs2_handle_query(const gs2_handle *H, int64_t *n, int64_t *nnz_l, int64_t *nnz_u, int64_t *bytes_stored,
                     int *lanes_per_row, int *levels_l, int *levels_u)
{
    if (!H) return GS2_ERR_ARG;
    const Handle &h = H->h;
    if (n) *n = h.n;
    if (nnz_l) *nnz_l = h.L.nnz;
    if (nnz_u) *nnz_u = h.U.nnz;
    if (bytes_stored)
        *bytes_stored = (h.L.padded + h.U.padded) * (int64_t)(4 + h.L.val_bytes) +
                        h.L.padded * (h.L.off ? 2 : 0) + h.U.padded * (h.U.off ? 2 : 0) +
                        8 * (h.L.nslices + h.U.nslices + 2) + 16 * h.n;
    if (lanes_per_row) *lanes_per_row = h.L.K;
    if (levels_l) *levels_l = h.nlev_l;
    if (levels_u) *levels_u = h.nlev_u;
    return GS2_OK;
}

int gs2_handle_schedule(const gs2_handle *H, int *format, int *lanes_per_row, int *rows_per_lane, int *vector_bytes,
                        int *lds_staging, int *xcd_ranges, int *ndiag_l, int *ndiag_u, int *tuned)
{
    if (!H) return GS2_ERR_ARG;
    const Handle &h = H->h;
    const bool dia = h.fmt == FMT_DIA;
    if (format) *format = !dia ? GS2_FORMAT_SELL : h.DL.b3 ? GS2_FORMAT_BLOCK3 : GS2_FORMAT_DIA;
    if (lanes_per_row) *lanes_per_row = h.L.K;
    if (rows_per_lane) *rows_per_lane = dia ? h.DL.R : 0;
    if (vector_bytes) *vector_bytes = dia ? h.DL.R * h.DL.val_bytes : 0;
    if (lds_staging) *lds_staging = dia ? h.lds : 0;
    if (xcd_ranges) *xcd_ranges = dia ? h.remap : 0;
    if (ndiag_l) *ndiag_l = h.DL.ndiag;
    if (ndiag_u) *ndiag_u = h.DU.ndiag;
    if (tuned) *tuned = h.tuned;
    return GS2_OK;
}

} // extern "C"
