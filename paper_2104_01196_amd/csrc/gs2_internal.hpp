// Internal definitions shared by the HIP sources of libgs2 (gfx950 only).
//
// Data layout.  The preconditioner works on the symmetrically scaled matrix
// Ah = S_l A S_r with S_r = |D|^-1/2 and S_l = sign(D) S_r, whose diagonal is
// one.  GS2 is invariant under this change of variables in exact arithmetic:
// (L + D)^{-1} = S_r (Lh + I)^{-1} S_l, and every Neumann partial sum
// transforms the same way, so the inner recurrence g <- D^{-1}(r - wLg) of
// eq. (jacobi) becomes g <- rh - w Lh g with no division (Section 4).  The
// strictly lower part Lh and strictly upper part Uh are stored apart from A
// (as the paper's GS2 code stores its triangles, Section 6) in a sliced-ELL
// layout made for 64-wide wavefronts:
//
//   * K lanes work on one row, so a slice holds C = 64/K consecutive rows and
//     is processed by one wavefront;
//   * a slice stores T steps of 64 entries; at step t, lane l = r*K + q holds
//     entry t*K + q of local row r, so every load of a wavefront reads 64
//     consecutive values (fully coalesced);
//   * rows shorter than the slice's longest row are padded with (own column,
//     value 0) entries.
//
// The natural row order is kept (no row sorting within slices).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gs2.h"

namespace gs2 {

constexpr int WAVE = 64;
constexpr int NUM_XCD = 8;

#define GS2_TRY_HIP(expr)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            std::fprintf(stderr, "gs2: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                                  \
            return e_ == hipErrorOutOfMemory ? GS2_ERR_NOMEM : GS2_ERR_HIP;                          \
        }                                                                                            \
    } while (0)

#define GS2_TRY(expr)                  \
    do {                               \
        int st_ = (expr);              \
        if (st_ != GS2_OK) return st_; \
    } while (0)

// ------------------------------------------------------------ device helpers

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remap so that each XCD walks one contiguous range of logical
// blocks: neighbouring rows then share an XCD's L2, which is where the x / g
// gathers of a stencil hit.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks)
{
    const int64_t q = nblocks / NUM_XCD, r = nblocks % NUM_XCD;
    const int64_t x = bid % NUM_XCD, k = bid / NUM_XCD;
    return x * q + (x < r ? x : r) + k;
}

// Cross-lane data movement within a DPP row (16 lanes) uses the DPP operand
// modifiers of the VALU instead of LDS-routed permutes.  Controls (CDNA ISA,
// DPP_CTRL): quad_perm [1,0,3,2] = lane ^ 1, quad_perm [2,3,0,1] = lane ^ 2,
// row_half_mirror = 7 - lane within each half row, row_mirror = 15 - lane
// within each row.  Lanes whose source is inactive read 0.
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double read_lane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ __forceinline__ float read_lane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over a group of K consecutive lanes (K a power of two <= 64); every
// lane of the group receives the sum.  Up to 16 lanes: pairs, quads, half
// rows and rows are combined with DPP moves (after each step every lane of
// the group holds the same value: the two operands of each addition are the
// same pair of partial sums).  Across rows the four row sums are read into
// scalar registers and added in a fixed order.  All 64 lanes must be active.
template <int K, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    static_assert(K >= 1 && K <= WAVE && (K & (K - 1)) == 0, "K must be a power of two <= 64");
    if constexpr (K >= 2) v += dpp_move<DPP_XOR1>(v);
    if constexpr (K >= 4) v += dpp_move<DPP_XOR2>(v);
    if constexpr (K >= 8) v += dpp_move<DPP_HALF_MIRROR>(v);
    if constexpr (K >= 16) v += dpp_move<DPP_MIRROR>(v);
    if constexpr (K == 32) {
        const T a = read_lane(v, 0) + read_lane(v, 16), b = read_lane(v, 32) + read_lane(v, 48);
        v = (threadIdx.x & 32) ? b : a;
    }
    if constexpr (K == 64) v = (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return group_sum<WAVE>(v);
}

// value type conversions used by the kernels
template <typename T>
__device__ __forceinline__ float to_f(T v)
{
    return static_cast<float>(v);
}
template <>
__device__ __forceinline__ float to_f<_Float16>(_Float16 v)
{
    return static_cast<float>(v);
}

// --------------------------------------------------------------- host side

// One triangle (strictly lower or upper part of Ah) in sliced-ELL layout.
struct Sell {
    int64_t n = 0;
    int K = 1;  // lanes per row
    int C = 64; // rows per slice
    int64_t nslices = 0;
    int64_t nnz = 0;    // real entries
    int64_t padded = 0; // stored entries (multiple of 64 per slice)
    int64_t *slice_ptr = nullptr;
    int32_t *col = nullptr;
    // col - row - off_min of every stored entry as an unsigned 16-bit number
    // when the offsets of the whole triangle span at most 65535 (the usual
    // case for mesh matrices in their natural ordering), else null.  The
    // streaming kernels then read 2 instead of 4 index bytes per entry.
    uint16_t *off = nullptr;
    int off_min = 0;
    void *val = nullptr;
    int val_bytes = 8;
    // stream the values and offsets past the caches (set for large triangles)
    int nt = 0;
    int idx_bytes() const { return off ? 2 : 4; }
    double stored_bytes() const { return (double)padded * (val_bytes + idx_bytes()); }
};

// The sweep kernels load a triangle with the non-temporal policy once both
// triangles together store more than this: below it they stay in the 256 MB
// last-level cache from one pass to the next and the normal policy is
// faster (128^3 Laplacian, float64, 126 MB: 38.2 ms normal, 40.7 ms
// non-temporal); above it every pass streams them from HBM and keeping them
// out of the caches leaves those to the gathered vectors (192^3 problem:
// 425 / 255 / 170 MB in float64 / float32 / scaled float16: 260.5 / 244.0 /
// 238.8 ms normal, 252.1 / 239.1 / 236.4 ms non-temporal).
constexpr double NT_TRIANGLES_BYTES = 150e6;

// Bytes read before each timed pass of the setup's schedule timing: twice
// the last-level cache (256 MB), so that every candidate is timed with the
// triangles out of the caches, as a Krylov solve finds them (its basis
// passes between two applies evict them).  Timed back to back instead, the
// 192^3 problem's float32 triangles (170 MB) stayed in that cache and one
// row per lane timed within the 3 % margin of two, while in the solve it
// ran 17 % slower per inner pass (42.0 against 35.8 us).
constexpr size_t FLUSH_BYTES = size_t(512) << 20;

// Build the 16-bit column offsets of a sliced-ELL array (K lanes per row,
// slice pointers sp, padded entries, columns col; lane l of slice s holds row
// s * 64/K + l/K): *off = col - row - *off_min.  *off is left null when the
// offsets span more than 65535.
int build_col_offsets(int64_t nslices, int K, const int64_t *sp, const int32_t *col, int64_t padded, uint16_t **off,
                      int *off_min, hipStream_t s);

// One triangle in the diagonal-interleaved layout (chosen by the setup's
// timing when the triangle has few distinct offsets col - row, as stencil
// matrices in their natural ordering do).  Diagonal d holds, for every row
// i, the value of entry (i, i + off[d]) (0 where the triangle has none or
// the column falls outside the matrix).  Rows are grouped in blocks of 64 R
// (one wavefront, R rows per lane): lane l of block b owns rows
// b*64R + k*64 + l, k < R, and its R values of a diagonal are stored
// contiguously at b*64R + l*R, so they arrive in one R * b_v byte load
// while every gather x[row + off] of the wavefront reads 64 consecutive
// elements.  No column indices are stored.
constexpr int DIA_MAX = 32;   // most diagonals per triangle
constexpr int DIA_HALO = 64;  // LDS staging covers offsets |off| <= DIA_HALO
constexpr int DIA_THREADS = 256; // threads per workgroup of the passes on it
struct Dia {
    int ndiag = 0;
    int R = 1;          // rows (3-row blocks: nodes) per lane
    int64_t stride = 0; // entries per diagonal (rows or nodes padded to whole workgroups)
    int64_t nnz = 0;    // real entries
    int off[DIA_MAX] = {};
    void *val = nullptr;
    int val_bytes = 8;
    int nt = 0; // stream the values with the non-temporal policy
    // 3-row blocks (3 unknowns per node, node-major): off[] holds node
    // offsets c/3 - r/3, and plane 9 d + 3 j + b (j, b < 3) holds
    // a_{3i + j, 3(i + off[d]) + b} at node i's interleaved position
    int b3 = 0;
    double stored_bytes() const { return (double)ndiag * (b3 ? 9.0 : 1.0) * (double)stride * val_bytes; }
};

// The schedule the setup picked for the sweep kernels.
enum : int { FMT_SELL = 0, FMT_DIA = 1 };

struct GmresWork; // krylov.hip
struct CgWork;    // cg.hip

struct Handle {
    int64_t n = 0;
    int sweeps = 1, inner = 1, variant = GS2_FORWARD, precision = GS2_FP64;
    double omega = 1.0, gamma = 1.0;
    int compact = 0;
    int orth = 0;        // GMRES orthogonalisation (0 delayed CGS2, 1 CGS2)
    int stag_cycles = 0; // GMRES stagnation window in restart cycles (0 default, < 0 off)
    int spmv_fmt = 0;    // GMRES: layout request for the solver's copy of A (GS2_FORMAT_*)
    int basis_req = 0;   // GMRES: basis passes' loads in flight (0 timed, 1 wide, 2 narrow)
    double *flush = nullptr; // setup only: FLUSH_BYTES read before each timed pass (null: none)
    int block_waves = 4; // wavefronts per workgroup in the sweep kernels
    Sell L, U;
    // diagonal-interleaved copies of L and U, used by the GS2 / JR passes
    // when fmt == FMT_DIA (rows per lane dl.R, LDS staging if lds)
    int fmt = FMT_SELL, lds = 0, tuned = 0;
    // diagonal passes: walk each XCD through its own contiguous range of
    // workgroups (1) or dispatch them in order (0); timed with the rest
    int remap = 1;
    Dia DL, DU;
    // hybrid relaxation: `blocks` contiguous row blocks; L and U then hold the
    // block-local triangles and E the couplings between blocks, applied to
    // values frozen once per global sweep (`local_sweeps` local sweeps each)
    int blocks = 1, local_sweeps = 1;
    Sell E;
    void *yh = nullptr; // frozen copy of the iterate
    double *sl = nullptr, *sr = nullptr; // scaling vectors (float64)
    // persistent temporaries (Section 6: allocated once, live with the handle)
    void *xh = nullptr, *xh2 = nullptr, *rh = nullptr, *ga = nullptr, *gb = nullptr;
    // S_l v rounded to the working precision, formed once per apply by the
    // 32- and 16-bit forms on the diagonal layout (null in float64)
    void *sv = nullptr;
    // level sets (optional)
    int nlev_l = 0, nlev_u = 0;
    int32_t *lev_rows_l = nullptr, *lev_rows_u = nullptr; // rows grouped by level
    std::vector<int64_t> lev_ptr_l, lev_ptr_u;            // host offsets
    // multicolor ordering (optional)
    int ncolors = 0;
    int32_t *color_rows = nullptr; // rows grouped by color
    std::vector<int64_t> color_ptr;
    GmresWork *gw = nullptr;
    CgWork *cw = nullptr;
    const int *stop = nullptr; // device flag: kernels return at once when set (GMRES)
    // GMRES: the serial work that closes its previous Arnoldi step, run by one
    // extra workgroup of the next apply's first pass (consumed by that apply)
    struct FinJob {
        const double *part = nullptr;
        int nb = 0;
        void *st = nullptr;
    } fin;
    ~Handle();
};

// setup.hip
int setup_handle(Handle &h, const gs2_csr &A, const gs2_options &o, hipStream_t s, bool alloc_vecs);
void free_sell(Sell &S);
void free_dia(Dia &D);
int choose_lanes(double avg_len, int max_len);
// out[i] = in[0] + ... + in[i-1] for i < m (device arrays; synchronises s)
int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t m, hipStream_t s);

// sweep.hip
int apply_gs2(Handle &h, const double *v, double *z, hipStream_t s);
int apply_jr(Handle &h, int sweeps, double omega, const double *v, double *z, hipStream_t s);
int apply_trisolve(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s);
int apply_mtgs(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s);
int time_inner_pass(Handle &h, hipStream_t s, float *ms, bool with_resid = false);
int inner_residuals(Handle &h, const double *r, int inner, double *out, hipStream_t s);
// device address of the allocation-free entry point's fixed scratch on the
// current device (resolved once per device)
int noalloc_scratch(double **ptr);

// krylov.hip, cg.hip
void free_gmres_work(GmresWork *w);
void free_cg_work(CgWork *w);

inline size_t prec_bytes(int precision) { return precision == GS2_FP64 ? 8 : 4; }

// profile.hip: optional per-launch HIP-event timing with algorithmic bytes
enum ProfKid : int {
    PK_INNER = 0, PK_RESID, PK_FIRST_JR, PK_TRI, PK_SPMV_DOT, PK_CGS, PK_TRUE_RESID, PK_REDUCE, PK_GIVENS,
    PK_SCALE, PK_UPDATE_X, PK_BATCHED, PK_MISC, PK_SPMV, PK_PREP
};
bool prof_on();
// While one lives, the calling thread's launches are not recorded (the
// allocation-free entry points: recording creates events).
struct ProfPause {
    ProfPause();
    ~ProfPause();
};
void prof_begin(hipStream_t s, int kid, double bytes);
void prof_end(hipStream_t s);
void prof_set_step(int cycle, int step);
void prof_drop_from_step(int cycle, int kk);

struct Prof {
    hipStream_t s;
    bool on;
    Prof(hipStream_t s_, int kid, double bytes) : s(s_), on(prof_on())
    {
        if (on) prof_begin(s, kid, bytes);
    }
    ~Prof()
    {
        if (on) prof_end(s);
    }
};

} // namespace gs2

struct gs2_handle {
    gs2::Handle h;
};
