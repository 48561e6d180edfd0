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

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m)
{
    return __shfl_xor(v, m, WAVE);
}

// Sum over a group of K consecutive lanes (K a power of two <= 64); every
// lane of the group receives the sum.  The butterfly order is fixed, so the
// result is deterministic.
template <int K, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int o = K / 2; o > 0; o >>= 1) v += shfl_xor(v, o);
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
    void *val = nullptr;
    int val_bytes = 8;
};

struct GmresWork; // krylov.hip
struct CgWork;    // cg.hip

struct Handle {
    int64_t n = 0;
    int sweeps = 1, inner = 1, variant = GS2_FORWARD, precision = GS2_FP64;
    double omega = 1.0, gamma = 1.0;
    int compact = 0;
    int orth = 0;        // GMRES orthogonalisation (0 delayed CGS2, 1 CGS2)
    int block_waves = 4; // wavefronts per workgroup in the sweep kernels
    Sell L, U;
    // hybrid relaxation: `blocks` contiguous row blocks; L and U then hold the
    // block-local triangles and E the couplings between blocks, applied to
    // values frozen once per global sweep (`local_sweeps` local sweeps each)
    int blocks = 1, local_sweeps = 1;
    Sell E;
    void *yh = nullptr; // frozen copy of the iterate
    double *sl = nullptr, *sr = nullptr; // scaling vectors (float64)
    // persistent temporaries (Section 6: allocated once, live with the handle)
    void *xh = nullptr, *xh2 = nullptr, *rh = nullptr, *ga = nullptr, *gb = nullptr;
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
    ~Handle();
};

// setup.hip
int setup_handle(Handle &h, const gs2_csr &A, const gs2_options &o, hipStream_t s, bool alloc_vecs);
void free_sell(Sell &S);
int choose_lanes(double avg_len, int max_len);

// sweep.hip
int apply_gs2(Handle &h, const double *v, double *z, hipStream_t s);
int apply_jr(Handle &h, int sweeps, double omega, const double *v, double *z, hipStream_t s);
int apply_trisolve(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s);
int apply_mtgs(Handle &h, int variant, double omega, const double *v, double *z, hipStream_t s);
int time_inner_pass(Handle &h, hipStream_t s, float *ms);

// krylov.hip, cg.hip
void free_gmres_work(GmresWork *w);
void free_cg_work(CgWork *w);

inline size_t prec_bytes(int precision) { return precision == GS2_FP64 ? 8 : 4; }

// profile.hip: optional per-launch HIP-event timing with algorithmic bytes
enum ProfKid : int {
    PK_INNER = 0, PK_RESID, PK_FIRST_JR, PK_TRI, PK_SPMV_DOT, PK_CGS, PK_TRUE_RESID, PK_REDUCE, PK_GIVENS,
    PK_SCALE, PK_UPDATE_X, PK_BATCHED, PK_MISC
};
bool prof_on();
void prof_begin(hipStream_t s, int kid, double bytes);
void prof_end(hipStream_t s);
void prof_set_step(int cycle, int step);
void prof_drop_from_step(int cycle, int kk);
struct ProfSet; // event records captured into a graph
void prof_capture_begin();
ProfSet *prof_capture_end();
void prof_accumulate(ProfSet *ps, int kk);
void prof_free_set(ProfSet *ps);

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
