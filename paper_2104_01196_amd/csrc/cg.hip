// Preconditioned conjugate gradients in float64 (the Krylov solver of the
// paper's symmetric positive definite experiments, Sections 9 and 10), for
// use with the symmetric GS2 (SGS2) preconditioner.  Textbook recurrences;
// the recurrence residual decides when to stop, the true residual is then
// checked and the iteration restarts from it if it has drifted.  Every
// scalar (alpha, beta, the stopping test) is formed on the device; the host
// enqueues iterations in chunks and synchronises once per chunk, kernels
// return at once after the stopping test has fired.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>

#include "gs2_internal.hpp"

namespace gs2 {

constexpr int CT = 256;  // threads per workgroup
constexpr int CRB = 1024; // rows per workgroup of the vector kernels

struct CState {
    int it, done, maxit, status;
    double bnorm, rtol, rz, pq, rr, beta;
};

struct CgWork {
    int64_t n = 0;
    int nb = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;
    CState *st = nullptr, *hst = nullptr;
};

void free_cg_work(CgWork *w)
{
    if (!w) return;
    for (void *ptr : {(void *)w->r, (void *)w->z, (void *)w->p, (void *)w->q, (void *)w->part, (void *)w->st})
        if (ptr) (void)hipFree(ptr);
    if (w->hst) (void)hipHostFree(w->hst);
    delete w;
}

static int alloc_cg(CgWork **out, int64_t n)
{
    CgWork *w = new (std::nothrow) CgWork;
    if (!w) return GS2_ERR_NOMEM;
    w->n = n;
    w->nb = (int)std::max<int64_t>(1, (n + CRB - 1) / CRB);
    const size_t N = (size_t)std::max<int64_t>(n, 1);
    int st = GS2_OK;
    auto A = [&](void **p, size_t b) {
        if (st == GS2_OK && hipMalloc(p, b) != hipSuccess) st = GS2_ERR_NOMEM;
    };
    A((void **)&w->r, 8 * N);
    A((void **)&w->z, 8 * N);
    A((void **)&w->p, 8 * N);
    A((void **)&w->q, 8 * N);
    A((void **)&w->part, 8 * (size_t)w->nb);
    A((void **)&w->st, sizeof(CState));
    if (st == GS2_OK && hipHostMalloc((void **)&w->hst, sizeof(CState), hipHostMallocDefault) != hipSuccess)
        st = GS2_ERR_NOMEM;
    if (st != GS2_OK) {
        free_cg_work(w);
        return st;
    }
    *out = w;
    return GS2_OK;
}

__device__ __forceinline__ double cg_block_sum(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < CT / WAVE; ++i) s += red[i];
    return s;
}

// out = b - A x (when b != NULL) or out = A x, with partial sums of
// out.x2 (x2 = out when x2 == NULL).  K lanes per row.
template <int K>
__global__ __launch_bounds__(CT) void k_cg_spmv(int64_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci, const double *__restrict__ va,
                                                const double *__restrict__ x, const double *__restrict__ b,
                                                double *__restrict__ out, const double *__restrict__ x2,
                                                const int *__restrict__ stop, double *__restrict__ part)
{
    __shared__ double red[CT / WAVE];
    if (stop && *stop) return;
    const int64_t r0 = (int64_t)blockIdx.x * CRB;
    const int t = threadIdx.x, q = t & (K - 1);
    constexpr int RPP = CT / K;
    double s = 0.0;
    for (int pass = 0; pass < CRB / RPP; ++pass) {
        const int64_t row = r0 + pass * RPP + t / K;
        double acc = 0.0;
        if (row < n) {
            const int bb = rp[row], e = rp[row + 1];
            for (int p = bb + q; p < e; p += K) acc += va[p] * x[ci[p]];
        }
        acc = group_sum<K>(acc);
        if (q == 0 && row < n) {
            const double o = b ? b[row] - acc : acc;
            out[row] = o;
            s += o * (x2 ? x2[row] : o);
        }
    }
    s = cg_block_sum(s, red);
    if (t == 0) part[blockIdx.x] = s;
}

// sum of the partials into *dst; mode 0: plain store; 1: CG update check
// (rr, stopping test); 2: r.z -> beta and rz
__global__ __launch_bounds__(CT) void k_cg_reduce(const double *__restrict__ part, int nb, CState *__restrict__ st,
                                                  int mode, double *__restrict__ dst)
{
    __shared__ double red[CT / WAVE];
    if (mode != 0 && st->done) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += CT) s += part[b];
    s = cg_block_sum(s, red);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        *dst = s;
    } else if (mode == 1) {
        st->rr = s;
        st->it += 1;
        if (!isfinite(s)) {
            st->status = GS2_ERR_NONFINITE;
            st->done = 1;
        } else if (sqrt(s) <= st->rtol * st->bnorm || st->it >= st->maxit) {
            st->done = 1;
        }
    } else {
        st->beta = s / st->rz;
        st->rz = s;
    }
}

// x += alpha p, r -= alpha q (alpha = rz / pq), partial ||r||^2
__global__ __launch_bounds__(CT) void k_cg_update(int64_t n, const double *__restrict__ p,
                                                  const double *__restrict__ q, double *__restrict__ x,
                                                  double *__restrict__ r, const CState *__restrict__ st,
                                                  double *__restrict__ part)
{
    __shared__ double red[CT / WAVE];
    if (st->done) return;
    const double alpha = st->rz / st->pq;
    const int64_t r0 = (int64_t)blockIdx.x * CRB;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < CRB / CT; ++u) {
        const int64_t i = r0 + threadIdx.x + u * CT;
        if (i < n) {
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            s += ri * ri;
        }
    }
    s = cg_block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// partial r.z
__global__ __launch_bounds__(CT) void k_cg_dot(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                               const CState *__restrict__ st, double *__restrict__ part)
{
    __shared__ double red[CT / WAVE];
    if (st && st->done) return;
    const int64_t r0 = (int64_t)blockIdx.x * CRB;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < CRB / CT; ++u) {
        const int64_t i = r0 + threadIdx.x + u * CT;
        if (i < n) s += a[i] * b[i];
    }
    s = cg_block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p  (beta_mode 0: p = z)
__global__ void k_cg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                       const CState *__restrict__ st, int beta_mode)
{
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = beta_mode ? z[i] + st->beta * p[i] : z[i];
}

__global__ void k_cg_copy(int64_t n, const double *__restrict__ a, double *__restrict__ b, const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_cg_start(CState *__restrict__ st, int maxit_total, double rtol)
{
    if (threadIdx.x) return;
    st->done = 0;
    st->maxit = maxit_total;
    st->rtol = rtol;
}

static int cg_lanes(const gs2_csr &A)
{
    const double avg = A.n ? (double)A.nnz / (double)A.n : 1.0;
    return avg <= 8.0 ? 4 : avg <= 16.0 ? 8 : avg <= 32.0 ? 16 : avg <= 64.0 ? 32 : 64;
}

#define GS2_CG_DISPATCH(K, kern, grid, ...)                                  \
    do {                                                                     \
        switch (K) {                                                         \
        case 4: kern<4><<<grid, CT, 0, s>>>(__VA_ARGS__); break;             \
        case 8: kern<8><<<grid, CT, 0, s>>>(__VA_ARGS__); break;             \
        case 16: kern<16><<<grid, CT, 0, s>>>(__VA_ARGS__); break;           \
        case 32: kern<32><<<grid, CT, 0, s>>>(__VA_ARGS__); break;           \
        default: kern<64><<<grid, CT, 0, s>>>(__VA_ARGS__); break;           \
        }                                                                    \
    } while (0)

static int cg_impl(const gs2_csr &A, const double *b, double *x, double rtol, int maxit, int kind, gs2_handle *P,
                   gs2_solve_info *info, hipStream_t s)
{
    const int64_t n = A.n;
    CgWork *own = nullptr, *W = nullptr;
    if (P) {
        if (!P->h.cw || P->h.cw->n != n) {
            if (P->h.cw) free_cg_work(P->h.cw);
            P->h.cw = nullptr;
            GS2_TRY(alloc_cg(&P->h.cw, n));
        }
        W = P->h.cw;
    } else {
        GS2_TRY(alloc_cg(&own, n));
        W = own;
    }
    struct Guard {
        CgWork *w;
        gs2_handle *P;
        ~Guard()
        {
            if (w) free_cg_work(w);
            if (P) P->h.stop = nullptr;
        }
    } guard{own, P};
    CState *st = W->st;
    if (P) P->h.stop = &st->done;
    const int nb = W->nb, K = cg_lanes(A);
    const unsigned gN = (unsigned)nb, gE = (unsigned)((n + 255) / 256);
    const double spmv_b = 12.0 * (double)A.nnz + 4.0 * (n + 1) + 16.0 * n;
    auto prec = [&](const double *v, double *z) -> int {
        switch (kind) {
        case GS2_PREC_GS2: return apply_gs2(P->h, v, z, s);
        case GS2_PREC_JR: return apply_jr(P->h, P->h.sweeps, P->h.omega, v, z, s);
        case GS2_PREC_GS_TRISOLVE: return apply_trisolve(P->h, P->h.variant, P->h.omega, v, z, s);
        case GS2_PREC_MTGS: return apply_mtgs(P->h, P->h.variant, P->h.omega, v, z, s);
        default: k_cg_copy<<<gE, 256, 0, s>>>(n, v, z, &st->done); return GS2_OK;
        }
    };
    auto read_state = [&]() -> int {
        GS2_TRY_HIP(hipMemcpyAsync(W->hst, st, sizeof(CState), hipMemcpyDeviceToHost, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        return GS2_OK;
    };
    // ||b||, initial state
    {
        // staged in the pinned mirror (no copy from it is in flight here)
        CState init{};
        init.rtol = rtol;
        init.maxit = maxit;
        *W->hst = init;
        GS2_TRY_HIP(hipMemcpyAsync(st, W->hst, sizeof(CState), hipMemcpyHostToDevice, s));
    }
    k_cg_dot<<<gN, CT, 0, s>>>(n, b, b, nullptr, W->part);
    k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 0, &st->bnorm);
    GS2_TRY_HIP(hipGetLastError());
    GS2_TRY(read_state());
    const double bn2 = W->hst->bnorm;
    if (!std::isfinite(bn2)) return GS2_ERR_NONFINITE;
    if (bn2 == 0.0) {
        GS2_TRY_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        GS2_TRY_HIP(hipStreamSynchronize(s));
        info->converged = 1;
        return GS2_OK;
    }
    const double bnorm = std::sqrt(bn2);
    {
        CState init{}; // the mirror was last filled by read_state, which synchronised
        init.bnorm = bnorm;
        init.rtol = rtol;
        init.maxit = maxit;
        *W->hst = init;
        GS2_TRY_HIP(hipMemcpyAsync(st, W->hst, sizeof(CState), hipMemcpyHostToDevice, s));
    }
    int status = GS2_OK, runs = 0;
    for (;;) {
        // true residual r = b - A x
        {
            Prof pr(s, PK_TRUE_RESID, spmv_b + 8.0 * n);
            GS2_CG_DISPATCH(K, k_cg_spmv, gN, n, A.rowptr, A.colind, A.val, x, b, W->r, nullptr, nullptr, W->part);
        }
        k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 0, &st->rr);
        GS2_TRY_HIP(hipGetLastError());
        GS2_TRY(read_state());
        const CState hs = *W->hst;
        if (hs.status != GS2_OK) { status = hs.status; break; }
        const double rel = std::sqrt(hs.rr) / bnorm;
        info->relres = rel;
        info->iterations = hs.it;
        if (!std::isfinite(rel)) { status = GS2_ERR_NONFINITE; break; }
        if (rel <= rtol) { info->converged = 1; break; }
        if (hs.it >= maxit) { status = GS2_NOT_CONVERGED; break; }
        if (runs++ > 0) info->restarts++;
        k_cg_start<<<1, 64, 0, s>>>(st, maxit, rtol);
        // z = M^-1 r, p = z, rz = r.z
        GS2_TRY(prec(W->r, W->z));
        k_cg_dot<<<gN, CT, 0, s>>>(n, W->r, W->z, st, W->part);
        k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 0, &st->rz);
        k_cg_p<<<gE, 256, 0, s>>>(n, W->z, W->p, st, 0);
        int chunk = 8;
        for (;;) {
            for (int c = 0; c < chunk; ++c) {
                {   // q = A p, p.q
                    Prof pr(s, PK_SPMV_DOT, spmv_b + 8.0 * n);
                    GS2_CG_DISPATCH(K, k_cg_spmv, gN, n, A.rowptr, A.colind, A.val, W->p, nullptr, W->q, W->p,
                                    &st->done, W->part);
                }
                k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 0, &st->pq);
                {
                    Prof pr(s, PK_CGS, 48.0 * n);
                    k_cg_update<<<gN, CT, 0, s>>>(n, W->p, W->q, x, W->r, st, W->part);
                }
                k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 1, nullptr);
                GS2_TRY(prec(W->r, W->z));
                k_cg_dot<<<gN, CT, 0, s>>>(n, W->r, W->z, st, W->part);
                k_cg_reduce<<<1, CT, 0, s>>>(W->part, nb, st, 2, nullptr);
                {
                    Prof pr(s, PK_SCALE, 24.0 * n);
                    k_cg_p<<<gE, 256, 0, s>>>(n, W->z, W->p, st, 1);
                }
            }
            GS2_TRY_HIP(hipGetLastError());
            GS2_TRY(read_state());
            if (W->hst->done) break;
            chunk = std::min(chunk * 2, 64);
        }
    }
    return status;
}

} // namespace gs2

using namespace gs2;

extern "C" int cg_solve(const gs2_csr *A, const double *b, double *x, double rtol, int maxit, int prec_kind,
                        gs2_handle *prec, gs2_solve_info *info, void *stream)
{
    gs2_solve_info local;
    gs2_solve_info *inf = info ? info : &local;
    std::memset(inf, 0, sizeof(*inf));
    const auto t0 = std::chrono::steady_clock::now();
    int st;
    if (!A || A->n <= 0 || A->n >= (int64_t(1) << 31) - 1 || !A->rowptr || !A->colind || !A->val || !b || !x ||
        !(rtol >= 0.0) || maxit < 0 || prec_kind < GS2_PREC_NONE || prec_kind > GS2_PREC_MTGS ||
        (prec_kind != GS2_PREC_NONE && !prec) || (prec && prec->h.n != A->n)) {
        st = GS2_ERR_ARG;
    } else if ((prec_kind == GS2_PREC_GS_TRISOLVE && prec->h.nlev_l == 0) ||
               (prec_kind == GS2_PREC_MTGS && prec->h.ncolors == 0)) {
        st = GS2_ERR_NO_LEVELS;
    } else {
        try {
            st = cg_impl(*A, b, x, rtol, maxit, prec_kind, prec, inf, (hipStream_t)stream);
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
