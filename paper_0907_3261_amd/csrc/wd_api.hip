// C ABI of the wdsolve library: context, setup, operator, preconditioner and
// the preconditioned block BiCGGR driver (Sec. 2, algorithm box; Sec. 3.3
// for the initial choices and the stopping rule).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "wd_internal.h"

using namespace wd;

namespace {

#define WD_TRY_HIP(expr)                           \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return WD_EHIP;      \
    } while (0)

size_t block_elems(const wd_ctx* c, int L) { return (size_t)12 * c->g.V * L; }

bool overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

// [a, a + na) and [b, b + nb) share a byte
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

int dev_alloc(void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return WD_ENOMEM;
    }
    return WD_OK;
}

void dev_free(void*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Workspace roles in ctx->ws
enum { WS_R = 0, WS_RT, WS_P, WS_V, WS_W, WS_F, WS_G, WS_U, WS_Y, WS_T1, WS_JT = 10, WS_T2 = 11 };

// Small device control block (after the L x L matrices in ctx->small)
struct Ctl {
    double norms[WD_MAX_L];
    double cond[2];  // condition estimates of the two L x L systems of the last iteration
    int status;
    int pad;
};

// ctx->small: eight L x L matrices (256 pairs each), 16 scalars, the control block
struct SmallLayout {
    double2* mats[8];
    double2 *C_r, *C_rn, *alpha, *gamma, *zeta;
    Ctl* ctl;
};

SmallLayout small_layout(wd_ctx* c) {
    SmallLayout s;
    for (int i = 0; i < 8; ++i) s.mats[i] = c->small + 256 * i;
    s.C_r = s.mats[0];
    s.C_rn = s.mats[1];
    s.alpha = s.mats[2];
    s.gamma = s.mats[3];
    s.zeta = c->small + 2048;
    s.ctl = reinterpret_cast<Ctl*>(c->small + 2064);
    return s;
}
constexpr size_t kSmallPairs = 2064 + (sizeof(Ctl) + 15) / 16 + 1;

int check_prec(int prec) { return (prec == WD_F64 || prec == WD_F32 || prec == WD_BF16) ? WD_OK : WD_EINVAL; }
// the Jacobi preconditioner also takes FP64 iterates with low-precision coefficients
bool coef_prec(int prec) { return prec == WD_F64_COEF_F32 || prec == WD_F64_COEF_BF16; }
Prec coef_of(int prec) { return prec == WD_F64_COEF_F32 ? Prec::F32 : Prec::BF16; }

// host copy of the squared column norms of an N x L block
int colnorms_host(wd_ctx* c, const double2* R, int L, double* out) {
    const size_t N = (size_t)12 * c->g.V;
    const int nb = gram_blocks(N);
    SmallLayout s = small_layout(c);
    WD_TRY_HIP(launch_colnorms(R, N, L, c->partial, nb, s.ctl->norms, c->stream));
    WD_TRY_HIP(hipMemcpyAsync(out, s.ctl->norms, sizeof(double) * L, hipMemcpyDeviceToHost, c->stream));
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

}  // namespace

namespace wd {

// The three low-precision block buffers (FP32-sized), allocated on first use;
// a buffer whose allocation failed earlier is tried again.
int lowp_ensure(wd_ctx* c) {
    const size_t bytes = block_elems(c, c->max_L) * sizeof(float2);
    for (int i = 0; i < 3; ++i) {
        if (c->lp[i]) continue;
        int r = dev_alloc(&c->lp[i], bytes);
        if (r != WD_OK) return r;
    }
    return WD_OK;
}

}  // namespace wd

extern "C" {

const char* wd_strerror(int code) {
    switch (code) {
        case WD_OK: return "ok";
        case WD_EINVAL: return "invalid argument";
        case WD_ENOMEM: return "device allocation failed";
        case WD_EHIP: return "HIP runtime error";
        case WD_ENAN: return "non-finite value in a residual";
        case WD_ESTATE: return "call out of order (links or parameters not set)";
        case WD_NOT_CONVERGED: return "not converged within max_iter";
        case WD_BREAKDOWN: return "breakdown: singular L x L system or zero step";
        case WD_DIVERGED: return "diverged: residual above diverge_at";
        case WD_STAGNATED: return "stagnated: no improvement within stagnate_window";
        default: return "unknown code";
    }
}

long long wd_volume(const wd_ctx* c) { return c ? (long long)c->g.V : -1; }

int wd_destroy(wd_ctx* c) {
    if (!c) return WD_EINVAL;
    dev_free((void*&)c->f.U);
    dev_free((void*&)c->f.T);
    for (int p = 0; p < 3; ++p) {
        dev_free(c->f.Uk[p]);
        dev_free(c->f.Ti[p]);
        dev_free(c->f.Tp[p]);
        dev_free(c->f.Tc[p]);
    }
    for (auto& w : c->ws) dev_free((void*&)w);
    for (auto& w : c->lp) dev_free(w);
    for (auto& w : c->tb) dev_free((void*&)w);
    dev_free((void*&)c->partial);
    dev_free((void*&)c->small);
    dev_free((void*&)c->theta);
    dev_free((void*&)c->U32);
    dev_free(c->learn_mem);
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    delete c;
    return WD_OK;
}

int wd_create(wd_ctx** out, const int dims[4], int bc_t, int max_L, void* hip_stream) {
    if (!out || !dims) return WD_EINVAL;
    *out = nullptr;
    for (int m = 0; m < 4; ++m)
        if (dims[m] < 2) return WD_EINVAL;
    if (bc_t != 0 && bc_t != 1) return WD_EINVAL;
    if (max_L < 1 || max_L > WD_MAX_L) return WD_EINVAL;
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    // site indices are 32-bit, and the stencil kernels address a field plane with 32-bit
    // byte offsets (16 bytes per site in FP64)
    if (V > (1LL << 28)) return WD_EINVAL;
    wd_ctx* c = new (std::nothrow) wd_ctx();
    if (!c) return WD_ENOMEM;
    c->g.lx = dims[0];
    c->g.ly = dims[1];
    c->g.lz = dims[2];
    c->g.lt = dims[3];
    c->g.V = (int)V;
    c->g.sxy = dims[0] * dims[1];
    c->g.sxyz = dims[0] * dims[1] * dims[2];
    c->bc_t = bc_t;
    c->max_L = max_L;
    c->stream = (hipStream_t)hip_stream;
    int r = WD_OK;
    const size_t links = (size_t)4 * 9 * V, clov = (size_t)2 * 18 * V;
    r = r ? r : dev_alloc((void**)&c->f.U, links * 16);
    r = r ? r : dev_alloc((void**)&c->f.T, clov * 16);
    const size_t psz[3] = {16, 8, 4};
    for (int p = 0; p < 3 && !r; ++p) {
        r = r ? r : dev_alloc(&c->f.Uk[p], links * psz[p]);
        r = r ? r : dev_alloc(&c->f.Ti[p], clov * psz[p]);
        r = r ? r : dev_alloc(&c->f.Tp[p], clov * psz[p]);
        r = r ? r : dev_alloc(&c->f.Tc[p], clov * psz[p]);
    }
    for (auto& w : c->ws) r = r ? r : dev_alloc((void**)&w, block_elems(c, max_L) * 16);
    r = r ? r : dev_alloc((void**)&c->partial, (size_t)512 * partial_stride() * 16);
    r = r ? r : dev_alloc((void**)&c->small, kSmallPairs * 16);
    r = r ? r : dev_alloc((void**)&c->U32, links * 8);
    r = r ? r : dev_alloc((void**)&c->theta, (size_t)WD_LEARNED_LAYERS * WD_LEARNED_DIRS * 16 * 8);
    if (!r && hipHostMalloc((void**)&c->host_ctl, sizeof(Ctl)) != hipSuccess) r = WD_ENOMEM;
    if (r) {
        wd_destroy(c);
        return r;
    }
    *out = c;
    return WD_OK;
}

int wd_set_links(wd_ctx* c, const double* U, int on_device) {
    if (!c || !U) return WD_EINVAL;
    const size_t n = (size_t)4 * 9 * c->g.V;
    const double2* src = (const double2*)U;
    void* staging = nullptr;
    if (!on_device) {
        // stage through the T2 workspace block (large enough: 36 V <= 12 V max_L only if
        // max_L >= 3), otherwise through a temporary allocation
        if (n <= block_elems(c, c->max_L)) {
            staging = c->ws[WS_T2];
        } else {
            int r = dev_alloc(&staging, n * 16);
            if (r) return r;
        }
        if (hipMemcpyAsync(staging, U, n * 16, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            if (staging != c->ws[WS_T2]) dev_free(staging);
            return WD_EHIP;
        }
        src = (const double2*)staging;
    }
    hipError_t e = launch_links_from_abi(src, c->f.U, c->g, c->bc_t, c->stream);
    if (e == hipSuccess) e = launch_convert(c->f.U, c->U32, Prec::F32, 1.0, n, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (staging && staging != c->ws[WS_T2]) dev_free(staging);
    if (e != hipSuccess) return WD_EHIP;
    c->have_links = true;
    c->have_params = false;
    return WD_OK;
}

int wd_set_params(wd_ctx* c, double kappa, double csw, int jacobi_kind) {
    if (!c) return WD_EINVAL;
    if (!c->have_links) return WD_ESTATE;
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return WD_EINVAL;
    if (jacobi_kind != WD_JACOBI_BLOCK && jacobi_kind != WD_JACOBI_POINT) return WD_EINVAL;
    const size_t V = c->g.V, links = (size_t)36 * V, clov = (size_t)36 * V;
    const size_t psize[3] = {16, 8, 4};
    hipStream_t s = c->stream;
    c->have_params = false;
    c->g.vt &= ~kCoefTiled;  // the fields below are written in the standard layout, then tiled
    double2* Ti64 = (double2*)c->f.Ti[0];
    WD_TRY_HIP(launch_clover(c->f.U, c->f.T, Ti64, c->g, kappa, csw, s));
    WD_TRY_HIP(launch_point_form(c->f.T, (double2*)c->f.Tp[0], V, s));
    WD_TRY_HIP(launch_convert(c->f.U, c->f.Uk[0], Prec::F64, kappa, links, s));
    WD_TRY_HIP(launch_convert(c->f.T, c->f.Tc[0], Prec::F64, 1.0, clov, s));
    for (int p = 1; p < 3; ++p) {
        const Prec pr = (Prec)p;
        // FP32 / BF16 links keep their first two rows (planes [mu][6][V]); the hop kernels
        // rebuild the third from them
        for (int mu = 0; mu < 4; ++mu)
            WD_TRY_HIP(launch_convert(c->f.U + (size_t)mu * 9 * V, (char*)c->f.Uk[p] + (size_t)mu * 6 * V * psize[p], pr,
                                      kappa, (size_t)6 * V, s));
        WD_TRY_HIP(launch_convert(Ti64, c->f.Ti[p], pr, 1.0, clov, s));
        WD_TRY_HIP(launch_convert((const double2*)c->f.Tp[0], c->f.Tp[p], pr, 1.0, clov, s));
        WD_TRY_HIP(launch_convert(c->f.T, c->f.Tc[p], pr, 1.0, clov, s));
    }
    // the hop kernels' FP64 fields in the tiled layout: each 64-site tile's links and 6x6 blocks
    // one contiguous run (see coef_site); f.T, which wd_get_clover returns, stays standard.
    // The copy goes through an idle workspace block (no allocation here: a large temporary
    // freed before the low-precision blocks are allocated was measured to slow the BF16
    // sweep by 40 %); with max_L < 3 that block is too small and the fields stay standard.
    void* tmp = block_elems(c, c->max_L) >= clov ? (void*)c->ws[WS_T2] : nullptr;
    if (coef_tiled_ok(c->g) && tmp) {
        hipError_t e = hipSuccess;
        auto tile = [&](void* f, int np, int pb) {
            if (e == hipSuccess) e = launch_tile_field(f, tmp, V, np, pb, s);
            if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, (size_t)np * V * pb, hipMemcpyDeviceToDevice, s);
        };
        tile(c->f.Uk[0], 36, 16);
        tile(c->f.Ti[0], 36, 16);
        tile(c->f.Tp[0], 36, 16);
        tile(c->f.Tc[0], 36, 16);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return WD_EHIP;
        c->g.vt |= kCoefTiled;
    }
    WD_TRY_HIP(hipStreamSynchronize(s));
    c->kappa = kappa;
    c->csw = csw;
    c->jacobi_kind = jacobi_kind;
    c->have_params = true;
    return WD_OK;
}

int wd_get_clover(wd_ctx* c, int which, double* out_host) {
    if (!c || !out_host || (which != 0 && which != 1)) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    const size_t V = c->g.V;
    std::vector<double2> packed(36 * V);
    const void* src = which == 0 ? (const void*)c->f.T : c->f.Ti[0];
    WD_TRY_HIP(hipMemcpyAsync(packed.data(), src, 36 * V * 16, hipMemcpyDeviceToHost, c->stream));
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    double2* out = (double2*)out_host;
    // T^{-1} is one of the hop kernels' fields, kept tiled when the lattice allows it
    const bool tiled = which == 1 && (c->g.vt & kCoefTiled);
    auto at = [&](size_t plane, size_t s) -> const double2& {
        return tiled ? packed[((s / 64) * 36 + plane) * 64 + s % 64] : packed[plane * V + s];
    };
    for (size_t s = 0; s < V; ++s)
        for (int ch = 0; ch < 2; ++ch) {
            double2* m = out + (s * 2 + ch) * 36;
            for (int i = 0; i < 3; ++i) {
                const double2 d = at(ch * 18 + i, s);
                m[(2 * i) * 6 + 2 * i] = make_double2(d.x, 0.0);
                m[(2 * i + 1) * 6 + 2 * i + 1] = make_double2(d.y, 0.0);
            }
            for (int i = 0; i < 6; ++i)
                for (int j = i + 1; j < 6; ++j) {
                    const double2 o = at(ch * 18 + 3 + herm_index(i, j), s);
                    m[i * 6 + j] = o;
                    m[j * 6 + i] = make_double2(o.x, -o.y);
                }
        }
    return WD_OK;
}

int wd_set_layout(wd_ctx* c, int layout) {
    if (!c || (layout != WD_LAYOUT_STANDARD && layout != WD_LAYOUT_TILED)) return WD_EINVAL;
    if (layout == WD_LAYOUT_TILED && !tiled_ok(c->g)) return WD_EINVAL;
    c->g.vt = (c->g.vt & ~kVecTiled) | (layout == WD_LAYOUT_TILED ? kVecTiled : 0);
    return WD_OK;
}

int wd_apply(wd_ctx* c, const void* X, void* Y, int L, int prec) {
    if (!c || !X || !Y) return WD_EINVAL;
    if (L < 1 || L > c->max_L || check_prec(prec)) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    if (overlap(X, Y, block_elems(c, L) * 16)) return WD_EINVAL;
    if (prec == WD_F64) {
        WD_TRY_HIP(launch_apply_A(c, (const double2*)X, (double2*)Y, L, c->stream));
    } else {
        int r = lowp_ensure(c);
        if (r) return r;
        WD_TRY_HIP(launch_apply_A_lowp(c, (const double2*)X, (double2*)Y, L, (Prec)prec, c->stream));
    }
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

int jacobi_precond(wd_ctx* c, const void* R, void* Z, int L, int j, int prec) {
    if (!c || !R || !Z) return WD_EINVAL;
    if (L < 1 || L > c->max_L || j < 0 || (check_prec(prec) && !coef_prec(prec))) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    if (overlap(R, Z, block_elems(c, L) * 16)) return WD_EINVAL;
    if (coef_prec(prec)) {
        WD_TRY_HIP(launch_jacobi_coef(c, (const double2*)R, (double2*)Z, L, j, coef_of(prec), c->stream));
        WD_TRY_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }
    if (prec != WD_F64) {
        int r = lowp_ensure(c);
        if (r) return r;
    }
    WD_TRY_HIP(launch_jacobi(c, (const double2*)R, (double2*)Z, L, j, (Prec)prec, c->stream));
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

int wd_hop_repeat(wd_ctx* c, const void* X, const void* R, void* Y, int L, int mode, int prec, int nrep) {
    if (!c || !X || !Y || (mode == 1 && !R)) return WD_EINVAL;
    if (L < 1 || L > c->max_L || nrep < 1 || (mode != 0 && mode != 1)) return WD_EINVAL;
    if (check_prec(prec) && !(coef_prec(prec) && mode == 1)) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    const size_t bytes = block_elems(c, L) * 16;
    if (overlap(X, Y, bytes) || (mode == 1 && overlap(R, Y, bytes))) return WD_EINVAL;
    if (coef_prec(prec)) {
        for (int i = 0; i < nrep; ++i)
            WD_TRY_HIP(launch_sweep_coef(c, (const double2*)X, (const double2*)R, (double2*)Y, L, coef_of(prec),
                                         c->stream));
        WD_TRY_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }
    if (prec != WD_F64) {
        int r = lowp_ensure(c);
        if (r) return r;
        WD_TRY_HIP(launch_hop_repeat_lowp(c, (const double2*)X, (const double2*)R, (double2*)Y, L, mode, (Prec)prec,
                                          nrep, c->stream));
        WD_TRY_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }
    for (int i = 0; i < nrep; ++i) {
        if (mode == 0)
            WD_TRY_HIP(launch_apply_A(c, (const double2*)X, (double2*)Y, L, c->stream));
        else
            WD_TRY_HIP(launch_sweep_f64(c, (const double2*)X, (const double2*)R, (double2*)Y, L, c->stream));
    }
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

int wd_block_gram(wd_ctx* c, const void* P, const void* Q, int L, void* C) {
    if (!c || !P || !Q || !C) return WD_EINVAL;
    if (L < 1 || L > c->max_L) return WD_EINVAL;
    const size_t N = (size_t)12 * c->g.V;
    const int nb = gram_blocks(N);
    WD_TRY_HIP(launch_gram_partials((const double2*)P, (const double2*)Q, N, L, c->partial, nb, c->stream));
    WD_TRY_HIP(launch_reduce_gram(c->partial, nb, L, (double2*)C, c->stream));
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

int wd_small_solve(wd_ctx* c, const void* M, const void* RHS, int L, void* Z) {
    if (!c || !M || !RHS || !Z) return WD_EINVAL;
    if (L < 1 || L > WD_MAX_L) return WD_EINVAL;
    SmallLayout s = small_layout(c);
    WD_TRY_HIP(launch_small_solve((const double2*)M, (const double2*)RHS, L, (double2*)Z, &s.ctl->status,
                                  c->stream));
    int st = 0;
    WD_TRY_HIP(hipMemcpyAsync(&st, &s.ctl->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return st ? WD_BREAKDOWN : WD_OK;
}

int wd_learned_pairs(wd_ctx* c, const void* B, const void* X, const void* Xsnap, int n, int L, void* Rp, void* Ep) {
    if (!c || !B || !X || !Xsnap || !Rp || !Ep || n < 1 || L < 1 || L > c->max_L) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    const size_t N = (size_t)12 * c->g.V, blk = N * L * 16, all = blk * n;
    const void* in[3] = {B, X, Xsnap};
    const size_t in_n[3] = {blk, blk, all};
    for (int i = 0; i < 3; ++i)
        if (ranges_overlap(in[i], in_n[i], Rp, all) || ranges_overlap(in[i], in_n[i], Ep, all)) return WD_EINVAL;
    if (ranges_overlap(Rp, all, Ep, all)) return WD_EINVAL;
    for (int k = 0; k < n; ++k) {
        const double2* xs = (const double2*)Xsnap + (size_t)k * N * L;
        double2* r = (double2*)Rp + (size_t)k * N * L;
        double2* e = (double2*)Ep + (size_t)k * N * L;
        WD_TRY_HIP(launch_apply_A(c, xs, c->ws[WS_T1], L, c->stream));                  // A X_k
        WD_TRY_HIP(launch_axpby_block((const double2*)B, c->ws[WS_T1], r, N * L, c->stream));  // B - A X_k
        WD_TRY_HIP(launch_axpby_block((const double2*)X, xs, e, N * L, c->stream));      // e = X - X_k
    }
    WD_TRY_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

// ---------------------------------------------------------------------------
// Preconditioned block BiCGGR (and the block BiCGSTAB foil)
// ---------------------------------------------------------------------------
namespace {

struct Solver {
    wd_ctx* c;
    int L;      // width of the block being solved
    int Ltot;   // columns of the whole solve
    size_t N;
    int nb;
    int j;
    int precond;
    Prec pin;
    int coef = 0;  // Jacobi with FP64 iterates: 0, or the storage (Prec) of its links and A_D^{-1}
    SmallLayout sl;
    SolverBufs bufs;
    long long mvm_paper = 0, mvm_actual = 0;  // operator applications, summed over columns
    double bytes = 0.0;                       // algorithmic HBM bytes of the launched kernels

    double2* ws(int i) { return c->ws[i]; }
    // one pass over n N x L blocks
    void blocks(double n) { bytes += n * 192.0 * L * c->g.V; }

    int applyM(const double2* in, double2* out) {
        if (precond == WD_PRECOND_LEARNED) {
            // scratch: the Jacobi temporary and T1, both idle while M is applied (the recovery
            // point and a cycle's best iterate live in T2)
            WD_TRY_HIP(launch_learned(c, in, out, L, pin, c->ws[WS_JT], c->ws[WS_T1], c->stream));
            mvm_actual += (long long)WD_LEARNED_LAYERS * L;
            // three layers: links read once per site, one input and one output block each
            // (FP32: 288 + 192 L B per site, with the first input and last output in FP64)
            bytes += pin == Prec::F64 ? (double)c->g.V * 3 * (576.0 + 384.0 * L)
                                      : (double)c->g.V * (3 * (288.0 + 192.0 * L) + 2 * 96.0 * L);
            return WD_OK;
        }
        if (precond == WD_PRECOND_JACOBI && j > 0 && coef) {
            WD_TRY_HIP(launch_jacobi_coef(c, in, out, L, j, (Prec)coef, c->stream));
            mvm_actual += (long long)(j - 1) * L;
            // FP64 vectors; A_D^{-1} (576 B per site in FP64) at 1/2 or 1/4, the links as two of
            // their three rows (384 B at FP64 size) at 1/2 or 1/4
            const double cs = coef == (int)Prec::F32 ? 0.5 : 0.25;
            bytes += (double)c->g.V * (576.0 * cs + 384.0 * L + (j - 1) * (960.0 * cs + 576.0 * L));
        } else if (precond == WD_PRECOND_JACOBI && j > 0 && pin != Prec::F64) {
            WD_TRY_HIP(launch_jacobi(c, in, out, L, j, pin, c->stream));
            mvm_actual += (long long)(j - 1) * L;
            // s: storage size relative to FP64.  The first sweep reads the FP64 right-hand side and
            // stores its rounded copy and G_1; the middle sweeps read and write storage format;
            // the last writes FP64 (j = 1: FP64 in, FP64 out).
            const double s = pin == Prec::F32 ? 0.5 : 0.25, Lf = L;
            const double coefs = 960.0 * s;  // two-row links and A_D^{-1}
            bytes += (double)c->g.V *
                     (j == 1 ? 576.0 * s + 384.0 * Lf
                             : (576.0 * s + 192.0 * Lf + 384.0 * Lf * s) + (j - 2) * (coefs + 576.0 * Lf * s) +
                                   (coefs + 384.0 * Lf * s + 192.0 * Lf));
        } else if (precond == WD_PRECOND_JACOBI && j > 0) {
            WD_TRY_HIP(launch_jacobi(c, in, out, L, j, pin, c->stream));
            mvm_actual += (long long)(j - 1) * L;
            bytes += (double)c->g.V * (bytes_first_sweep(L) + (j - 1) * bytes_sweep(L));
        } else {
            WD_TRY_HIP(launch_copy(out, in, N * L, c->stream));
            blocks(2);
        }
        mvm_paper += (long long)j * L;
        return WD_OK;
    }
    int applyA(const double2* in, double2* out, bool paper = true) {
        WD_TRY_HIP(launch_apply_A(c, in, out, L, c->stream));
        if (paper) mvm_paper += L;
        mvm_actual += L;
        bytes += (double)c->g.V * bytes_apply(L);
        return WD_OK;
    }
    int gram_into(const double2* P, const double2* Q, double2* C) {
        WD_TRY_HIP(launch_gram_partials(P, Q, N, L, c->partial, nb, c->stream));
        WD_TRY_HIP(launch_reduce_gram(c->partial, nb, L, C, c->stream));
        blocks(2);
        return WD_OK;
    }
    int copy(double2* dst, const double2* src) {
        WD_TRY_HIP(launch_copy(dst, src, N * L, c->stream));
        blocks(2);
        return WD_OK;
    }
    // squared column norms of an N x L block, on the host (synchronises)
    int norms(const double2* Rb, double* out) {
        blocks(1);
        return colnorms_host(c, Rb, L, out);
    }
    int fetch_ctl(Ctl* h) {
        WD_TRY_HIP(hipMemcpyAsync(h, sl.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
        WD_TRY_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }
};

// State of one solve: options, the whole block's column norms, and what the
// runs of all (sub-)blocks report.
struct Driver {
    Solver S;
    wd_solve_opts op{};
    double tol = 0.0;
    int max_iter = 0, max_restarts = 0, stag = 0, cycle_stag = 0;
    static constexpr int max_cycles = 200;
    double diverge_at = 0.0;
    double cycle_tol = -1.0;  // > 0: Krylov cycles of an inexact M
    int fb_j = 0;             // Jacobi steps of the FP64 fallback
    double bnorm[WD_MAX_L] = {};
    int iters = 0, total_iters = 0, restarts = 0, cycles = 0, snaps = 0, splits = 0, min_block = WD_MAX_L;
    bool fell_back = false;
    bool snap_untile = false;  // the solve runs tiled for a standard-layout caller: snapshots go back
    double cond_max = 0.0;
    long long snap_clock = 0;
    int hist_pos = 0;
    double true_rel[WD_MAX_L] = {}, rec_rel[WD_MAX_L] = {};

    void record(double res, double gap, double cond) {
        if (hist_pos < op.history_len) {
            if (op.history) op.history[hist_pos] = res;
            if (op.gap_history) op.gap_history[hist_pos] = gap;
            if (op.cond_history) op.cond_history[hist_pos] = cond;
        }
        ++hist_pos;
    }
    // largest per-column ||R - (B - A X)|| / ||b|| over the columns [col0, col0 + L) (diagnostic)
    int gap(const double2* B, const double2* X, const double2* R, int col0, double* out) {
        Solver& s = S;
        double2* T1 = s.ws(WS_T1);
        const size_t n = s.N * s.L;
        int r = s.applyA(X, T1, false);
        if (r) return r;
        WD_TRY_HIP(launch_axpby_block(B, T1, T1, n, s.c->stream));  // B - A X
        WD_TRY_HIP(launch_axpby_block(R, T1, T1, n, s.c->stream));  // R - (B - A X)
        s.blocks(6);
        double g2[WD_MAX_L];
        if ((r = s.norms(T1, g2))) return r;
        double m = 0.0;
        for (int i = 0; i < s.L; ++i) m = std::fmax(m, std::sqrt(g2[i]) / bnorm[col0 + i]);
        *out = m;
        return WD_OK;
    }
    // FP64 true residual of columns [col0, col0 + L); returns the largest
    int true_residual(const double2* B, const double2* X, int col0, double* tmax) {
        Solver& s = S;
        double2* T1 = s.ws(WS_T1);
        int r = s.applyA(X, T1, false);
        if (r) return r;
        WD_TRY_HIP(launch_axpby_block(B, T1, T1, s.N * s.L, s.c->stream));
        s.blocks(3);
        double tr2[WD_MAX_L];
        if ((r = s.norms(T1, tr2))) return r;
        *tmax = 0.0;
        for (int i = 0; i < s.L; ++i) {
            true_rel[col0 + i] = std::sqrt(tr2[i]) / bnorm[col0 + i];
            *tmax = std::fmax(*tmax, std::isfinite(true_rel[col0 + i]) ? true_rel[col0 + i] : INFINITY);
        }
        return WD_OK;
    }
};

constexpr int kCycleEnd = 100;  // internal run status: restart from X

// Solve the columns [col0, col0 + L) of the system; B and X point at the first
// of them.  Runs the block BiCGGR iteration, its Krylov cycles and FP64
// fallback for an inexact M, true-residual restarts and, after a failed FP64
// run, the recursive split of the block into halves.
int solve_block(Driver& D, const double2* B, double2* X, int col0, int L, bool use_x0) {
    Solver& S = D.S;
    wd_ctx* c = S.c;
    const size_t N = S.N;
    hipStream_t st = c->stream;
    S.L = L;
    if (L < D.min_block) D.min_block = L;
    const double* bnorm = D.bnorm + col0;
    double* rec_rel = D.rec_rel + col0;
    double2 *R = S.ws(WS_R), *Rt = S.ws(WS_RT), *P = S.ws(WS_P), *V = S.ws(WS_V), *W = S.ws(WS_W),
            *F = S.ws(WS_F), *G = S.ws(WS_G), *U = S.ws(WS_U), *Y = S.ws(WS_Y), *T1 = S.ws(WS_T1);
    double2* Xrec = S.ws(WS_T2);  // recovery point of a run (a cycle's best iterate when cycling)
    const bool whole = col0 == 0 && L == S.Ltot;
    Ctl* hc = reinterpret_cast<Ctl*>(c->host_ctl);
    int r = WD_OK;
    int status = WD_NOT_CONVERGED;
    for (;;) {
        ++D.cycles;
        const bool cycling = D.cycle_tol > 0.0;
        // ---- initialisation: R0 = B - A X0, P0 = R0, Rt0 = R0, F0 = M R0, V0 = W0 = A F0
        if (use_x0) {
            if ((r = S.applyA(X, T1))) return r;
            WD_TRY_HIP(launch_axpby_block(B, T1, R, N * L, st));
            S.blocks(3);
        } else {
            WD_TRY_HIP(launch_zero(X, N * L, st));
            S.blocks(1);
            if ((r = S.copy(R, B))) return r;
            S.mvm_paper += L;  // R0 = B - A X0 counts as one application (Table 1 convention)
        }
        if ((r = S.copy(P, R))) return r;
        if ((r = S.copy(Rt, R))) return r;
        if ((r = S.applyM(R, F))) return r;
        if ((r = S.applyA(F, W))) return r;
        if ((r = S.copy(V, W))) return r;
        if ((r = S.gram_into(Rt, R, S.sl.C_r))) return r;
        WD_TRY_HIP(launch_zero(reinterpret_cast<double2*>(S.sl.ctl), (sizeof(Ctl) + 15) / 16, st));
        double rn2[WD_MAX_L];
        if ((r = S.norms(R, rn2))) return r;
        double res = 0.0;
        for (int i = 0; i < L; ++i) {
            rec_rel[i] = std::sqrt(rn2[i]) / bnorm[i];
            res = std::fmax(res, rec_rel[i]);
        }
        if (!std::isfinite(res)) return WD_ENAN;
        D.record(res, 0.0, 0.0);
        int iters = 0;
        int run_status = WD_NOT_CONVERGED;
        const double res0 = res;
        double best = res, saved = res;
        int best_k = 0;
        // the recovery point starts as the run's initial X
        if (use_x0) {
            if ((r = S.copy(Xrec, X))) return r;
        } else {
            WD_TRY_HIP(launch_zero(Xrec, N * L, st));
            S.blocks(1);
        }
        if (res <= D.tol) run_status = WD_OK;
        for (int k = 0; run_status == WD_NOT_CONVERGED && k < D.max_iter; ++k) {
            // alpha and zeta; after the first iteration the P / V update of the previous one
            // has already left Rt^H V, Tr[W^H R] and Tr[W^H W] in the partial blocks
            if (k == 0) {
                WD_TRY_HIP(launch_gram1(Rt, V, W, R, N, L, c->partial, S.nb, st));
                S.blocks(4);
            }
            WD_TRY_HIP(launch_solve_alpha(c->partial, S.nb, L, S.bufs, st));
            // U = (P - zeta V) alpha ; G = M U ; Y = A G
            WD_TRY_HIP(launch_update_U(P, V, S.sl.zeta, S.sl.alpha, U, N, L, st));
            S.blocks(3);
            const long long mp = S.mvm_paper, ma = S.mvm_actual;
            if ((r = S.applyM(U, G))) return r;
            if ((r = S.applyA(G, Y))) return r;
            // X += zeta F + G ; R -= zeta W + Y ; Rt^H R_{k+1}, norms ; gamma
            WD_TRY_HIP(launch_update_XR_gram(X, R, F, G, W, Y, Rt, S.sl.zeta, N, L, c->partial, S.nb, st));
            S.blocks(9);
            WD_TRY_HIP(launch_solve_gamma(c->partial, S.nb, L, S.bufs, st));
            if ((r = S.fetch_ctl(hc))) return r;
            if (hc->status & 1) {  // alpha system singular: X and R were left unchanged
                S.mvm_paper = mp;
                S.mvm_actual = ma;
                run_status = WD_BREAKDOWN;
                break;
            }
            iters = k + 1;
            ++D.snap_clock;
            if (whole && D.snaps < D.op.snap_count && D.snap_clock % D.op.snap_every == 0) {
                double2* slot = (double2*)D.op.x_snap + (size_t)D.snaps * N * L;
                if (D.snap_untile)
                    WD_TRY_HIP(launch_retile(X, slot, c->g.V, L, false, st));
                else
                    WD_TRY_HIP(launch_copy(slot, X, N * L, st));
                S.blocks(2);
                ++D.snaps;
            }
            res = 0.0;
            bool nan = (hc->status & 4) != 0;
            for (int i = 0; i < L; ++i) {
                rec_rel[i] = std::sqrt(hc->norms[i]) / bnorm[i];
                if (!std::isfinite(rec_rel[i])) nan = true;
                res = std::fmax(res, rec_rel[i]);
            }
            const double cond = std::fmax(hc->cond[0], hc->cond[1]);
            D.cond_max = std::fmax(D.cond_max, cond);
            double gapv = 0.0;
            if (D.op.gap_history && (r = D.gap(B, X, R, col0, &gapv))) return r;
            D.record(res, gapv, cond);
            if (nan) {
                run_status = WD_ENAN;
                break;
            }
            if (res <= D.tol) {
                run_status = WD_OK;
                break;
            }
            if (cycling && res <= D.cycle_tol * res0) {
                run_status = kCycleEnd;
                break;
            }
            if (res > D.diverge_at) {
                run_status = WD_DIVERGED;
                break;
            }
            if (res < best) {
                best = res;
                best_k = k + 1;
                if (cycling && (r = S.copy(Xrec, X))) return r;
            } else if (k + 1 - best_k >= (cycling ? D.cycle_stag : D.stag)) {
                run_status = WD_STAGNATED;
                break;
            }
            if (!cycling && res < 0.1 * saved) {
                if ((r = S.copy(Xrec, X))) return r;
                saved = res;
            }
            // rank loss of the block: a singular gamma system, or a condition estimate past the limit
            if ((hc->status & 2) || (D.op.cond_limit > 0.0 && !(cond <= D.op.cond_limit))) {
                run_status = WD_BREAKDOWN;
                break;
            }
            // F = M R_{k+1} ; W = A F
            if ((r = S.applyM(R, F))) return r;
            if ((r = S.applyA(F, W))) return r;
            // P = R + U gamma ; V = W + Y gamma, with the next iteration's Gram products
            WD_TRY_HIP(launch_update_PV_gram(P, V, R, W, U, Y, S.sl.gamma, Rt, N, L, c->partial, S.nb, st));
            S.blocks(7);
        }
        D.iters = iters;
        D.total_iters += iters;
        // an inexact M whose cycle stalled, blew up or broke down.  Unless the caller turned the
        // fallback off, the solve starts again from X0 = 0 (so R~0 = R0 = B, as in a plain solve)
        // with the FP64 Jacobi preconditioner: restarted from the inexact iterate, FP64 block
        // BiCGGR close to the critical kappa can level off above a 1e-12 residual.  Without the
        // fallback X returns to the cycle's best iterate.
        if (cycling && (run_status == WD_STAGNATED || run_status == WD_DIVERGED || run_status == WD_BREAKDOWN ||
                        run_status == WD_NOT_CONVERGED)) {
            if (!D.op.no_fallback && run_status != WD_NOT_CONVERGED) {
                S.precond = D.fb_j > 0 ? WD_PRECOND_JACOBI : WD_PRECOND_NONE;
                S.j = D.fb_j;
                S.pin = Prec::F64;
                S.coef = 0;
                D.cycle_tol = -1.0;
                D.fell_back = true;
                use_x0 = false;
                continue;
            }
            if ((r = S.copy(X, Xrec))) return r;
        }
        if (run_status == kCycleEnd && D.cycles < D.max_cycles) {
            use_x0 = true;
            continue;
        }
        if (run_status == kCycleEnd) run_status = WD_NOT_CONVERGED;
        status = run_status;
        if (status == WD_ENAN) return WD_ENAN;
        if (!cycling && status != WD_OK) {
            // a diverged or stagnated FP64 run goes back to its recovery point unless the last
            // iterate is at least as good (a breakdown stops on a sound iterate; at max_iter the
            // last iterate is returned)
            if ((status == WD_DIVERGED || status == WD_STAGNATED) && res > saved && (r = S.copy(X, Xrec)))
                return r;
            if (status != WD_NOT_CONVERGED) {
                if (S.precond == WD_PRECOND_LEARNED && !D.op.no_fallback) {
                    // a learned M that fails is replaced by the FP64 Jacobi preconditioner, from X = 0
                    S.precond = D.fb_j > 0 ? WD_PRECOND_JACOBI : WD_PRECOND_NONE;
                    S.j = D.fb_j;
                    S.pin = Prec::F64;
                    S.coef = 0;
                    D.fell_back = true;
                    use_x0 = false;
                    continue;
                }
                if (L > 1 && !D.op.no_split) {
                    // Sec. 3.3's remedy, a block with fewer columns: each half of the block
                    // is solved on its own from the current X (recursively)
                    ++D.splits;
                    const int La = (L + 1) / 2;
                    const int ra = solve_block(D, B, X, col0, La, true);
                    if (ra < 0) return ra;
                    const int rb = solve_block(D, B + (size_t)La * N, X + (size_t)La * N, col0 + La, L - La, true);
                    if (rb < 0) return rb;
                    S.L = L;
                    return ra != WD_OK ? ra : rb;
                }
                if (D.restarts < D.max_restarts) {
                    ++D.restarts;
                    use_x0 = true;
                    continue;
                }
            }
        }
        // ---- true residual ||B - A X|| / ||B|| in FP64
        double tmax = 0.0;
        if ((r = D.true_residual(B, X, col0, &tmax))) return r;
        if (status == WD_OK && tmax > D.tol) {
            if (D.restarts < D.max_restarts) {
                ++D.restarts;
                use_x0 = true;
                continue;
            }
            status = WD_NOT_CONVERGED;
        }
        break;
    }
    return status;
}

// Block BiCGSTAB on the whole block (the foil): same initialisation, stopping
// rule, recovery point and true-residual restarts as above.
int stab_solve(Driver& D, const double2* B, double2* X, bool use_x0) {
    Solver& S = D.S;
    wd_ctx* c = S.c;
    const size_t N = S.N;
    const int L = S.L;
    hipStream_t st = c->stream;
    D.min_block = L;
    const SmallLayout& sl = S.sl;
    double2 *R = S.ws(WS_R), *Rt = S.ws(WS_RT), *P = S.ws(WS_P), *V = S.ws(WS_V), *Ph = S.ws(WS_F),
            *Sb = S.ws(WS_U), *Sh = S.ws(WS_G), *T = S.ws(WS_Y), *T1 = S.ws(WS_T1);
    double2* Xrec = S.ws(WS_T2);
    // L x L matrices: Rt^H R, Rt^H V, alpha, beta, Rt^H T, T^H S, T^H T; omega in the scalars
    double2 *C_r = sl.mats[0], *C_v = sl.mats[1], *alpha = sl.mats[2], *beta = sl.mats[3], *C_t = sl.mats[4],
            *C_ts = sl.mats[5], *C_tt = sl.mats[6], *omega = sl.zeta + 4;
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0), zero = make_double2(0.0, 0.0);
    int* flags = &sl.ctl->status;
    Ctl* hc = reinterpret_cast<Ctl*>(c->host_ctl);
    int r = WD_OK;
    int status = WD_NOT_CONVERGED;
    for (;;) {
        ++D.cycles;
        if (use_x0) {
            if ((r = S.applyA(X, T1))) return r;
            WD_TRY_HIP(launch_axpby_block(B, T1, R, N * L, st));
            S.blocks(3);
        } else {
            WD_TRY_HIP(launch_zero(X, N * L, st));
            S.blocks(1);
            if ((r = S.copy(R, B))) return r;
            S.mvm_paper += L;
        }
        if ((r = S.copy(P, R))) return r;
        if ((r = S.copy(Rt, R))) return r;
        if ((r = S.gram_into(Rt, R, C_r))) return r;
        WD_TRY_HIP(launch_zero(reinterpret_cast<double2*>(sl.ctl), (sizeof(Ctl) + 15) / 16, st));
        double rn2[WD_MAX_L];
        if ((r = S.norms(R, rn2))) return r;
        double res = 0.0;
        for (int i = 0; i < L; ++i) {
            D.rec_rel[i] = std::sqrt(rn2[i]) / D.bnorm[i];
            res = std::fmax(res, D.rec_rel[i]);
        }
        if (!std::isfinite(res)) return WD_ENAN;
        D.record(res, 0.0, 0.0);
        int iters = 0, run_status = WD_NOT_CONVERGED;
        double best = res, saved = res;
        int best_k = 0;
        if (use_x0) {
            if ((r = S.copy(Xrec, X))) return r;
        } else {
            WD_TRY_HIP(launch_zero(Xrec, N * L, st));
            S.blocks(1);
        }
        if (res <= D.tol) run_status = WD_OK;
        for (int k = 0; run_status == WD_NOT_CONVERGED && k < D.max_iter; ++k) {
            if ((r = S.applyM(P, Ph))) return r;                     // Ph = M P
            if ((r = S.applyA(Ph, V))) return r;                     // V = A Ph
            if ((r = S.gram_into(Rt, V, C_v))) return r;             // Rt^H V
            WD_TRY_HIP(launch_small_solve_scaled(C_v, C_r, L, one, alpha, flags, 1, &sl.ctl->cond[0], st));
            WD_TRY_HIP(launch_block_comb(Sb, R, nullptr, V, nullptr, alpha, one, zero, mone, zero, nullptr, 0, N, L,
                                         st));                       // S = R - V alpha
            S.blocks(3);
            if ((r = S.applyM(Sb, Sh))) return r;                    // Sh = M S
            if ((r = S.applyA(Sh, T))) return r;                     // T = A Sh
            if ((r = S.gram_into(T, Sb, C_ts))) return r;
            if ((r = S.gram_into(T, T, C_tt))) return r;
            WD_TRY_HIP(launch_stab_omega(C_ts, C_tt, L, omega, flags, 2, st));
            // X += Ph alpha + omega Sh ; R = S - omega T
            WD_TRY_HIP(launch_block_comb(X, X, Sh, Ph, nullptr, alpha, one, one, one, zero, omega, 2, N, L, st));
            WD_TRY_HIP(launch_block_comb(R, Sb, T, nullptr, nullptr, nullptr, one, mone, zero, zero, omega, 2, N, L,
                                         st));
            S.blocks(4 + 3);
            WD_TRY_HIP(launch_colnorms(R, N, L, c->partial, S.nb, sl.ctl->norms, st));
            S.blocks(1);
            if ((r = S.fetch_ctl(hc))) return r;
            iters = k + 1;
            res = 0.0;
            bool nan = false;
            for (int i = 0; i < L; ++i) {
                D.rec_rel[i] = std::sqrt(hc->norms[i]) / D.bnorm[i];
                if (!std::isfinite(D.rec_rel[i])) nan = true;
                res = std::fmax(res, D.rec_rel[i]);
            }
            const double cond = hc->cond[0];
            D.cond_max = std::fmax(D.cond_max, cond);
            double gapv = 0.0;
            if (D.op.gap_history && (r = D.gap(B, X, R, 0, &gapv))) return r;
            D.record(res, gapv, cond);
            if (nan) {
                run_status = WD_ENAN;
                break;
            }
            if (hc->status & 3) {  // singular Rt^H V or zero Tr[T^H T]
                run_status = WD_BREAKDOWN;
                break;
            }
            if (res <= D.tol) {
                run_status = WD_OK;
                break;
            }
            if (res > D.diverge_at) {
                run_status = WD_DIVERGED;
                break;
            }
            if (res < best) {
                best = res;
                best_k = k + 1;
            } else if (k + 1 - best_k >= D.stag) {
                run_status = WD_STAGNATED;
                break;
            }
            if (res < 0.1 * saved) {
                if ((r = S.copy(Xrec, X))) return r;
                saved = res;
            }
            if (D.op.cond_limit > 0.0 && !(cond <= D.op.cond_limit)) {
                run_status = WD_BREAKDOWN;
                break;
            }
            // beta: (Rt^H V) beta = -Rt^H T ; P = R + (P - omega V) beta ; Rt^H R_{k+1}
            if ((r = S.gram_into(Rt, T, C_t))) return r;
            WD_TRY_HIP(launch_small_solve_scaled(C_v, C_t, L, mone, beta, flags, 1, nullptr, st));
            WD_TRY_HIP(launch_block_comb(P, R, nullptr, P, V, beta, one, zero, one, mone, omega, 8, N, L, st));
            S.blocks(4);
            if ((r = S.gram_into(Rt, R, C_r))) return r;
        }
        D.iters = iters;
        D.total_iters += iters;
        status = run_status;
        if (status == WD_ENAN) return WD_ENAN;
        if (status != WD_OK) {
            if ((status == WD_DIVERGED || status == WD_STAGNATED) && res > saved && (r = S.copy(X, Xrec)))
                return r;
            if (status != WD_NOT_CONVERGED && D.restarts < D.max_restarts) {
                ++D.restarts;
                use_x0 = true;
                continue;
            }
        }
        double tmax = 0.0;
        if ((r = D.true_residual(B, X, 0, &tmax))) return r;
        if (status == WD_OK && tmax > D.tol) {
            if (D.restarts < D.max_restarts) {
                ++D.restarts;
                use_x0 = true;
                continue;
            }
            status = WD_NOT_CONVERGED;
        }
        break;
    }
    return status;
}

void fill_info(const Driver& D, int rc, double secs, int L, wd_solve_info* info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->status = rc;
    info->iterations = D.iters;
    info->total_iterations = D.total_iters;
    info->restarts = D.restarts;
    info->cycles = D.cycles;
    info->fallback = D.fell_back ? 1 : 0;
    info->snapshots = D.snaps;
    info->mvm_paper = D.S.mvm_paper / L;
    info->mvm_actual = D.S.mvm_actual / L;
    info->seconds = secs;
    info->bytes_alg = D.S.bytes;
    for (int i = 0; i < L; ++i) {
        info->true_residual[i] = D.true_rel[i];
        info->recursive_residual[i] = D.rec_rel[i];
    }
    info->cond_max = D.cond_max;
    info->splits = D.splits;
    info->min_block = D.min_block;
}

// Argument checks and set-up shared by both solvers; returns 0 or an error.
int solve_setup(wd_ctx* c, const void* Bv, void* Xv, int L, double tol, const wd_solve_opts* o, bool stab,
                Driver& D) {
    if (!c || !Bv || !Xv) return WD_EINVAL;
    if (L < 1 || L > c->max_L || !(tol > 0.0)) return WD_EINVAL;
    if (!c->have_params) return WD_ESTATE;
    wd_solve_opts& op = D.op;
    if (o) op = *o;
    if (op.precond != WD_PRECOND_NONE && op.precond != WD_PRECOND_JACOBI && op.precond != WD_PRECOND_LEARNED)
        return WD_EINVAL;
    if (op.j < 0 || (check_prec(op.prec_inner) && !coef_prec(op.prec_inner))) return WD_EINVAL;
    if (op.snap_count < 0 || (op.snap_count > 0 && (!op.x_snap || op.snap_every < 1))) return WD_EINVAL;
    if (op.history_len < 0) return WD_EINVAL;
    if (stab && (op.precond == WD_PRECOND_LEARNED || op.prec_inner != WD_F64 || op.snap_count > 0))
        return WD_EINVAL;
    if (op.precond == WD_PRECOND_LEARNED) {
        if (op.prec_inner == WD_BF16 || coef_prec(op.prec_inner)) return WD_EINVAL;
        if (!c->have_theta) return WD_ESTATE;
        int r0 = learned_ensure(c);
        if (r0) return r0;
    }
    const size_t N = (size_t)12 * c->g.V;
    const size_t blk_bytes = N * L * 16;
    if (overlap(Bv, Xv, blk_bytes)) return WD_EINVAL;
    if (op.snap_count > 0 && (ranges_overlap(op.x_snap, blk_bytes * op.snap_count, Bv, blk_bytes) ||
                              ranges_overlap(op.x_snap, blk_bytes * op.snap_count, Xv, blk_bytes)))
        return WD_EINVAL;
    if ((op.prec_inner == WD_F32 || op.prec_inner == WD_BF16) && op.precond == WD_PRECOND_JACOBI) {
        int r = lowp_ensure(c);
        if (r) return r;
    }
    // FP64 fallback for an inexact M whose cycles stall: Jacobi in FP64 with the caller's j (M = I if 0)
    D.fb_j = op.j;
    if (op.precond != WD_PRECOND_JACOBI) op.j = 0;
    D.tol = tol;
    D.max_iter = op.max_iter > 0 ? op.max_iter : 5000;
    D.max_restarts = op.max_restarts >= 0 ? op.max_restarts : 3;
    D.stag = op.stagnate_window > 0 ? op.stagnate_window : 200;
    D.cycle_stag = op.stagnate_window > 0 ? op.stagnate_window : 20;  // no-improvement limit of a cycle
    D.diverge_at = op.diverge_at > 0 ? op.diverge_at : 1e2;
    // Krylov cycles for an inexact M (low-precision storage of the Jacobi preconditioner)
    const bool inexact_M = (op.prec_inner == WD_F32 || op.prec_inner == WD_BF16) &&
                           (op.precond == WD_PRECOND_LEARNED || (op.precond == WD_PRECOND_JACOBI && op.j > 0));
    D.cycle_tol = op.cycle_tol;
    if (D.cycle_tol == 0.0) D.cycle_tol = inexact_M ? (op.prec_inner == WD_F32 ? 1e-4 : 1e-1) : -1.0;
    Solver& S = D.S;
    S.c = c;
    S.L = L;
    S.Ltot = L;
    S.N = N;
    S.nb = gram_blocks(N);
    S.j = op.j;
    S.precond = op.precond;
    S.coef = coef_prec(op.prec_inner) ? (int)coef_of(op.prec_inner) : 0;
    S.pin = S.coef ? Prec::F64 : (Prec)op.prec_inner;
    S.sl = small_layout(c);
    S.bufs = SolverBufs{S.sl.C_r,       S.sl.C_rn,         S.sl.alpha,          S.sl.gamma,
                        S.sl.zeta,      S.sl.ctl->norms,   &S.sl.ctl->status,   S.sl.ctl->cond};
    return WD_OK;
}

// The two blocks a solve in the tiled layout needs for a caller of the standard
// one, allocated on first use (a failed allocation is tried again next time).
int tiled_ensure(wd_ctx* c) {
    for (auto& b : c->tb) {
        if (b) continue;
        int r = dev_alloc((void**)&b, block_elems(c, c->max_L) * 16);
        if (r) return r;
    }
    return WD_OK;
}

int solve_common(wd_ctx* c, const void* Bv, void* Xv, int L, double tol, const wd_solve_opts* o,
                 wd_solve_info* info, bool stab) {
    Driver D;
    int rc = solve_setup(c, Bv, Xv, L, tol, o, stab, D);
    if (rc) return rc;  // argument errors: nothing modified
    const auto t0 = std::chrono::steady_clock::now();
    const double2* B = (const double2*)Bv;
    double2* X = (double2*)Xv;
    // A caller of the standard layout gets the solve in the tiled one (its stencils run
    // faster): B and X are copied into the tiled layout here, X back at the end and every
    // snapshot as it is taken; without the two blocks of memory the solve stays in the
    // standard layout.
    const bool retile = !(c->g.vt & kVecTiled) && tiled_ok(c->g) && tiled_ensure(c) == WD_OK;
    D.snap_untile = retile;
    rc = hipStreamSynchronize(c->stream) == hipSuccess ? WD_OK : WD_EHIP;
    if (rc == WD_OK && retile) {
        if (launch_retile(B, c->tb[0], c->g.V, L, true, c->stream) != hipSuccess ||
            (D.op.use_x0 && launch_retile(X, c->tb[1], c->g.V, L, true, c->stream) != hipSuccess))
            rc = WD_EHIP;
        D.S.blocks(D.op.use_x0 ? 4 : 2);
        B = c->tb[0];
        X = c->tb[1];
        c->g.vt |= kVecTiled;
    }
    if (rc == WD_OK) {
        double bn2[WD_MAX_L];
        rc = D.S.norms(B, bn2);
        for (int i = 0; i < L && rc == WD_OK; ++i) {
            if (!std::isfinite(bn2[i])) rc = WD_ENAN;
            else if (bn2[i] == 0.0) rc = WD_EINVAL;
            else D.bnorm[i] = std::sqrt(bn2[i]);
        }
    }
    const bool ran = rc == WD_OK;
    if (ran) rc = stab ? stab_solve(D, B, X, D.op.use_x0 != 0) : solve_block(D, B, X, 0, L, D.op.use_x0 != 0);
    if (retile) {
        // X back into the caller's layout, whatever the outcome of the iteration
        c->g.vt &= ~kVecTiled;
        if (ran) {
            if (launch_retile(X, (double2*)Xv, c->g.V, L, false, c->stream) != hipSuccess && rc >= 0) rc = WD_EHIP;
            D.S.blocks(2);
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc >= 0) rc = WD_EHIP;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(D, rc, secs, L, info);
    return rc;
}

}  // namespace

int bbicggr_solve(wd_ctx* c, const void* Bv, void* Xv, int L, double tol, const wd_solve_opts* o,
                  wd_solve_info* info) {
    return solve_common(c, Bv, Xv, L, tol, o, info, false);
}

int bbicgstab_solve(wd_ctx* c, const void* Bv, void* Xv, int L, double tol, const wd_solve_opts* o,
                    wd_solve_info* info) {
    return solve_common(c, Bv, Xv, L, tol, o, info, true);
}

}  // extern "C"
