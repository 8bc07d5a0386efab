// Tall-skinny block kernels of the outer block BiCGGR iteration (Sec. 2,
// algorithm box): the L x L products Rt_0^H V_k and Rt_0^H R_{k+1}, the
// traces Tr[W^H R] and Tr[W^H W], column norms, the fused updates
//   U = (P - zeta V) alpha,   X += zeta F + G,   R -= zeta W + Y,
//   P = R + U gamma,  V = W + Y gamma,
// and the FP64 LU solves of the L x L systems for alpha and gamma.
//
// The Gram products are dense contractions over N rows and run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64): lane l of a wavefront loads column
// l % 16 of 4 consecutive rows (row group l / 16); the same lane data feeds
// both MFMA operands, so one instruction accumulates sum_k conj(P[k,i]) Q[k,j]
// over 4 rows into a 16 x 16 tile (L <= 16).  Complex products take four real
// MFMAs.  Reductions run in two passes with a fixed order (per-workgroup
// partials, then one workgroup), so results are deterministic.
#include "wd_internal.h"

namespace wd {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kWG = 256;         // threads per workgroup of the row kernels
constexpr int kPStride = 272;    // complex entries per partial block: 16x16 tile + 16 extras
constexpr int kMaxPartial = 512;
// 4-row groups per wavefront and loop trip in the Gram kernels: eight keep 8 (k_gram) or
// 32 (k_gram1) loads of each lane in flight
constexpr int kRG = 8;

struct GramAcc {
    dbl4 re, im;
};

__device__ __forceinline__ void gram_zero(GramAcc& a) {
    a.re = dbl4{0.0, 0.0, 0.0, 0.0};
    a.im = dbl4{0.0, 0.0, 0.0, 0.0};
}

// acc += conj(a)^T b over the 4 rows held by the wavefront (a, b: this lane's element)
__device__ __forceinline__ void gram_step(GramAcc& acc, cx<double> a, cx<double> b) {
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, acc.re, 0, 0, 0);
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, acc.re, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, acc.im, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.re, acc.im, 0, 0, 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum the per-wave 16x16 tiles of the workgroup and write the partial tile.
// Output layout of v_mfma_f64_16x16x4f64 (measured): lane l holds
// D[l/16 + 4 v][l % 16] in accumulator element v = 0..3.
__device__ __forceinline__ void gram_store(const GramAcc& acc, double2* __restrict__ out, double2* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = lane & 15, rg = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) sh[w * 256 + (rg + 4 * v) * 16 + j] = make_double2(acc.re[v], acc.im[v]);
    __syncthreads();
    const int e = threadIdx.x;  // kWG == 256 entries
    double2 s = sh[e];
#pragma unroll
    for (int q = 1; q < kWG / 64; ++q) {
        s.x += sh[q * 256 + e].x;
        s.y += sh[q * 256 + e].y;
    }
    out[e] = s;
}

// Per-column squared norms held per lane (column = lane % 16) -> extras[0..15]
__device__ __forceinline__ void colsum_store(double v, double2* __restrict__ out, double* shd) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 16) shd[w * 16 + lane] = v;
    __syncthreads();
    if (threadIdx.x < 16) {
        double s = 0.0;
        for (int q = 0; q < kWG / 64; ++q) s += shd[q * 16 + threadIdx.x];
        out[256 + threadIdx.x] = make_double2(s, 0.0);
    }
}

struct RowRange {
    size_t r0, r1;
};
__device__ __forceinline__ RowRange block_rows(size_t N, int nb) {
    const size_t per = ((N + nb - 1) / nb + 63) / 64 * 64;
    const size_t r0 = (size_t)blockIdx.x * per;
    return {r0, r0 + per < N ? r0 + per : N};
}

// ---- plain Gram P^H Q
__global__ void __launch_bounds__(kWG) k_gram(const double2* __restrict__ P, const double2* __restrict__ Q, size_t N,
                                              int L, double2* __restrict__ partial, int nb) {
    __shared__ double2 sh[kWG / 64 * 256];
    const RowRange rr = block_rows(N, nb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, q = lane >> 4;
    const bool colok = col < L;
    GramAcc acc;
    gram_zero(acc);
    for (size_t n0 = rr.r0 + 4 * kRG * w; n0 < rr.r1; n0 += 4 * kRG * (kWG / 64)) {
        cx<double> a[kRG], b[kRG];
#pragma unroll
        for (int r = 0; r < kRG; ++r) {
            const size_t n = n0 + 4 * r + q;
            const bool ok = colok && n < rr.r1;
            a[r] = ok ? StF64::ld(P, (size_t)col * N + n) : cx<double>{0.0, 0.0};
            b[r] = ok ? StF64::ld(Q, (size_t)col * N + n) : cx<double>{0.0, 0.0};
        }
#pragma unroll
        for (int r = 0; r < kRG; ++r) gram_step(acc, a[r], b[r]);
    }
    gram_store(acc, partial + (size_t)blockIdx.x * kPStride, sh);
}

// ---- Gram1: Rt^H V (tile), Tr[W^H R] (extra 0), Tr[W^H W] (extra 1)
__global__ void __launch_bounds__(kWG) k_gram1(const double2* __restrict__ Rt, const double2* __restrict__ V,
                                               const double2* __restrict__ W, const double2* __restrict__ R, size_t N,
                                               int L, double2* __restrict__ partial, int nb) {
    __shared__ double2 sh[kWG / 64 * 256];
    const RowRange rr = block_rows(N, nb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, q = lane >> 4;
    const bool colok = col < L;
    GramAcc acc;
    gram_zero(acc);
    double twr_re = 0, twr_im = 0, tww = 0;
    for (size_t n0 = rr.r0 + 4 * kRG * w; n0 < rr.r1; n0 += 4 * kRG * (kWG / 64)) {
        cx<double> a[kRG], b[kRG], ww[kRG], rv[kRG];
#pragma unroll
        for (int r = 0; r < kRG; ++r) {
            const size_t n = n0 + 4 * r + q;
            const bool ok = colok && n < rr.r1;
            const size_t idx = (size_t)col * N + n;
            a[r] = ok ? StF64::ld(Rt, idx) : cx<double>{0.0, 0.0};
            b[r] = ok ? StF64::ld(V, idx) : cx<double>{0.0, 0.0};
            ww[r] = ok ? StF64::ld(W, idx) : cx<double>{0.0, 0.0};
            rv[r] = ok ? StF64::ld(R, idx) : cx<double>{0.0, 0.0};
        }
#pragma unroll
        for (int r = 0; r < kRG; ++r) {
            gram_step(acc, a[r], b[r]);
            const cx<double> p = cmulc(ww[r], rv[r]);
            twr_re += p.re;
            twr_im += p.im;
            tww += ww[r].re * ww[r].re + ww[r].im * ww[r].im;
        }
    }
    double2* out = partial + (size_t)blockIdx.x * kPStride;
    gram_store(acc, out, sh);
    __syncthreads();
    double* shd = reinterpret_cast<double*>(sh);
    twr_re = wave_sum(twr_re);
    twr_im = wave_sum(twr_im);
    tww = wave_sum(tww);
    if (lane == 0) {
        shd[w * 3 + 0] = twr_re;
        shd[w * 3 + 1] = twr_im;
        shd[w * 3 + 2] = tww;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0, a1 = 0, a2 = 0;
        for (int q2 = 0; q2 < kWG / 64; ++q2) {
            a0 += shd[q2 * 3 + 0];
            a1 += shd[q2 * 3 + 1];
            a2 += shd[q2 * 3 + 2];
        }
        out[256] = make_double2(a0, a1);
        out[257] = make_double2(a2, 0.0);
    }
}

// ---- column norms only (extras)
__global__ void __launch_bounds__(kWG) k_colnorms(const double2* __restrict__ R, size_t N, int L,
                                                  double2* __restrict__ partial, int nb) {
    __shared__ double shd[kWG / 64 * 16];
    const RowRange rr = block_rows(N, nb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, q = lane >> 4;
    double nrm = 0.0;
    if (col < L)
        for (size_t n0 = rr.r0 + 16 * w; n0 < rr.r1; n0 += 16 * (kWG / 64)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const size_t n = n0 + 4 * r + q;
                if (n < rr.r1) {
                    const cx<double> v = StF64::ld(R, (size_t)col * N + n);
                    nrm += v.re * v.re + v.im * v.im;
                }
            }
        }
    colsum_store(nrm, partial + (size_t)blockIdx.x * kPStride, shd);
}

// ---------------------------------------------------------------------------
// Single-workgroup reduction of partials and L x L solves
// ---------------------------------------------------------------------------
constexpr int kRT = 1024;  // threads of the reduce/solve kernels

// Reduce E = L*L tile entries (if tile) plus n_extra extras over nb partial
// blocks, in a fixed order, into out[0..E).
__device__ void reduce_partials(const double2* __restrict__ partial, int nb, int L, bool tile, int n_extra,
                                double2* out, double2* scratch /* kRT entries */) {
    const int nt = tile ? L * L : 0;
    const int E = nt + n_extra;
    const int G = kRT / E;  // >= 3 since E <= 272
    const int t = threadIdx.x;
    const int g = t / E, e = t % E;
    double2 s = make_double2(0.0, 0.0);
    if (g < G) {
        const int idx = (e < nt) ? (e / L) * 16 + (e % L) : 256 + (e - nt);
        for (int b = g; b < nb; b += G) {
            const double2 v = partial[(size_t)b * kPStride + idx];
            s.x += v.x;
            s.y += v.y;
        }
        scratch[g * E + e] = s;
    }
    __syncthreads();
    if (t < E) {
        double2 a = scratch[t];
        for (int q = 1; q < G; ++q) {
            a.x += scratch[q * E + t].x;
            a.y += scratch[q * E + t].y;
        }
        out[t] = a;
    }
    __syncthreads();
}

__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }
__device__ __forceinline__ double cabs2(cx<double> a) { return a.re * a.re + a.im * a.im; }

struct SolveShared {
    double2 scratch[kRT];
    double2 red[16 * 16 + 16];
    double2 M[256], RHS[256], sol[256];
    double2 aug[16 * 32];
    double fac[2 * 16];
    double scale;
    double pmin, pmax;  // smallest and largest pivot modulus of the last factorisation
    int piv;
    int flag;
};

// Solve M Z = RHS (L x L row-major in shared memory) by LU with partial
// pivoting into sm.sol (row-major).  Returns false (uniformly across the
// workgroup) on a pivot below 1e-14 max|M| or a non-finite entry.  The
// ratio sm.pmax / sm.pmin of the pivot moduli is a cheap estimate of the
// condition of M (a lower bound of it for this pivot order).
__device__ bool lu_solve_shared(SolveShared& sm, int L) {
    const int t = threadIdx.x;
    const int W2 = 2 * L;
    if (t == 0) {
        sm.flag = 0;
        sm.pmin = INFINITY;
        sm.pmax = 0.0;
    }
    __syncthreads();
    if (t < L * W2) {
        const int r = t / W2, c = t % W2;
        const double2 v = (c < L) ? sm.M[r * L + c] : sm.RHS[r * L + (c - L)];
        sm.aug[r * W2 + c] = v;
        if (!finite2(v)) atomicOr(&sm.flag, 1);
    }
    __syncthreads();
    if (sm.flag) return false;
    if (t == 0) {
        double m = 0.0;
        for (int r = 0; r < L; ++r)
            for (int c = 0; c < L; ++c) {
                const double2 v = sm.aug[r * W2 + c];
                m = fmax(m, sqrt(v.x * v.x + v.y * v.y));
            }
        sm.scale = m;
        if (m == 0.0) sm.flag = 1;
    }
    __syncthreads();
    if (sm.flag) return false;
    const double thr = 1e-14 * sm.scale;
    for (int k = 0; k < L; ++k) {
        if (t == 0) {
            int p = k;
            double best = -1.0;
            for (int r = k; r < L; ++r) {
                const double2 v = sm.aug[r * W2 + k];
                const double m = v.x * v.x + v.y * v.y;
                if (m > best) {
                    best = m;
                    p = r;
                }
            }
            const double pm = sqrt(best);
            if (!(pm >= thr)) sm.flag = 1;
            sm.pmin = fmin(sm.pmin, pm);
            sm.pmax = fmax(sm.pmax, pm);
            sm.piv = p;
        }
        __syncthreads();
        if (sm.flag) return false;
        const int p = sm.piv;
        if (p != k && t < W2) {
            const double2 a = sm.aug[k * W2 + t];
            sm.aug[k * W2 + t] = sm.aug[p * W2 + t];
            sm.aug[p * W2 + t] = a;
        }
        __syncthreads();
        if (t < L - k - 1) {
            const int r = k + 1 + t;
            const cx<double> piv = {sm.aug[k * W2 + k].x, sm.aug[k * W2 + k].y};
            const cx<double> num = {sm.aug[r * W2 + k].x, sm.aug[r * W2 + k].y};
            const double d = 1.0 / cabs2(piv);
            const cx<double> f = cmulc(piv, num);  // conj(piv) num / |piv|^2 = num / piv
            sm.fac[2 * t] = f.re * d;
            sm.fac[2 * t + 1] = f.im * d;
        }
        __syncthreads();
        const int rows = L - k - 1, cols = W2 - k;
        for (int id = t; id < rows * cols; id += kRT) {
            const int r = k + 1 + id / cols, c = k + id % cols;
            const cx<double> f = {sm.fac[2 * (r - k - 1)], sm.fac[2 * (r - k - 1) + 1]};
            const cx<double> pk = {sm.aug[k * W2 + c].x, sm.aug[k * W2 + c].y};
            cx<double> v = {sm.aug[r * W2 + c].x, sm.aug[r * W2 + c].y};
            v = v - f * pk;
            sm.aug[r * W2 + c] = make_double2(v.re, v.im);
        }
        __syncthreads();
    }
    // back substitution, one thread per right-hand-side column
    if (t < L) {
        for (int k = L - 1; k >= 0; --k) {
            cx<double> x = {sm.aug[k * W2 + L + t].x, sm.aug[k * W2 + L + t].y};
            for (int c = k + 1; c < L; ++c) {
                const cx<double> a = {sm.aug[k * W2 + c].x, sm.aug[k * W2 + c].y};
                const cx<double> sv = {sm.sol[c * L + t].x, sm.sol[c * L + t].y};
                x = x - a * sv;
            }
            const cx<double> piv = {sm.aug[k * W2 + k].x, sm.aug[k * W2 + k].y};
            const double d = 1.0 / cabs2(piv);
            const cx<double> q = cmulc(piv, x);
            sm.sol[k * L + t] = make_double2(q.re * d, q.im * d);
        }
    }
    __syncthreads();
    return true;
}

__global__ void __launch_bounds__(kRT) k_reduce_gram(const double2* __restrict__ partial, int nb, int L,
                                                     double2* __restrict__ C) {
    __shared__ SolveShared sm;
    reduce_partials(partial, nb, L, true, 0, sm.red, sm.scratch);
    if ((int)threadIdx.x < L * L) C[threadIdx.x] = sm.red[threadIdx.x];
}

__global__ void __launch_bounds__(kRT) k_reduce_extras(const double2* __restrict__ partial, int nb, int n,
                                                       double* __restrict__ out) {
    __shared__ SolveShared sm;
    reduce_partials(partial, nb, 1, false, n, sm.red, sm.scratch);
    if ((int)threadIdx.x < n) out[threadIdx.x] = sm.red[threadIdx.x].x;
}

__device__ __forceinline__ double cond_of(const SolveShared& sm, bool ok) {
    return ok ? sm.pmax / sm.pmin : INFINITY;
}

// Z = M^{-1} (c RHS) for a complex scale c, by LU in LDS; on failure Z = 0.
// status_bit 0: *status = ok ? 0 : 1; otherwise *status |= status_bit on
// failure.  cond (may be null) receives the pivot-ratio condition estimate.
__global__ void __launch_bounds__(kRT) k_small_solve(const double2* __restrict__ M, const double2* __restrict__ RHS,
                                                     int L, double2 c, double2* __restrict__ Z,
                                                     int* __restrict__ status, int status_bit,
                                                     double* __restrict__ cond) {
    __shared__ SolveShared sm;
    const int t = threadIdx.x;
    if (t < L * L) {
        sm.M[t] = M[t];
        const double2 r = RHS[t];
        sm.RHS[t] = make_double2(c.x * r.x - c.y * r.y, c.x * r.y + c.y * r.x);
    }
    __syncthreads();
    const bool ok = lu_solve_shared(sm, L);
    if (t < L * L) Z[t] = ok ? sm.sol[t] : make_double2(0.0, 0.0);
    if (t == 0) {
        if (status_bit == 0) status[0] = ok ? 0 : 1;
        else if (!ok) status[0] |= status_bit;
        if (cond) cond[0] = cond_of(sm, ok);
    }
}

// Status bits of the solver flags
constexpr int kAlphaBreak = 1, kGammaBreak = 2, kNaN = 4;

// alpha: (Rt^H V) alpha = Rt^H R_k ; zeta = Tr[W^H R] / Tr[W^H W].  On a
// breakdown alpha = 0 and zeta = 0, so the following updates leave X and R
// unchanged.
__global__ void __launch_bounds__(kRT) k_solve_alpha(const double2* __restrict__ partial, int nb, int L,
                                                     SolverBufs b) {
    __shared__ SolveShared sm;
    const int t = threadIdx.x;
    reduce_partials(partial, nb, L, true, 2, sm.red, sm.scratch);
    if (t < L * L) {
        sm.M[t] = sm.red[t];
        sm.RHS[t] = b.C_r[t];
    }
    __syncthreads();
    const double2 twr = sm.red[L * L], tww = sm.red[L * L + 1];
    bool ok = lu_solve_shared(sm, L);
    ok = ok && finite2(twr) && isfinite(tww.x) && tww.x > 0.0;
    if (t < L * L) b.alpha[t] = ok ? sm.sol[t] : make_double2(0.0, 0.0);
    if (t == 0) {
        b.cond[0] = cond_of(sm, ok);
        b.zeta[0] = ok ? make_double2(twr.x / tww.x, twr.y / tww.x) : make_double2(0.0, 0.0);
        b.zeta[1] = twr;
        b.zeta[2] = tww;
        if (!ok) b.status[0] |= kAlphaBreak;
    }
}

// norms of R_{k+1}; gamma: (Rt^H R_k) gamma = Rt^H R_{k+1} / zeta; then C_r <- C_rn.
__global__ void __launch_bounds__(kRT) k_solve_gamma(const double2* __restrict__ partial, int nb, int L,
                                                     SolverBufs b) {
    __shared__ SolveShared sm;
    const int t = threadIdx.x;
    reduce_partials(partial, nb, L, true, L, sm.red, sm.scratch);
    const cx<double> z = StF64::ld(b.zeta, 0);
    const double zz = cabs2(z);
    if (t < L * L) {
        sm.M[t] = b.C_r[t];
        const double2 c = sm.red[t];
        // c / z = c conj(z) / |z|^2
        sm.RHS[t] = zz > 0.0 ? make_double2((c.x * z.re + c.y * z.im) / zz, (c.y * z.re - c.x * z.im) / zz)
                             : make_double2(0.0, 0.0);
    }
    if (t < L) {
        const double v = sm.red[L * L + t].x;
        b.norms[t] = v;
        if (!isfinite(v)) atomicOr(b.status, kNaN);
    }
    __syncthreads();
    bool ok = lu_solve_shared(sm, L);
    ok = ok && zz > 0.0;
    if (t < L * L) {
        b.gamma[t] = ok ? sm.sol[t] : make_double2(0.0, 0.0);
        b.C_r[t] = sm.red[t];
        b.C_rn[t] = sm.red[t];
    }
    if (t == 0) {
        b.cond[1] = cond_of(sm, ok);
        if (!ok) b.status[0] |= kGammaBreak;
    }
}

// ---------------------------------------------------------------------------
// Row-wise L x L right multiplications (one thread per row, L compile-time)
// ---------------------------------------------------------------------------
// The Gram tile Rt^H S over the kWG rows [c0, c0 + kWG) of one chunk, where S
// is staged in LDS as sS[col][row - c0] by the update above it: each wave takes
// 64 rows, lane (col = lane % 16, q = lane / 16) feeds rows 4 r + q.
template <int L>
__device__ __forceinline__ void gram_chunk(GramAcc& acc, const double2* __restrict__ Rt, const double2 (*sS)[kWG + 1],
                                           size_t N, size_t c0, size_t r1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, q = lane >> 4;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int rl = 64 * w + 4 * r + q;
        const size_t n = c0 + rl;
        const bool ok = col < L && n < r1;
        const cx<double> a = ok ? StF64::ld(Rt, (size_t)col * N + n) : cx<double>{0.0, 0.0};
        cx<double> b = {0.0, 0.0};
        if (ok) b = {sS[col][rl].x, sS[col][rl].y};
        gram_step(acc, a, b);
    }
}

// P = R + U gamma, V = W + Y gamma (Sec. 2, the last two updates of an
// iteration), fused with the Gram products that open the next iteration:
// Rt^H V (tile), Tr[W^H R] (extra 0) and Tr[W^H W] (extra 1), written to the
// partial blocks as k_gram1 writes them.
template <int L>
__global__ void __launch_bounds__(kWG) k_update_PV_gram(double2* __restrict__ P, double2* __restrict__ V,
                                                        const double2* __restrict__ R, const double2* __restrict__ W,
                                                        const double2* __restrict__ U, const double2* __restrict__ Y,
                                                        const double2* __restrict__ gamma,
                                                        const double2* __restrict__ Rt, size_t N,
                                                        double2* __restrict__ partial, int nb) {
    __shared__ double2 sS[L][kWG + 1];
    __shared__ double2 sh[kWG / 64 * 256];
    const RowRange rr = block_rows(N, nb);
    GramAcc acc;
    gram_zero(acc);
    double twr_re = 0, twr_im = 0, tww = 0;
    for (size_t c0 = rr.r0; c0 < rr.r1; c0 += kWG) {
        const size_t n = c0 + threadIdx.x;
        if (n < rr.r1) {
            cx<double> u[L], y[L];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                u[i] = StF64::ld(U, (size_t)i * N + n);
                y[i] = StF64::ld(Y, (size_t)i * N + n);
            }
#pragma unroll
            for (int j = 0; j < L; ++j) {
                cx<double> p = StF64::ld(R, (size_t)j * N + n);
                cx<double> v = StF64::ld(W, (size_t)j * N + n);
                const cx<double> wr = cmulc(v, p);
                twr_re += wr.re;
                twr_im += wr.im;
                tww += v.re * v.re + v.im * v.im;
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const cx<double> gm = StF64::ld(gamma, i * L + j);
                    cfma(p, u[i], gm);
                    cfma(v, y[i], gm);
                }
                StF64::st(P, (size_t)j * N + n, p);
                StF64::st(V, (size_t)j * N + n, v);
                sS[j][threadIdx.x] = make_double2(v.re, v.im);
            }
        }
        __syncthreads();
        gram_chunk<L>(acc, Rt, sS, N, c0, rr.r1);
        __syncthreads();
    }
    double2* out = partial + (size_t)blockIdx.x * kPStride;
    gram_store(acc, out, sh);
    __syncthreads();
    double* shd = reinterpret_cast<double*>(sh);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    twr_re = wave_sum(twr_re);
    twr_im = wave_sum(twr_im);
    tww = wave_sum(tww);
    if (lane == 0) {
        shd[w * 3 + 0] = twr_re;
        shd[w * 3 + 1] = twr_im;
        shd[w * 3 + 2] = tww;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0, a1 = 0, a2 = 0;
        for (int q2 = 0; q2 < kWG / 64; ++q2) {
            a0 += shd[q2 * 3 + 0];
            a1 += shd[q2 * 3 + 1];
            a2 += shd[q2 * 3 + 2];
        }
        out[256] = make_double2(a0, a1);
        out[257] = make_double2(a2, 0.0);
    }
}

// X += zeta F + G, R -= zeta W + Y (Sec. 2), fused with the products the
// gamma system needs: the squared column norms of R_{k+1} (extras 0..L-1)
// and Rt^H R_{k+1} (tile).
template <int L>
__global__ void __launch_bounds__(kWG) k_update_XR_gram(double2* __restrict__ X, double2* __restrict__ R,
                                                        const double2* __restrict__ F, const double2* __restrict__ G,
                                                        const double2* __restrict__ W, const double2* __restrict__ Y,
                                                        const double2* __restrict__ zp,
                                                        const double2* __restrict__ Rt, size_t N,
                                                        double2* __restrict__ partial, int nb) {
    __shared__ double2 sS[L][kWG + 1];
    __shared__ double2 sh[kWG / 64 * 256];
    const RowRange rr = block_rows(N, nb);
    const cx<double> z = StF64::ld(zp, 0);
    GramAcc acc;
    gram_zero(acc);
    double nrm[L];
#pragma unroll
    for (int i = 0; i < L; ++i) nrm[i] = 0.0;
    for (size_t c0 = rr.r0; c0 < rr.r1; c0 += kWG) {
        const size_t n = c0 + threadIdx.x;
        if (n < rr.r1) {
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const size_t idx = (size_t)i * N + n;
                cx<double> x = StF64::ld(X, idx);
                cfma(x, z, StF64::ld(F, idx));
                x = x + StF64::ld(G, idx);
                StF64::st(X, idx, x);
                cx<double> rn = StF64::ld(R, idx) - StF64::ld(Y, idx);
                cfma(rn, -z, StF64::ld(W, idx));
                StF64::st(R, idx, rn);
                nrm[i] += rn.re * rn.re + rn.im * rn.im;
                sS[i][threadIdx.x] = make_double2(rn.re, rn.im);
            }
        }
        __syncthreads();
        gram_chunk<L>(acc, Rt, sS, N, c0, rr.r1);
        __syncthreads();
    }
    double2* out = partial + (size_t)blockIdx.x * kPStride;
    gram_store(acc, out, sh);
    __syncthreads();
    double* shd = reinterpret_cast<double*>(sh);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const double v = wave_sum(nrm[i]);
        if (lane == 0) shd[w * 16 + i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        double sum = 0.0;
        if ((int)threadIdx.x < L)
            for (int q2 = 0; q2 < kWG / 64; ++q2) sum += shd[q2 * 16 + threadIdx.x];
        out[256 + threadIdx.x] = make_double2(sum, 0.0);
    }
}

template <int L>
__global__ void __launch_bounds__(kWG) k_update_U(const double2* __restrict__ P, const double2* __restrict__ V,
                                                  const double2* __restrict__ zp, const double2* __restrict__ alpha,
                                                  double2* __restrict__ U, size_t N) {
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const cx<double> z = StF64::ld(zp, 0);
    cx<double> s[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        s[i] = StF64::ld(P, (size_t)i * N + n);
        cfma(s[i], -z, StF64::ld(V, (size_t)i * N + n));
    }
#pragma unroll
    for (int j = 0; j < L; ++j) {
        cx<double> u = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < L; ++i) cfma(u, s[i], StF64::ld(alpha, i * L + j));
        StF64::st(U, (size_t)j * N + n, u);
    }
}

// X += zeta F + G ; R <- R - zeta W - Y ; per-column ||R||^2 into the partial
// extras (one thread per row, L columns; coalesced across the wavefront).
// R = B - AX elementwise; R may be AX (each element is read before it is written)
__global__ void k_axpby(const double2* __restrict__ B, const double2* AX, double2* R, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 b = B[i], a = AX[i];
    R[i] = make_double2(b.x - a.x, b.y - a.y);
}

__global__ void k_copy(double2* __restrict__ d, const double2* __restrict__ s, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

__global__ void k_fill0(double2* __restrict__ d, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = make_double2(0.0, 0.0);
}

// A coefficient field [np][V] into the tiled order [V/64][np][64]; one thread per
// element of the output.
template <typename T>
__global__ void k_tile_field(const T* __restrict__ in, T* __restrict__ out, size_t V, int np) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * (size_t)np) return;
    const size_t tile = i / ((size_t)np * 64), r = i - tile * np * 64, p = r / 64;
    out[i] = in[p * V + tile * 64 + (r % 64)];
}

// Block vector of L columns between the standard layout (row k*V + s) and the
// tiled one (row (s/64)*768 + k*64 + s%64); one thread per element of the tiled
// side, so each 64-site run of a plane is one 1 KB read or write on both sides.
template <bool TO_TILED>
__global__ void k_retile(const double2* __restrict__ in, double2* __restrict__ out, size_t V, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t N = 12 * V, col = i / N, r = i - col * N;
    const size_t tile = r / 768, k = (r % 768) / 64, s = tile * 64 + (r % 64);
    const size_t std_i = col * N + k * V + s;
    if (TO_TILED) out[i] = in[std_i];
    else out[std_i] = in[i];
}

// ---------------------------------------------------------------------------
// Block BiCGSTAB helpers (the foil of block BiCGGR)
// ---------------------------------------------------------------------------
// out[:, j] = a A[:, j] + b B[:, j] + sum_i (c C[:, i] + d D[:, i]) M[i, j],
// one thread per row.  Null blocks are left out; the scalars a, b, c, d are
// multiplied by the device scalar *w where bits 1, 2, 4, 8 of wmask say so.
// A row's C and D entries are all read before any of its outputs is written
// and out[:, j] reads only A[:, j] and B[:, j] before it is written, so out
// may be the same block as A, C or D.
template <int L>
__global__ void __launch_bounds__(kWG) k_block_comb(double2* out, const double2* A, const double2* Bm,
                                                    const double2* C, const double2* D,
                                                    const double2* __restrict__ M, double2 a, double2 b, double2 c,
                                                    double2 d, const double2* __restrict__ w, int wmask, size_t N) {
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    cx<double> sa = {a.x, a.y}, sb = {b.x, b.y}, sc = {c.x, c.y}, sd = {d.x, d.y};
    if (w) {
        const cx<double> wv = StF64::ld(w, 0);
        if (wmask & 1) sa = sa * wv;
        if (wmask & 2) sb = sb * wv;
        if (wmask & 4) sc = sc * wv;
        if (wmask & 8) sd = sd * wv;
    }
    cx<double> s[L];
    const bool mix = (C != nullptr || D != nullptr) && M != nullptr;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        s[i] = {0.0, 0.0};
        if (mix && C) cfma(s[i], sc, StF64::ld(C, (size_t)i * N + n));
        if (mix && D) cfma(s[i], sd, StF64::ld(D, (size_t)i * N + n));
    }
#pragma unroll
    for (int j = 0; j < L; ++j) {
        cx<double> v = {0.0, 0.0};
        if (A) cfma(v, sa, StF64::ld(A, (size_t)j * N + n));
        if (Bm) cfma(v, sb, StF64::ld(Bm, (size_t)j * N + n));
        if (mix)
#pragma unroll
            for (int i = 0; i < L; ++i) cfma(v, s[i], StF64::ld(M, i * L + j));
        StF64::st(out, (size_t)j * N + n, v);
    }
}

// omega = Tr[T^H S] / Tr[T^H T] from the two L x L Gram matrices; on a zero or
// non-finite denominator omega = 0 and bit is set in *status.
__global__ void k_stab_omega(const double2* __restrict__ Cts, const double2* __restrict__ Ctt, int L,
                             double2* __restrict__ omega, int* __restrict__ status, int bit) {
    if (threadIdx.x != 0) return;
    double nr = 0.0, ni = 0.0, dd = 0.0;
    for (int i = 0; i < L; ++i) {
        nr += Cts[i * L + i].x;
        ni += Cts[i * L + i].y;
        dd += Ctt[i * L + i].x;
    }
    const bool ok = isfinite(nr) && isfinite(ni) && isfinite(dd) && dd > 0.0;
    omega[0] = ok ? make_double2(nr / dd, ni / dd) : make_double2(0.0, 0.0);
    if (!ok) status[0] |= bit;
}

inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t partial_stride() { return kPStride; }

int gram_blocks(size_t N) {
    size_t nb = (N + 4095) / 4096;
    if (nb < 1) nb = 1;
    if (nb > kMaxPartial) nb = kMaxPartial;
    return (int)nb;
}

hipError_t launch_gram_partials(const double2* P, const double2* Q, size_t N, int L, double2* partial, int nb,
                                hipStream_t s) {
    k_gram<<<nb, kWG, 0, s>>>(P, Q, N, L, partial, nb);
    return hipGetLastError();
}

hipError_t launch_reduce_gram(const double2* partial, int nb, int L, double2* C, hipStream_t s) {
    k_reduce_gram<<<1, kRT, 0, s>>>(partial, nb, L, C);
    return hipGetLastError();
}

hipError_t launch_small_solve(const double2* M, const double2* RHS, int L, double2* Z, int* status, hipStream_t s) {
    k_small_solve<<<1, kRT, 0, s>>>(M, RHS, L, make_double2(1.0, 0.0), Z, status, 0, nullptr);
    return hipGetLastError();
}

hipError_t launch_small_solve_scaled(const double2* M, const double2* RHS, int L, double2 c, double2* Z, int* status,
                                     int status_bit, double* cond, hipStream_t s) {
    k_small_solve<<<1, kRT, 0, s>>>(M, RHS, L, c, Z, status, status_bit, cond);
    return hipGetLastError();
}

hipError_t launch_gram1(const double2* Rt, const double2* V, const double2* W, const double2* R, size_t N, int L,
                        double2* partial, int nb, hipStream_t s) {
    k_gram1<<<nb, kWG, 0, s>>>(Rt, V, W, R, N, L, partial, nb);
    return hipGetLastError();
}

hipError_t launch_solve_alpha(const double2* partial, int nb, int L, const SolverBufs& b, hipStream_t s) {
    k_solve_alpha<<<1, kRT, 0, s>>>(partial, nb, L, b);
    return hipGetLastError();
}

hipError_t launch_solve_gamma(const double2* partial, int nb, int L, const SolverBufs& b, hipStream_t s) {
    k_solve_gamma<<<1, kRT, 0, s>>>(partial, nb, L, b);
    return hipGetLastError();
}

#define WD_L_SWITCH(L, CALL)          \
    switch (L) {                      \
        case 1: CALL(1); break;       \
        case 2: CALL(2); break;       \
        case 3: CALL(3); break;       \
        case 4: CALL(4); break;       \
        case 5: CALL(5); break;       \
        case 6: CALL(6); break;       \
        case 7: CALL(7); break;       \
        case 8: CALL(8); break;       \
        case 9: CALL(9); break;       \
        case 10: CALL(10); break;     \
        case 11: CALL(11); break;     \
        case 12: CALL(12); break;     \
        case 13: CALL(13); break;     \
        case 14: CALL(14); break;     \
        case 15: CALL(15); break;     \
        case 16: CALL(16); break;     \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_update_U(const double2* P, const double2* V, const double2* zeta, const double2* alpha,
                           double2* U, size_t N, int L, hipStream_t s) {
#define WD_CALL_U(l) k_update_U<l><<<nblk(N, kWG), kWG, 0, s>>>(P, V, zeta, alpha, U, N)
    WD_L_SWITCH(L, WD_CALL_U)
#undef WD_CALL_U
    return hipGetLastError();
}

hipError_t launch_update_PV_gram(double2* P, double2* V, const double2* R, const double2* W, const double2* U,
                                 const double2* Y, const double2* gamma, const double2* Rt, size_t N, int L,
                                 double2* partial, int nb, hipStream_t s) {
#define WD_CALL_PVG(l) k_update_PV_gram<l><<<nb, kWG, 0, s>>>(P, V, R, W, U, Y, gamma, Rt, N, partial, nb)
    WD_L_SWITCH(L, WD_CALL_PVG)
#undef WD_CALL_PVG
    return hipGetLastError();
}

hipError_t launch_update_XR_gram(double2* X, double2* R, const double2* F, const double2* G, const double2* W,
                                 const double2* Y, const double2* Rt, const double2* zeta, size_t N, int L,
                                 double2* partial, int nb, hipStream_t s) {
#define WD_CALL_XRG(l) k_update_XR_gram<l><<<nb, kWG, 0, s>>>(X, R, F, G, W, Y, zeta, Rt, N, partial, nb)
    WD_L_SWITCH(L, WD_CALL_XRG)
#undef WD_CALL_XRG
    return hipGetLastError();
}

hipError_t launch_block_comb(double2* out, const double2* A, const double2* Bm, const double2* C, const double2* D,
                             const double2* M, double2 a, double2 b, double2 c, double2 d, const double2* w, int wmask,
                             size_t N, int L, hipStream_t s) {
#define WD_CALL_COMB(l) k_block_comb<l><<<nblk(N, kWG), kWG, 0, s>>>(out, A, Bm, C, D, M, a, b, c, d, w, wmask, N)
    WD_L_SWITCH(L, WD_CALL_COMB)
#undef WD_CALL_COMB
    return hipGetLastError();
}

hipError_t launch_stab_omega(const double2* Cts, const double2* Ctt, int L, double2* omega, int* status, int bit,
                             hipStream_t s) {
    k_stab_omega<<<1, 64, 0, s>>>(Cts, Ctt, L, omega, status, bit);
    return hipGetLastError();
}

hipError_t launch_axpby_block(const double2* B, const double2* AX, double2* R, size_t n, hipStream_t s) {
    k_axpby<<<nblk(n, 256), 256, 0, s>>>(B, AX, R, n);
    return hipGetLastError();
}

hipError_t launch_colnorms(const double2* R, size_t N, int L, double2* partial, int nb, double* norms,
                           hipStream_t s) {
    k_colnorms<<<nb, kWG, 0, s>>>(R, N, L, partial, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce_extras<<<1, kRT, 0, s>>>(partial, nb, L, norms);
    return hipGetLastError();
}

hipError_t launch_copy(double2* dst, const double2* src, size_t n, hipStream_t s) {
    k_copy<<<nblk(n, 256), 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_zero(double2* dst, size_t n, hipStream_t s) {
    k_fill0<<<nblk(n, 256), 256, 0, s>>>(dst, n);
    return hipGetLastError();
}

hipError_t launch_tile_field(const void* src, void* dst, size_t V, int np, int pair_bytes, hipStream_t s) {
    if (V % 64 != 0) return hipErrorInvalidValue;
    const size_t n = V * (size_t)np;
    switch (pair_bytes) {
        case 16: k_tile_field<double2><<<nblk(n, 256), 256, 0, s>>>((const double2*)src, (double2*)dst, V, np); break;
        case 8: k_tile_field<float2><<<nblk(n, 256), 256, 0, s>>>((const float2*)src, (float2*)dst, V, np); break;
        case 4: k_tile_field<uint32_t><<<nblk(n, 256), 256, 0, s>>>((const uint32_t*)src, (uint32_t*)dst, V, np); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_retile(const double2* src, double2* dst, size_t V, int L, bool to_tiled, hipStream_t s) {
    if (V % 64 != 0) return hipErrorInvalidValue;
    const size_t n = (size_t)12 * V * L;
    if (to_tiled)
        k_retile<true><<<nblk(n, 256), 256, 0, s>>>(src, dst, V, n);
    else
        k_retile<false><<<nblk(n, 256), 256, 0, s>>>(src, dst, V, n);
    return hipGetLastError();
}

}  // namespace wd
