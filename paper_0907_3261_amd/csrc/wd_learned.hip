// Learned linear gauge-covariant preconditioner M_theta = L_2 L_1 L_0 with
//   (L psi)(x) = W_0 psi(x) + sum_mu [ W_{+mu} U_mu(x) psi(x+mu) + W_{-mu} U_mu(x-mu)^dag psi(x-mu) ],
// W complex 4 x 4 on spin, U on colour, FP32 storage and arithmetic.  It is
// the "better preconditioner than Jacobi" direction the paper names as
// future work (Sec. 4), kept linear so the outer block BiCGGR is unchanged.
//
// Kernels: one layer (the adjoint layer is the same kernel with weights
// W_0^dag, W_{+-mu} -> W_{-+mu}^dag), the weight gradient
// dl/dRe W_d + i dl/dIm W_d = 2 sum_{x,c,i} g(x) (S_d z)(x)^dag, the loss
// mean_i ||y_i - e_i||^2 / ||e_i||^2 with its gradient, and Adam.
#include <cmath>
#include <type_traits>
#include <complex>
#include <cstring>
#include <vector>

#include "wd_internal.h"

using namespace wd;

namespace {

constexpr int kNL = WD_LEARNED_LAYERS, kND = WD_LEARNED_DIRS;

// S_d psi for one column at site s: returns 12 complex (index 3*spin + colour).  V:
// sites (the links' plane stride); KS, vs, vnb: the plane stride of the block vector
// and the element offsets of s and nb in it (standard or tiled layout).
template <class SZ>
__device__ __forceinline__ void shifted(const float2* __restrict__ U, const typename SZ::P* __restrict__ Z, size_t V,
                                        size_t KS, int d, int s, int nb, uint32_t vs, uint32_t vnb,
                                        cx<float> (&q)[12]) {
    if (d == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const auto v = SZ::ld(Z, (size_t)k * KS + vs);
            q[k] = {(float)v.re, (float)v.im};
        }
        return;
    }
    const int mu = (d - 1) >> 1;
    const bool fwd = (d & 1) != 0;
    const int ls = fwd ? s : nb;
    cx<float> u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = StF32::ld(U, (size_t)(mu * 9 + k) * V + ls);
    cx<float> p[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const auto v = SZ::ld(Z, (size_t)k * KS + vnb);
        p[k] = {(float)v.re, (float)v.im};
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<float> r = {0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (fwd)
                    cfma(r, u[a * 3 + b], p[3 * sp + b]);
                else
                    cfmac(r, u[b * 3 + a], p[3 * sp + b]);
            }
            q[3 * sp + a] = r;
        }
}

__device__ __forceinline__ int neighbour(const Geom& g, int s, int d) {
    if (d == 0) return s;
    const int mu = (d - 1) >> 1;
    const int step = (d & 1) ? 1 : -1;
    int c[4] = {s % g.lx, (s / g.lx) % g.ly, (s / g.sxy) % g.lz, s / g.sxyz};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    c[mu] = (c[mu] + step + ext[mu]) % ext[mu];
    return c[0] + g.lx * (c[1] + g.ly * (c[2] + g.lz * c[3]));
}

// Operands of one term W_d (U or U^dag or 1) psi(nb): the link and the CT input spinors.
template <class R, int CT>
struct Term {
    cx<R> u[9];
    cx<R> p[CT][12];
};

// Issue the loads of a term.  KIND: 0 self term, 1 forward hop (link at the site),
// 2 backward hop (daggered link at the neighbour).  vnb: element offset of the input
// site in a plane of the block vector, KS its plane stride.
template <int KIND, class SI, class SL, class R, int CT>
__device__ __forceinline__ void term_load(Term<R, CT>& t, const typename SL::P* __restrict__ U, int mu, int ls,
                                          const typename SI::P* __restrict__ Zin, size_t V, size_t KS, size_t col0,
                                          uint32_t vnb) {
    if (KIND != 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) t.u[k] = SL::ld(U, (size_t)(mu * 9 + k) * V + ls);
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const typename SI::P* zc = Zin + (col0 + c) * 12 * V;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const auto v = SI::ld(zc, (size_t)k * KS + vnb);
            t.p[c][k] = {(R)v.re, (R)v.im};
        }
    }
}

// acc += W_d (U or U^dag or 1) psi for the CT columns of a loaded term
template <int KIND, class R, int CT>
__device__ __forceinline__ void term_apply(const Term<R, CT>& t, const float2* __restrict__ Wd, cx<R> (&acc)[CT][12]) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        // source spin tt: q = (U or U^dag or 1) psi_tt, then acc[sp] += W[sp][tt] q
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            cx<R> q[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (KIND == 0) {
                    q[a] = t.p[c][3 * tt + a];
                } else {
                    cx<R> r = {R(0), R(0)};
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        if (KIND == 1)
                            cfma(r, t.u[a * 3 + b], t.p[c][3 * tt + b]);
                        else
                            cfmac(r, t.u[b * 3 + a], t.p[c][3 * tt + b]);
                    }
                    q[a] = r;
                }
            }
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const float2 wv = Wd[sp * 4 + tt];
                const cx<R> w = {(R)wv.x, (R)wv.y};
#pragma unroll
                for (int a = 0; a < 3; ++a) cfma(acc[c][3 * sp + a], w, q[a]);
            }
        }
    }
}

// One layer: thread (site, tile) accumulates CT columns, so each link and
// weight is loaded once per tile.  SI / SO: storage of input / output, SL:
// storage (and arithmetic precision) of the links.  W: 9 x 16 complex
// (row-major 4 x 4 per direction; direction 1 + 2 mu is the forward hop,
// 2 + 2 mu the backward one), FP32.  Columns [c0 + tile*CT, + CT) of the
// block vectors; every tile of the launch is complete.  In FP32 the nine
// terms are software-pipelined: the operands of the next term are in flight
// while the current one is accumulated.
template <class SI, class SO, class SL, int CT>
__global__ void __launch_bounds__(256) k_layer(const Geom g, const SiteMap sm, const typename SL::P* __restrict__ U,
                                               const float2* __restrict__ W, const typename SI::P* __restrict__ Zin,
                                               typename SO::P* __restrict__ Zout, const int c0, const int ntile) {
    using R = typename SL::R;
    const size_t V = g.V;
    const int s = map_site(g, sm, blockIdx.x, threadIdx.x);
    const int tile = blockIdx.y * blockDim.y + threadIdx.y;
    if (s < 0 || tile >= ntile) return;
    const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / g.sxy) % g.lz, t = s / g.sxyz;
    const int co[4] = {x, y, z, t};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    const int str[4] = {1, g.lx, g.sxy, g.sxyz};
    const size_t col0 = (size_t)(c0 + tile * CT);
    auto fwd_site = [&](int mu) {
        return (co[mu] + 1 == ext[mu]) ? s - (ext[mu] - 1) * str[mu] : s + str[mu];
    };
    auto bwd_site = [&](int mu) { return (co[mu] == 0) ? s + (ext[mu] - 1) * str[mu] : s - str[mu]; };
    const size_t KS = vec_plane(g);
    const auto vo = [&](int n) { return vec_site(g, n); };
    cx<R> acc[CT][12];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[c][k] = {R(0), R(0)};
    if constexpr (sizeof(R) == 4) {
        // FP32: two operand sets, the next term's loads in flight during the current term
        Term<R, CT> A, B;  // A: self and backward terms, B: forward terms
        term_load<0, SI, SL>(A, U, 0, s, Zin, V, KS, col0, vo(s));
        term_load<1, SI, SL>(B, U, 0, s, Zin, V, KS, col0, vo(fwd_site(0)));
        term_apply<0>(A, W, acc);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            const int bw = bwd_site(mu);
            term_load<2, SI, SL>(A, U, mu, bw, Zin, V, KS, col0, vo(bw));
            term_apply<1>(B, W + (1 + 2 * mu) * 16, acc);
            if (mu < 3) term_load<1, SI, SL>(B, U, mu + 1, s, Zin, V, KS, col0, vo(fwd_site(mu + 1)));
            term_apply<2>(A, W + (2 + 2 * mu) * 16, acc);
        }
    } else {
        // FP64: one operand set (two would halve the occupancy)
        Term<R, CT> A;
        term_load<0, SI, SL>(A, U, 0, s, Zin, V, KS, col0, vo(s));
        term_apply<0>(A, W, acc);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            term_load<1, SI, SL>(A, U, mu, s, Zin, V, KS, col0, vo(fwd_site(mu)));
            term_apply<1>(A, W + (1 + 2 * mu) * 16, acc);
            const int bw = bwd_site(mu);
            term_load<2, SI, SL>(A, U, mu, bw, Zin, V, KS, col0, vo(bw));
            term_apply<2>(A, W + (2 + 2 * mu) * 16, acc);
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        typename SO::P* oc = Zout + (col0 + c) * 12 * V;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            SO::st(oc, (size_t)k * KS + vo(s),
                   cx<typename SO::R>{(typename SO::R)acc[c][k].re, (typename SO::R)acc[c][k].im});
    }
}

// Adjoint weights: W'_0 = W_0^dag, W'_{+mu} = W_{-mu}^dag, W'_{-mu} = W_{+mu}^dag
__global__ void k_adjoint_weights(const float2* __restrict__ W, float2* __restrict__ Wa) {
    const int t = threadIdx.x;  // 9 * 16
    if (t >= kND * 16) return;
    const int d = t / 16, i = (t % 16) / 4, j = t % 4;
    int src = d;
    if (d > 0) src = (d & 1) ? d + 1 : d - 1;
    const float2 v = W[src * 16 + j * 4 + i];
    Wa[t] = make_float2(v.x, -v.y);
}

constexpr int kGB = 256;  // threads of the reduction kernels

// partial[(col * gridDim.x + block) * 16 + e] = sum over this block's sites of
//   2 sum_a g[3 s + a] conj((S_d z)[3 t + a]),  e = 4 s + t
template <class SZ>
__global__ void __launch_bounds__(kGB) k_wgrad(const Geom g, const float2* __restrict__ U,
                                               const typename SZ::P* __restrict__ Z, const float2* __restrict__ Gr,
                                               int d, double2* __restrict__ partial) {
    __shared__ double sh[kGB / 64][32];
    const size_t V = g.V, KS = vec_plane(g);
    const int col = blockIdx.y;
    const typename SZ::P* zc = Z + (size_t)col * 12 * V;
    const float2* gc = Gr + (size_t)col * 12 * V;
    double acc[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) acc[e] = 0.0;
    for (int s = blockIdx.x * kGB + threadIdx.x; s < g.V; s += gridDim.x * kGB) {
        cx<float> q[12], gv[12];
        const int nb = neighbour(g, s, d);
        const uint32_t vs = vec_site(g, s);
        shifted<SZ>(U, zc, V, KS, d, s, nb, vs, vec_site(g, nb), q);
#pragma unroll
        for (int k = 0; k < 12; ++k) gv[k] = StF32::ld(gc, (size_t)k * KS + vs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                cx<float> r = {0.f, 0.f};
#pragma unroll
                for (int a = 0; a < 3; ++a) cfma(r, gv[3 * sp + a], conj(q[3 * t + a]));
                acc[2 * (sp * 4 + t)] += 2.0 * r.re;
                acc[2 * (sp * 4 + t) + 1] += 2.0 * r.im;
            }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        double v = acc[e];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sh[w][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        double re = 0.0, im = 0.0;
        for (int q = 0; q < kGB / 64; ++q) {
            re += sh[q][2 * threadIdx.x];
            im += sh[q][2 * threadIdx.x + 1];
        }
        partial[((size_t)col * gridDim.x + blockIdx.x) * 16 + threadIdx.x] = make_double2(re, im);
    }
}

// out[e] = sum_p partial[p * 16 + e] (fixed order), e < 16
__global__ void __launch_bounds__(kGB) k_reduce16(const double2* __restrict__ partial, int np,
                                                  double2* __restrict__ out) {
    __shared__ double2 sh[kGB];
    const int e = threadIdx.x & 15, gq = threadIdx.x >> 4;  // 16 groups
    double2 s = make_double2(0.0, 0.0);
    for (int p = gq; p < np; p += kGB / 16) {
        const double2 v = partial[(size_t)p * 16 + e];
        s.x += v.x;
        s.y += v.y;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        double2 a = sh[threadIdx.x];
        for (int q = 1; q < kGB / 16; ++q) {
            a.x += sh[q * 16 + threadIdx.x].x;
            a.y += sh[q * 16 + threadIdx.x].y;
        }
        out[threadIdx.x] = a;
    }
}

// g = (y - e) / (||e_col||^2 P) in FP32; partial[block] = sum |y - e|^2 / ||e_col||^2
__global__ void __launch_bounds__(kGB) k_loss(const float2* __restrict__ Y, const double2* __restrict__ E,
                                              const double* __restrict__ en2, size_t n_per_col, int L,
                                              float2* __restrict__ Gr, double* __restrict__ partial) {
    __shared__ double sh[kGB / 64];
    const size_t n = n_per_col * L;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kGB + threadIdx.x; i < n; i += (size_t)gridDim.x * kGB) {
        const int col = (int)(i / n_per_col);
        const double inv = 1.0 / en2[col];
        const float2 y = Y[i];
        const double2 e = E[i];
        const double dr = (double)y.x - e.x, di = (double)y.y - e.y;
        acc += (dr * dr + di * di) * inv;
        const double sc = inv / L;
        Gr[i] = make_float2((float)(dr * sc), (float)(di * sc));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < kGB / 64; ++q) s += sh[q];
        partial[blockIdx.x] = s;
    }
}

// Residual-space loss: with Ay = A M r (FP64) and r, per element d = Ay - r; the loss partials
// sum |d|^2 / ||r||^2 per column, and out = gamma5 d / (||r||^2 L), the input of the second
// application of A in dl/d(conj y) = gamma5 A gamma5 d / (||r||^2 L) (gamma5 negates the lower
// spin pair, planes k = 6..11 of a column).  out may be Ay.  tiled: the block vectors'
// layout (the plane of element i follows from it).
__global__ void __launch_bounds__(kGB) k_res_loss(const double2* Ay, const double2* __restrict__ R,
                                                  const double* __restrict__ rn2, size_t n_per_col, int L,
                                                  double2* out, double* __restrict__ partial, int tiled) {
    __shared__ double sh[kGB / 64];
    const size_t n = n_per_col * L;
    const size_t plane = n_per_col / 12;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kGB + threadIdx.x; i < n; i += (size_t)gridDim.x * kGB) {
        const int col = (int)(i / n_per_col);
        const size_t row = i - (size_t)col * n_per_col;
        const int k = tiled ? (int)((row % 768) / 64) : (int)(row / plane);
        const double inv = 1.0 / rn2[col];
        const double2 a = Ay[i], r = R[i];
        const double dr = a.x - r.x, di = a.y - r.y;
        acc += (dr * dr + di * di) * inv;
        const double sc = (k >= 6 ? -inv : inv) / L;
        out[i] = make_double2(dr * sc, di * sc);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int q = 0; q < kGB / 64; ++q) sum += sh[q];
        partial[blockIdx.x] = sum;
    }
}

// FP32 activation -> FP64 block; gamma5 applied on request (the gradient's last factor)
__global__ void k_to_f64(const float2* __restrict__ src, double2* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = make_double2((double)src[i].x, (double)src[i].y);
}
__global__ void k_gamma5_to_f32(const double2* __restrict__ src, float2* __restrict__ dst, size_t n_per_col,
                                size_t n, int tiled) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t plane = n_per_col / 12, r = i % n_per_col;
    const int k = tiled ? (int)((r % 768) / 64) : (int)(r / plane);
    const double sg = k >= 6 ? -1.0 : 1.0;
    dst[i] = make_float2((float)(sg * src[i].x), (float)(sg * src[i].y));
}

__global__ void __launch_bounds__(kGB) k_reduce_loss(const double* __restrict__ partial, int np, int L,
                                                     double* __restrict__ out) {
    __shared__ double sh[kGB];
    double s = 0.0;
    for (int p = threadIdx.x; p < np; p += kGB) s += partial[p];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int q = 0; q < kGB; ++q) a += sh[q];
        out[0] = a / L;
    }
}

// Adam on the real and imaginary parts; G holds dl/dRe + i dl/dIm (FP64)
__global__ void k_adam(float2* __restrict__ theta, const double2* __restrict__ G, double2* __restrict__ m,
                       double2* __restrict__ v, int n, int t, double lr, double b1, double b2, double eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 g = G[i];
    double2 mi = m[i], vi = v[i];
    mi.x = b1 * mi.x + (1 - b1) * g.x;
    mi.y = b1 * mi.y + (1 - b1) * g.y;
    vi.x = b2 * vi.x + (1 - b2) * g.x * g.x;
    vi.y = b2 * vi.y + (1 - b2) * g.y * g.y;
    m[i] = mi;
    v[i] = vi;
    const double c1 = 1.0 / (1.0 - pow(b1, (double)t)), c2 = 1.0 / (1.0 - pow(b2, (double)t));
    float2 th = theta[i];
    th.x -= (float)(lr * (mi.x * c1) / (sqrt(vi.x * c2) + eps));
    th.y -= (float)(lr * (mi.y * c1) / (sqrt(vi.y * c2) + eps));
    theta[i] = th;
}

// One layer over L >= 3 columns with the links of a 64-site tile staged in LDS, as in the FP64
// hop kernel: wave mu first stores U_mu(x) and U_mu(x - mu) for the tile's sites, then wave w
// takes columns w, w + 4, ... one at a time through the nine terms (self, then forward and
// backward per mu, the order of k_layer, so the results are bit-identical), with the next
// term's input spinor in flight while the current term is applied.  The links are read from
// HBM once per tile instead of once per column.  A lane without a site takes lane 0's site
// and stores lane 0's values (unpredicated stores).
template <class SI, class SO, class SL>
__global__ void __launch_bounds__(256) k_layer_lds(const Geom g, const SiteMap sm, const typename SL::P* __restrict__ U,
                                                   const float2* __restrict__ W, const typename SI::P* __restrict__ Zin,
                                                   typename SO::P* __restrict__ Zout, const int L) {
    using R = typename SL::R;
    using PL = typename SL::P;
    __shared__ PL sU[72][64];
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int s0 = map_site(g, sm, blockIdx.x, lane);
    if (!__any(s0 >= 0)) return;  // the same for all four waves
    const int s = s0 >= 0 ? s0 : map_site(g, sm, blockIdx.x, 0);
    const size_t V = g.V;
    const int co[4] = {s % g.lx, (s / g.lx) % g.ly, (s / g.sxy) % g.lz, s / g.sxyz};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    const int str[4] = {1, g.lx, g.sxy, g.sxyz};
    int nb[9];  // input site of each term: self, then x+ x- y+ y- z+ z- t+ t-
    nb[0] = s;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        nb[1 + 2 * mu] = (co[mu] + 1 == ext[mu]) ? s - (ext[mu] - 1) * str[mu] : s + str[mu];
        nb[2 + 2 * mu] = (co[mu] == 0) ? s + (ext[mu] - 1) * str[mu] : s - str[mu];
    }
    {
        const int bw = (w == 0) ? nb[2] : (w == 1) ? nb[4] : (w == 2) ? nb[6] : nb[8];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sU[(2 * w) * 9 + k][lane] = U[(size_t)(w * 9 + k) * V + s];
            sU[(2 * w + 1) * 9 + k][lane] = U[(size_t)(w * 9 + k) * V + bw];
        }
    }
    __syncthreads();
    for (int c = w; c < L; c += 4) {
        // the LDS lane index is opaque per column so that the staged links are read where they
        // are used instead of all being hoisted into registers
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const typename SI::P* zc = Zin + (size_t)c * 12 * V;
        const size_t KS = vec_plane(g);
        cx<R> acc[1][12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0][k] = {R(0), R(0)};
        Term<R, 1> t[2];
        auto load_in = [&](Term<R, 1>& dst, int site) {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const auto v = SI::ld(zc, (size_t)k * KS + vec_site(g, site));
                dst.p[0][k] = {(R)v.re, (R)v.im};
            }
        };
        load_in(t[0], nb[0]);
        static_for<0, 9>([&](auto dc) {
            constexpr int D = decltype(dc)::value;
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (D + 1 < 9) load_in(t[(D + 1) % 2], nb[D + 1]);
            Term<R, 1>& cur = t[D % 2];
            if constexpr (D == 0) {
                term_apply<0>(cur, W, acc);
            } else {
                constexpr int mu = (D - 1) / 2;
                constexpr bool fwd = (D % 2) == 1;
                constexpr int plane0 = (fwd ? 2 * mu : 2 * mu + 1) * 9;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const PL v = sU[plane0 + k][ln];
                    cur.u[k] = {(R)v.x, (R)v.y};
                }
                term_apply<fwd ? 1 : 2>(cur, W + D * 16, acc);
            }
        });
        __builtin_amdgcn_sched_barrier(0);
        typename SO::P* oc = Zout + (size_t)c * 12 * V;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            SO::st(oc, (size_t)k * KS + vec_site(g, s),
                   cx<typename SO::R>{(typename SO::R)acc[0][k].re, (typename SO::R)acc[0][k].im});
    }
}

inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <class SI, class SO, class SL, int CT>
hipError_t launch_layer_ct(const wd_ctx* c, const typename SL::P* U, const float2* W, const void* in, void* out,
                           int c0, int ntile, hipStream_t s) {
    if (ntile <= 0) return hipSuccess;
    const int ty = ntile < 4 ? ntile : 4;
    // XCD-aware site order in rows of the hop kernels' map, four t-slices walked together
    // (a fifth to a third fewer fetched bytes than the plane-wide map at 32^3 x 64, L = 12)
    const SiteMap sm =
        make_site_map_rows(c->g, 12.0 * CT * ty * sizeof(typename SI::P) + 36.0 * sizeof(typename SL::P), 4);
    dim3 block(64, ty), grid(sm.nblk, (ntile + ty - 1) / ty);
    k_layer<SI, SO, SL, CT><<<grid, block, 0, s>>>(c->g, sm, U, W, (const typename SI::P*)in, (typename SO::P*)out,
                                                   c0, ntile);
    return hipGetLastError();
}

// One layer over L columns, one column per thread.  At 32^3 x 64 with twelve
// columns this is the fastest tiling in both precisions (two- and four-column
// tiles lose occupancy to their accumulators and operand sets, and spill).
constexpr int kLayerCT = 1;

template <class SI, class SO, class SL>
hipError_t launch_layer(const wd_ctx* c, const typename SL::P* U, const float2* W, const void* in, void* out, int L,
                        hipStream_t s) {
    if (std::is_same_v<SL, StF64> && L >= 3) {
        // FP64: LDS-staged links from three columns on (one workgroup per tile, all columns;
        // measured 12.8 against 15.2 ms per application of M at 32^3 x 64, L = 12; in FP32 the
        // register-tiled kernel with its next-term prefetch stays 3 % faster)
        // the same site map as the register-tiled layer (16 % fewer fetched bytes and 5 % faster
        // than the plane-wide map)
        const SiteMap sm = make_site_map_rows(c->g, 12.0 * L * sizeof(typename SI::P) + 72.0 * sizeof(typename SL::P), 4);
        dim3 block(64, 4), grid(sm.nblk);
        k_layer_lds<SI, SO, SL><<<grid, block, 0, s>>>(c->g, sm, U, W, (const typename SI::P*)in,
                                                       (typename SO::P*)out, L);
        return hipGetLastError();
    }
    return launch_layer_ct<SI, SO, SL, kLayerCT>(c, U, W, in, out, 0, L / kLayerCT, s);
}

template <class SI, class SO>
hipError_t launch_layer(const wd_ctx* c, const float2* W, const void* in, void* out, int L, hipStream_t s) {
    return launch_layer<SI, SO, StF32>(c, c->U32, W, in, out, L, s);
}

constexpr int kWgBlocks = 64;

struct LearnWs {
    float2* z[3];       // FP32 activations z1, z2, z3 (z0 is the FP64 input)
    float2* g[2];       // FP32 gradient ping-pong
    double2* gpart;     // weight-gradient partials
    double2* G;         // gradient (3 x 9 x 16)
    double2* m;         // Adam moments
    double2* v;
    float2* Wa;         // adjoint weights (9 x 16)
    double* lpart;      // loss partials
    double* en2;        // ||e||^2 per column of the current batch
    double* loss;
};

int learn_ws(wd_ctx* c, LearnWs& w) {
    // the learned workspace lives in the low-precision Jacobi buffers (3 blocks) plus a
    // dedicated set for training
    const size_t blk = (size_t)12 * c->g.V * c->max_L;
    if (!c->learn_mem) {
        const size_t bytes = 2 * blk * sizeof(float2) + (size_t)kWgBlocks * WD_MAX_L * 16 * sizeof(double2) +
                             3 * kNL * kND * 16 * sizeof(double2) + kND * 16 * sizeof(float2) +
                             4096 * sizeof(double) + WD_MAX_L * sizeof(double) + 64;
        if (hipMalloc(&c->learn_mem, bytes) != hipSuccess) {
            c->learn_mem = nullptr;
            (void)hipGetLastError();
            return WD_ENOMEM;
        }
        c->learn_bytes = bytes;
    }
    {
        const int r = lowp_ensure(c);
        if (r != WD_OK) return r;
    }
    char* p = (char*)c->learn_mem;
    w.z[0] = (float2*)c->lp[0];
    w.z[1] = (float2*)c->lp[1];
    w.z[2] = (float2*)c->lp[2];
    w.g[0] = (float2*)p;
    p += blk * sizeof(float2);
    w.g[1] = (float2*)p;
    p += blk * sizeof(float2);
    w.gpart = (double2*)p;
    p += (size_t)kWgBlocks * WD_MAX_L * 16 * sizeof(double2);
    w.G = (double2*)p;
    p += kNL * kND * 16 * sizeof(double2);
    w.m = (double2*)p;
    p += kNL * kND * 16 * sizeof(double2);
    w.v = (double2*)p;
    p += kNL * kND * 16 * sizeof(double2);
    w.Wa = (float2*)p;
    p += kND * 16 * sizeof(float2);
    w.lpart = (double*)p;
    p += 4096 * sizeof(double);
    w.en2 = (double*)p;
    p += WD_MAX_L * sizeof(double);
    w.loss = (double*)p;
    return WD_OK;
}

}  // namespace

namespace wd {

// Z = M_theta R (FP64 in and out).  FP32: layers in FP32 with the
// low-precision Jacobi buffers as scratch; FP64: layers in FP64 with two
// FP64 workspace blocks (t0, t1) as scratch.
hipError_t launch_learned(wd_ctx* c, const double2* R, double2* Z, int L, Prec p, double2* t0d, double2* t1d,
                          hipStream_t s) {
    if (p == Prec::F64) {
        const double2* U = c->f.U;
        hipError_t e = launch_layer<StF64, StF64, StF64>(c, U, c->theta, R, t0d, L, s);
        if (e == hipSuccess) e = launch_layer<StF64, StF64, StF64>(c, U, c->theta + kND * 16, t0d, t1d, L, s);
        if (e == hipSuccess) e = launch_layer<StF64, StF64, StF64>(c, U, c->theta + 2 * kND * 16, t1d, Z, L, s);
        return e;
    }
    float2* t0 = (float2*)c->lp[0];
    float2* t1 = (float2*)c->lp[1];
    hipError_t e = launch_layer<StF64, StF32>(c, c->theta, R, t0, L, s);
    if (e == hipSuccess) e = launch_layer<StF32, StF32>(c, c->theta + kND * 16, t0, t1, L, s);
    if (e == hipSuccess) e = launch_layer<StF32, StF64>(c, c->theta + 2 * kND * 16, t1, Z, L, s);
    return e;
}

// Loss of one batch into w.loss and dl/d(conj y) (FP32) into w.g[0], from the forward output
// w.z[2].  kind WD_LOSS_ERROR: ||y - e||^2 / ||e||^2; WD_LOSS_RESIDUAL: ||A y - r||^2 / ||r||^2,
// whose gradient needs two FP64 applications of A (scratch: the solver blocks T1 and the Jacobi
// temporary, ws[9] and ws[10], idle while training).
hipError_t batch_loss(wd_ctx* c, LearnWs& w, const double2* Rb, const double2* Eb, int L, int kind, hipStream_t s) {
    const size_t ncol = (size_t)12 * c->g.V, n = ncol * L;
    const unsigned lblocks = 1024;
    if (kind == WD_LOSS_ERROR) {
        hipError_t e = launch_colnorms(Eb, ncol, L, c->partial, gram_blocks(ncol), w.en2, s);
        if (e != hipSuccess) return e;
        k_loss<<<lblocks, kGB, 0, s>>>(w.z[2], Eb, w.en2, ncol, L, w.g[0], w.lpart);
        k_reduce_loss<<<1, kGB, 0, s>>>(w.lpart, lblocks, L, w.loss);
        return hipGetLastError();
    }
    double2* t1 = c->ws[9];
    double2* t2 = c->ws[10];
    hipError_t e = launch_colnorms(Rb, ncol, L, c->partial, gram_blocks(ncol), w.en2, s);
    if (e != hipSuccess) return e;
    k_to_f64<<<nblk(n, 256), 256, 0, s>>>(w.z[2], t1, n);
    if ((e = launch_apply_A(c, t1, t2, L, s)) != hipSuccess) return e;      // A y
    k_res_loss<<<lblocks, kGB, 0, s>>>(t2, Rb, w.en2, ncol, L, t1, w.lpart, c->g.vt & kVecTiled);  // gamma5 (A y - r) / ...
    k_reduce_loss<<<1, kGB, 0, s>>>(w.lpart, lblocks, L, w.loss);
    if ((e = launch_apply_A(c, t1, t2, L, s)) != hipSuccess) return e;      // A gamma5 (A y - r)
    k_gamma5_to_f32<<<nblk(n, 256), 256, 0, s>>>(t2, w.g[0], ncol, n, c->g.vt & kVecTiled);
    return hipGetLastError();
}

int learned_ensure(wd_ctx* c) {
    LearnWs w;
    return learn_ws(c, w);
}

}  // namespace wd

extern "C" {

int wd_set_learned(wd_ctx* c, const float* theta_host) {
    if (!c || !theta_host) return WD_EINVAL;
    for (int i = 0; i < 2 * kNL * kND * 16; ++i)
        if (!std::isfinite(theta_host[i])) return WD_EINVAL;
    if (hipMemcpyAsync(c->theta, theta_host, kNL * kND * 16 * sizeof(float2), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return WD_EHIP;
    c->have_theta = true;
    return WD_OK;
}

int wd_learned_init(wd_ctx* c, int kind) {
    if (!c || (kind != WD_LEARNED_INIT_IDENTITY && kind != WD_LEARNED_INIT_NEUMANN)) return WD_EINVAL;
    if (kind == WD_LEARNED_INIT_NEUMANN && !c->have_params) return WD_ESTATE;
    using C = std::complex<double>;
    const C I(0.0, 1.0);
    // chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]]
    const C sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}}, {{0.0, -I}, {I, 0.0}}, {{1.0, 0.0}, {0.0, -1.0}}};
    C gam[4][4][4] = {};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                gam[k][a][2 + b] = -I * sig[k][a][b];
                gam[k][2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 2; ++a) gam[3][a][2 + a] = gam[3][2 + a][a] = 1.0;
    const C coef[kNL] = {1.0, I, -I};
    std::vector<float> th(2 * kNL * kND * 16, 0.0f);
    for (int l = 0; l < kNL; ++l)
        for (int d = 0; d < kND; ++d)
            for (int r = 0; r < 4; ++r)
                for (int q = 0; q < 4; ++q) {
                    C w = 0.0;
                    if (d == 0) {
                        w = (r == q) ? 1.0 : 0.0;
                    } else if (kind == WD_LEARNED_INIT_NEUMANN) {
                        const int mu = (d - 1) / 2;
                        const double sgn = (d & 1) ? -1.0 : 1.0;  // +mu: 1 - gamma, -mu: 1 + gamma
                        w = coef[l] * c->kappa * ((r == q ? 1.0 : 0.0) + sgn * gam[mu][r][q]);
                    }
                    const size_t o = 2 * (((size_t)l * kND + d) * 16 + r * 4 + q);
                    th[o] = (float)w.real();
                    th[o + 1] = (float)w.imag();
                }
    return wd_set_learned(c, th.data());
}

int wd_get_learned(wd_ctx* c, float* theta_host) {
    if (!c || !theta_host) return WD_EINVAL;
    if (!c->have_theta) return WD_ESTATE;
    if (hipMemcpyAsync(theta_host, c->theta, kNL * kND * 16 * sizeof(float2), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return WD_EHIP;
    return WD_OK;
}

int wd_learned_apply(wd_ctx* c, const void* R, void* Z, int L, int prec) {
    if (!c || !R || !Z || L < 1 || L > c->max_L || (prec != WD_F64 && prec != WD_F32)) return WD_EINVAL;
    if (!c->have_links || !c->have_theta) return WD_ESTATE;
    const size_t bytes = (size_t)12 * c->g.V * L * 16;
    const char *a = (const char*)R, *b = (const char*)Z;
    if (a < b + bytes && b < a + bytes) return WD_EINVAL;
    int r = learned_ensure(c);
    if (r) return r;
    if (launch_learned(c, (const double2*)R, (double2*)Z, L, (Prec)prec, c->ws[10], c->ws[11], c->stream) !=
        hipSuccess)
        return WD_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return WD_EHIP;
    return WD_OK;
}

int wd_learned_train(wd_ctx* c, const void* Rp, const void* Ep, int n_pairs, int L, int steps, double lr,
                     int loss_kind, float* loss_hist) {
    if (loss_kind != WD_LOSS_ERROR && loss_kind != WD_LOSS_RESIDUAL) return WD_EINVAL;
    if (!c || !Rp || (!Ep && loss_kind == WD_LOSS_ERROR) || L < 1 || L > c->max_L || n_pairs < L || steps < 0 ||
        !(lr > 0.0))
        return WD_EINVAL;
    if (!c->have_links || !c->have_theta) return WD_ESTATE;
    if (loss_kind == WD_LOSS_RESIDUAL && !c->have_params) return WD_ESTATE;
    LearnWs w;
    int r = learn_ws(c, w);
    if (r) return r;
    hipStream_t s = c->stream;
    const size_t V = c->g.V, ncol = 12 * V;
    const int nbatch = n_pairs / L;
    const int nparam = kNL * kND * 16;
    // every normalising column (e, or r for the residual loss) must be non-zero and finite (a
    // snapshot equal to the solution gives e = 0, which the normalised loss cannot take)
    const void* Nv = loss_kind == WD_LOSS_ERROR ? Ep : Rp;
    for (int b = 0; b < nbatch; ++b) {
        double en2[WD_MAX_L];
        if (launch_colnorms((const double2*)Nv + (size_t)b * L * ncol, ncol, L, c->partial, gram_blocks(ncol), w.en2,
                            s) != hipSuccess ||
            hipMemcpyAsync(en2, w.en2, sizeof(double) * L, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return WD_EHIP;
        for (int i = 0; i < L; ++i)
            if (!(en2[i] > 0.0) || !std::isfinite(en2[i])) return WD_EINVAL;
    }
    if (launch_zero(w.m, nparam, s) != hipSuccess || launch_zero(w.v, nparam, s) != hipSuccess) return WD_EHIP;
    for (int step = 0; step < steps; ++step) {
        const int b = step % nbatch;
        const double2* Rb = (const double2*)Rp + (size_t)b * L * ncol;
        const double2* Eb = Ep ? (const double2*)Ep + (size_t)b * L * ncol : nullptr;
        // forward: z0 = R (FP64) -> z1 -> z2 -> y (FP32, kept for the loss)
        if (launch_layer<StF64, StF32>(c, c->theta, Rb, w.z[0], L, s) != hipSuccess) return WD_EHIP;
        if (launch_layer<StF32, StF32>(c, c->theta + kND * 16, w.z[0], w.z[1], L, s) != hipSuccess) return WD_EHIP;
        if (launch_layer<StF32, StF32>(c, c->theta + 2 * kND * 16, w.z[1], w.z[2], L, s) != hipSuccess)
            return WD_EHIP;
        // loss and dl/d(conj y)
        if (batch_loss(c, w, Rb, Eb, L, loss_kind, s) != hipSuccess) return WD_EHIP;
        // backward through layers 2, 1, 0
        int gi = 0;
        for (int l = kNL - 1; l >= 0; --l) {
            for (int d = 0; d < kND; ++d) {
                dim3 grid(kWgBlocks, L);
                if (l == 0)
                    k_wgrad<StF64><<<grid, kGB, 0, s>>>(c->g, c->U32, Rb, w.g[gi], d, w.gpart);
                else
                    k_wgrad<StF32><<<grid, kGB, 0, s>>>(c->g, c->U32, w.z[l - 1], w.g[gi], d, w.gpart);
                k_reduce16<<<1, kGB, 0, s>>>(w.gpart, kWgBlocks * L, w.G + (l * kND + d) * 16);
            }
            if (l > 0) {
                k_adjoint_weights<<<1, 192, 0, s>>>(c->theta + l * kND * 16, w.Wa);
                if (launch_layer<StF32, StF32>(c, w.Wa, w.g[gi], w.g[1 - gi], L, s) != hipSuccess) return WD_EHIP;
                gi = 1 - gi;
            }
        }
        if (hipGetLastError() != hipSuccess) return WD_EHIP;
        k_adam<<<nblk(nparam, 256), 256, 0, s>>>(c->theta, w.G, w.m, w.v, nparam, step + 1, lr, 0.9, 0.999, 1e-8);
        if (loss_hist) {
            double lv = 0.0;
            if (hipMemcpyAsync(&lv, w.loss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return WD_EHIP;
            loss_hist[step] = (float)lv;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return WD_EHIP;
    return WD_OK;
}

// Loss and gradient of the current theta on L pairs, without updating theta
// (G: host buffer of 3 * 9 * 16 complex128, dl/dRe + i dl/dIm).
int wd_learned_grad(wd_ctx* c, const void* R, const void* E, int L, int loss_kind, double* loss, double* G_host) {
    if (loss_kind != WD_LOSS_ERROR && loss_kind != WD_LOSS_RESIDUAL) return WD_EINVAL;
    if (!c || !R || (!E && loss_kind == WD_LOSS_ERROR) || !loss || !G_host || L < 1 || L > c->max_L)
        return WD_EINVAL;
    if (!c->have_links || !c->have_theta) return WD_ESTATE;
    if (loss_kind == WD_LOSS_RESIDUAL && !c->have_params) return WD_ESTATE;
    LearnWs w;
    int r = learn_ws(c, w);
    if (r) return r;
    hipStream_t s = c->stream;
    const double2* Rb = (const double2*)R;
    const double2* Eb = (const double2*)E;
    if (launch_layer<StF64, StF32>(c, c->theta, Rb, w.z[0], L, s) != hipSuccess) return WD_EHIP;
    if (launch_layer<StF32, StF32>(c, c->theta + kND * 16, w.z[0], w.z[1], L, s) != hipSuccess) return WD_EHIP;
    if (launch_layer<StF32, StF32>(c, c->theta + 2 * kND * 16, w.z[1], w.z[2], L, s) != hipSuccess) return WD_EHIP;
    if (batch_loss(c, w, Rb, Eb, L, loss_kind, s) != hipSuccess) return WD_EHIP;
    int gi = 0;
    for (int l = kNL - 1; l >= 0; --l) {
        for (int d = 0; d < kND; ++d) {
            dim3 grid(kWgBlocks, L);
            if (l == 0)
                k_wgrad<StF64><<<grid, kGB, 0, s>>>(c->g, c->U32, Rb, w.g[gi], d, w.gpart);
            else
                k_wgrad<StF32><<<grid, kGB, 0, s>>>(c->g, c->U32, w.z[l - 1], w.g[gi], d, w.gpart);
            k_reduce16<<<1, kGB, 0, s>>>(w.gpart, kWgBlocks * L, w.G + (l * kND + d) * 16);
        }
        if (l > 0) {
            k_adjoint_weights<<<1, 192, 0, s>>>(c->theta + l * kND * 16, w.Wa);
            if (launch_layer<StF32, StF32>(c, w.Wa, w.g[gi], w.g[1 - gi], L, s) != hipSuccess) return WD_EHIP;
            gi = 1 - gi;
        }
    }
    if (hipGetLastError() != hipSuccess) return WD_EHIP;
    if (hipMemcpyAsync(loss, w.loss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return WD_EHIP;
    if (hipMemcpyAsync(G_host, w.G, kNL * kND * 16 * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess)
        return WD_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return WD_EHIP;
    return WD_OK;
}

}  // extern "C"
