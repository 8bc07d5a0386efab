// Multi-right-hand-side Wilson-clover hopping kernels: the operator
// Y = A X and the sweeps of the Jacobi preconditioner (Sec. 2).
//
// One thread owns one lattice site and a tile of CT columns; the tiles of
// a site block sit in the same workgroup (threadIdx.y), so each gauge link
// fetched from HBM is reused from cache by all column tiles and from
// registers by the CT columns of a thread.  Spinor and link arrays are
// site-fastest (structure of arrays), so each load instruction of a
// wavefront reads 64 consecutive sites.
//
// The hop uses the rank-2 spin projectors of the chiral basis: for the
// forward hop (1 - g_mu) psi = (h, -B^dag h) with h = u - B d, for the
// backward hop (1 + g_mu) psi = (h, B^dag h) with h = u + B d, where u and d
// are the upper and lower spin pairs and g_mu = [[0, B], [B^dag, 0]] with
// B = -i s_k (k = x, y, z) and B = 1 (t).  Only the two-spinor h is
// multiplied by the link.
//
// Modes:
//   APPLY  Y = T X - kappa H X                     (the operator A)
//   JBLOCK Y = T^{-1} (Rh + kappa H X)             (Jacobi sweep, A_D = T)
//   JPOINT Y = D^{-1} (Rh + kappa H X - (T - D) X) (Jacobi sweep, A_D = diag T)
// The links arrive pre-multiplied by kappa.
#include <type_traits>

#include "wd_internal.h"

namespace wd {

namespace {

enum { APPLY = 0, JBLOCK = 1, JPOINT = 2 };

// Load the 18 pairs of one chiral 6x6 Hermitian block (packed) and expand to
// a full matrix held as 6 real diagonal entries and 15 complex upper entries.
// C is the field base; plane k of it starts at C + k*V; boff is the site's
// byte offset inside a plane.  S: storage of the block, R: compute type (the
// stored values are widened on load when R is wider).
template <class S, typename R = typename S::R>
struct Herm6 {
    R d[6];
    cx<R> o[15];
    template <bool NT = false>
    __device__ __forceinline__ void load(const typename S::P* __restrict__ C, int chir, uint32_t boff, size_t V) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const typename S::P* q = C + (size_t)(chir * 18 + i) * V;
            const cx<typename S::R> p = NT ? S::ldb_nt(q, boff) : S::ldb(q, boff);
            d[2 * i] = (R)p.re;
            d[2 * i + 1] = (R)p.im;
        }
#pragma unroll
        for (int p = 0; p < 15; ++p) {
            const typename S::P* q = C + (size_t)(chir * 18 + 3 + p) * V;
            const cx<typename S::R> v = NT ? S::ldb_nt(q, boff) : S::ldb(q, boff);
            o[p] = {(R)v.re, (R)v.im};
        }
    }
    // element (i, j) as a complex number
    __device__ __forceinline__ cx<R> at(int i, int j) const {
        if (i == j) return cx<R>{d[i], R(0)};
        if (i < j) return o[herm_index(i, j)];
        return conj(o[herm_index(j, i)]);
    }
};

// acc (+/-)= link-multiplied hop contribution of direction MU from the projected
// two-spinor h (h0: first spin component, h1: second; 3 colours each), whose
// lower spin pair is rebuilt after the colour multiply.
// FWD: link U applied to h = u - B d; BWD: U^dag applied to h = u + B d.
template <typename R, int MU, bool FWD, bool ADD>
__device__ __forceinline__ void hop_mul_acc(cx<R> (&acc)[12], const cx<R> (&u)[9], const cx<R> (&h0)[3],
                                            const cx<R> (&h1)[3]) {
    // colour: g = U h (forward) or U^dag h (backward)
    cx<R> g0[3], g1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> r0 = {R(0), R(0)}, r1 = {R(0), R(0)};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (FWD) {
                cfma(r0, u[a * 3 + b], h0[b]);
                cfma(r1, u[a * 3 + b], h1[b]);
            } else {
                cfmac(r0, u[b * 3 + a], h0[b]);
                cfmac(r1, u[b * 3 + a], h1[b]);
            }
        }
        g0[a] = r0;
        g1[a] = r1;
    }
    // reconstruct the lower spin pair and accumulate
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> l2, l3;
        if (MU == 0) {
            l2 = FWD ? tmi(g1[a]) : ti(g1[a]);
            l3 = FWD ? tmi(g0[a]) : ti(g0[a]);
        } else if (MU == 1) {
            l2 = FWD ? -g1[a] : g1[a];
            l3 = FWD ? g0[a] : -g0[a];
        } else if (MU == 2) {
            l2 = FWD ? tmi(g0[a]) : ti(g0[a]);
            l3 = FWD ? ti(g1[a]) : tmi(g1[a]);
        } else {
            l2 = FWD ? -g0[a] : g0[a];
            l3 = FWD ? -g1[a] : g1[a];
        }
        if (ADD) {
            acc[a] = acc[a] + g0[a];
            acc[3 + a] = acc[3 + a] + g1[a];
            acc[6 + a] = acc[6 + a] + l2;
            acc[9 + a] = acc[9 + a] + l3;
        } else {
            acc[a] = acc[a] - g0[a];
            acc[3 + a] = acc[3 + a] - g1[a];
            acc[6 + a] = acc[6 + a] - l2;
            acc[9 + a] = acc[9 + a] - l3;
        }
    }
}

// The projected two-spinor of direction MU from a full neighbour spinor p
// (index 3*spin + colour).
template <typename R, int MU, bool FWD>
__device__ __forceinline__ void project(const cx<R> (&p)[12], cx<R> (&h0)[3], cx<R> (&h1)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> s0 = p[c], s1 = p[3 + c], s2 = p[6 + c], s3 = p[9 + c];
        if (MU == 0) {
            h0[c] = FWD ? s0 + ti(s3) : s0 - ti(s3);
            h1[c] = FWD ? s1 + ti(s2) : s1 - ti(s2);
        } else if (MU == 1) {
            h0[c] = FWD ? s0 + s3 : s0 - s3;
            h1[c] = FWD ? s1 - s2 : s1 + s2;
        } else if (MU == 2) {
            h0[c] = FWD ? s0 + ti(s2) : s0 - ti(s2);
            h1[c] = FWD ? s1 - ti(s3) : s1 + ti(s3);
        } else {
            h0[c] = FWD ? s0 - s2 : s0 + s2;
            h1[c] = FWD ? s1 - s3 : s1 + s3;
        }
    }
}

// acc (+/-)= projected-and-multiplied hop contribution of direction MU.
template <typename R, int MU, bool FWD, bool ADD>
__device__ __forceinline__ void hop_dir(cx<R> (&acc)[12], const cx<R> (&u)[9], const cx<R> (&p)[12]) {
    cx<R> h0[3], h1[3];
    project<R, MU, FWD>(p, h0, h1);
    hop_mul_acc<R, MU, FWD, ADD>(acc, u, h0, h1);
}

// Links stored in FP32 or BF16 keep only their first two rows (12 reals,
// "reconstruct-12"): for U in SU(3) the third row is the complex conjugate of
// the cross product of the first two.  The stored rows carry kappa, so the
// product carries kappa^2 and is scaled by 1/kappa; a link whose sign was
// flipped for the antiperiodic time boundary has its first two rows flipped,
// which leaves their cross product unchanged, so the third row is negated
// there (neg).
template <class SC>
constexpr bool kCompressedLinks = sizeof(typename SC::P) < 16;

template <typename R>
__device__ __forceinline__ void third_row(cx<R> (&u)[9], R invk, bool neg) {
    const R f = neg ? -invk : invk;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        const cx<R> w = u[b1] * u[3 + b2] - u[b2] * u[3 + b1];
        u[6 + b] = {f * w.re, -f * w.im};
    }
}

// One hop direction for the CT columns of this thread: the link is loaded
// once and applied to every column.  Xc is the wave-uniform base of the
// thread's first column; link_off and nb_off are byte offsets of the link's
// site and of the neighbour site inside one plane; V is the number of sites
// (the plane stride of the links and 12 V the column stride of the block
// vector), KS the block vector's plane stride.  LT: the links may be tiled
// (FP64 fields), with their plane stride in LS (V, or 64 when tiled).  SC: storage of the links
// (widened to the compute type of S on load; FP32 and BF16 links are stored
// as two rows, planes [mu][6][V], and completed by third_row).
template <class S, int MU, bool FWD, bool ADD, int CT, bool NT = false, class SC = S, bool LT = false>
__device__ __forceinline__ void hop_all(cx<typename S::R> (&acc)[CT][12], const typename SC::P* __restrict__ Uk,
                                        const typename S::P* __restrict__ Xc, uint32_t link_off, uint32_t nb_off,
                                        size_t V, size_t KS, typename S::R invk = 0, bool neg = false,
                                        size_t LS = 0) {
    using R = typename S::R;
    // keep each direction's loads and arithmetic together: without this fence
    // the scheduler hoists the loads of all eight directions and spills
    __builtin_amdgcn_sched_barrier(0);
    cx<R> u[9];
    if constexpr (kCompressedLinks<SC>) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const cx<typename SC::R> v = SC::ldb(Uk + (size_t)(MU * 6 + k) * (LT ? LS : V), link_off);
            u[k] = {(R)v.re, (R)v.im};
        }
        third_row<R>(u, invk, neg);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const cx<typename SC::R> v = SC::ldb(Uk + (size_t)(MU * 9 + k) * (LT ? LS : V), link_off);
            u[k] = {(R)v.re, (R)v.im};
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        cx<R> p[12];
        const typename S::P* xc = Xc + (size_t)c * 12 * V;
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k] = NT ? S::ldb_nt(xc + (size_t)k * KS, nb_off) : S::ldb(xc + (size_t)k * KS, nb_off);
        hop_dir<R, MU, FWD, ADD>(acc[c], u, p);
    }
}

template <class SY, typename R>
__device__ __forceinline__ void store_out(typename SY::P* base, uint32_t boff, cx<R> v) {
    SY::stb_nt(base, boff, cx<typename SY::R>{(typename SY::R)v.re, (typename SY::R)v.im});
}

// SF: storage of the X / Rh inputs (and compute type); SY: storage of the
// output; SC: storage of the links and clover (default SF; FP64 vectors with
// FP32 or BF16 coefficients widen the coefficients on load).
// NTP: bit 0 streams the clover / T^{-1} loads (read once per launch), bit 1
// the time-direction neighbour loads (their reuse distance exceeds the L2).
template <class SF, class SY, int CT, int MODE, int NTP = 0, class SC = SF>
__global__ void __launch_bounds__(256)
    k_hop(const Geom g, const SiteMap sm, const typename SC::P* __restrict__ Uk, const typename SC::P* __restrict__ Cl,
          const typename SF::P* __restrict__ X, const typename SF::P* __restrict__ Rh, typename SY::P* __restrict__ Y,
          const int col_begin, const int ntiles, const double invk_d, const int bc_t) {
    using R = typename SF::R;
    using PF = typename SF::P;
    using PY = typename SY::P;
    const int s = map_site(g, sm, blockIdx.x, threadIdx.x);
    // blockDim.x == 64: threadIdx.y is the same for the whole wavefront
    const int tile = __builtin_amdgcn_readfirstlane(threadIdx.y);
    if (tile >= ntiles || s < 0) return;
    const int c0 = col_begin + tile * CT;
    const size_t V = g.V;
    const size_t cs = 12 * V;        // column stride of a block vector
    const size_t KS = vec_plane(g);  // its plane stride (standard or tiled layout)

    const int x = s % g.lx;
    const int y = (s / g.lx) % g.ly;
    const int z = (s / g.sxy) % g.lz;
    const int t = s / g.sxyz;
    const int n_bx = (x == 0) ? s + (g.lx - 1) : s - 1;
    const int n_by = (y == 0) ? s + (g.ly - 1) * g.lx : s - g.lx;
    const int n_bz = (z == 0) ? s + (g.lz - 1) * g.sxy : s - g.sxy;
    const int n_bt = (t == 0) ? s + (g.lt - 1) * g.sxyz : s - g.sxyz;
    // byte offsets of the sites in a plane of the block vector
    const uint32_t PB = sizeof(PF);
    const auto vo = [&](int n) -> uint32_t { return vec_site(g, n) * PB; };
    const uint32_t o_s = vo(s);
    const uint32_t o_y = vec_site(g, s) * (uint32_t)sizeof(PY);  // the output may have another pair size
    const uint32_t o_fx = vo((x == g.lx - 1) ? s - (g.lx - 1) : s + 1);
    const uint32_t o_bx = vo(n_bx);
    const uint32_t o_fy = vo((y == g.ly - 1) ? s - (g.ly - 1) * g.lx : s + g.lx);
    const uint32_t o_by = vo(n_by);
    const uint32_t o_fz = vo((z == g.lz - 1) ? s - (g.lz - 1) * g.sxy : s + g.sxy);
    const uint32_t o_bz = vo(n_bz);
    const uint32_t o_ft = vo((t == g.lt - 1) ? s - (g.lt - 1) * g.sxyz : s + g.sxyz);
    const uint32_t o_bt = vo(n_bt);
    const PF* Xc = X + (size_t)c0 * cs;
    // byte offsets of the same sites in the coefficient fields (links: co, 36 planes; 6x6
    // blocks: cb, 36 planes) and their plane stride CKS.  Only FP64 fields may be tiled (LT);
    // the FP32 / BF16 instantiations keep the plain site addressing, whose generated code is
    // the faster one for the VALU-bound BF16 sweep.
    constexpr uint32_t PC = sizeof(typename SC::P);
    constexpr bool LT = PC == 16;
    const size_t CKS = LT ? coef_plane<PC>(g) : V;
    const auto co = [&](int n) -> uint32_t {
        if constexpr (LT) return coef_site<PC>(g, n, 36) * PC;
        else return (uint32_t)n * PC;
    };
    const auto cb = co;

    cx<R> acc[CT][12];
    if (MODE == APPLY) {
        // acc = T X(s), one chiral block at a time
#pragma unroll
        for (int chir = 0; chir < 2; ++chir) {
            Herm6<SC, R> T;
            T.template load<(NTP & 1) != 0>(Cl, chir, cb(s), CKS);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                cx<R> v[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) v[k] = SF::ldb(Xc + (size_t)c * cs + (size_t)(6 * chir + k) * KS, o_s);
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cx<R> r = {R(0), R(0)};
#pragma unroll
                    for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), v[j]);
                    acc[c][6 * chir + i] = r;
                }
            }
        }
    } else {
        const PF* Rc = Rh + (size_t)c0 * cs;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
#pragma unroll
            for (int k = 0; k < 12; ++k)
                acc[c][k] = SF::ldb_nt(Rc + (size_t)c * cs + (size_t)k * KS, o_s);
        }
    }

    constexpr bool ADD = (MODE != APPLY);
    // compressed links: 1/kappa, and the antiperiodic sign of the time links on the last slice
    // (the forward link of t = Lt - 1, the backward link seen from t = 0)
    const R invk = (R)invk_d;
    const bool neg_ft = bc_t && t == g.lt - 1, neg_bt = bc_t && t == 0;
    hop_all<SF, 0, true, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(s), o_fx, V, KS, invk, false, CKS);
    hop_all<SF, 0, false, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(n_bx), o_bx, V, KS, invk, false, CKS);
    hop_all<SF, 1, true, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(s), o_fy, V, KS, invk, false, CKS);
    hop_all<SF, 1, false, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(n_by), o_by, V, KS, invk, false, CKS);
    hop_all<SF, 2, true, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(s), o_fz, V, KS, invk, false, CKS);
    hop_all<SF, 2, false, ADD, CT, false, SC, LT>(acc, Uk, Xc, co(n_bz), o_bz, V, KS, invk, false, CKS);
    hop_all<SF, 3, true, ADD, CT, (NTP & 2) != 0, SC, LT>(acc, Uk, Xc, co(s), o_ft, V, KS, invk, neg_ft, CKS);
    hop_all<SF, 3, false, ADD, CT, (NTP & 2) != 0, SC, LT>(acc, Uk, Xc, co(n_bt), o_bt, V, KS, invk, neg_bt, CKS);
    __builtin_amdgcn_sched_barrier(0);

    PY* Yc = Y + (size_t)c0 * cs;
    if (MODE == APPLY) {
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int k = 0; k < 12; ++k) store_out<SY>(Yc + (size_t)c * cs + (size_t)k * KS, o_y, acc[c][k]);
    } else {
#pragma unroll
        for (int chir = 0; chir < 2; ++chir) {
            Herm6<SC, R> T;
            T.template load<(NTP & 1) != 0>(Cl, chir, cb(s), CKS);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                {
                    cx<R> xs[6];
                    if (MODE == JPOINT) {
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            xs[k] = SF::ldb(Xc + (size_t)c * cs + (size_t)(6 * chir + k) * KS, o_s);
                    }
#pragma unroll
                    for (int i = 0; i < 6; ++i) {
                        cx<R> r;
                        if (MODE == JBLOCK) {
                            r = {R(0), R(0)};
#pragma unroll
                            for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), acc[c][6 * chir + j]);
                        } else {
                            // point reading: the diagonal slots hold 1/d
                            cx<R> q = acc[c][6 * chir + i];
#pragma unroll
                            for (int j = 0; j < 6; ++j)
                                if (j != i) q = q - T.at(i, j) * xs[j];
                            r = T.d[i] * q;
                        }
                        store_out<SY>(Yc + (size_t)c * cs + (size_t)(6 * chir + i) * KS, o_y, r);
                    }
                }
            }
        }
    }
}

// Chiral 6x6 block chir of a clover-type field staged in LDS (planes chir*18 + i).
__device__ __forceinline__ void herm_from_lds(Herm6<StF64>& T, const double2 (*sT)[64], int chir, int lane) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double2 p = sT[chir * 18 + i][lane];
        T.d[2 * i] = p.x;
        T.d[2 * i + 1] = p.y;
    }
#pragma unroll
    for (int p = 0; p < 15; ++p) {
        const double2 v = sT[chir * 18 + 3 + p][lane];
        T.o[p] = {v.x, v.y};
    }
}

// Jacobi iterates between sweeps (FP64, three or more columns) are stored in
// time-diagonal form: planes k < 6 hold a = u + d and planes k >= 6 hold
// b = u - d, where u and d are the upper and lower spin pairs (k = 3*spin +
// colour).  In the chiral basis gamma_t = [[0, 1], [1, 0]], so the forward
// time hop needs only h = u - d = b of its neighbour and the backward one
// only h = u + d = a: each time-direction neighbour load reads six planes
// instead of twelve.  The other directions rebuild u = (a + b) / 2 and
// d = (a - b) / 2 (a rounding of the last bit, well inside the FP64
// tolerance).  The right-hand side and the final output of M stay in the
// standard form.
enum { FMT_IN_TD = 1, FMT_OUT_TD = 2 };

// FP64 hop kernel for three or more columns, same modes as k_hop.  A
// workgroup owns a tile of 64 sites.  Its four waves first stage in LDS the
// links of the tile's eight hops (wave mu: U_mu(x) and U_mu(x - mu)) and the
// site's 6x6 blocks (T, T^{-1} or the point form), 108 KB, read from HBM once
// per tile instead of once per column tile.  Then wave w takes columns w,
// w + 4, ... one at a time through all eight directions, with the next
// direction's neighbour spinor in flight while the current one is applied.
// Keeping one column per wave in flight (instead of three) also keeps the
// neighbour reuse of a column within the XCD's L2.  FMT: time-diagonal input
// and / or output (sweeps only); with FMT = 0 the arithmetic and its order
// are k_hop's (bit-identical results).
template <int MODE, int FMT = 0, class SC = StF64, int VT = 0>
__global__ void __launch_bounds__(256)
    k_hop_f64(const Geom g, const SiteMap sm, const typename SC::P* __restrict__ Uk,
              const typename SC::P* __restrict__ Cl, const double2* __restrict__ X, const double2* __restrict__ Rh,
              double2* __restrict__ Y, const int L, const double invk = 0.0, const int bc_t = 0) {
    static_assert(MODE != APPLY || FMT == 0, "the operator takes and returns the standard form");
    constexpr bool TD_IN = (FMT & FMT_IN_TD) != 0, TD_OUT = (FMT & FMT_OUT_TD) != 0;
    __shared__ double2 sU[72][64];
    __shared__ double2 sT[36][64];
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int s0 = map_site(g, sm, blockIdx.x, lane);
    // the site depends on the block and the lane only, so all four waves agree on this exit
    if (!__any(s0 >= 0)) return;
    // a lane without a site (partial tile) takes the site of lane 0, which always has one: it
    // repeats lane 0's arithmetic bit for bit and stores the same values to the same addresses,
    // which keeps the stores unpredicated (a predicated store doubles the register use here)
    const int s = s0 >= 0 ? s0 : map_site(g, sm, blockIdx.x, 0);
    const size_t V = g.V;
    const size_t cs = 12 * V;         // column stride of a block vector
    // the block-vector layout is a template argument here (VT = g.vt & kVecTiled), so that the plane
    // stride of the tiled layout is a constant of the address arithmetic
    const size_t KS = VT ? (size_t)64 : V;  // plane stride of a block vector
    const auto vsite = [](int n) -> uint32_t { return VT ? (uint32_t)((n >> 6) * 768 + (n & 63)) : (uint32_t)n; };
    const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / g.sxy) % g.lz, t = s / g.sxyz;
    constexpr uint32_t PB = 16;
    int nb[8];  // the neighbours x+, x-, y+, y-, z+, z-, t+, t-
    nb[0] = (x == g.lx - 1) ? s - (g.lx - 1) : s + 1;
    nb[1] = (x == 0) ? s + (g.lx - 1) : s - 1;
    nb[2] = (y == g.ly - 1) ? s - (g.ly - 1) * g.lx : s + g.lx;
    nb[3] = (y == 0) ? s + (g.ly - 1) * g.lx : s - g.lx;
    nb[4] = (z == g.lz - 1) ? s - (g.lz - 1) * g.sxy : s + g.sxy;
    nb[5] = (z == 0) ? s + (g.lz - 1) * g.sxy : s - g.sxy;
    nb[6] = (t == g.lt - 1) ? s - (g.lt - 1) * g.sxyz : s + g.sxyz;
    nb[7] = (t == 0) ? s + (g.lt - 1) * g.sxyz : s - g.sxyz;
    uint32_t on[8];  // byte offsets of the neighbours' spinors inside a plane of a column
#pragma unroll
    for (int d = 0; d < 8; ++d) on[d] = vsite(nb[d]) * PB;
    const uint32_t o_s = vsite(s) * PB;
    {
        // coefficient fields in storage SC: FP64, or FP32 / BF16 (two-row links, completed by
        // third_row, and 6x6 blocks, all widened to FP64 here, once per tile)
        constexpr uint32_t PC = sizeof(typename SC::P);
        constexpr int NPL = kCompressedLinks<SC> ? 24 : 36;  // planes of the link field
        const size_t CKS = coef_plane<PC>(g);
        const int sb = (w == 0) ? nb[1] : (w == 1) ? nb[3] : (w == 2) ? nb[5] : nb[7];
        const uint32_t c_s = coef_site<PC>(g, s, NPL) * PC, c_b = coef_site<PC>(g, sb, NPL) * PC;
        const uint32_t t_s = coef_site<PC>(g, s, 36) * PC;
        if constexpr (kCompressedLinks<SC>) {
            const bool neg_f = (w == 3) && bc_t && t == g.lt - 1, neg_b = (w == 3) && bc_t && t == 0;
            cx<double> uf[9], ub[9];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const typename SC::P* pl = Uk + (size_t)(w * 6 + k) * CKS;
                const cx<typename SC::R> f = SC::ldb(pl, c_s), b = SC::ldb(pl, c_b);
                uf[k] = {(double)f.re, (double)f.im};
                ub[k] = {(double)b.re, (double)b.im};
            }
            third_row<double>(uf, invk, neg_f);
            third_row<double>(ub, invk, neg_b);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                sU[(2 * w) * 9 + k][lane] = make_double2(uf[k].re, uf[k].im);
                sU[(2 * w + 1) * 9 + k][lane] = make_double2(ub[k].re, ub[k].im);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const typename SC::P* pl = Uk + (size_t)(w * 9 + k) * CKS;
                const cx<typename SC::R> f = SC::ldb(pl, c_s), b = SC::ldb(pl, c_b);
                sU[(2 * w) * 9 + k][lane] = make_double2((double)f.re, (double)f.im);
                sU[(2 * w + 1) * 9 + k][lane] = make_double2((double)b.re, (double)b.im);
            }
        }
        // the blocks are read by this tile only: streamed, so they do not take L2 room from the
        // neighbour spinors and links other tiles reuse (measured 1-2 % faster)
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const cx<typename SC::R> v = SC::ldb_nt(Cl + (size_t)(w * 9 + j) * CKS, t_s);
            sT[w * 9 + j][lane] = make_double2((double)v.re, (double)v.im);
        }
    }
    __syncthreads();
    constexpr bool ADD = MODE != APPLY;
    for (int c = w; c < L; c += 4) {
        // the LDS lane index is made opaque per column, so that the compiler re-reads the staged
        // links and blocks in every column instead of hoisting all 108 of them into registers
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const double2* xc = X + (size_t)c * cs;
        cx<double> acc[12];
        if (MODE == APPLY) {
#pragma unroll
            for (int chir = 0; chir < 2; ++chir) {
                Herm6<StF64> T;
                herm_from_lds(T, sT, chir, ln);
                cx<double> v[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) v[k] = StF64::ldb(xc + (size_t)(6 * chir + k) * KS, o_s);
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cx<double> r = {0.0, 0.0};
#pragma unroll
                    for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), v[j]);
                    acc[6 * chir + i] = r;
                }
            }
        } else {
            const double2* rc = Rh + (size_t)c * cs;
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = StF64::ldb_nt(rc + (size_t)k * KS, o_s);
        }
        // neighbour spinor of direction d.  The sweeps stream the time-direction neighbours, as
        // k_hop does; the operator, whose site map walks four t-slices together, loads them like
        // the others (measured 1.8 % faster there, no gain in the sweeps).  In the time-diagonal
        // form the time hops load only the half they project onto.
        constexpr bool T_NT = MODE != APPLY;
        cx<double> p[2][12];
        auto load_dir = [&](cx<double>(&dst)[12], int d) {
            if (TD_IN && d >= 6) {
                const int k0 = (d == 6) ? 6 : 0;  // t+: b = u - d, t-: a = u + d
#pragma unroll
                for (int k = 0; k < 6; ++k) dst[k] = StF64::ldb_nt(xc + (size_t)(k0 + k) * KS, on[d]);
                return;
            }
#pragma unroll
            for (int k = 0; k < 12; ++k)
                dst[k] = (T_NT && d >= 6) ? StF64::ldb_nt(xc + (size_t)k * KS, on[d]) : StF64::ldb(xc + (size_t)k * KS, on[d]);
        };
        load_dir(p[0], 0);
        static_for<0, 8>([&](auto dc) {
            constexpr int D = decltype(dc)::value;
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (D + 1 < 8) load_dir(p[(D + 1) % 2], D + 1);
            cx<double> u[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double2 v = sU[D * 9 + k][ln];
                u[k] = {v.x, v.y};
            }
            cx<double>(&q)[12] = p[D % 2];
            if constexpr (TD_IN && D >= 6) {
                // the loaded half is the projected two-spinor itself
                cx<double> h0[3] = {q[0], q[1], q[2]}, h1[3] = {q[3], q[4], q[5]};
                hop_mul_acc<double, 3, D == 6, ADD>(acc, u, h0, h1);
            } else {
                if constexpr (TD_IN) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const cx<double> av = q[k], bv = q[k + 6];
                        q[k] = 0.5 * (av + bv);
                        q[k + 6] = 0.5 * (av - bv);
                    }
                }
                hop_dir<double, D / 2, (D % 2) == 0, ADD>(acc, u, q);
            }
        });
        __builtin_amdgcn_sched_barrier(0);
        double2* yc = Y + (size_t)c * cs;
        if (MODE == APPLY) {
#pragma unroll
            for (int k = 0; k < 12; ++k) StF64::stb_nt(yc + (size_t)k * KS, o_s, acc[k]);
        } else {
            cx<double> out[12];
#pragma unroll
            for (int chir = 0; chir < 2; ++chir) {
                Herm6<StF64> T;
                herm_from_lds(T, sT, chir, ln);
                cx<double> xs[6];
                if (MODE == JPOINT) {
                    if constexpr (TD_IN) {
                        // own site, back to the standard form: u = (a + b) / 2, d = (a - b) / 2
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            const cx<double> av = StF64::ldb(xc + (size_t)k * KS, o_s);
                            const cx<double> bv = StF64::ldb(xc + (size_t)(k + 6) * KS, o_s);
                            xs[k] = chir == 0 ? 0.5 * (av + bv) : 0.5 * (av - bv);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 6; ++k) xs[k] = StF64::ldb(xc + (size_t)(6 * chir + k) * KS, o_s);
                    }
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cx<double> r;
                    if (MODE == JBLOCK) {
                        r = {0.0, 0.0};
#pragma unroll
                        for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), acc[6 * chir + j]);
                    } else {
                        // point reading: the diagonal slots hold 1/d
                        cx<double> q = acc[6 * chir + i];
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            if (j != i) q = q - T.at(i, j) * xs[j];
                        r = T.d[i] * q;
                    }
                    if constexpr (TD_OUT) {
                        out[6 * chir + i] = r;
                    } else {
                        StF64::stb_nt(yc + (size_t)(6 * chir + i) * KS, o_s, r);
                    }
                }
            }
            if constexpr (TD_OUT) {
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    StF64::stb_nt(yc + (size_t)k * KS, o_s, out[k] + out[k + 6]);
                    StF64::stb_nt(yc + (size_t)(k + 6) * KS, o_s, out[k] - out[k + 6]);
                }
            }
        }
    }
}

// FP32 / BF16 hop kernel for three or more columns (used for FP32): the LDS-staged
// structure of k_hop_f64 in the compute type (float).  The staging rebuilds the third row of
// every two-row link once per tile (instead of once per column tile) and widens
// the links and the 6x6 blocks to float, 54 KB of LDS; the arithmetic and its
// order are k_hop's, so the results are bit-identical to it.
template <class SF, class SY, int MODE>
__global__ void __launch_bounds__(256)
    k_hop_lds_lp(const Geom g, const SiteMap sm, const typename SF::P* __restrict__ Uk,
                 const typename SF::P* __restrict__ Cl, const typename SF::P* __restrict__ X,
                 const typename SF::P* __restrict__ Rh, typename SY::P* __restrict__ Y, const int L,
                 const float invk, const int bc_t) {
    using R = typename SF::R;
    using PF = typename SF::P;
    static_assert(sizeof(R) == 4, "FP32 compute");
    __shared__ float2 sU[72][64];
    __shared__ float2 sT[36][64];
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int s0 = map_site(g, sm, blockIdx.x, lane);
    if (!__any(s0 >= 0)) return;  // the same for all four waves
    // a lane without a site takes lane 0's site (unpredicated stores, as in k_hop_f64)
    const int s = s0 >= 0 ? s0 : map_site(g, sm, blockIdx.x, 0);
    const size_t V = g.V;
    const size_t cs = 12 * V;         // column stride of a block vector
    const size_t KS = vec_plane(g);   // its plane stride (standard or tiled layout)
    const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / g.sxy) % g.lz, t = s / g.sxyz;
    constexpr uint32_t PB = sizeof(PF);
    int nb[8];  // the neighbours x+, x-, y+, y-, z+, z-, t+, t-
    nb[0] = (x == g.lx - 1) ? s - (g.lx - 1) : s + 1;
    nb[1] = (x == 0) ? s + (g.lx - 1) : s - 1;
    nb[2] = (y == g.ly - 1) ? s - (g.ly - 1) * g.lx : s + g.lx;
    nb[3] = (y == 0) ? s + (g.ly - 1) * g.lx : s - g.lx;
    nb[4] = (z == g.lz - 1) ? s - (g.lz - 1) * g.sxy : s + g.sxy;
    nb[5] = (z == 0) ? s + (g.lz - 1) * g.sxy : s - g.sxy;
    nb[6] = (t == g.lt - 1) ? s - (g.lt - 1) * g.sxyz : s + g.sxyz;
    nb[7] = (t == 0) ? s + (g.lt - 1) * g.sxyz : s - g.sxyz;
    uint32_t on[8];  // byte offsets of the neighbours' spinors inside a plane of a column
#pragma unroll
    for (int d = 0; d < 8; ++d) on[d] = vec_site(g, nb[d]) * PB;
    const uint32_t o_s = vec_site(g, s) * PB;
    // the site in the coefficient fields (two-row links: 24 planes; blocks: 36)
    const size_t CKS = coef_plane<PB>(g);
    const uint32_t c_s = coef_site<PB>(g, s, 24) * PB, t_s = coef_site<PB>(g, s, 36) * PB;
    {
        // wave mu: the two stored rows of U_mu(x) and U_mu(x - mu), completed by third_row (the
        // antiperiodic sign of the time links on the last slice, seen from t = Lt - 1 forward and
        // from t = 0 backward), then stored in LDS as full 3 x 3 float matrices
        const uint32_t ob = coef_site<PB>(g, (w == 0) ? nb[1] : (w == 1) ? nb[3] : (w == 2) ? nb[5] : nb[7], 24) * PB;
        const bool neg_f = (w == 3) && bc_t && t == g.lt - 1, neg_b = (w == 3) && bc_t && t == 0;
        cx<R> uf[9], ub[9];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const PF* pl = Uk + (size_t)(w * 6 + k) * CKS;
            uf[k] = SF::ldb(pl, c_s);
            ub[k] = SF::ldb(pl, ob);
        }
        third_row<R>(uf, invk, neg_f);
        third_row<R>(ub, invk, neg_b);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sU[(2 * w) * 9 + k][lane] = make_float2(uf[k].re, uf[k].im);
            sU[(2 * w + 1) * 9 + k][lane] = make_float2(ub[k].re, ub[k].im);
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const cx<R> v = SF::ldb_nt(Cl + (size_t)(w * 9 + j) * CKS, t_s);
            sT[w * 9 + j][lane] = make_float2(v.re, v.im);
        }
    }
    __syncthreads();
    constexpr bool ADD = MODE != APPLY;
    for (int c = w; c < L; c += 4) {
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const PF* xc = X + (size_t)c * cs;
        cx<R> acc[12];
        auto herm = [&](Herm6<StF32>& T, int chir) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float2 q = sT[chir * 18 + i][ln];
                T.d[2 * i] = q.x;
                T.d[2 * i + 1] = q.y;
            }
#pragma unroll
            for (int q = 0; q < 15; ++q) {
                const float2 v = sT[chir * 18 + 3 + q][ln];
                T.o[q] = {v.x, v.y};
            }
        };
        if (MODE == APPLY) {
#pragma unroll
            for (int chir = 0; chir < 2; ++chir) {
                Herm6<StF32> T;
                herm(T, chir);
                cx<R> v[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) v[k] = SF::ldb(xc + (size_t)(6 * chir + k) * KS, o_s);
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cx<R> r = {R(0), R(0)};
#pragma unroll
                    for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), v[j]);
                    acc[6 * chir + i] = r;
                }
            }
        } else {
            const PF* rc = Rh + (size_t)c * cs;
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = SF::ldb_nt(rc + (size_t)k * KS, o_s);
        }
        cx<R> p[2][12];
        auto load_dir = [&](cx<R>(&dst)[12], int d) {
#pragma unroll
            for (int k = 0; k < 12; ++k)
                dst[k] = (d >= 6) ? SF::ldb_nt(xc + (size_t)k * KS, on[d]) : SF::ldb(xc + (size_t)k * KS, on[d]);
        };
        load_dir(p[0], 0);
        static_for<0, 8>([&](auto dc) {
            constexpr int D = decltype(dc)::value;
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (D + 1 < 8) load_dir(p[(D + 1) % 2], D + 1);
            cx<R> u[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float2 v = sU[D * 9 + k][ln];
                u[k] = {v.x, v.y};
            }
            hop_dir<R, D / 2, (D % 2) == 0, ADD>(acc, u, p[D % 2]);
        });
        __builtin_amdgcn_sched_barrier(0);
        typename SY::P* yc = Y + (size_t)c * cs;
        const uint32_t o_y = vec_site(g, s) * (uint32_t)sizeof(typename SY::P);
        if (MODE == APPLY) {
#pragma unroll
            for (int k = 0; k < 12; ++k) store_out<SY>(yc + (size_t)k * KS, o_y, acc[k]);
        } else {
#pragma unroll
            for (int chir = 0; chir < 2; ++chir) {
                Herm6<StF32> T;
                herm(T, chir);
                cx<R> xs[6];
                if (MODE == JPOINT) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) xs[k] = SF::ldb(xc + (size_t)(6 * chir + k) * KS, o_s);
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cx<R> r;
                    if (MODE == JBLOCK) {
                        r = {R(0), R(0)};
#pragma unroll
                        for (int j = 0; j < 6; ++j) cfma(r, T.at(i, j), acc[6 * chir + j]);
                    } else {
                        cx<R> q = acc[6 * chir + i];
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            if (j != i) q = q - T.at(i, j) * xs[j];
                        r = T.d[i] * q;
                    }
                    store_out<SY>(yc + (size_t)(6 * chir + i) * KS, o_y, r);
                }
            }
        }
    }
}

// First Jacobi sweep from G_0 = 0: Y = A_D^{-1} R (site-local, no hop).
// SI: input storage, SF: compute (and clover) storage, SY: output storage,
// SC: clover storage when it differs from SF (widened on load); with
// RL != nullptr the input is also written out in format SF (the
// low-precision copy of the right-hand side used by later sweeps).
template <class SI, class SF, class SY, int MODE, class SC = SF>
__global__ void __launch_bounds__(256)
    k_first_sweep(const Geom g, const typename SC::P* __restrict__ Cl, const typename SI::P* __restrict__ Rin,
                  typename SF::P* __restrict__ RL, typename SY::P* __restrict__ Y, const int L) {
    // one thread per site; the site's A_D^{-1} block stays in registers for all L columns
    using R = typename SF::R;
    const size_t V = g.V;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t cs = 12 * V;        // column stride of a block vector
    const size_t KS = vec_plane(g);  // its plane stride (standard or tiled layout)
    const uint32_t vs = vec_site(g, s);
    const uint32_t oF = vs * sizeof(typename SF::P);
    const uint32_t oI = vs * sizeof(typename SI::P);
    const uint32_t oY = vs * sizeof(typename SY::P);
    constexpr int PC = sizeof(typename SC::P);
    const uint32_t oC = coef_site<PC>(g, s, 36) * PC;
    const size_t CKS = coef_plane<PC>(g);
#pragma unroll
    for (int chir = 0; chir < 2; ++chir) {
        Herm6<SC, R> T;
        T.load(Cl, chir, oC, CKS);
        for (int col = 0; col < L; ++col) {
            const typename SI::P* Rc = Rin + (size_t)col * cs;
            cx<R> v[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const auto w = SI::ldb_nt(Rc + (size_t)(6 * chir + k) * KS, oI);
                v[k] = {(R)w.re, (R)w.im};
                if (RL != nullptr) {
                    // later sweeps read the rounded copy; use the same rounded value here
                    SF::stb(RL + (size_t)col * cs + (size_t)(6 * chir + k) * KS, oF, v[k]);
                    v[k] = SF::rnd(v[k]);
                }
            }
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                cx<R> o = {R(0), R(0)};
                if (MODE == JBLOCK) {
#pragma unroll
                    for (int j = 0; j < 6; ++j) cfma(o, T.at(r, j), v[j]);
                } else {
                    o = T.d[r] * v[r];
                }
                store_out<SY>(Y + (size_t)col * cs + (size_t)(6 * chir + r) * KS, oY, o);
            }
        }
    }
}

template <class S>
__global__ void k_from_lowp(const typename S::P* __restrict__ src, double2* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const auto v = S::ld(src, i);
    dst[i] = make_double2((double)v.re, (double)v.im);
}

// Streaming-load policy of the hop kernel: the time-direction neighbours are
// streamed (measured about 5 % faster at 32^3 x 64, L = 12 than no streaming,
// streaming the clover as well, or both).
constexpr int kHopNTP = 2;

// Columns per thread for L right-hand sides.  FP32 / BF16 storage takes
// four-column tiles from L = 10 on (measured a few per cent faster than three
// at L = 12; FP64 is fastest with three).
int tile_cols(int L, bool lowp) {
    if (L <= 2) return 1;
    if (L <= 8) return 2;
    if (L <= 12) return (lowp && L >= 10) ? 4 : 3;
    return 4;
}

// What the compressed links need besides the field: 1/kappa and the time boundary condition.
struct LinkInfo {
    double invk;
    int bc_t;
};
LinkInfo link_info(const wd_ctx* c) { return {c->kappa != 0.0 ? 1.0 / c->kappa : 0.0, c->bc_t}; }

template <class SF, class SY, int MODE, int CT, class SC = SF>
hipError_t launch_hop_ct(const Geom& g, const LinkInfo& li, const void* Uk, const void* Cl, const void* X,
                         const void* Rh, void* Y, int col_begin, int ntiles, hipStream_t s) {
    if (ntiles > 4) return hipErrorInvalidValue;  // at most 4 wavefronts (256 threads) per site tile
    const double bytes_site = 12.0 * CT * ntiles * sizeof(typename SF::P) + 72.0 * sizeof(typename SC::P);
    const SiteMap sm = make_site_map(g, bytes_site);
    dim3 block(64, ntiles), grid(sm.nblk);
    using PF = typename SF::P;
    using PY = typename SY::P;
    using PC = typename SC::P;
    k_hop<SF, SY, CT, MODE, kHopNTP, SC><<<grid, block, 0, s>>>(g, sm, (const PC*)Uk, (const PC*)Cl, (const PF*)X,
                                                             (const PF*)Rh, (PY*)Y, col_begin, ntiles, li.invk,
                                                             li.bc_t);
    return hipGetLastError();
}

template <class SF, class SY, int MODE, class SC = SF>
hipError_t launch_hop_cols(const Geom& g, const LinkInfo& li, const void* Uk, const void* Cl, const void* X,
                           const void* Rh, void* Y, int CT, int col_begin, int ntiles, hipStream_t s) {
    switch (CT) {
        case 1: return launch_hop_ct<SF, SY, MODE, 1, SC>(g, li, Uk, Cl, X, Rh, Y, col_begin, ntiles, s);
        case 2: return launch_hop_ct<SF, SY, MODE, 2, SC>(g, li, Uk, Cl, X, Rh, Y, col_begin, ntiles, s);
        case 3: return launch_hop_ct<SF, SY, MODE, 3, SC>(g, li, Uk, Cl, X, Rh, Y, col_begin, ntiles, s);
        case 4: return launch_hop_ct<SF, SY, MODE, 4, SC>(g, li, Uk, Cl, X, Rh, Y, col_begin, ntiles, s);
        default: return hipErrorInvalidValue;
    }
}

// L columns: launches of up to four tiles of CT columns, then one launch for
// the remainder (fewer than CT columns).
template <class SF, class SY, int MODE, class SC = SF>
hipError_t launch_hop_t(const Geom& g, const LinkInfo& li, const void* Uk, const void* Cl, const void* X,
                        const void* Rh, void* Y, int L, hipStream_t s) {
    if constexpr (std::is_same_v<SF, StF64> && std::is_same_v<SY, StF64>) {
        // FP64 vectors from three columns on: the LDS-staged kernel (measured faster at every
        // L >= 3 at 32^3 x 64; with one or two columns the staging cannot be shared by enough
        // waves); the links and blocks may be stored in FP32 or BF16 (SC)
        if (L >= 3) {
            // t-slices walked together: four for the operator, two for the sweeps (measured at
            // 32^3 x 64, L = 12 in the tiled layout: A X 3.53 against 3.61 ms with one slice at
            // a time; the sweep reads 18.2 instead of 20.1 GB in the same time)
            const SiteMap sm = make_site_map_rows(g, 12.0 * L * 16 + 72.0 * 16, MODE == APPLY ? 4 : 2);
            dim3 block(64, 4), grid(sm.nblk);
            if (g.vt & kVecTiled)
                k_hop_f64<MODE, 0, SC, 1><<<grid, block, 0, s>>>(
                    g, sm, (const typename SC::P*)Uk, (const typename SC::P*)Cl, (const double2*)X,
                    (const double2*)Rh, (double2*)Y, L, li.invk, li.bc_t);
            else
                k_hop_f64<MODE, 0, SC, 0><<<grid, block, 0, s>>>(
                    g, sm, (const typename SC::P*)Uk, (const typename SC::P*)Cl, (const double2*)X,
                    (const double2*)Rh, (double2*)Y, L, li.invk, li.bc_t);
            return hipGetLastError();
        }
    }
    if constexpr (std::is_same_v<SF, StF32> && std::is_same_v<SC, SF>) {
        // FP32 from three columns on: the LDS-staged kernel (sweep 2.51 against 2.96 ms at
        // 32^3 x 64, L = 12; BF16 keeps the register-tiled kernel, whose four-column tiles share
        // each rebuilt link: 1.42 against 1.52 ms LDS-staged)
        if (L >= 3) {
            const SiteMap sm = make_site_map_rows(g, 12.0 * L * sizeof(typename SF::P) + 72.0 * 8);
            dim3 block(64, 4), grid(sm.nblk);
            k_hop_lds_lp<SF, SY, MODE><<<grid, block, 0, s>>>(g, sm, (const typename SF::P*)Uk,
                                                             (const typename SF::P*)Cl, (const typename SF::P*)X,
                                                             (const typename SF::P*)Rh, (typename SY::P*)Y, L,
                                                             (float)li.invk, li.bc_t);
            return hipGetLastError();
        }
    }
    const int CT = tile_cols(L, sizeof(typename SF::P) < 16);
    const int full = L / CT, rem = L % CT;
    hipError_t e = hipSuccess;
    for (int t0 = 0; t0 < full && e == hipSuccess; t0 += 4) {
        const int nt = full - t0 < 4 ? full - t0 : 4;
        e = launch_hop_cols<SF, SY, MODE, SC>(g, li, Uk, Cl, X, Rh, Y, CT, t0 * CT, nt, s);
    }
    if (e != hipSuccess || rem == 0) return e;
    return launch_hop_cols<SF, SY, MODE, SC>(g, li, Uk, Cl, X, Rh, Y, rem, full * CT, 1, s);
}

template <class SI, class SF, class SY, class SC = SF>
hipError_t launch_first(const wd_ctx* c, const void* Cl, const void* Rin, void* RL, void* Y, int L, hipStream_t s) {
    const unsigned nb = (unsigned)((c->g.V + 255) / 256);
    if (c->jacobi_kind == WD_JACOBI_POINT)
        k_first_sweep<SI, SF, SY, JPOINT, SC><<<nb, 256, 0, s>>>(c->g, (const typename SC::P*)Cl,
                                                                  (const typename SI::P*)Rin, (typename SF::P*)RL,
                                                                  (typename SY::P*)Y, L);
    else
        k_first_sweep<SI, SF, SY, JBLOCK, SC><<<nb, 256, 0, s>>>(c->g, (const typename SC::P*)Cl,
                                                                  (const typename SI::P*)Rin, (typename SF::P*)RL,
                                                                  (typename SY::P*)Y, L);
    return hipGetLastError();
}

template <class SF, class SY, class SC = SF>
hipError_t launch_sweep(const wd_ctx* c, int pi, const void* X, const void* Rh, void* Y, int L, hipStream_t s) {
    if (c->jacobi_kind == WD_JACOBI_POINT)
        return launch_hop_t<SF, SY, JPOINT, SC>(c->g, link_info(c), c->f.Uk[pi], c->f.Tp[pi], X, Rh, Y, L, s);
    return launch_hop_t<SF, SY, JBLOCK, SC>(c->g, link_info(c), c->f.Uk[pi], c->f.Ti[pi], X, Rh, Y, L, s);
}

// One FP64 sweep of three or more columns with the iterates in the format FMT
// (FMT_IN_TD / FMT_OUT_TD: time-diagonal input / output).
template <int FMT, class SC = StF64>
hipError_t launch_sweep_td(const wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, hipStream_t s) {
    const SiteMap sm = make_site_map_rows(c->g, 12.0 * L * 16 + 72.0 * 16, 2);
    dim3 block(64, 4), grid(sm.nblk);
    constexpr int pi = std::is_same_v<SC, StF64> ? 0 : std::is_same_v<SC, StF32> ? 1 : 2;
    using PC = typename SC::P;
    const LinkInfo li = link_info(c);
    const bool pt = c->jacobi_kind == WD_JACOBI_POINT;
    const PC* U = (const PC*)c->f.Uk[pi];
    const PC* C = (const PC*)(pt ? c->f.Tp[pi] : c->f.Ti[pi]);
    if (pt && (c->g.vt & kVecTiled))
        k_hop_f64<JPOINT, FMT, SC, 1><<<grid, block, 0, s>>>(c->g, sm, U, C, X, R, Y, L, li.invk, li.bc_t);
    else if (pt)
        k_hop_f64<JPOINT, FMT, SC, 0><<<grid, block, 0, s>>>(c->g, sm, U, C, X, R, Y, L, li.invk, li.bc_t);
    else if (c->g.vt & kVecTiled)
        k_hop_f64<JBLOCK, FMT, SC, 1><<<grid, block, 0, s>>>(c->g, sm, U, C, X, R, Y, L, li.invk, li.bc_t);
    else
        k_hop_f64<JBLOCK, FMT, SC, 0><<<grid, block, 0, s>>>(c->g, sm, U, C, X, R, Y, L, li.invk, li.bc_t);
    return hipGetLastError();
}

// Sweeps 2 .. j of a Jacobi application with FP64 iterates (coefficients in SC): from three
// columns on with the iterates between sweeps in the time-diagonal form, else in the standard
// form through launch_sweep.  `first` holds the first sweep's output; the result lands in Z.
template <class SC>
hipError_t sweep_chain(wd_ctx* c, int pi, const double2* R, double2* Z, double2* tmp, double2* out, int L, int j,
                       hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int i = 2; i <= j && e == hipSuccess; ++i) {
        double2* in = out;
        out = ((j - i) % 2 == 0) ? Z : tmp;
        if (L >= 3 && j >= 3) {
            // the second sweep reads the standard output of the first, the last one writes Z in
            // the standard form
            if (i == 2)
                e = launch_sweep_td<FMT_OUT_TD, SC>(c, in, R, out, L, s);
            else if (i < j)
                e = launch_sweep_td<FMT_IN_TD | FMT_OUT_TD, SC>(c, in, R, out, L, s);
            else
                e = launch_sweep_td<FMT_IN_TD, SC>(c, in, R, out, L, s);
        } else {
            e = launch_sweep<StF64, StF64, SC>(c, pi, in, R, out, L, s);
        }
    }
    return e;
}

// j sweeps with FP64 vectors and arithmetic and the links and A_D^{-1} of
// storage format SC (FP32 or BF16): a fixed linear operator, unlike the
// low-precision form, whose rounding of the vectors makes it nonlinear.
template <class SC>
hipError_t jacobi_coef(wd_ctx* c, int pi, const double2* R, double2* Z, int L, int j, hipStream_t s) {
    const void* clf = (c->jacobi_kind == WD_JACOBI_POINT) ? c->f.Tp[pi] : c->f.Ti[pi];
    double2* tmp = c->ws[10];
    double2* out = ((j - 1) % 2 == 0) ? Z : tmp;
    hipError_t e = launch_first<StF64, StF64, StF64, SC>(c, clf, R, nullptr, out, L, s);
    if (e != hipSuccess) return e;
    return sweep_chain<SC>(c, pi, R, Z, tmp, out, L, j, s);
}

// j sweeps in storage format S (FP32 or BF16), FP64 in and out.
template <class S>
hipError_t jacobi_lowp(wd_ctx* c, int pi, const double2* R, double2* Z, int L, int j, hipStream_t s) {
    const void* clf = (c->jacobi_kind == WD_JACOBI_POINT) ? c->f.Tp[pi] : c->f.Ti[pi];
    void* rl = c->lp[2];
    if (j == 1) return launch_first<StF64, S, StF64>(c, clf, R, nullptr, Z, L, s);
    hipError_t e = launch_first<StF64, S, S>(c, clf, R, rl, c->lp[0], L, s);
    if (e != hipSuccess) return e;
    int cur = 0;
    for (int i = 2; i < j; ++i) {
        e = launch_sweep<S, S>(c, pi, c->lp[cur], rl, c->lp[1 - cur], L, s);
        if (e != hipSuccess) return e;
        cur = 1 - cur;
    }
    return launch_sweep<S, StF64>(c, pi, c->lp[cur], rl, Z, L, s);
}

}  // namespace

hipError_t launch_apply_A(const wd_ctx* c, const double2* X, double2* Y, int L, hipStream_t s) {
    // Tc[0]: T in the hop kernels' field layout (f.T keeps the standard one)
    return launch_hop_t<StF64, StF64, APPLY>(c->g, link_info(c), c->f.Uk[0], c->f.Tc[0], X, nullptr, Y, L, s);
}

hipError_t launch_sweep_f64(const wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, hipStream_t s) {
    // the sweep jacobi_precond runs most often: from three columns on, the middle sweep with
    // time-diagonal input and output
    if (L >= 3) return launch_sweep_td<FMT_IN_TD | FMT_OUT_TD>(c, X, R, Y, L, s);
    return launch_sweep<StF64, StF64>(c, 0, X, R, Y, L, s);
}

hipError_t launch_sweep_coef(const wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, Prec coef,
                             hipStream_t s) {
    // as launch_sweep_f64: from three columns on, the middle sweep (time-diagonal in and out)
    if (coef == Prec::F32)
        return L >= 3 ? launch_sweep_td<FMT_IN_TD | FMT_OUT_TD, StF32>(c, X, R, Y, L, s)
                      : launch_sweep<StF64, StF64, StF32>(c, 1, X, R, Y, L, s);
    if (coef == Prec::BF16)
        return L >= 3 ? launch_sweep_td<FMT_IN_TD | FMT_OUT_TD, StBF16>(c, X, R, Y, L, s)
                      : launch_sweep<StF64, StF64, StBF16>(c, 2, X, R, Y, L, s);
    return hipErrorInvalidValue;
}

hipError_t launch_apply_A_lowp(wd_ctx* c, const double2* X, double2* Y, int L, Prec p, hipStream_t s) {
    const size_t n = (size_t)12 * c->g.V * L;
    hipError_t e = launch_to_lowp(X, c->lp[0], p, n, s);
    if (e != hipSuccess) return e;
    if (p == Prec::F32)
        return launch_hop_t<StF32, StF64, APPLY>(c->g, link_info(c), c->f.Uk[1], c->f.Tc[1], c->lp[0], nullptr, Y, L,
                                                 s);
    return launch_hop_t<StBF16, StF64, APPLY>(c->g, link_info(c), c->f.Uk[2], c->f.Tc[2], c->lp[0], nullptr, Y, L, s);
}

hipError_t launch_jacobi_coef(wd_ctx* c, const double2* R, double2* Z, int L, int j, Prec coef, hipStream_t s) {
    if (j == 0) return launch_copy(Z, R, (size_t)12 * c->g.V * L, s);
    if (coef == Prec::F32) return jacobi_coef<StF32>(c, 1, R, Z, L, j, s);
    if (coef == Prec::BF16) return jacobi_coef<StBF16>(c, 2, R, Z, L, j, s);
    return hipErrorInvalidValue;
}

hipError_t launch_jacobi(wd_ctx* c, const double2* R, double2* Z, int L, int j, Prec p, hipStream_t s) {
    const size_t n = (size_t)12 * c->g.V * L;
    if (j == 0) return launch_copy(Z, R, n, s);
    if (p == Prec::F32) return jacobi_lowp<StF32>(c, 1, R, Z, L, j, s);
    if (p == Prec::BF16) return jacobi_lowp<StBF16>(c, 2, R, Z, L, j, s);
    const void* clf = (c->jacobi_kind == WD_JACOBI_POINT) ? c->f.Tp[0] : c->f.Ti[0];
    // FP64: alternate between Z and the scratch block so that sweep j lands in Z
    double2* tmp = c->ws[10];
    double2* out = ((j - 1) % 2 == 0) ? Z : tmp;
    hipError_t e = launch_first<StF64, StF64, StF64>(c, clf, R, nullptr, out, L, s);
    if (e != hipSuccess) return e;
    return sweep_chain<StF64>(c, 0, R, Z, tmp, out, L, j, s);
}

// Throughput measurement in FP32 / BF16 storage: X (and R) are rounded into
// the low-precision buffers once, then the kernel runs nrep times on them.
// mode 0: Y = A X with FP64 output; mode 1: a middle Jacobi sweep with
// low-precision input and output (the output stays in the third buffer).
hipError_t launch_hop_repeat_lowp(wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, int mode, Prec p,
                                  int nrep, hipStream_t s) {
    const size_t n = (size_t)12 * c->g.V * L;
    const int pi = p == Prec::F32 ? 1 : 2;
    hipError_t e = launch_to_lowp(X, c->lp[0], p, n, s);
    if (e == hipSuccess && mode == 1) e = launch_to_lowp(R, c->lp[2], p, n, s);
    for (int i = 0; i < nrep && e == hipSuccess; ++i) {
        if (mode == 0)
            e = p == Prec::F32
                    ? launch_hop_t<StF32, StF64, APPLY>(c->g, link_info(c), c->f.Uk[1], c->f.Tc[1], c->lp[0], nullptr,
                                                        Y, L, s)
                    : launch_hop_t<StBF16, StF64, APPLY>(c->g, link_info(c), c->f.Uk[2], c->f.Tc[2], c->lp[0],
                                                         nullptr, Y, L, s);
        else
            e = p == Prec::F32 ? launch_sweep<StF32, StF32>(c, pi, c->lp[0], c->lp[2], c->lp[1], L, s)
                               : launch_sweep<StBF16, StBF16>(c, pi, c->lp[0], c->lp[2], c->lp[1], L, s);
    }
    return e;
}

}  // namespace wd
