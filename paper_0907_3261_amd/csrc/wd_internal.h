// Internal declarations of the wdsolve library: device data layouts,
// complex arithmetic, storage formats and the kernel launchers shared by the
// translation units.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <cstddef>
#include <cstdint>

#include "../../include/wdsolve.h"

namespace wd {

// ---------------------------------------------------------------------------
// Complex numbers over a compute real R (double or float)
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// i * a and -i * a
template <typename R>
__host__ __device__ __forceinline__ cx<R> ti(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> tmi(cx<R> a) { return {a.im, -a.re}; }
// a += b * c, a += conj(b) * c
template <typename R>
__host__ __device__ __forceinline__ void cfma(cx<R>& a, cx<R> b, cx<R> c) {
    a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
    a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}
template <typename R>
__host__ __device__ __forceinline__ void cfmac(cx<R>& a, cx<R> b, cx<R> c) {
    a.re = fma(b.re, c.re, fma(b.im, c.im, a.re));
    a.im = fma(b.re, c.im, fma(-b.im, c.re, a.im));
}

// ---------------------------------------------------------------------------
// Storage formats of complex pairs in device memory
// ---------------------------------------------------------------------------
// Every field lives as an array of complex "pairs" (re, im) in one of three
// storage formats; kernels load into and compute in the format's real R.
//
// ldb/stb address a pair by a wave-uniform plane base pointer plus a 32-bit
// per-lane byte offset, which maps to the scalar-base + vector-offset form
// of the global memory instructions (one offset register serves every plane
// of a field instead of one 64-bit address per load).
#define WD_BYTE_OFFSET_ACCESSORS                                                        \
    __device__ __forceinline__ static cx<R> ldb(const P* base, uint32_t boff) {         \
        return ld(reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + boff), 0); \
    }                                                                                   \
    __device__ __forceinline__ static void stb(P* base, uint32_t boff, cx<R> v) {       \
        st(reinterpret_cast<P*>(reinterpret_cast<char*>(base) + boff), 0, v);          \
    }                                                                                   \
    __device__ __forceinline__ static cx<R> ldb_nt(const P* base, uint32_t boff) {      \
        return ld_nt(reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + boff)); \
    }                                                                                   \
    __device__ __forceinline__ static void stb_nt(P* base, uint32_t boff, cx<R> v) {    \
        st_nt(reinterpret_cast<P*>(reinterpret_cast<char*>(base) + boff), v);          \
    }
typedef double wd_dvec2 __attribute__((ext_vector_type(2)));
typedef float wd_fvec2 __attribute__((ext_vector_type(2)));

// Non-temporal ("streaming") accesses are used for data touched once per
// kernel (outputs, right-hand sides) so they do not evict reused neighbours.
struct StF64 {
    using R = double;
    using P = double2;
    static constexpr int bytes = 16;
    __device__ __forceinline__ static cx<R> ld_nt(const P* p) {
        const wd_dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const wd_dvec2*>(p));
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st_nt(P* p, cx<R> v) {
        __builtin_nontemporal_store(wd_dvec2{v.re, v.im}, reinterpret_cast<wd_dvec2*>(p));
    }
    __device__ __forceinline__ static cx<R> ld(const P* p, size_t i) {
        P v = p[i];
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st(P* p, size_t i, cx<R> v) { p[i] = make_double2(v.re, v.im); }
    __device__ __forceinline__ static cx<R> rnd(cx<R> v) { return v; }
    WD_BYTE_OFFSET_ACCESSORS
};

struct StF32 {
    using R = float;
    using P = float2;
    static constexpr int bytes = 8;
    __device__ __forceinline__ static cx<R> ld_nt(const P* p) {
        const wd_fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const wd_fvec2*>(p));
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st_nt(P* p, cx<R> v) {
        __builtin_nontemporal_store(wd_fvec2{v.re, v.im}, reinterpret_cast<wd_fvec2*>(p));
    }
    __device__ __forceinline__ static cx<R> ld(const P* p, size_t i) {
        P v = p[i];
        return {v.x, v.y};
    }
    __device__ __forceinline__ static void st(P* p, size_t i, cx<R> v) { p[i] = make_float2(v.re, v.im); }
    __device__ __forceinline__ static cx<R> rnd(cx<R> v) { return v; }
    WD_BYTE_OFFSET_ACCESSORS
};

// bfloat16 pair packed in 32 bits: low half = re, high half = im.  The
// conversion is the gfx950 packed convert (round to nearest even, NaN kept).
typedef __bf16 wd_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float re, float im) {
    const wd_fvec2 f = {re, im};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, wd_bf16x2));
}
struct StBF16 {
    using R = float;
    using P = uint32_t;
    static constexpr int bytes = 4;
    __device__ __forceinline__ static cx<R> ld_nt(const P* p) {
        const uint32_t v = __builtin_nontemporal_load(p);
        return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
    }
    __device__ __forceinline__ static void st_nt(P* p, cx<R> v) { __builtin_nontemporal_store(pack_bf16(v.re, v.im), p); }
    __device__ __forceinline__ static cx<R> ld(const P* p, size_t i) {
        uint32_t v = p[i];
        return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
    }
    __device__ __forceinline__ static void st(P* p, size_t i, cx<R> v) {
        p[i] = pack_bf16(v.re, v.im);
    }
    // value after a round trip through the storage format
    __device__ __forceinline__ static cx<R> rnd(cx<R> v) {
        const uint32_t b = pack_bf16(v.re, v.im);
        return {__uint_as_float(b << 16), __uint_as_float(b & 0xffff0000u)};
    }
    WD_BYTE_OFFSET_ACCESSORS
};

// Compile-time loop: f(std::integral_constant<int, D>) for D = D0 .. N - 1, so
// that the loop index can select template arguments (hop direction, term).
template <int D, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (D < N) {
        f(std::integral_constant<int, D>{});
        static_for<D + 1, N>(f);
    }
}

// ---------------------------------------------------------------------------
// Lattice geometry
// ---------------------------------------------------------------------------
struct Geom {
    int lx, ly, lz, lt;
    int V;          // number of sites
    int sxy;        // lx*ly
    int sxyz;       // lx*ly*lz
    // layout flags: bit 0 (kVecTiled) block vectors in the tiled layout (needs V % 64 == 0),
    // bit 1 (kCoefTiled) the hop kernels' FP64 coefficient fields tiled (both below)
    int vt = 0;
};
enum { kVecTiled = 1, kCoefTiled = 2 };

// Device data layouts (all "pair" arrays, site index fastest):
//   links      [mu][a*3+b][V]               4*9 pairs per site
//   clover     [chirality c][18][V]         per 6x6 Hermitian block: entries
//              0..2 hold the six real diagonal elements as (d0,d1),(d2,d3),(d4,d5),
//              entries 3..17 the upper off-diagonal elements (i<j) in row order
//   block vec  standard: [column][k = 3*spin+colour][V]
//              tiled:    [column][V/64][k][64]: the 12 planes of a 64-site tile of a
//              column are contiguous (12 KB in FP64), so a tile's spinors touch one
//              memory page instead of twelve planes 16 V bytes apart.  Within a
//              column it is a permutation of the rows, so the block updates, Grams and
//              norms, which treat a column as a plain vector, work on either layout.
__host__ __device__ constexpr int herm_index(int i, int j) {  // i < j, 6x6
    return i * 6 - i * (i + 1) / 2 + (j - i - 1);
}

// Element offset of site s inside a column of a block vector (plane k adds k times
// vec_plane), in the layout of g.
__host__ __device__ __forceinline__ uint32_t vec_site(const Geom& g, int s) {
    return (g.vt & kVecTiled) ? (uint32_t)((s >> 6) * 768 + (s & 63)) : (uint32_t)s;
}
__host__ __device__ __forceinline__ size_t vec_plane(const Geom& g) {
    return (g.vt & kVecTiled) ? (size_t)64 : (size_t)g.V;
}
// the tiled layout needs whole tiles and 32-bit byte offsets inside an FP64 column
inline bool tiled_ok(const Geom& g) { return g.V % 64 == 0 && (long long)g.V * 192 <= 0xFFFFFFFFLL; }

// The FP64 coefficient fields of the hop kernels (kappa-scaled links, T, T^{-1},
// the point form; np planes of V pairs each) are kept tiled when the lattice
// allows it: [V/64][np][64], so that a tile's links or 6x6 blocks are one
// contiguous run (measured 1.5 % off the FP64 sweep and 1.4 % off A X at 32^3 x 64,
// L = 12).  The FP32 and BF16 fields stay [np][V]: tiled, they gained nothing in the
// LDS-staged kernels.  This is
// private to the library (kCoefTiled, set by wd_set_params); 32-bit byte offsets over a
// whole FP64 field of 36 planes need V <= 2^32 / 576.  PB: the field's pair size.
inline bool coef_tiled_ok(const Geom& g) { return g.V % 64 == 0 && (long long)g.V * 576 <= 0xFFFFFFFFLL; }
template <int PB>
__host__ __device__ __forceinline__ uint32_t coef_site(const Geom& g, int s, int np) {
    return (PB == 16 && (g.vt & kCoefTiled)) ? (uint32_t)((s >> 6) * np * 64 + (s & 63)) : (uint32_t)s;
}
template <int PB>
__host__ __device__ __forceinline__ size_t coef_plane(const Geom& g) {
    return (PB == 16 && (g.vt & kCoefTiled)) ? (size_t)64 : (size_t)g.V;
}

// Workgroup index -> tile index such that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int nx = 8;
    const int q = nb / nx, r = nb % nx;
    const int x = b % nx, i = b / nx;
    return x * q + (x < r ? x : r) + i;
}

// Site tiles of the stencil kernels.  The hardware hands workgroup b to
// XCD b % 8.  XCD k owns the sub-lattice Lx x [y-range] x [z-range] x Lt
// (y split ny ways, z split nz = 8 / ny ways) and walks it t-slice by
// t-slice, z-plane by z-plane, 64-site tiles of its (x, y) rows fastest.  A
// site's y-neighbour was then read one row earlier and its z-neighbour one
// plane (Lx * Ly / ny sites) earlier, both in the XCD's L2 when the plane is
// small enough, which is what ny is chosen for; its t-neighbour was read one
// slab-slice earlier and is served by the shared MALL, as are the faces
// between XCDs, whose neighbours are processed at the same time.  Lattices
// with Lz * Ly too small for the split use contiguous site ranges.
struct SiteMap {
    int mode;    // 1: XCD sub-lattices, 0: contiguous ranges
    int ny;      // y split
    int nz;      // z split
    int tpp;     // 64-site tiles per plane of a sub-lattice (max over XCDs)
    int nblk;    // workgroups in the grid
    int nt = 1;  // t split (ny * nz * nt = 8)
    int tb = 1;  // t-slices walked together: planes go (t block, z, t within the block)
};

// Site of this lane, or -1.
__device__ __forceinline__ int map_site(const Geom& g, const SiteMap& m, int b, int lane) {
    if (m.mode == 1) {
        const int k = b & 7, i = b >> 3;
        const int ky = k % m.ny, kr = k / m.ny, kz = kr % m.nz, kt = kr / m.nz;
        const int y0 = (ky * g.ly) / m.ny, ny = ((ky + 1) * g.ly) / m.ny - y0;
        const int z0 = (kz * g.lz) / m.nz, nz = ((kz + 1) * g.lz) / m.nz - z0;
        const int t0 = (kt * g.lt) / m.nt, nt = ((kt + 1) * g.lt) / m.nt - t0;
        const int plane = i / m.tpp, tip = i - plane * m.tpp;
        if (plane >= nz * nt) return -1;
        // planes in blocks of tb t-slices: within a block z-plane by z-plane, the tb slices of
        // a z-plane one after the other (tb = 1: slice by slice); a last partial block is
        // shorter
        const int blk = plane / (nz * m.tb), r = plane - blk * (nz * m.tb);
        const int tbn = nt - blk * m.tb < m.tb ? nt - blk * m.tb : m.tb;
        const int z = z0 + r / tbn, t = t0 + blk * m.tb + (r - (r / tbn) * tbn);
        const int xy = tip * 64 + lane;
        if (xy >= g.lx * ny) return -1;
        const int y = y0 + xy / g.lx, x = xy - (xy / g.lx) * g.lx;
        return x + g.lx * (y + g.ly * (z + g.lz * t));
    }
    const int lin = xcd_remap(b, m.nblk);
    const int s = lin * 64 + lane;
    return s < g.V ? s : -1;
}

// bytes_site: bytes per site a stencil launch keeps reusing (input block
// vector plus links and clover)
inline SiteMap make_site_map(const Geom& g, double bytes_site) {
    SiteMap m{};
    const double budget = 2.0 * 1024 * 1024;
    for (int ny = 1; ny <= 8; ny *= 2) {
        const int nz = 8 / ny;
        if (g.ly < ny || g.lz < nz) continue;
        const int rows = (g.ly + ny - 1) / ny;
        m.mode = 1;
        m.ny = ny;
        m.nz = nz;
        m.tpp = (g.lx * rows + 63) / 64;
        m.nblk = 8 * ((g.lz + nz - 1) / nz) * g.lt * m.tpp;
        if (g.lx * rows * bytes_site <= budget) break;  // else try a finer y split
    }
    if (m.mode == 0) m.nblk = (g.V + 63) / 64;
    return m;
}

// Site map of the LDS-staged kernels: the finest y split (y x z = 8 x 1, then
// 4 x 2, ...) whose per-XCD planes still hold whole 64-site tiles, so that an
// XCD walks few rows of every z-plane, plane by plane (measured 3 % faster than
// the L2-budget split at 32^3 x 64, L = 12); else the budget rule above.  With
// tb > 1 the XCD walks tb t-slices together, so a site's time neighbours inside
// the block are read while still in the L2.
inline SiteMap make_site_map_rows(const Geom& g, double bytes_site, int tb = 1) {
    for (int ny = 8; ny >= 1; ny /= 2) {
        const int nz = 8 / ny;
        if (g.ly % ny != 0 || g.lz < nz) continue;
        const int rows = g.ly / ny;
        if ((g.lx * rows) % 64 != 0) continue;
        SiteMap m{};
        m.mode = 1;
        m.ny = ny;
        m.nz = nz;
        m.tpp = g.lx * rows / 64;
        m.nblk = 8 * ((g.lz + nz - 1) / nz) * g.lt * m.tpp;
        m.tb = tb < 1 ? 1 : (tb > g.lt ? g.lt : tb);
        return m;
    }
    return make_site_map(g, bytes_site);
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Fields {
    double2* U = nullptr;      // FP64 links, antiperiodic sign folded in (clover, learned layers)
    double2* T = nullptr;      // FP64 clover T (operator A)
    // per precision (index Prec): kappa-scaled links, T^{-1} (block reading),
    // point form (1/diag(T) on the diagonal slots, T's off-diagonals), T
    void* Uk[3] = {};
    void* Ti[3] = {};
    void* Tp[3] = {};
    void* Tc[3] = {};
};

enum class Prec { F64 = 0, F32 = 1, BF16 = 2 };

}  // namespace wd

struct wd_ctx {
    wd::Geom g;
    int bc_t = 0;
    int max_L = 0;
    hipStream_t stream = nullptr;
    bool have_links = false;
    bool have_params = false;
    double kappa = 0, csw = 0;
    int jacobi_kind = WD_JACOBI_BLOCK;
    wd::Fields f;
    // solver workspace: N x max_L FP64 blocks
    double2* ws[12] = {};
    // low-precision Jacobi iterates: two ping-pong blocks and the right-hand side copy
    void* lp[3] = {};
    // B and X of a solve run in the tiled layout for a caller of the standard one
    double2* tb[2] = {};
    // reduction partials and small control data
    double2* partial = nullptr;
    int n_partial_blocks = 0;
    double2* small = nullptr;     // L x L matrices, scalars (see wd_blas.hip)
    int* dstatus = nullptr;
    double* host_ctl = nullptr;   // pinned host mirror of per-iteration control data
    // learned preconditioner: FP32 links (unscaled), weights, training workspace
    float2* U32 = nullptr;
    float2* theta = nullptr;
    bool have_theta = false;
    void* learn_mem = nullptr;
    size_t learn_bytes = 0;
};

namespace wd {

// ---- setup (wd_setup.hip)
hipError_t launch_links_from_abi(const double2* Uabi, double2* U, const Geom& g, int bc_t, hipStream_t s);
hipError_t launch_clover(const double2* U, double2* T, double2* Ti, const Geom& g, double kappa, double csw,
                         hipStream_t s);
// dst = scale * src, stored in precision p (n complex pairs)
hipError_t launch_convert(const double2* src, void* dst, Prec p, double scale, size_t n, hipStream_t s);
// point form of T: diagonal slots replaced by 1/diag, off-diagonal slots kept
hipError_t launch_point_form(const double2* T, double2* Tp, size_t V, hipStream_t s);
// convert an FP64 block vector to precision p and back
hipError_t launch_to_lowp(const double2* src, void* dst, Prec p, size_t n, hipStream_t s);

// ---- Wilson hopping kernels (wd_dslash.hip)
// Y = A X (FP64)
hipError_t launch_apply_A(const wd_ctx* c, const double2* X, double2* Y, int L, hipStream_t s);
// Z = M R with j sweeps in precision p; tmp is a scratch block of L columns
hipError_t launch_jacobi(wd_ctx* c, const double2* R, double2* Z, int L, int j, Prec p, hipStream_t s);
// Z = M R with j sweeps of FP64 vectors and arithmetic, links and A_D^{-1} stored in precision coef
hipError_t launch_jacobi_coef(wd_ctx* c, const double2* R, double2* Z, int L, int j, Prec coef, hipStream_t s);
// one such sweep (FP64 vectors, coefficients in precision coef)
hipError_t launch_sweep_coef(const wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, Prec coef,
                             hipStream_t s);
// one Jacobi sweep Y = A_D^{-1}(R + kappa H X) in FP64
hipError_t launch_sweep_f64(const wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, hipStream_t s);
// algorithmic HBM bytes per site of the kernels (FP64 storage, L columns)
inline double bytes_apply(int L) { return 1152.0 + 384.0 * L; }
inline double bytes_sweep(int L) { return 1152.0 + 576.0 * L; }
inline double bytes_first_sweep(int L) { return 576.0 + 384.0 * L; }
// low precision application of A (diagnostic): Y (FP64) = A X computed in p
hipError_t launch_apply_A_lowp(wd_ctx* c, const double2* X, double2* Y, int L, Prec p, hipStream_t s);
hipError_t launch_hop_repeat_lowp(wd_ctx* c, const double2* X, const double2* R, double2* Y, int L, int mode, Prec p,
                                  int nrep, hipStream_t s);

// ---- learned preconditioner (wd_learned.hip): Z = M_theta R, FP64 in and out
hipError_t launch_learned(wd_ctx* c, const double2* R, double2* Z, int L, Prec p, double2* t0, double2* t1,
                          hipStream_t s);
int learned_ensure(wd_ctx* c);
int lowp_ensure(wd_ctx* c);  // allocates the three low-precision block buffers

// ---- block kernels (wd_blas.hip)
size_t partial_stride();  // complex entries per partial block
int gram_blocks(size_t N);
// partials of P^H Q over rows (nb blocks)
hipError_t launch_gram_partials(const double2* P, const double2* Q, size_t N, int L, double2* partial, int nb,
                                hipStream_t s);
// reduce partials -> C (L x L row-major) on the device
hipError_t launch_reduce_gram(const double2* partial, int nb, int L, double2* C, hipStream_t s);
hipError_t launch_small_solve(const double2* M, const double2* RHS, int L, double2* Z, int* status, hipStream_t s);
// Z = M^{-1} (c RHS); status_bit 0: *status = ok ? 0 : 1, else *status |= status_bit on failure;
// cond (may be null): pivot-ratio condition estimate of M
hipError_t launch_small_solve_scaled(const double2* M, const double2* RHS, int L, double2 c, double2* Z, int* status,
                                     int status_bit, double* cond, hipStream_t s);
// out = a A + b B + (c C + d D) M (N x L blocks, L x L matrix M; see k_block_comb)
hipError_t launch_block_comb(double2* out, const double2* A, const double2* Bm, const double2* C, const double2* D,
                             const double2* M, double2 a, double2 b, double2 c, double2 d, const double2* w, int wmask,
                             size_t N, int L, hipStream_t s);
// omega = Tr[Cts] / Tr[Ctt]
hipError_t launch_stab_omega(const double2* Cts, const double2* Ctt, int L, double2* omega, int* status, int bit,
                             hipStream_t s);

// solver-specific fused kernels
struct SolverBufs {
    double2* C_r;      // Rt^H R_k           (L x L)
    double2* C_rn;     // Rt^H R_{k+1}       (L x L)
    double2* alpha;    // L x L
    double2* gamma;    // L x L
    double2* zeta;     // [0] = zeta, [1] = Tr W^H R, [2] = Tr W^H W
    double* norms;     // L squared column norms of R_{k+1}
    int* status;       // breakdown / nan flags
    double* cond;      // [0]: condition estimate of Rt^H V_k, [1]: of Rt^H R_k
};
hipError_t launch_gram1(const double2* Rt, const double2* V, const double2* W, const double2* R, size_t N, int L,
                        double2* partial, int nb, hipStream_t s);
hipError_t launch_solve_alpha(const double2* partial, int nb, int L, const SolverBufs& b, hipStream_t s);
hipError_t launch_update_U(const double2* P, const double2* V, const double2* zeta, const double2* alpha,
                           double2* U, size_t N, int L, hipStream_t s);
hipError_t launch_solve_gamma(const double2* partial, int nb, int L, const SolverBufs& b, hipStream_t s);
hipError_t launch_update_PV_gram(double2* P, double2* V, const double2* R, const double2* W, const double2* U,
                                 const double2* Y, const double2* gamma, const double2* Rt, size_t N, int L,
                                 double2* partial, int nb, hipStream_t s);
hipError_t launch_update_XR_gram(double2* X, double2* R, const double2* F, const double2* G, const double2* W,
                                 const double2* Y, const double2* Rt, const double2* zeta, size_t N, int L,
                                 double2* partial, int nb, hipStream_t s);
// residual helpers
hipError_t launch_axpby_block(const double2* B, const double2* AX, double2* R, size_t n, hipStream_t s);  // R = B - AX
hipError_t launch_colnorms(const double2* R, size_t N, int L, double2* partial, int nb, double* norms,
                           hipStream_t s);
hipError_t launch_copy(double2* dst, const double2* src, size_t n, hipStream_t s);
hipError_t launch_zero(double2* dst, size_t n, hipStream_t s);
// an L-column block vector from the standard into the tiled layout (to_tiled) or back
hipError_t launch_retile(const double2* src, double2* dst, size_t V, int L, bool to_tiled, hipStream_t s);
// a coefficient field of np planes of V pairs of pair_bytes (16, 8 or 4) from [np][V] into
// [V/64][np][64]
hipError_t launch_tile_field(const void* src, void* dst, size_t V, int np, int pair_bytes, hipStream_t s);

}  // namespace wd
