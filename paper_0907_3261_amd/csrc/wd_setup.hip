// Setup kernels: gauge-field layout, clover field strength and site matrices
// T(x) = T_+ (+) T_- with their inverses, and precision conversions.
//
// The clover term is the O(a) improvement of the operator that the paper's
// Sec. 2 uses without printing it; the form is the standard
// T = 1 - kappa c_SW sum_{mu<nu} sigma_{mu nu} F_{mu nu} with
// F_{mu nu} = (Q - Q^dag)/(8i) from the four plaquette leaves at x.
//
// In the chiral gamma basis sigma_{jk} = -eps_{jkl} diag(s_l, s_l) and
// sigma_{k4} = diag(s_k, -s_k), so T is block diagonal in chirality:
//   T_pm = 1 - kappa c_SW [[B3, B1 - i B2], [B1 + i B2, -B3]]  (3x3 colour blocks)
// with B1 = -F_yz pm F_xt, B2 = F_xz pm F_yt, B3 = -F_xy pm F_zt.
#include "wd_internal.h"

namespace wd {

namespace {

struct M3 {
    cx<double> e[9];
};

__device__ __forceinline__ M3 load_link(const double2* __restrict__ U, int mu, int s, size_t V) {
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = StF64::ld(U, (size_t)(mu * 9 + k) * V + s);
    return m;
}

__device__ __forceinline__ M3 mul(const M3& a, const M3& b) {  // a b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> acc = a.e[i * 3 + 0] * b.e[0 * 3 + j];
            cfma(acc, a.e[i * 3 + 1], b.e[1 * 3 + j]);
            cfma(acc, a.e[i * 3 + 2], b.e[2 * 3 + j]);
            r.e[i * 3 + j] = acc;
        }
    return r;
}

__device__ __forceinline__ M3 mul_nd(const M3& a, const M3& b) {  // a b^dag
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) acc = acc + a.e[i * 3 + k] * conj(b.e[j * 3 + k]);
            r.e[i * 3 + j] = acc;
        }
    return r;
}

__device__ __forceinline__ M3 mul_dn(const M3& a, const M3& b) {  // a^dag b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) acc = acc + conj(a.e[k * 3 + i]) * b.e[k * 3 + j];
            r.e[i * 3 + j] = acc;
        }
    return r;
}

// ABI layout U[mu][s][a][b] -> device layout [mu][a*3+b][s]; the antiperiodic
// time boundary is folded into the links on the last time slice.
__global__ void k_links_from_abi(const double2* __restrict__ Uabi, double2* __restrict__ U, Geom g, int bc_t) {
    const size_t V = g.V;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V * 9) return;
    const int ab = (int)(i % 9);
    const size_t s = (i / 9) % V;
    const int mu = (int)(i / (9 * V));
    double2 v = Uabi[i];
    if (bc_t && mu == 3 && (int)(s / g.sxyz) == g.lt - 1) {
        v.x = -v.x;
        v.y = -v.y;
    }
    U[(size_t)(mu * 9 + ab) * V + s] = v;
}

struct Nb {
    int s;
    int f[4], b[4];  // s +- mu
};

__device__ __forceinline__ int step(const Geom& g, int s, int mu, int d) {
    int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / g.sxy) % g.lz, t = s / g.sxyz;
    int c[4] = {x, y, z, t};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    c[mu] = (c[mu] + d + ext[mu]) % ext[mu];
    return c[0] + g.lx * (c[1] + g.ly * (c[2] + g.lz * c[3]));
}

// F_{mu nu}(x) for the site s (Hermitian 3x3, no trace subtraction).
__device__ M3 field_strength(const double2* __restrict__ U, const Geom& g, int s, int mu, int nu) {
    const size_t V = g.V;
    const int s_pm = step(g, s, mu, 1), s_mm = step(g, s, mu, -1);
    const int s_pn = step(g, s, nu, 1), s_mn = step(g, s, nu, -1);
    const int s_mm_pn = step(g, s_mm, nu, 1);
    const int s_mm_mn = step(g, s_mm, nu, -1);
    const int s_pm_mn = step(g, s_pm, nu, -1);
    const M3 umu = load_link(U, mu, s, V), unu = load_link(U, nu, s, V);
    // leaf 1: U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^dag
    M3 q = mul_nd(mul(umu, load_link(U, nu, s_pm, V)), mul(unu, load_link(U, mu, s_pn, V)));
    // leaf 2: U_nu(x) [U_nu(x-mu) U_mu(x-mu+nu)]^dag U_mu(x-mu)
    const M3 umu_mm = load_link(U, mu, s_mm, V);
    M3 l2 = mul(mul_nd(unu, mul(load_link(U, nu, s_mm, V), load_link(U, mu, s_mm_pn, V))), umu_mm);
    // leaf 3: [U_nu(x-mu-nu) U_mu(x-mu)]^dag [U_mu(x-mu-nu) U_nu(x-nu)]
    const M3 unu_mn = load_link(U, nu, s_mn, V);
    M3 l3 = mul_dn(mul(load_link(U, nu, s_mm_mn, V), umu_mm), mul(load_link(U, mu, s_mm_mn, V), unu_mn));
    // leaf 4: U_nu(x-nu)^dag [U_mu(x-nu) U_nu(x+mu-nu)] U_mu(x)^dag
    M3 l4 = mul_nd(mul_dn(unu_mn, mul(load_link(U, mu, s_mn, V), load_link(U, nu, s_pm_mn, V))), umu);
    M3 F;
#pragma unroll
    for (int k = 0; k < 9; ++k) q.e[k] = q.e[k] + l2.e[k] + l3.e[k] + l4.e[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // (Q_ab - conj(Q_ba)) / (8 i) = -i/8 (Q_ab - conj(Q_ba))
            cx<double> d = q.e[a * 3 + b] - conj(q.e[b * 3 + a]);
            F.e[a * 3 + b] = {d.im * 0.125, -d.re * 0.125};
        }
    return F;
}

// Invert a 6x6 complex matrix by Gauss-Jordan elimination with partial pivoting.
__device__ void invert6(cx<double> (&a)[6][6], cx<double> (&inv)[6][6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) inv[i][j] = {i == j ? 1.0 : 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int p = k;
        double best = a[k][k].re * a[k][k].re + a[k][k].im * a[k][k].im;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            double m = a[r][k].re * a[r][k].re + a[r][k].im * a[r][k].im;
            if (m > best) {
                best = m;
                p = r;
            }
        }
        // swap rows k and p with selects only (no dynamic register indexing)
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const bool sw = (r == p);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                cx<double> t1 = a[k][j], t2 = a[r][j];
                a[k][j] = sw ? t2 : t1;
                a[r][j] = sw ? t1 : t2;
                cx<double> u1 = inv[k][j], u2 = inv[r][j];
                inv[k][j] = sw ? u2 : u1;
                inv[r][j] = sw ? u1 : u2;
            }
        }
        const cx<double> piv = a[k][k];
        const double den = 1.0 / (piv.re * piv.re + piv.im * piv.im);
        const cx<double> pinv = {piv.re * den, -piv.im * den};
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            a[k][j] = pinv * a[k][j];
            inv[k][j] = pinv * inv[k][j];
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (r == k) continue;
            const cx<double> f = a[r][k];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                a[r][j] = a[r][j] - f * a[k][j];
                inv[r][j] = inv[r][j] - f * inv[k][j];
            }
        }
    }
}

__device__ __forceinline__ void store_herm(double2* __restrict__ out, int chir, int s, size_t V,
                                           const cx<double> (&m)[6][6]) {
    // diagonal (real parts) in slots 0..2; Hermitian-averaged upper triangle in 3..17
#pragma unroll
    for (int i = 0; i < 3; ++i)
        out[(size_t)(chir * 18 + i) * V + s] = make_double2(m[2 * i][2 * i].re, m[2 * i + 1][2 * i + 1].re);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            const cx<double> u = m[i][j], l = m[j][i];
            out[(size_t)(chir * 18 + 3 + herm_index(i, j)) * V + s] =
                make_double2(0.5 * (u.re + l.re), 0.5 * (u.im - l.im));
        }
}

__global__ void __launch_bounds__(64) k_clover(const double2* __restrict__ U, double2* __restrict__ T,
                                               double2* __restrict__ Ti, Geom g, double kc) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = g.V;
    // planes: xy xz xt yz yt zt
    M3 F[6];
    int pidx = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) F[pidx++] = field_strength(U, g, s, mu, nu);
    const M3 &Fxy = F[0], &Fxz = F[1], &Fxt = F[2], &Fyz = F[3], &Fyt = F[4], &Fzt = F[5];
    for (int chir = 0; chir < 2; ++chir) {
        const double sg = chir == 0 ? 1.0 : -1.0;
        cx<double> m[6][6];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int k = a * 3 + b;
                const cx<double> B1 = (-1.0) * Fyz.e[k] + sg * Fxt.e[k];
                const cx<double> B2 = Fxz.e[k] + sg * Fyt.e[k];
                const cx<double> B3 = (-1.0) * Fxy.e[k] + sg * Fzt.e[k];
                const double d = (a == b) ? 1.0 : 0.0;
                // [[B3, B1 - i B2], [B1 + i B2, -B3]]
                m[a][b] = cx<double>{d, 0.0} - kc * B3;
                m[3 + a][3 + b] = cx<double>{d, 0.0} + kc * B3;
                m[a][3 + b] = (-kc) * (B1 - ti(B2));
                m[3 + a][b] = (-kc) * (B1 + ti(B2));
            }
        store_herm(T, chir, s, V, m);
        cx<double> inv[6][6];
        invert6(m, inv);
        store_herm(Ti, chir, s, V, inv);
    }
}

template <class S>
__global__ void k_convert(const double2* __restrict__ src, typename S::P* __restrict__ dst, double scale, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 v = src[i];
    S::st(dst, i, cx<typename S::R>{(typename S::R)(scale * v.x), (typename S::R)(scale * v.y)});
}

__global__ void k_point_form(const double2* __restrict__ T, double2* __restrict__ Tp, size_t V) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 36 * V) return;
    const size_t slot = (i / V) % 18;
    double2 v = T[i];
    if (slot < 3) v = make_double2(1.0 / v.x, 1.0 / v.y);
    Tp[i] = v;
}

inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_links_from_abi(const double2* Uabi, double2* U, const Geom& g, int bc_t, hipStream_t s) {
    const size_t n = (size_t)4 * g.V * 9;
    k_links_from_abi<<<nblk(n, 256), 256, 0, s>>>(Uabi, U, g, bc_t);
    return hipGetLastError();
}

hipError_t launch_clover(const double2* U, double2* T, double2* Ti, const Geom& g, double kappa, double csw,
                         hipStream_t s) {
    k_clover<<<nblk(g.V, 64), 64, 0, s>>>(U, T, Ti, g, kappa * csw);
    return hipGetLastError();
}

hipError_t launch_convert(const double2* src, void* dst, Prec p, double scale, size_t n, hipStream_t s) {
    switch (p) {
        case Prec::F64:
            k_convert<StF64><<<nblk(n, 256), 256, 0, s>>>(src, (double2*)dst, scale, n);
            break;
        case Prec::F32:
            k_convert<StF32><<<nblk(n, 256), 256, 0, s>>>(src, (float2*)dst, scale, n);
            break;
        case Prec::BF16:
            k_convert<StBF16><<<nblk(n, 256), 256, 0, s>>>(src, (uint32_t*)dst, scale, n);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_point_form(const double2* T, double2* Tp, size_t V, hipStream_t s) {
    k_point_form<<<nblk(36 * V, 256), 256, 0, s>>>(T, Tp, V);
    return hipGetLastError();
}

hipError_t launch_to_lowp(const double2* src, void* dst, Prec p, size_t n, hipStream_t s) {
    return launch_convert(src, dst, p, 1.0, n, s);
}

}  // namespace wd
