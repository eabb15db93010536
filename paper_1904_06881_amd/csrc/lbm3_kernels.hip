// HIP kernels (gfx950) of the ternary high-density-ratio free-energy LBM
// with wetting walls (Bala et al., arXiv:1904.06881).
//
// Data layout in HBM: populations SoA [Q][QS] (x fastest; QS = array_stride
// of the node count, the arrays padded apart), two buffers per set (push
// streaming writes the other one); fields rho, phi in the compute type, two
// buffers (the FP16 storage decodes with the previous step's fields); in 3D
// F and mu_phi [D + 1][QS]; at tau_g = 1 in 3D the five values (a, phi, v)
// of g^eq [5][QS] in place of a second g set.  A step is two launches in 2D
// and four in 3D:
//   k_moments      rho, phi of every fluid node from its populations (2D, or
//                  3D with stored g);
//   k_moments_imp  (3D, tau_g = 1) the same as a march of 64 x 4 tiles along
//                  the wall axis, g rebuilt from the five values of each
//                  source node staged through a 3-plane LDS ring;
//   k_ghost        (3D) wall ghost layers of rho, phi;
//   k_fused        per block an in-plane tile (x in 2D, x-y in 3D) marching
//                  along the wall axis: a 5-plane LDS ring of rho, phi with
//                  halo 3 (in 2D the wall ghost layers are filled in the
//                  block), a 3-plane LDS ring of -P and mu_phi with halo 1,
//                  then force, entropic collision of f, LBGK of g and push
//                  streaming with halfway bounce-back for one plane at a time;
//   k_stencil      (3D) the same march up to the force, writing F and mu_phi;
//   k_collide      (3D) one thread per fluid node: the fused kernel's
//                  collision and streaming, and LBGK of g or, at tau_g = 1,
//                  the five values of g^eq (k_fused does all of it in 3D too
//                  when one kernel is asked for).
// The _batch variants run the same per-node arithmetic for many simulations
// in one launch.  k_ghost also fills the ghost layers for initialisation and
// export.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lbm3_internal.h"

namespace lbm3k {

// ------------------------------------------------------------ lattice ----
// velocity i = sum_a (c_a + 1) 3^(D-1-a): x most significant
__host__ __device__ constexpr int cdir(int D, int i, int a)
{
    return D == 2 ? (a == 0 ? i / 3 - 1 : (a == 1 ? i % 3 - 1 : 0))
                  : (a == 0 ? i / 9 - 1 : (a == 1 ? (i / 3) % 3 - 1 : i % 3 - 1));
}
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wgt(int D, int i)
{
    return D == 2 ? w1(cdir(2, i, 0)) * w1(cdir(2, i, 1))
                  : w1(cdir(3, i, 0)) * w1(cdir(3, i, 1)) * w1(cdir(3, i, 2));
}
// index of -P_ab in the symmetric storage: 2D xx xy yy; 3D xx xy xz yy yz zz
__host__ __device__ constexpr int sym(int D, int a, int b)
{
    return D == 2 ? a + b
                  : (a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : (b == 0 ? a : (b == 1 ? 2 + a : 5)));
}

template <int PREC> struct Ty;
template <> struct Ty<P64> { using S = double; using R = double; };
template <> struct Ty<P32> { using S = float; using R = float; };
template <> struct Ty<P16> { using S = _Float16; using R = float; };

__device__ __forceinline__ int wrapi(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// a / b: correctly rounded in FP64; in FP32 a times the hardware reciprocal
// (about 1 ulp), well inside the FP32 path's error budget
template <typename R> __device__ __forceinline__ R fdiv(R a, R b) { return a / b; }
template <> __device__ __forceinline__ float fdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Storage codecs.  FP16: f_i stored as f_i / (w_i rho_node) - 1 and the rest
// g as g_0 - phi_node, with rho_node, phi_node the fields the writer holds
// for the node the value is stored at; other g raw.
template <int PREC, int D>
__device__ __forceinline__ typename Ty<PREC>::R dec_f(typename Ty<PREC>::S s, int i,
                                                      typename Ty<PREC>::R rn)
{
    using R = typename Ty<PREC>::R;
    if constexpr (PREC == P16) return (R)wgt(D, i) * rn * ((R)1 + (R)s);
    else return (R)s;
}
template <int PREC, int D>
__device__ __forceinline__ typename Ty<PREC>::S enc_f(typename Ty<PREC>::R v, int i,
                                                      typename Ty<PREC>::R rn)
{
    using S = typename Ty<PREC>::S;
    using R = typename Ty<PREC>::R;
    if constexpr (PREC == P16) return (S)(fdiv(v, (R)wgt(D, i) * rn) - (R)1);
    else return (S)v;
}
template <int PREC, int D>
__device__ __forceinline__ typename Ty<PREC>::R dec_g(typename Ty<PREC>::S s, int i,
                                                      typename Ty<PREC>::R pn)
{
    using R = typename Ty<PREC>::R;
    constexpr int rest = (D == 2 ? 9 : 27) / 2;
    if constexpr (PREC == P16) return i == rest ? (R)s + pn : (R)s;
    else return (R)s;
}
template <int PREC, int D>
__device__ __forceinline__ typename Ty<PREC>::S enc_g(typename Ty<PREC>::R v, int i,
                                                      typename Ty<PREC>::R pn)
{
    using S = typename Ty<PREC>::S;
    constexpr int rest = (D == 2 ? 9 : 27) / 2;
    if constexpr (PREC == P16) return i == rest ? (S)(v - pn) : (S)v;
    else return (S)v;
}

// ------------------------------------------------------ thermodynamics ---
template <typename R> struct Thermo {
    R rho_l, drho, inv_drho, chi, inv_chi, a, b, T, C, psi0, hl1, hl2, hl3, lam2, lam3, krr, kpp, kx;
    __device__ void load(const KParams &k)
    {
        rho_l = (R)k.rho_l; drho = (R)k.drho; inv_drho = (R)(1.0 / k.drho);
        chi = (R)k.chi; inv_chi = (R)(1.0 / k.chi);
        a = (R)k.a; b = (R)k.b; T = (R)k.T; C = (R)k.C; psi0 = (R)k.psi0;
        hl1 = (R)(0.5 * k.lam1); hl2 = (R)(0.5 * k.lam2); hl3 = (R)(0.5 * k.lam3);
        lam2 = (R)k.lam2; lam3 = (R)k.lam3;
        krr = (R)k.krr; kpp = (R)k.kpp; kx = (R)k.kx;
    }
};

template <typename R> __device__ __forceinline__ R gfun(R x) { return x * (x - (R)0.5) * (x - (R)1); }

// log1p: the library's in FP64; in FP32, for |y| < 0.28 the atanh series
// 2 (s + s^3/3 + ... + s^9/9), s = y/(2 + y) (|s| < 0.14, truncation < 1e-9
// relative), else the hardware log2 of 1 + y; about 3 ulp at worst
template <typename R> __device__ __forceinline__ R flog1p(R y) { return log1p(y); }
template <> __device__ __forceinline__ float flog1p<float>(float y)
{
    const float s = y * __builtin_amdgcn_rcpf(2.0f + y), s2 = s * s;
    float p = 1.0f / 9.0f;
    p = p * s2 + 1.0f / 7.0f;
    p = p * s2 + 1.0f / 5.0f;
    p = p * s2 + 1.0f / 3.0f;
    p = p * s2 + 1.0f;
    const float series = 2.0f * s * p;
    const float direct = __builtin_amdgcn_logf(1.0f + y) * 0.69314718055994531f;
    return fabsf(y) < 0.28f ? series : direct;
}
// log: the library's in FP64, the hardware log2 times ln 2 in FP32
template <typename R> __device__ __forceinline__ R flog(R v) { return log(v); }
template <> __device__ __forceinline__ float flog<float>(float v) { return __builtin_amdgcn_logf(v) * 0.69314718055994531f; }
// sqrt: correctly rounded in FP64, the hardware square root in FP32
template <typename R> __device__ __forceinline__ R fsqrt(R v) { return sqrt(v); }
template <> __device__ __forceinline__ float fsqrt<float>(float v) { return __builtin_amdgcn_sqrtf(v); }

// Bulk chemical potentials and free energy (Eqs. 2, 4-7, 11-12, 15): C1 from
// rho, C2/C3 from rho and phi; dPsi and Psi of the Carnahan-Starling EOS; the
// rho derivative of the lambda2/lambda3 wells is +(lambda2 g(C2) +
// lambda3 g(C3))/Delta_rho (dC2/drho = dC3/drho = 1/(2 Delta_rho)).
template <typename R>
__device__ __forceinline__ void bulk(const Thermo<R> &t, R rho, R phi, R &mrb, R &mpb, R &fb)
{
    R C1 = (t.rho_l - rho) * t.inv_drho;
    R ph = phi * t.inv_chi;
    R C2 = (R)0.5 * ((R)1 + ph - C1);
    R C3 = (R)0.5 * ((R)1 - ph - C1);
    R br = t.b * rho;
    R d = br - (R)4;
    R id = fdiv((R)1, d);
    R lr = flog(rho);
    R dpsi = t.C - (R)2 * t.a * rho + t.T * ((R)1 + lr) + (R)16 * t.T * (br - (R)12) * id * id * id;
    R psi = rho * (t.C - t.a * rho - (R)8 * t.T * (br - (R)6) * id * id + t.T * lr);
    R g2 = gfun(C2), g3 = gfun(C3);
    mrb = t.hl1 * dpsi + (t.lam2 * g2 + t.lam3 * g3) * t.inv_drho;
    mpb = (t.lam2 * g2 - t.lam3 * g3) * t.inv_chi;
    R a2 = C2 * ((R)1 - C2), a3 = C3 * ((R)1 - C3);
    fb = t.hl1 * (psi - t.psi0) + t.hl2 * a2 * a2 + t.hl3 * a3 * a3;
}

// mu_rho, mu_phi (Eqs. 11-18 with one cross coefficient k_x) and -P
// (Eqs. 19-20) from the fields and their stencils.  NP = D(D+1)/2.
template <int D, typename R>
__device__ __forceinline__ void thermo(const Thermo<R> &t, R rho, R phi, const R *G, const R *H,
                                       R Lr, R Lp, R &mur, R &mup, R *mP)
{
    R mrb, mpb, fb;
    bulk(t, rho, phi, mrb, mpb, fb);
    mur = mrb - t.krr * Lr - t.kx * Lp;
    mup = mpb - t.kpp * Lp - t.kx * Lr;
    R p0 = rho * mrb + phi * mpb - fb;
    R GG = 0, HH = 0, GH = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) { GG += G[a] * G[a]; HH += H[a] * H[a]; GH += G[a] * H[a]; }
    R iso = p0 - t.krr * (rho * Lr + (R)0.5 * GG) - t.kpp * (phi * Lp + (R)0.5 * HH) -
            t.kx * (rho * Lp + phi * Lr + GH);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            R v = t.krr * G[a] * G[b] + t.kpp * H[a] * H[b] + t.kx * (G[a] * H[b] + H[a] * G[b]);
            if (a == b) v += iso;
            mP[sym(D, a, b)] = -v;
        }
}

// Link pressure of the ideal part of the force,
// 2 rho_x rho_y / (rho_x + rho_y + 4 sqrt(rho_x rho_y)), from qx = sqrt(rho_x)
// and qy = sqrt(rho_y): equals rho/3 for equal densities; its lattice
// divergence keeps an exponential density profile an exact steady state of
// the product-form ELBM.
template <typename R> __device__ __forceinline__ R link_q(R qx, R qy)
{
    const R m = qx * qy, s = qx + qy;
    return fdiv((R)2 * m * m, s * s + (R)2 * m);
}
// The same from the densities (one square root per link; in FP32 the
// hardware reciprocal and square root, as in the rest of the FP32 path).
template <typename R> __device__ __forceinline__ R link_p(R rx, R ry)
{
    return fdiv((R)2 * rx * ry, rx + ry + (R)4 * fsqrt(rx * ry));
}

// ------------------------------------------------------------ equilibria -
// f_i^eq = rho w_i prod_a A(u_a) B(u_a)^{c_ia}, Eqs. 25-27, from per-axis
// factors fac[a][c+1] = w1(c) A(u_a) B(u_a)^c: f^eq_i = rho prod_a fac[a][c_ia + 1].
template <typename R>
__device__ __forceinline__ void feq_factors(R u, R *fac)
{
    R s = fsqrt((R)1 + (R)3 * u * u);
    R A = (R)2 - s;
    R B = fdiv((R)2 * u + s, (R)1 - u);
    fac[0] = fdiv((R)(1.0 / 6.0) * A, B);
    fac[1] = (R)(2.0 / 3.0) * A;
    fac[2] = (R)(1.0 / 6.0) * A * B;
}

template <int D, typename R>
__device__ __forceinline__ void feq(R rho, const R *u, R *fe)
{
    constexpr int Q = D == 2 ? 9 : 27;
    R fac[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a) feq_factors(u[a], fac[a]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R v = rho * fac[0][cdir(D, i, 0) + 1] * fac[1][cdir(D, i, 1) + 1];
        if constexpr (D == 3) v *= fac[2][cdir(D, i, 2) + 1];
        fe[i] = v;
    }
}

// The velocity the collision uses, u + du, has reached the lattice speed:
// |u + du| >= 1 (counted as an instability next to NaN and rho <= 0)
template <int D, typename R> __device__ __forceinline__ bool too_fast(const R *u, const R *du)
{
    R s = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) s += (u[a] + du[a]) * (u[a] + du[a]);
    return s >= (R)1;
}

// Entropic alpha: non-trivial root of H(f' + alpha Delta) = H(f'), Eqs. 30-32,
// as G(alpha) = sum f'[(1 + alpha x) log1p(alpha x) - alpha x] - alpha K,
// x = Delta/f', K = sum f' x log1p(x): the terms linear in ln(f^eq/w) and
// alpha sum Delta vanish because Delta carries no mass or momentum, and
// leaving them out keeps the root free of their rounding.  The expansion of
// G about alpha = 2 gives alpha_s = 2 + (S3 - 2 S4)/(3 S2 - 4 S3), S_k =
// sum f' x^k.  kind: 0 small deviation (max|x| < eps: alpha_s is the root to
// O(x^3)), 1 Newton root, 2 fallback (non-positive f' or no convergence).
// Newton starts from alpha_s (one step fewer than from alpha = 2 on typical
// interface states); its iterates are kept in (1, alpha_max), alpha_max =
// min_{x<0} -1/x the positivity limit.  It stops when |step| < tol or when a step below 10 tol
// fails to halve the previous one (resolved to rounding).  On return dx holds
// x (is_x = true) or, after a non-positive f', still Delta.
template <int Q, typename R>
__device__ __forceinline__ R entropic_alpha(const R *fp, R *dx, R eps, R tol, int maxit, int &kind,
                                            bool &is_x)
{
    bool pos = true;
#pragma unroll
    for (int i = 0; i < Q; ++i) pos = pos && (fp[i] > (R)0);
    if (!pos) { kind = 2; is_x = false; return (R)2; }
    is_x = true;
    R xmax = 0, xmin = 0;
    R S2 = 0, S3 = 0, S4 = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R x = fdiv(dx[i], fp[i]);
        dx[i] = x;
        xmax = fmax(xmax, fabs(x));
        xmin = fmin(xmin, x);
        const R x2 = x * x;
        S2 += fp[i] * x2;
        S3 += fp[i] * x2 * x;
        S4 += fp[i] * x2 * x2;
    }
    // min over x < 0 of -1/x is -1/min(x) (the division is monotone)
    const R amax = xmin < (R)0 ? fdiv((R)-1, xmin) : (R)INFINITY;
    const R den = (R)3 * S2 - (R)4 * S3;
    const R as = den > (R)0 ? (R)2 + fdiv(S3 - (R)2 * S4, den) : (R)2;
    if (xmax < eps) { kind = 0; return as; }
    R K = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) K += fp[i] * dx[i] * flog1p(dx[i]);
    R al;
    if (den > (R)0 && as > (R)1 && as < amax) al = as;
    else al = ((R)2 < amax) ? (R)2 : (R)0.5 * ((R)1 + amax);
    const R stag = (R)10 * tol;
    R prev = (R)INFINITY;
    for (int it = 0; it < maxit; ++it) {
        R G = 0, G1 = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R ax = al * dx[i];
            const R la = flog1p(ax);
            G += fp[i] * (((R)1 + ax) * la - ax);
            G1 += fp[i] * dx[i] * la;
        }
        G -= al * K;
        G1 -= K;
        if (!(G1 > (R)0)) break;
        R an = al - fdiv(G, G1);
        if (an >= amax) an = (R)0.5 * (al + amax);
        if (an <= (R)1) an = (R)0.5 * (al + (R)1);
        const R st = fabs(an - al);
        if (st < tol || (st < stag && st > (R)0.5 * prev)) { kind = 1; return an; }
        prev = st;
        al = an;
    }
    kind = 2;
    return ((R)2 < amax) ? (R)2 : amax;
}

// ------------------------------------------------------------ collision --
// Per-axis equilibrium factors at u and at u + du and their differences
// (FP32).  With s = sqrt(1 + 3u^2), A = 2 - s and B = (2u + s)/(1 - u)
// (Eq. 27) the factors (A/6B, 2A/3, AB/6) sum to 1 and their first moment
// is u exactly; in FP32 the c = -1 factor is computed and the others are
// taken from these two identities, so that the equilibrium carries the
// node's mass and momentum to rounding (computed through A and B their
// errors bias both, by 1e-8 per step).  The c = -1 difference is formed
// without cancellation: A(u + du) - A(u) = -3 du (2u + du)/(s + s') and
// B(u + du) - B(u) = (2 du + (s' - s)(1 - u) + s du)/((1 - u)(1 - u - du)).
template <typename R>
__device__ __forceinline__ void feq_factor_steps(R u, R du, R *fe, R *fd, R *dd)
{
    // no contraction into fused multiply-adds, so that every kernel that
    // inlines this rounds it the same way
#pragma clang fp contract(off)
    const R ud = u + du;
    const R s = fsqrt((R)1 + (R)3 * u * u), sd = fsqrt((R)1 + (R)3 * ud * ud);
    const R A = (R)2 - s;
    const R B = fdiv((R)2 * u + s, (R)1 - u), Bd = fdiv((R)2 * ud + sd, (R)1 - ud);
    const R dA = fdiv((R)-3 * du * ((R)2 * u + du), s + sd);
    const R dB = fdiv((R)2 * du - dA * ((R)1 - u) + s * du, ((R)1 - u) * ((R)1 - ud));
    fe[0] = fdiv((R)(1.0 / 6.0) * A, B);
    dd[0] = fdiv((R)(1.0 / 6.0) * (dA * B - A * dB), B * Bd);
    fd[0] = fe[0] + dd[0];
    fe[2] = fe[0] + u;
    fd[2] = fd[0] + ud;
    dd[2] = dd[0] + du;
    fe[1] = (R)1 - fe[0] - fe[2];
    fd[1] = (R)1 - fd[0] - fd[2];
    dd[1] = -(dd[0] + dd[2]);
}

// ELBM step of one node (Eqs. 24-32): on entry f holds the node's stored
// populations, on return f* = f' + alpha beta Delta, with the mirror state
// f' = f + f^eq(rho, u + du) - f^eq(rho, u) and Delta = f^eq(rho, u + du) - f'
// = f^eq(rho, u) - f.  Returns the alpha kind (0 small deviation, 1 Newton,
// 2 fallback), or -1 when alpha = 2 is forced.
template <int D, typename R>
__device__ __forceinline__ int collide_f(R *f, R r0, const R *u, const R *du, R beta, R aeps, R atol, int maxit,
                                         bool alpha2)
{
    constexpr int Q = D == 2 ? 9 : 27;
    R dl[Q];
    if constexpr (sizeof(R) == 4) {
        // FP32: the forcing term f^eq(u + du) - f^eq(u) is small against
        // either equilibrium, so it is formed from the factor differences
        // (a telescoping product) instead of subtracting two rounded
        // equilibria; Delta as f^eq(u) - f.  Not contracted into fused
        // multiply-adds, so that every kernel rounds it the same way.
#pragma clang fp contract(off)
        R fe[3][3], fd[3][3], dd[3][3];
#pragma unroll
        for (int a = 0; a < D; ++a) feq_factor_steps(u[a], du[a], fe[a], fd[a], dd[a]);
        // per population e = rho prod_a fe_a and the telescoped difference
        // rho [dd_0 fd_1 (fd_2) + fe_0 dd_1 (fd_2) (+ fe_0 fe_1 dd_2)], from
        // products over the leading axes shared by the populations
        R ez[3], fz[3], dz[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ez[k] = r0 * fe[D - 1][k];
            fz[k] = r0 * fd[D - 1][k];
            dz[k] = r0 * dd[D - 1][k];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int kx = cdir(D, i, 0) + 1, ky = cdir(D, i, 1) + 1, kz = D == 3 ? cdir(D, i, 2) + 1 : 1;
            R e, dme;
            if constexpr (D == 3) {
                const R pxy = fe[0][kx] * fe[1][ky];
                const R xy = dd[0][kx] * fd[1][ky] + fe[0][kx] * dd[1][ky];
                e = pxy * ez[kz];
                dme = xy * fz[kz] + pxy * dz[kz];
            } else {
                e = fe[0][kx] * ez[ky];
                dme = dd[0][kx] * fz[ky] + fe[0][kx] * dz[ky];
            }
            dl[i] = e - f[i];  // Delta
            f[i] += dme;       // mirror state f'
        }
    } else {
        R fe[3][3], fd[3][3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            feq_factors(u[a], fe[a]);
            feq_factors(u[a] + du[a], fd[a]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            R e = r0 * fe[0][cdir(D, i, 0) + 1] * fe[1][cdir(D, i, 1) + 1];
            R d = r0 * fd[0][cdir(D, i, 0) + 1] * fd[1][cdir(D, i, 1) + 1];
            if constexpr (D == 3) {
                e *= fe[2][cdir(D, i, 2) + 1];
                d *= fd[2][cdir(D, i, 2) + 1];
            }
            R fpi = f[i] + d - e;
            dl[i] = d - fpi;  // Delta
            f[i] = fpi;       // mirror state f'
        }
    }
    R al = (R)2;
    bool is_x = false;
    int kind = -1;
    if (!alpha2) al = entropic_alpha<Q, R>(f, dl, aeps, atol, maxit, kind, is_x);
    const R ab = al * beta;
    if (is_x) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] += ab * (dl[i] * f[i]);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] += ab * dl[i];
    }
    if constexpr (sizeof(R) == 4) {
        // FP32: the rest population takes the node's mass minus the moving
        // ones.  The equilibrium's per-axis factors round to a sum slightly
        // above 1 (2/3 + 2 (1/6) = 1 + 3e-8 at rest), which otherwise adds
        // that fraction of the mass at every node and step (1.6e-4 after
        // 2000 steps of a 128 x 64 drop).
        R m = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i != Q / 2) m += f[i];
        f[Q / 2] = r0 - m;
    }
    return kind;
}

// g^eq(phi, v), v = u + du/2 (Eqs. 33-35): g^eq_i = w_i (a + v.c_i (b +
// c v.c_i)) with a = 3 Gamma mu_phi - 1.5 phi |v|^2, b = 3 phi, c = 4.5 phi
// for i other than the rest velocity; g^eq_rest = phi - (the sum of the
// others, in population order).
// Evaluated without contraction, so the moments pass that rebuilds g from
// (a, phi, v) at tau_g = 1 gets the very values the collision produced.
template <int D, typename R>
__device__ __forceinline__ R geq_a(const R *v, R p0, R mup, R Gam)
{
#pragma clang fp contract(off)
    R vv = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) vv += v[a] * v[a];
    return (R)3 * Gam * mup - (R)1.5 * p0 * vv;
}
template <int D, typename R>
__device__ __forceinline__ R geq_i(int i, const R *v, R ca, R cb, R cc)
{
#pragma clang fp contract(off)
    R vc = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (cdir(D, i, a) != 0) vc += (R)cdir(D, i, a) * v[a];
    return (R)wgt(D, i) * (ca + vc * (cb + cc * vc));
}
template <int D, typename R>
__device__ __forceinline__ R geq_rest(const R *v, R p0, R ca)
{
#pragma clang fp contract(off)
    constexpr int Q = D == 2 ? 9 : 27;
    const R cb = (R)3 * p0, cc = (R)4.5 * p0;
    R sum = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (i != Q / 2) sum += geq_i<D, R>(i, v, ca, cb, cc);
    return p0 - sum;
}

// LBGK for g (Eqs. 33-35).  At tau_g = 1 (itg = 1) g* = g^eq exactly (the
// stored g is not needed, and FRESH callers do not load it); otherwise
// g* = g + (g^eq - g)/tau_g.
template <int D, typename R, bool FRESH = false>
__device__ __forceinline__ void collide_g(R *gg, const R *v, R p0, R mup, R Gam, R itg)
{
    constexpr int Q = D == 2 ? 9 : 27;
    const R ca = geq_a<D, R>(v, p0, mup, Gam), cb = (R)3 * p0, cc = (R)4.5 * p0;
    const bool one = itg == (R)1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (i == Q / 2) continue;
        const R ge = geq_i<D, R>(i, v, ca, cb, cc);
        if constexpr (FRESH) gg[i] = ge;
        else gg[i] = one ? ge : gg[i] + (ge - gg[i]) * itg;
    }
    const R gr = geq_rest<D, R>(v, p0, ca);
    if constexpr (FRESH) gg[Q / 2] = gr;
    else gg[Q / 2] = one ? gr : gg[Q / 2] + (gr - gg[Q / 2]) * itg;
}

// Raw buffer access to one array of n elements at a uniform base: the
// resource (base, size) lives in scalar registers and each lane supplies a
// 32-bit byte offset, so no 64-bit address arithmetic is spent per access;
// accesses beyond the array read 0 and drop the store.  Every array of a
// simulation is below 4 GiB (checked when the handle is created).
template <typename T> __device__ __forceinline__ __amdgpu_buffer_rsrc_t arr(const T *base, unsigned n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(n * (unsigned)sizeof(T)), 0x00020000);
}
template <typename T> __device__ __forceinline__ T ld32(__amdgpu_buffer_rsrc_t r, unsigned byte_off)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
    else if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0));
}
template <typename T> __device__ __forceinline__ void st32(__amdgpu_buffer_rsrc_t r, unsigned byte_off, T v)
{
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, byte_off, 0, 0);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, byte_off, 0, 0);
}

// The uniform pointer p in scalar registers, opaque to the compiler: buffer
// resources built from it are built where they are used, not hoisted out of
// a loop or ahead of the arithmetic, where many of them outgrow the scalar
// registers and spill into vector lanes.
template <typename T> __device__ __forceinline__ T *opaque(T *p)
{
    const unsigned long long v = (unsigned long long)p;
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (T *)(((unsigned long long)hi << 32) | lo);
}

// -------------------------------------------------------------- moments --
// Nodes per thread of the moments kernel: in 2D, 16-byte loads of V
// consecutive nodes when the plane stride is a multiple of V (then so are
// the fluid range's start and length and every population array's offset);
// in 3D one (27 wide loads per set outgrow the registers, measured slower).
template <int D, int PREC> constexpr int mom_vec() { return D == 3 ? 1 : (PREC == P64 ? 2 : 4); }
inline int mom_width(const KParams &kp, int prec)
{
    const int v = kp.D == 3 ? 1 : (prec == P64 ? 2 : 4);
    return kp.PS % v == 0 ? v : 1;
}

// rho, phi of the fluid nodes of thread t (counted from the first fluid
// plane): V nodes in one group, summed per node in population order
template <int D, int PREC, int V>
__device__ __forceinline__ void moments_nodes(const KParams &kp, const typename Ty<PREC>::S *__restrict__ f,
                                              const typename Ty<PREC>::S *__restrict__ g,
                                              const typename Ty<PREC>::R *__restrict__ rprev,
                                              const typename Ty<PREC>::R *__restrict__ pprev,
                                              typename Ty<PREC>::R *__restrict__ rho,
                                              typename Ty<PREC>::R *__restrict__ phi, long long t)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    using VS = S __attribute__((ext_vector_type(V)));
    using VR = R __attribute__((ext_vector_type(V)));
    constexpr int Q = D == 2 ? 9 : 27;
    const long long first = kp.walls ? kp.PS : 0;
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    if (t * V >= count) return;
    const long long n = first + t * V;
    VR rp = (R)0, pp = (R)0;
    if constexpr (PREC == P16) {
        rp = *(const VR *)(rprev + n);
        pp = *(const VR *)(pprev + n);
    }
    VS fv[Q], gv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fv[i] = *(const VS *)(f + (long long)i * kp.QS + n);
        gv[i] = *(const VS *)(g + (long long)i * kp.QS + n);
    }
    VR r = (R)0, ph = (R)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            r[j] += dec_f<PREC, D>(fv[i][j], i, rp[j]);
            ph[j] += dec_g<PREC, D>(gv[i][j], i, pp[j]);
        }
    }
    *(VR *)(rho + n) = r;
    *(VR *)(phi + n) = ph;
}

template <int D, int PREC>
__device__ __forceinline__ void moments_node(const KParams &kp, const typename Ty<PREC>::S *__restrict__ f,
                                             const typename Ty<PREC>::S *__restrict__ g,
                                             const typename Ty<PREC>::R *__restrict__ rprev,
                                             const typename Ty<PREC>::R *__restrict__ pprev,
                                             typename Ty<PREC>::R *__restrict__ rho,
                                             typename Ty<PREC>::R *__restrict__ phi, long long t)
{
    constexpr int V = mom_vec<D, PREC>();
    if (kp.PS % V == 0) moments_nodes<D, PREC, V>(kp, f, g, rprev, pprev, rho, phi, t);
    else moments_nodes<D, PREC, 1>(kp, f, g, rprev, pprev, rho, phi, t);
}

template <int D, int PREC>
__global__ void __launch_bounds__(256)
k_moments(KParams kp, const typename Ty<PREC>::S *__restrict__ f, const typename Ty<PREC>::S *__restrict__ g,
          const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
          typename Ty<PREC>::R *__restrict__ rho, typename Ty<PREC>::R *__restrict__ phi)
{
    moments_node<D, PREC>(kp, f, g, rprev, pprev, rho, phi, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// A buffer pointer read from a simulation descriptor, re-derived from the
// descriptor array (a kernel argument, known to be global memory) so that
// the accesses through it compile to global instead of flat instructions
// (flat ones also count against the LDS wait counter): the same address.
template <typename T>
__device__ __forceinline__ T *on_global(const SimDesc *base, const void *p)
{
    return (T *)((const char *)base + (long long)((uintptr_t)p - (uintptr_t)base));
}

// Blocks of a launch go to the 8 XCDs in turn (block b to XCD b mod 8),
// each with its own L2: renumbered so that every XCD walks one contiguous
// eighth of the grid and finds the rows and planes around its nodes in its
// own L2.  A bijection on [0, nb) (identity for the last nb mod 8 blocks).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned per = nb / 8u;
    if (b >= per * 8u) return b;
    return (b % 8u) * per + b / 8u;
}

// The g populations that streaming delivers to a fluid node when tau_g = 1
// with collisions (3D two-kernel step), from the (a, phi, v) that the
// collision stored at every node: g_i(x) = g^eq_i at the source x - c_i,
// or for a population bounced back at a wall g^eq of the opposite velocity
// at x itself, and the rest population g^eq_rest(x).  get(cx, cy, cz, k)
// returns value k of (a, phi, v0, v1, v2) at x - c; low / high: the node
// lies on the first / last fluid plane of a walled grid.  The values are
// those the collision computed; sink(i, g_i) sees them in population order.
template <typename R, typename Get, typename Sink>
__device__ __forceinline__ void implicit_g(Get get, bool low, bool high, Sink sink)
{
    constexpr int D = 3, Q = 27;
    const R oa = get(0, 0, 0, 0), op = get(0, 0, 0, 1);
    const R ov[3] = {get(0, 0, 0, 2), get(0, 0, 0, 3), get(0, 0, 0, 4)};
    const R ob = (R)3 * op, oc = (R)4.5 * op;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cdir(D, i, 0), cy = cdir(D, i, 1), cz = cdir(D, i, 2);
        if (i == Q / 2) {
            sink(i, geq_rest<D, R>(ov, op, oa));
        } else if ((cz > 0 && low) || (cz < 0 && high)) {
            sink(i, geq_i<D, R>(Q - 1 - i, ov, oa, ob, oc));
        } else {
            const R sa = get(cx, cy, cz, 0), sp = get(cx, cy, cz, 1);
            const R sv[3] = {get(cx, cy, cz, 2), get(cx, cy, cz, 3), get(cx, cy, cz, 4)};
            sink(i, geq_i<D, R>(i, sv, sa, (R)3 * sp, (R)4.5 * sp));
        }
    }
}

// The implicit-g moments pass as a march: block b of a simulation takes the
// TX x TY tile (b mod tiles) through the `chunk` consecutive fluid planes of
// chunk (b / tiles), keeping the five values of three planes (tile and ring)
// in an LDS ring, so that each plane is staged once per tile instead of
// three times.  The same values and sums as the stored-g pass.  The buffer
// resources of the 27 population arrays and the five value arrays are
// rebuilt in every plane from bases the compiler cannot see through: held
// across the loop, those 32 resources (128 scalar registers) spill into
// vector lanes, and their reloads took a third of the loop's vector
// instructions.  imp false (batched steps only): g is still stored (the
// first step after an initialisation or an export), phi = the sum of the
// stored g and nothing is staged.
constexpr int kImpTX = 64, kImpTY = 4;
template <int PREC, int TX, int TY>
__device__ __forceinline__ void moments_march(const KParams &kp, const typename Ty<PREC>::S *__restrict__ f,
                                              const typename Ty<PREC>::S *__restrict__ g,
                                              const typename Ty<PREC>::R *__restrict__ gp,
                                              const typename Ty<PREC>::R *__restrict__ rprev,
                                              const typename Ty<PREC>::R *__restrict__ pprev,
                                              typename Ty<PREC>::R *__restrict__ rho,
                                              typename Ty<PREC>::R *__restrict__ phi, int chunk, unsigned b, bool imp,
                                              typename Ty<PREC>::R (*s_p)[5][(TY + 2) * (TX + 2)])
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    constexpr int Q = 27, EX = TX + 2, EY = TY + 2, CELLS = EY * EX;
    constexpr unsigned SR = sizeof(R), SS = sizeof(S);
    const int nx = kp.nx, ny = kp.ny, nw = kp.nw;
    const bool walls = kp.walls != 0;
    const unsigned N = (unsigned)kp.N, PS = (unsigned)kp.PS;
    const unsigned QS = (unsigned)kp.QS;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, ntiles = ntx * nty;
    const int tile = (int)(b % (unsigned)ntiles), ch = (int)(b / (unsigned)ntiles);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int planes = walls ? nw - 2 : nw;
    const int q0 = ch * chunk, q1 = q0 + chunk < planes ? q0 + chunk : planes;
    const int off0 = walls ? 1 : 0;
    // stage plane pz (any plane, ghost planes included) into ring slot `slot`
    auto stage = [&](int slot, int pz) {
        if (!walls) pz = pz < 0 ? pz + nw : (pz >= nw ? pz - nw : pz);
        for (int c = threadIdx.x; c < CELLS; c += TX * TY) {
            const int lx = c % EX, ly = c / EX;
            // periodic wrap without a division (a tile may pass the end of a
            // small grid more than once)
            int gx = x0 + lx - 1, gy = y0 + ly - 1;
            if (gx < 0) gx += nx;
            while (gx >= nx) gx -= nx;
            if (gy < 0) gy += ny;
            while (gy >= ny) gy -= ny;
            const unsigned off = ((unsigned)pz * PS + (unsigned)gy * (unsigned)nx + (unsigned)gx) * SR;
            const R *gb = opaque(gp);
#pragma unroll
            for (int k = 0; k < 5; ++k) s_p[slot][k][c] = ld32<R>(arr(gb + (size_t)k * QS, N), off);
        }
    };
    const int lx = (int)threadIdx.x % TX, ly = (int)threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool in = x < nx && y < ny;
    const int l0 = (ly + 1) * EX + lx + 1;
    if (imp) {
        stage(0, q0 + off0 - 1);
        stage(1, q0 + off0);
    }
    for (int q = q0; q < q1; ++q) {
        const int pz = q + off0;
        const int sm = (q - q0) % 3, sc = (q - q0 + 1) % 3, sp = (q - q0 + 2) % 3;
        if (imp) stage(sp, pz + 1);
        const unsigned n = (unsigned)pz * PS + (unsigned)y * (unsigned)nx + (unsigned)x;
        S fr[Q];
        R rp = 0;
        if (in) {
            const S *fb = opaque(f);
#pragma unroll
            for (int i = 0; i < Q; ++i) fr[i] = ld32<S>(arr(fb + (size_t)i * QS, N), n * SS);
            // FP16 storage: offsets decoded with the density they were encoded with
            if constexpr (PREC == P16) rp = ld32<R>(arr(rprev, N), n * SR);
        }
        __syncthreads();
        if (in) {
            R r = 0, ph = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) r += dec_f<PREC, 3>(fr[i], i, rp);
            if (imp) {
                // the source x - c lies in plane pz - cz: below (sm), this (sc) or above (sp)
                auto get = [&](int cx, int cy, int cz, int k) {
                    const int sl = cz > 0 ? sm : (cz < 0 ? sp : sc);
                    return s_p[sl][k][l0 - cy * EX - cx];
                };
                implicit_g<R>(get, walls && pz == 1, walls && pz == nw - 2, [&](int, R gv) { ph += gv; });
            } else {
                R pp = 0;
                if constexpr (PREC == P16) pp = ld32<R>(arr(pprev, N), n * SR);
                const S *gb = opaque(g);
#pragma unroll
                for (int i = 0; i < Q; ++i) ph += dec_g<PREC, 3>(ld32<S>(arr(gb + (size_t)i * QS, N), n * SS), i, pp);
            }
            st32<R>(arr(rho, N), n * SR, r);
            st32<R>(arr(phi, N), n * SR, ph);
        }
        __syncthreads();
    }
}

// The single-simulation pass, its blocks renumbered so that each XCD takes a
// contiguous range of tiles and chunks.
template <int PREC, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_moments_imp(KParams kp, const typename Ty<PREC>::S *__restrict__ f, const typename Ty<PREC>::R *__restrict__ gp,
              const typename Ty<PREC>::R *__restrict__ rprev, typename Ty<PREC>::R *__restrict__ rho,
              typename Ty<PREC>::R *__restrict__ phi, int chunk)
{
    using R = typename Ty<PREC>::R;
    __shared__ R s_p[3][5][(TY + 2) * (TX + 2)];
    moments_march<PREC, TX, TY>(kp, f, nullptr, gp, rprev, nullptr, rho, phi, chunk,
                                xcd_block(blockIdx.x, gridDim.x), true, s_p);
}

// planes per block of the marching moments pass: about 4096 blocks
inline int imp_chunk(const KParams &kp, long long ntiles)
{
    const long long planes = kp.walls ? kp.nw - 2 : kp.nw;
    long long c = (ntiles * planes + 4095) / 4096;
    if (c < 1) c = 1;
    if (c > planes) c = planes;
    return (int)c;
}

// planes per block and blocks of the march of one simulation
int moments_march_chunk(const KParams &kp)
{
    return imp_chunk(kp, (long long)((kp.nx + kImpTX - 1) / kImpTX) * ((kp.ny + kImpTY - 1) / kImpTY));
}
static long long moments_march_blocks(const KParams &kp)
{
    const long long planes = kp.walls ? kp.nw - 2 : kp.nw;
    const long long ntiles = (long long)((kp.nx + kImpTX - 1) / kImpTX) * ((kp.ny + kImpTY - 1) / kImpTY);
    const long long chunk = moments_march_chunk(kp);
    return ntiles * ((planes + chunk - 1) / chunk);
}

// implicit_g at fluid node n with the values gathered from global memory
template <int PREC, typename Sink>
__device__ __forceinline__ void implicit_g_global(const KParams &kp, const typename Ty<PREC>::R *__restrict__ gp,
                                                  unsigned n, Sink sink)
{
    using R = typename Ty<PREC>::R;
    constexpr unsigned SR = sizeof(R);
    const unsigned N = (unsigned)kp.N, PS = (unsigned)kp.PS;
    const unsigned QS = (unsigned)kp.QS;
    const int nx = kp.nx, ny = kp.ny, nw = kp.nw;
    const bool walls = kp.walls != 0;
    const int x = (int)(n % (unsigned)nx), y = (int)((n / (unsigned)nx) % (unsigned)ny), p = (int)(n / PS);
    auto get = [&](int cx, int cy, int cz, int k) {
        const int sx = x - cx < 0 ? x - cx + nx : (x - cx >= nx ? x - cx - nx : x - cx);
        const int sy = y - cy < 0 ? y - cy + ny : (y - cy >= ny ? y - cy - ny : y - cy);
        const int sz = walls ? p - cz : (p - cz < 0 ? p - cz + nw : (p - cz >= nw ? p - cz - nw : p - cz));
        const unsigned off = ((unsigned)sz * PS + (unsigned)sy * (unsigned)nx + (unsigned)sx) * SR;
        return ld32<R>(arr(gp + (size_t)k * QS, N), off);
    };
    implicit_g<R>(get, walls && p == 1, walls && p == nw - 2, sink);
}

// The implicit g written out as populations (before anything that reads the
// stored g: observables, exports).
template <int PREC>
__global__ void __launch_bounds__(256)
k_g_materialize(KParams kp, const typename Ty<PREC>::R *__restrict__ gp, const typename Ty<PREC>::R *__restrict__ pcur,
                typename Ty<PREC>::S *__restrict__ g)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const unsigned n = (unsigned)((kp.walls ? kp.PS : 0) + t), N = (unsigned)kp.N;
    const unsigned QS = (unsigned)kp.QS;
    // FP16 storage: the rest population as an offset from the field phi the
    // next reader decodes it with (the current one)
    R pn = 0;
    if constexpr (PREC == P16) pn = ld32<R>(arr(pcur, N), n * (unsigned)sizeof(R));
    implicit_g_global<PREC>(kp, gp, n, [&](int i, R v) {
        st32<S>(arr(g + (size_t)i * QS, N), n * (unsigned)sizeof(S), enc_g<PREC, 3>(v, i, pn));
    });
}

// One launch over many simulations: block b belongs to simulation sim[b];
// `phase` is the parity of the steps taken since the descriptors were
// written, `first` whether this is the first of them.  A simulation with an
// implicit-g array (3D, tau_g = 1) takes the march of the single-simulation
// pass (blocks of 64 x 4 tiles and its descriptor's chunk of planes), with
// g implicit or, at the first step, still stored; the others one thread per
// node.
template <int D, int PREC>
__global__ void __launch_bounds__(256)
k_moments_batch(const SimDesc *__restrict__ d, const int *__restrict__ sim, int phase, int first)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    const SimDesc &sd = d[sim[blockIdx.x]];
    const KParams &kp = sd.kp;
    const int pc = sd.pc ^ phase, fc = sd.fc ^ phase;
    const long long t = (long long)(blockIdx.x - sd.mblk0) * blockDim.x + threadIdx.x;
    if constexpr (D == 3) {
        // simulations with an implicit-g array take the march (its block
        // count, moments_march_blocks), their g implicit or still stored
        __shared__ R s_p[3][5][(kImpTY + 2) * (kImpTX + 2)];
        if (sd.gp) {
            moments_march<PREC, kImpTX, kImpTY>(kp, on_global<const S>(d, sd.f[pc]), on_global<const S>(d, sd.g[pc]),
                                                on_global<const R>(d, sd.gp), on_global<const R>(d, sd.rho[fc]),
                                                on_global<const R>(d, sd.phi[fc]), on_global<R>(d, sd.rho[1 - fc]),
                                                on_global<R>(d, sd.phi[1 - fc]), sd.mchunk, blockIdx.x - sd.mblk0,
                                                !first || sd.gimp0, s_p);
            return;
        }
    }
    moments_node<D, PREC>(kp, on_global<const S>(d, sd.f[pc]), on_global<const S>(d, sd.g[pc]),
                          on_global<const R>(d, sd.rho[fc]), on_global<const R>(d, sd.phi[fc]),
                          on_global<R>(d, sd.rho[1 - fc]), on_global<R>(d, sd.phi[1 - fc]), t);
}

// ----------------------------------------------------------- ghost layers
// Interface detection (paper's rules, cascade 1-3 then 4-5 override):
// 0 = 1-2 (theta21), 1 = 1-3 (theta31), 2 = 2-3 (theta23).
template <typename R>
__device__ __forceinline__ int classify(R ngr, R ngp, R dot, R r, R ph, R rho_l, R drho, R chi, R ratio)
{
    int k;
    if (ngr * chi < ratio * drho * ngp) k = 2;
    else if (dot < (R)0) k = 1;
    else k = 0;
    if (r > (R)0.5 * rho_l && ph < (R)-0.95 * chi) k = 1;
    if (r > (R)0.5 * rho_l && ph > (R)0.95 * chi) k = 0;
    return k;
}

// linear interpolation along the wall at offset l, Eq. 47; get(dx, dy, r, p)
// returns the first fluid layer at in-plane offset (dx, dy) from the node
template <typename R, typename Get>
__device__ __forceinline__ void interp2(Get get, R l, R &r, R &ph)
{
    R l0 = floor(l), l1 = l0 + (R)1;
    R r0, p0;
    get((int)l0, 0, r0, p0);
    if (l == l0) { r = r0; ph = p0; return; }  // exact lattice copy at integer shifts
    R r1, p1;
    get((int)l1, 0, r1, p1);
    r = (r1 - r0) * l + (l1 * r0 - l0 * r1);
    ph = (p1 - p0) * l + (l1 * p0 - l0 * p1);
}

// plane through the three corners of the unit cell nearest to (lx, ly),
// Eqs. 48-49
template <typename R>
__device__ __forceinline__ R plane3(const R *X, const R *Y, const R *Cv, R lx, R ly)
{
    R x1 = X[0], x2 = X[1], x3 = X[2], y1 = Y[0], y2 = Y[1], y3 = Y[2];
    R c1 = Cv[0], c2 = Cv[1], c3 = Cv[2];
    R A = y2 * c1 - y3 * c1 - y1 * c2 + y3 * c2 + y1 * c3 - y2 * c3;
    R B = -x2 * c1 + x3 * c1 + x1 * c2 - x3 * c2 - x1 * c3 + x2 * c3;
    R Cc = -x3 * y2 * c1 + x2 * y3 * c1 + x3 * y1 * c2 - x1 * y3 * c2 - x2 * y1 * c3 + x1 * y2 * c3;
    R Dd = -x2 * y1 + x3 * y1 + x1 * y2 - x3 * y2 - x1 * y3 + x2 * y3;
    return (A * lx + B * ly + Cc) / Dd;
}

template <typename R, typename Get>
__device__ __forceinline__ void interp3(Get get, R lx, R ly, R &r, R &ph)
{
    R x0 = floor(lx), y0 = floor(ly);
    R fx = lx - x0, fy = ly - y0;
    const int cx[4] = {0, 1, 0, 1}, cy[4] = {0, 0, 1, 1};
    int drop = 0;
    R dmax = (R)-1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        R d = (fx - cx[k]) * (fx - cx[k]) + (fy - cy[k]) * (fy - cy[k]);
        if (d > dmax) { dmax = d; drop = k; }
    }
    R X[3], Y[3], Cr[3], Cp[3];
    int m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k == drop) continue;
        X[m] = x0 + cx[k];
        Y[m] = y0 + cy[k];
        get((int)X[m], (int)Y[m], Cr[m], Cp[m]);
        ++m;
    }
    r = plane3(X, Y, Cr, lx, ly);
    ph = plane3(X, Y, Cp, lx, ly);
}

// cot(theta) of the three interface pairs at one wall, in registers: the
// empty asm keeps the compiler from turning the selects back into an indexed
// load from the parameter block (a memory access and a wait per use)
template <typename R>
__device__ __forceinline__ void wall_cots(const KParams &kp, int wall, R (&c)[3])
{
    R a0 = (R)kp.cot[0][0], a1 = (R)kp.cot[0][1], a2 = (R)kp.cot[0][2];
    R b0 = (R)kp.cot[1][0], b1 = (R)kp.cot[1][1], b2 = (R)kp.cot[1][2];
    asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(b0), "+v"(b1), "+v"(b2));
    c[0] = wall == 0 ? a0 : b0;
    c[1] = wall == 0 ? a1 : b1;
    c[2] = wall == 0 ? a2 : b2;
}

// Ghost-layer values of one wall node (Sec. IV): copy of the first fluid
// layer for the force method, else the geometric wetting condition with the
// contact angle of the interface found by the detection rules (cot: the
// wall's cot(theta) per pair, from wall_cots).
template <int D, typename R, typename Get>
__device__ __forceinline__ void ghost_value(const KParams &kp, const R (&cot)[3], Get get, R &out_r, R &out_p)
{
    R r0, p0;
    get(0, 0, r0, p0);
    out_r = r0;
    out_p = p0;
    if (kp.wetting == 0) return;
    R drho = (R)kp.drho, chi = (R)kp.chi;
    R gr[2] = {0, 0}, gp[2] = {0, 0};
    R ra, pa, rb, pb;
    get(1, 0, ra, pa);
    get(-1, 0, rb, pb);
    gr[0] = (R)0.5 * (ra - rb);
    gp[0] = (R)0.5 * (pa - pb);
    if constexpr (D == 3) {
        get(0, 1, ra, pa);
        get(0, -1, rb, pb);
        gr[1] = (R)0.5 * (ra - rb);
        gp[1] = (R)0.5 * (pa - pb);
    }
    R ngr = sqrt(gr[0] * gr[0] + gr[1] * gr[1]);
    R ngp = sqrt(gp[0] * gp[0] + gp[1] * gp[1]);
    if (ngr < (R)1e-12 * drho && ngp < (R)1e-12 * drho) return;
    R dot = gr[0] * gp[0] + gr[1] * gp[1];
    int cls = classify(ngr, ngp, dot, r0, p0, (R)kp.rho_l, drho, chi, (R)kp.detect_ratio);
    const R ct = cls == 0 ? cot[0] : (cls == 1 ? cot[1] : cot[2]);
    const R *gc = cls == 2 ? gp : gr;
    R ngc = cls == 2 ? ngp : ngr;
    if (kp.wetting == 2) {
        // geometric extrapolation (Eqs. 45-46), per field along m, kept
        // within the bulk range widened to the first-layer value (the plain
        // extrapolation can give a negative gas-side density)
        if (ngc != (R)0) {
            R m0 = gc[0] / ngc, m1 = gc[1] / ngc;
            const R re = r0 + ct * (gr[0] * m0 + gr[1] * m1);
            const R pe = p0 + ct * (gp[0] * m0 + gp[1] * m1);
            const R rlo = fmin(r0, (R)kp.rho_g), rhi = fmax(r0, (R)kp.rho_l);
            const R plo = fmin(p0, -chi), phi_ = fmax(p0, chi);
            out_r = re < rlo ? rlo : (re > rhi ? rhi : re);
            out_p = pe < plo ? plo : (pe > phi_ ? phi_ : pe);
        }
    } else if constexpr (D == 2) {
        // shift by cot(theta) toward the measuring phase (+grad c)
        R sg = gc[0] > (R)0 ? (R)1 : (gc[0] < (R)0 ? (R)-1 : (R)0);
        interp2(get, sg * ct, out_r, out_p);
    } else {
        if (ngc != (R)0) interp3(get, ct * gc[0] / ngc, ct * gc[1] / ngc, out_r, out_p);
    }
}

template <int D, typename R>
__device__ __forceinline__ void ghost_node(const KParams &kp, R *__restrict__ rho, R *__restrict__ phi, int t)
{
    int nx = kp.nx, ny = kp.ny;
    int np = (D == 2) ? nx : nx * ny;  // ghost nodes per wall
    if (t >= 2 * np) return;
    int wall = t / np;
    int k = t % np;
    int i = k % nx, j = (D == 2) ? 0 : k / nx;
    int kg = wall == 0 ? 0 : kp.nw - 1, kf = wall == 0 ? 1 : kp.nw - 2;
    long long bf = (long long)kf * kp.PS, ng = (long long)kg * kp.PS + i + (long long)nx * j;
    auto get = [&](int dx, int dy, R &r, R &ph) {
        long long n = bf + wrapi(i + dx, nx) + (D == 3 ? (long long)nx * wrapi(j + dy, ny) : 0);
        r = rho[n];
        ph = phi[n];
    };
    R out_r, out_p, cot[3];
    wall_cots<R>(kp, wall, cot);
    ghost_value<D, R>(kp, cot, get, out_r, out_p);
    rho[ng] = out_r;
    phi[ng] = out_p;
}

template <int D, typename R>
__global__ void __launch_bounds__(256)
k_ghost(KParams kp, R *__restrict__ rho, R *__restrict__ phi)
{
    ghost_node<D, R>(kp, rho, phi, blockIdx.x * blockDim.x + threadIdx.x);
}

template <int D, typename R>
__global__ void __launch_bounds__(256)
k_ghost_batch(const SimDesc *__restrict__ d, const int *__restrict__ sim, int phase)
{
    const SimDesc &sd = d[sim[blockIdx.x]];
    const KParams &kp = sd.kp;
    const int fc = sd.fc ^ phase;
    ghost_node<D, R>(kp, on_global<R>(d, sd.rho[1 - fc]), on_global<R>(d, sd.phi[1 - fc]),
                     (blockIdx.x - sd.gblk0) * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- fused --
// wrap of v into [0, n) for |v| < 2n (one conditional each way)
// Planes [pb, pe) of block row `by` along the wall axis.  In the small 2D
// class, when its chunks hold more than one plane, the six planes next to
// each wall run one per block: they hold the wetting films' interfaces (most
// Newton solves of alpha) and the ghost fill, and with every block of such a
// launch resident at once the slowest block sets its duration (measured 6 %
// faster than uniform two-plane chunks on a 2048 x 64 channel).
//
// With one plane per block (chunk 1) the same small 2D class instead takes
// the two planes next to each wall first (edge -1): those blocks fill the
// ghost layers and run longest, and blocks start in index order.
__host__ __device__ inline int wall_edge(const KParams &kp, bool small2d, int chunk)
{
    const int planes = kp.walls ? kp.nw - 2 : kp.nw;
    if (small2d && kp.walls && chunk == 1 && planes >= 4) return -1;
    return (small2d && kp.walls && chunk > 1 && planes > 12 + chunk) ? 6 : 0;
}
__host__ __device__ inline void chunk_range(const KParams &kp, int edge, int chunk, int by, int &pb, int &pe)
{
    const int pf0 = kp.walls ? 1 : 0, pf1 = kp.walls ? kp.nw - 1 : kp.nw;
    if (edge < 0) {
        // planes 1, nw - 2, 2, nw - 3, then 3 .. nw - 4
        pb = by < 4 ? ((by & 1) ? kp.nw - 2 - (by >> 1) : 1 + (by >> 1)) : by - 1;
        pe = pb + 1;
        return;
    }
    if (edge == 0) {
        pb = pf0 + by * chunk;
        pe = pb + chunk < pf1 ? pb + chunk : pf1;
        return;
    }
    const int nmid = (pf1 - pf0 - 2 * edge + chunk - 1) / chunk;
    if (by < edge) {
        pb = pf0 + by;
        pe = pb + 1;
    } else if (by < edge + nmid) {
        pb = pf0 + edge + (by - edge) * chunk;
        pe = pb + chunk < pf1 - edge ? pb + chunk : pf1 - edge;
    } else {
        pb = pf1 - edge + (by - edge - nmid);
        pe = pb + 1;
    }
}
__host__ __device__ inline int chunk_count(const KParams &kp, int edge, int chunk)
{
    const int planes = kp.walls ? kp.nw - 2 : kp.nw;
    if (edge < 0) return planes;
    return edge ? 2 * edge + (planes - 2 * edge + chunk - 1) / chunk : (planes + chunk - 1) / chunk;
}

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// general wrap without a division (setup only)
__device__ __forceinline__ int wrapl(int v, int n)
{
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// One block updates a TX x TY tile (TY = 1 in 2D) of every plane in its
// chunk with NTH >= TX TY threads; NTH = (TX + 2)(TY + 2) in 2D makes the
// -P stage one pass per plane.  In 2D the wall ghost layers of rho, phi are
// filled by the blocks themselves from the first fluid layer (and written
// back for their own nodes), so a step is the moments kernel and this one;
// in 3D the ghost-layer kernel runs in between.
//
// SPLIT: the stencil pass of the two-kernel step instead (3D): the same
// march and force, then F and mu_phi go to fmu ([D + 1][QS]) and the
// populations are left to k_collide.
// ONE: every chunk is one plane (no march loop, so the compiler's counts of
// memory operations in flight need not merge a loop's back edge).
template <int D, int PREC, int TX, int TY, int NTH, bool SPLIT = false, bool ONE = false>
__device__ __forceinline__ void
fused_tile(const KParams &kp, const typename Ty<PREC>::S *__restrict__ fin, const typename Ty<PREC>::S *__restrict__ gin,
           typename Ty<PREC>::S *__restrict__ fout, typename Ty<PREC>::S *__restrict__ gout,
           typename Ty<PREC>::R *__restrict__ rho, typename Ty<PREC>::R *__restrict__ phi,
           const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
           unsigned long long *__restrict__ cnt, int chunk, int bx, int by,
           typename Ty<PREC>::R *__restrict__ fmu = nullptr)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    constexpr int Q = D == 2 ? 9 : 27;
    constexpr int HF = 3;                        // halo of the rho, phi tile
    constexpr int FW = TX + 2 * HF, FH = D == 3 ? TY + 2 * HF : 1, FS = FW * FH;
    constexpr int TW = TX + 2, TH = D == 3 ? TY + 2 : 1, TS = TW * TH;
    constexpr int NP = D * (D + 1) / 2;
    constexpr int WA = D - 1;                    // wall (march) axis component
    constexpr int NLD = (FS + NTH - 1) / NTH;    // field elements loaded per thread and plane
    constexpr int NIP = D == 3 ? 9 : 3;          // in-plane neighbour offsets
    __shared__ R s_r[5][FS];
    __shared__ R s_p[5][FS];
    // QR: keep sqrt(rho) in a ring for the link pressures (one square root
    // per field element instead of one per link); the small 2D tile, whose
    // run time is the latency of its plane stages, takes it per link
    constexpr bool QR = !(D == 2 && NTH <= 64);
    __shared__ R s_q[5][QR ? FS : 1];
    __shared__ R s_t[3][NP + 1][TS];
    __shared__ int s_cnt[4];

    const int tid = threadIdx.x;
    const int nx = kp.nx, ny = kp.ny, nw = kp.nw;
    const unsigned N = (unsigned)kp.N, PS = (unsigned)kp.PS;
    const unsigned QS = (unsigned)kp.QS;
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (bx % ntx) * TX;
    const int y0 = (D == 3) ? (bx / ntx) * TY : 0;
    int pb, pe;
    chunk_range(kp, wall_edge(kp, D == 2 && NTH <= 64, chunk), chunk, by, pb, pe);
    if (pb >= pe) return;
    if (tid < 4) s_cnt[tid] = 0;

    Thermo<R> th;
    th.load(kp);
    const R beta = (R)kp.beta, itg = (R)kp.inv_tau_g, Gam = (R)kp.Gamma;
    const R aeps = (R)kp.alpha_eps, atol = (R)kp.alpha_tol;
    const bool collide = !(kp.flags & 1u), alpha2 = (kp.flags & 2u) != 0;
    const bool walls = kp.walls != 0;

    // in-plane indices of the field elements this thread loads (fixed for
    // the march) and whether the element is one of the block's own nodes
    unsigned ld_idx[NLD];
    unsigned own = 0;
#pragma unroll
    for (int m = 0; m < NLD; ++m) {
        int k = tid + m * NTH;
        // threads beyond the tile's elements load the last element again
        // (one address, so their loads cost one cache line per wave)
        const int ka = k < FS ? k : FS - 1;
        int lx = ka % FW, ly = ka / FW;
        unsigned v = (unsigned)wrapl(x0 + lx - HF, nx);
        if constexpr (D == 3) v += (unsigned)nx * (unsigned)wrapl(y0 + ly - HF, ny);
        ld_idx[m] = v;
        bool o = k < FS && lx >= HF && lx < TX + HF && x0 + lx - HF < nx;  // k >= FS: not own
        if constexpr (D == 3) o = o && ly >= HF && ly < TY + HF && y0 + ly - HF < ny;
        own |= (o ? 1u : 0u) << m;
    }
    auto plane = [&](int q) { return walls ? q : wrapl(q, nw); };

    // 2D: the block fills the wall ghost layers itself (one launch fewer per
    // step); 3D: they come filled from the ghost-layer kernel
    constexpr bool GK = D == 2;

    // plane q of rho, phi into the LDS ring (ghost layers: ghost_plane), in
    // two halves: fetch issues the loads into registers, commit stores them,
    // so a plane's loads can be in flight while the previous one is worked on.
    // Every thread loads, whether or not the element is used (planes beyond
    // the walls read the nearest stored plane, surplus threads the tile's
    // last element): with no load under a branch the compiler's counts of
    // loads in flight stay exact, and a wait for one plane does not also wait
    // for the loads issued after it.
    auto has_fields = [&](int q) {
        if (walls && (q < 0 || q > nw - 1)) return false;
        return !(GK && walls && (q == 0 || q == nw - 1));
    };
    auto fetch_into = [&](int q, R *dr, R *dp) {
        const int qc = walls ? (q < 0 ? 0 : (q > nw - 1 ? nw - 1 : q)) : q;
        const unsigned base = (unsigned)plane(qc) * PS;
#pragma unroll
        for (int m = 0; m < NLD; ++m) {
            dr[m] = rho[base + ld_idx[m]];
            dp[m] = phi[base + ld_idx[m]];
        }
    };
    auto commit_from = [&](int q, const R *dr, const R *dp) {
        if (!has_fields(q)) return;
        const int slot = (q + 10) % 5;
#pragma unroll
        for (int m = 0; m < NLD; ++m) {
            int k = tid + m * NTH;
            if (NLD * NTH == FS || k < FS) {
                s_r[slot][k] = dr[m];
                if constexpr (QR) s_q[slot][k] = fsqrt(dr[m]);
                s_p[slot][k] = dp[m];
            }
        }
    };
    R pre_r[NLD], pre_p[NLD];
    auto fetch = [&](int q) { fetch_into(q, pre_r, pre_p); };
    auto commit = [&](int q) { commit_from(q, pre_r, pre_p); };

    // Wall ghost layer q (0 or nw - 1) over the tile and a halo of 2 (Sec. IV)
    // from the first fluid layer, which is in the ring; the wetting condition
    // reads it within the tile's halo of HF = 3 from LDS and, where a contact
    // angle's |cot| exceeds 1 (interpolation shifts beyond one node), further
    // out along the wall from rho, phi.  The two cases are separate code, so
    // that the common one has no global loads (whose waits would also wait
    // for the population loads in flight).
    auto ghost_plane = [&](int q) {
        if constexpr (!GK) return;
        const int wall = q == 0 ? 0 : 1;
        const int kf = wall == 0 ? 1 : nw - 2;
        const int sg = (q + 10) % 5, sf = (kf + 10) % 5;
        const unsigned bf = (unsigned)kf * PS, bg = (unsigned)q * PS;
        R cot[3];
        wall_cots<R>(kp, wall, cot);
        const bool far = kp.wetting == 1 && (fabs(cot[0]) > (R)1 || fabs(cot[1]) > (R)1 || fabs(cot[2]) > (R)1);
        auto run = [&](auto far_t) {
            constexpr bool FAR = decltype(far_t)::value;
            for (int m = 0; m < NLD; ++m) {
                const int k = tid + m * NTH;
                if (NLD * NTH != FS && k >= FS) continue;
                const int lx = k % FW, ly = k / FW;
                if (lx < HF - 2 || lx >= FW - HF + 2 || (D == 3 && (ly < HF - 2 || ly >= FH - HF + 2))) continue;
                // the LDS read is unconditional (clamped index) and the global
                // one overrides it, so the two are not merged into one flat load
                auto get = [&](int dx, int dy, R &r, R &ph) {
                    const int jx = lx + dx, jy = ly + dy;
                    const int cx = jx < 0 ? 0 : (jx >= FW ? FW - 1 : jx), cy = jy < 0 ? 0 : (jy >= FH ? FH - 1 : jy);
                    r = s_r[sf][cy * FW + cx];
                    ph = s_p[sf][cy * FW + cx];
                    if constexpr (FAR) {
                        if (jx != cx || jy != cy) {
                            unsigned n = bf + (unsigned)wrapl(x0 + jx - HF, nx);
                            if constexpr (D == 3) n += (unsigned)nx * (unsigned)wrapl(y0 + jy - HF, ny);
                            r = rho[n];
                            ph = phi[n];
                        }
                    }
                };
                R gr_, gp_;
                ghost_value<D, R>(kp, cot, get, gr_, gp_);
                s_r[sg][k] = gr_;
                if constexpr (QR) s_q[sg][k] = fsqrt(gr_);
                s_p[sg][k] = gp_;
                if (own & (1u << m)) {
                    rho[bg + ld_idx[m]] = gr_;
                    phi[bg + ld_idx[m]] = gp_;
                }
            }
        };
        if (far)
            run(std::true_type{});
        else
            run(std::false_type{});
    };

    auto compute_T = [&](int q) {
        if (walls && (q < 1 || q > nw - 2)) return;
        const int st = (q + 10) % 3;
        const int sm = (q + 9) % 5, s0 = (q + 10) % 5, sp = (q + 11) % 5;
        for (int k = tid; k < TS; k += NTH) {
            int hx = k % TW, hy = k / TW;
            int fc = (D == 3 ? (hy + HF - 1) * FW : 0) + hx + HF - 1;
            R G[3] = {0, 0, 0}, H[3] = {0, 0, 0}, Lr = 0, Lp = 0;
            R r0 = s_r[s0][fc], p0 = s_p[s0][fc];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (i == Q / 2) continue;
                const int cw = cdir(D, i, WA);
                const int off = cdir(D, i, 0) + (D == 3 ? cdir(D, i, 1) * FW : 0);
                const int sl = cw < 0 ? sm : (cw > 0 ? sp : s0);
                R rn = s_r[sl][fc + off], pn = s_p[sl][fc + off];
                const R w3 = (R)(3.0 * wgt(D, i)), w6 = (R)(6.0 * wgt(D, i));
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    if (cdir(D, i, a) != 0) {
                        G[a] += (R)(cdir(D, i, a)) * w3 * rn;
                        H[a] += (R)(cdir(D, i, a)) * w3 * pn;
                    }
                }
                Lr += w6 * (rn - r0);
                Lp += w6 * (pn - p0);
            }
            R mur, mup, mP[NP];
            thermo<D, R>(th, r0, p0, G, H, Lr, Lp, mur, mup, mP);
#pragma unroll
            for (int c = 0; c < NP; ++c) s_t[st][c][k] = mP[c];
            s_t[st][NP][k] = mup;
        }
    };

    const int tx = tid % TX, ty = tid / TX;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = tid < TX * TY && x < nx && (D == 2 || y < ny);
    const int fcen = (D == 3 ? (ty + HF) * FW : 0) + tx + HF;
    const int tcen = (D == 3 ? (ty + 1) * TW : 0) + tx + 1;
    // in-plane indices of x + (cx, cy) for every in-plane offset (surplus
    // threads take the last node of the row, so their addresses stay valid)
    unsigned nb[NIP];
#pragma unroll
    for (int k = 0; k < NIP; ++k) {
        const int cx = (D == 3 ? k / 3 : k) - 1, cy = D == 3 ? k % 3 - 1 : 0;
        unsigned v = (unsigned)wrap1(min(x, nx - 1) + cx, nx);
        if constexpr (D == 3) v += (unsigned)nx * (unsigned)wrap1(min(y, ny - 1) + cy, ny);
        nb[k] = v;
    }

    // This plane's f loads are issued before the field stage, so that their
    // latency overlaps the stencil work; the g loads too where registers
    // allow (2D), else (3D) after the f collision but before the f stores:
    // loads and stores retire in order, so a load issued behind the stores
    // would wait for them.  Every thread loads (inactive ones a valid node).
    constexpr bool PG = D == 2;
    S fr[Q], gr[PG ? Q : 1];
    // population stores: non-temporal in the small 2D class (measured 2 %
    // faster per step on a 2048 x 64 channel; on larger grids the next
    // step's moments kernel then read them more slowly)
    auto put = [&](S *dst, S v) {
        if constexpr (D == 2 && NTH <= 64)
            __builtin_nontemporal_store(v, dst);
        else
            *dst = v;
    };
    auto load_pops = [&](int p) {
        if constexpr (!SPLIT) {
            const unsigned n = (unsigned)p * PS + nb[NIP / 2];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                fr[i] = fin[(size_t)i * QS + n];
                if constexpr (PG) gr[i] = gin[(size_t)i * QS + n];
            }
        }
    };

    // prologue: fields pb-2 .. pb+2 (the five planes' loads in flight
    // together), -P planes pb-1 .. pb.  (Issuing the first plane's
    // populations here as well measured slower on a 2048 x 64 channel:
    // 38 loads per thread in flight at the kernel's start.)
    {
        R pr[4][NLD], pp[4][NLD];
#pragma unroll
        for (int j = 0; j < 4; ++j) fetch_into(pb - 2 + j, pr[j], pp[j]);
        fetch(pb + 2);
#pragma unroll
        for (int j = 0; j < 4; ++j) commit_from(pb - 2 + j, pr[j], pp[j]);
    }
    __syncthreads();
    if (GK && walls && (pb - 2 <= 0 || pb + 1 >= nw - 1)) {
        for (int q = pb - 2; q <= pb + 1; ++q)
            if (q == 0 || q == nw - 1) ghost_plane(q);
        __syncthreads();
    }
    compute_T(pb - 1);
    compute_T(pb);
    // in-plane index of population i's target
    auto nbi = [&](int i) -> unsigned {
        return D == 3 ? nb[(cdir(D, i, 0) + 1) * 3 + cdir(D, i, 1) + 1] : nb[cdir(D, i, 0) + 1];
    };
    // alpha kinds of the wave's nodes and its nodes with |u + du| >= 1,
    // counted per plane with ballots
    unsigned long long wave_cnt[4] = {0, 0, 0, 0};
    auto wc = [&](int k) { return k == 0 ? wave_cnt[0] : (k == 1 ? wave_cnt[1] : (k == 2 ? wave_cnt[2] : wave_cnt[3])); };
    // small 2D class: the block's own running counts (every lane loads, so
    // the load is not under a branch), stored back at the end
    constexpr bool OWNSLOT = D == 2 && NTH <= 64 && !SPLIT;
    unsigned long long *const bslot = OWNSLOT ? cnt + (size_t)(kCntSlots + by * ntx + bx) * kCntStride : nullptr;
    unsigned long long run_cnt = 0;
    if constexpr (OWNSLOT) run_cnt = bslot[tid < 4 ? tid : 3];

    if (ONE) pe = pb + 1;
    for (int p = pb; p < pe; ++p) {
        // the far ghost layer from plane p + 1, before this plane's loads
        if (GK && walls && p + 2 == nw - 1) ghost_plane(p + 2);
        const unsigned n = (unsigned)p * PS + nb[NIP / 2];
        load_pops(p);
        commit(p + 2);
        if (!ONE && p + 1 < pe) fetch(p + 3);
        __syncthreads();
        compute_T(p + 1);
        __syncthreads();
        int kind_p = -1;
        bool fast_p = false;
        if (active) {
            const int sm = (p + 9) % 5, s0 = (p + 10) % 5, sp = (p + 11) % 5;
            const int tm = (p + 9) % 3, t0 = (p + 10) % 3, tp = (p + 11) % 3;
            const R r0 = s_r[s0][fcen], p0 = s_p[s0][fcen], q0 = QR ? s_q[s0][fcen] : (R)0;
            const bool first = walls && (p == 1 || p == nw - 2);
            R F[3] = {0, 0, 0};
            if (first) {
                // wall rule (Sec. IV): the pressure tensor, not defined on
                // the solid nodes, loses its wall-normal derivatives and takes
                // in-layer central differences; the ideal part needs only rho,
                // which the ghost layer holds, and keeps its wall-normal link
#pragma unroll
                for (int b = 0; b < D - 1; ++b) {
                    const int ot = b == 0 ? 1 : TW, of = b == 0 ? 1 : FW;
#pragma unroll
                    for (int a = 0; a < D; ++a)
                        F[a] += (R)0.5 * (s_t[t0][sym(D, a, b)][tcen + ot] - s_t[t0][sym(D, a, b)][tcen - ot]);
                    if constexpr (QR)
                        F[b] += link_q(q0, s_q[s0][fcen + of]) - link_q(q0, s_q[s0][fcen - of]);
                    else
                        F[b] += link_p(r0, s_r[s0][fcen + of]) - link_p(r0, s_r[s0][fcen - of]);
                }
                if constexpr (QR)
                    F[WA] += link_q(q0, s_q[sp][fcen]) - link_q(q0, s_q[sm][fcen]);
                else
                    F[WA] += link_p(r0, s_r[sp][fcen]) - link_p(r0, s_r[sm][fcen]);
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (i == Q / 2) continue;
                    const int cw = cdir(D, i, WA);
                    const int offt = cdir(D, i, 0) + (D == 3 ? cdir(D, i, 1) * TW : 0);
                    const int offf = cdir(D, i, 0) + (D == 3 ? cdir(D, i, 1) * FW : 0);
                    const int slt = cw < 0 ? tm : (cw > 0 ? tp : t0);
                    const int slf = cw < 0 ? sm : (cw > 0 ? sp : s0);
                    const R w3 = (R)(3.0 * wgt(D, i)), w6 = (R)(6.0 * wgt(D, i));
                    const R pl = QR ? link_q(q0, s_q[slf][fcen + offf]) : link_p(r0, s_r[slf][fcen + offf]);
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        R acc = 0;
#pragma unroll
                        for (int b = 0; b < D; ++b)
                            if (cdir(D, i, b) != 0) acc += (R)cdir(D, i, b) * s_t[slt][sym(D, a, b)][tcen + offt];
                        F[a] += w3 * acc;
                        if (cdir(D, i, a) != 0) F[a] += w6 * (R)cdir(D, i, a) * pl;
                    }
                }
            }
            if (walls && kp.wetting == 0) {
                R rrel = (r0 - (R)kp.rho_g) * th.inv_drho, prel = p0 * th.inv_chi;
                if (p == 2) F[WA] -= (R)(1.0 / 6.0) * rrel * ((R)kp.kw[0][0] + prel * (R)kp.kw[0][1]);
                if (p == nw - 3) F[WA] += (R)(1.0 / 6.0) * rrel * ((R)kp.kw[1][0] + prel * (R)kp.kw[1][1]);
            }
            if constexpr (SPLIT) {
#pragma unroll
                for (int a = 0; a < D; ++a) fmu[(size_t)a * QS + n] = F[a];
                fmu[(size_t)D * QS + n] = s_t[t0][NP][tcen];
            } else {
                R rp = (R)0, pp = (R)0;
                if constexpr (PREC == P16) { rp = rprev[n]; pp = pprev[n]; }
                R f[Q];
                R j[3] = {0, 0, 0};
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    f[i] = dec_f<PREC, D>(fr[i], i, rp);
#pragma unroll
                    for (int a = 0; a < D; ++a)
                        if (cdir(D, i, a) != 0) j[a] += (R)cdir(D, i, a) * f[i];
                }
                R u[3], du[3], v[3];
                const R ir = fdiv((R)1, r0);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    u[a] = j[a] * ir;
                    du[a] = F[a] * ir;
                    v[a] = u[a] + (R)0.5 * du[a];
                }
                fast_p = collide && too_fast<D, R>(u, du);
                if (collide) kind_p = collide_f<D, R>(f, r0, u, du, beta, aeps, atol, kp.alpha_maxit, alpha2);
                // g populations (Eqs. 33-35 below), loaded ahead of the f stores
                R gg[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const S *gi = gin + (size_t)i * QS;
                    gg[i] = dec_g<PREC, D>(PG ? gr[PG ? i : 0] : gi[n], i, pp);
                }
                // stream f: push to x + c_i, halfway bounce-back at the walls
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int cw = cdir(D, i, WA);
                    const int pt = p + cw;
                    if (walls && (pt < 1 || pt > nw - 2)) {
                        S *fo = fout + (size_t)(Q - 1 - i) * QS;
                        put(&fo[n], enc_f<PREC, D>(f[i], Q - 1 - i, r0));
                    } else {
                        const int offf = cdir(D, i, 0) + (D == 3 ? cdir(D, i, 1) * FW : 0);
                        const int slf = cw < 0 ? sm : (cw > 0 ? sp : s0);
                        const unsigned nt = (unsigned)plane(pt) * PS + nbi(i);
                        S *fo = fout + (size_t)i * QS;
                        put(&fo[nt], enc_f<PREC, D>(f[i], i, s_r[slf][fcen + offf]));
                    }
                }
                // g: LBGK toward g^eq(phi, v) (Eqs. 33-35)
                if (collide) collide_g<D, R>(gg, v, p0, s_t[t0][NP][tcen], Gam, itg);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int cw = cdir(D, i, WA);
                    const int pt = p + cw;
                    if (walls && (pt < 1 || pt > nw - 2)) {
                        S *go = gout + (size_t)(Q - 1 - i) * QS;
                        put(&go[n], enc_g<PREC, D>(gg[i], Q - 1 - i, p0));
                    } else {
                        const int offf = cdir(D, i, 0) + (D == 3 ? cdir(D, i, 1) * FW : 0);
                        const int slf = cw < 0 ? sm : (cw > 0 ? sp : s0);
                        const unsigned nt = (unsigned)plane(pt) * PS + nbi(i);
                        S *go = gout + (size_t)i * QS;
                        put(&go[nt], enc_g<PREC, D>(gg[i], i, s_p[slf][fcen + offf]));
                    }
                }
            }
        }
        if constexpr (!SPLIT) {
            wave_cnt[0] += __popcll(__ballot(kind_p == 1));
            wave_cnt[1] += __popcll(__ballot(kind_p == 0));
            wave_cnt[2] += __popcll(__ballot(kind_p == 2));
            wave_cnt[3] += __popcll(__ballot(fast_p));
        }
        __syncthreads();
    }
    if constexpr (SPLIT) return;
    // alpha statistics: one add per wave and kind (a one-wave block adds to
    // its counter slot directly; the small 2D class stores its own slot)
    unsigned long long *slot = cnt + (size_t)((bx + by * 7) & (kCntSlots - 1)) * kCntStride;
    if constexpr (OWNSLOT) {
        if (tid < 4) bslot[tid] = run_cnt + wc(tid);
    } else if constexpr (NTH <= 64) {
        if (tid < 4 && wc(tid)) atomicAdd(&slot[tid], wc(tid));
    } else {
        if ((tid & 63) == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (wave_cnt[k]) atomicAdd(&s_cnt[k], (int)wave_cnt[k]);
        __syncthreads();
        if (tid < 4 && s_cnt[tid]) atomicAdd(&slot[tid], (unsigned long long)s_cnt[tid]);
    }
}

#define LBM3_FUSED_ATTR                                                                                     \
    __launch_bounds__(NTH)                                                                                  \
    __attribute__((amdgpu_waves_per_eu(D == 3 ? (PREC == P64 ? 1 : 2) : (PREC == P64 ? 2 : (NTH <= 64 ? 3 : 4)))))

template <int D, int PREC, int TX, int TY, int NTH, bool ONE = false>
__global__ void LBM3_FUSED_ATTR
k_fused(KParams kp, const typename Ty<PREC>::S *__restrict__ fin, const typename Ty<PREC>::S *__restrict__ gin,
        typename Ty<PREC>::S *__restrict__ fout, typename Ty<PREC>::S *__restrict__ gout,
        typename Ty<PREC>::R *__restrict__ rho, typename Ty<PREC>::R *__restrict__ phi,
        const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
        unsigned long long *__restrict__ cnt, int chunk)
{
    fused_tile<D, PREC, TX, TY, NTH, false, ONE>(kp, fin, gin, fout, gout, rho, phi, rprev, pprev, cnt, chunk,
                                                 blockIdx.x, blockIdx.y);
}

template <int D, int PREC, int TX, int TY, int NTH>
__global__ void LBM3_FUSED_ATTR
k_fused_batch(const SimDesc *__restrict__ d, const int *__restrict__ sim, int phase)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    const SimDesc &sd = d[sim[blockIdx.x]];
    const KParams &kp = sd.kp;
    const int pc = sd.pc ^ phase, fc = sd.fc ^ phase;
    const int local = blockIdx.x - sd.fblk0;
    fused_tile<D, PREC, TX, TY, NTH>(kp, on_global<const S>(d, sd.f[pc]), on_global<const S>(d, sd.g[pc]),
                                     on_global<S>(d, sd.f[1 - pc]), on_global<S>(d, sd.g[1 - pc]),
                                     on_global<R>(d, sd.rho[1 - fc]), on_global<R>(d, sd.phi[1 - fc]),
                                     on_global<const R>(d, sd.rho[fc]), on_global<const R>(d, sd.phi[fc]),
                                     on_global<unsigned long long>(d, sd.counters), sd.chunk, local % sd.ntiles,
                                     local / sd.ntiles);
}

// ------------------------------------------------------ 3D stencil pass --
// The 1D factors of the isotropic D3Q27 stencils: with w_i the product of
// w1(c) = 2/3, 1/6, 1/6 over the axes, sum_i w_i q(x + c_i) = S_x S_y S_z q,
// grad_x q = 3 sum_i w_i c_ix q(x + c_i) = D_x S_y S_z q (and cyclic), and
// lap q = 6 (S_x S_y S_z q - q), with S = (1/6, 2/3, 1/6) and D = (-1/2, 0,
// 1/2).  The divergence of -P uses the same gradient stencil on each column.
template <typename R> __device__ __forceinline__ R sm3(R m, R c, R p)
{
    return (R)(2.0 / 3.0) * c + (R)(1.0 / 6.0) * (m + p);
}
template <typename R> __device__ __forceinline__ R df3(R m, R p) { return (R)0.5 * (p - m); }

// Stencil pass of the two-kernel 3D step (Sec. II A-C, Sec. IV): per block an
// in-plane TX x TY tile marching along the wall axis over the planes of its
// chunk.  Each plane q: the z factors of the rho, phi stencils from three
// planes of fields held in registers (tile + halo 2), then the y and the x
// factors through LDS, giving grad, lap of rho and phi on tile + halo 1, mu
// and -P there (Eqs. 11-20), kept in registers for three planes; then the
// force on the tile for the plane below: the z factors of div(-P) in
// registers, y and x through LDS, plus the ideal part as the lattice
// divergence of the link pressure of sqrt(rho), and the first-fluid-layer
// wall rule and force-method wall force of Sec. IV.  Writes F and mu_phi
// ([D + 1][QS]).
template <int PREC, int TX, int TY>
__device__ __forceinline__ void force_march3(const KParams &kp, const typename Ty<PREC>::R *__restrict__ rho,
                                             const typename Ty<PREC>::R *__restrict__ phi,
                                             typename Ty<PREC>::R *__restrict__ fmu, int chunk, int bx, int by)
{
    using R = typename Ty<PREC>::R;
    constexpr int NT = TX * TY;
    constexpr int W2 = TX + 4, H2 = TY + 4, E2 = W2 * H2;  // tile + halo 2
    constexpr int W1 = TX + 2, H1 = TY + 2, E1 = W1 * H1;  // tile + halo 1
    constexpr int EY = W2 * (TY + 2);                      // y pass of the fields
    constexpr int ED = W1 * TY;                            // y pass of the divergence
    constexpr int FE = (E2 + NT - 1) / NT, TE = (E1 + NT - 1) / NT, YE = (EY + NT - 1) / NT, DE = (ED + NT - 1) / NT;
    // The field stage (s_z, s_c, s_y) and the force stage (s_w, s_mu, s_d)
    // of a plane share one LDS area, a barrier apart: 24 KB per block in
    // FP32 instead of 43, so that the registers (128), not the LDS, bound
    // the blocks per CU (four instead of three; 12 % faster on 256^3).
    constexpr int EA = 6 * E2 + 6 * EY, EB = 9 * E1 + 6 * ED;
    __shared__ R s_u[EA > EB ? EA : EB];
    __shared__ R s_q[3][E2];        // 1/sqrt(rho) of three planes (ring)
    R (*const s_z)[E2] = (R (*)[E2])s_u;               // S_z rho, D_z rho, S_z phi, D_z phi
    R (*const s_c)[E2] = (R (*)[E2])(s_u + 4 * E2);    // rho, phi of the plane
    R (*const s_y)[EY] = (R (*)[EY])(s_u + 6 * E2);    // S_y S_z rho, D_y S_z rho, S_y D_z rho, same for phi
    R (*const s_w)[E1] = (R (*)[E1])s_u;               // S_z of -P xx xy xz yy yz, D_z of -P xz yz zz
                                                       // (first layer: -P xx..yz)
    R *const s_mu = s_u + 8 * E1;                      // mu_phi of the output plane
    R (*const s_d)[ED] = (R (*)[ED])(s_u + 9 * E1);    // S_y S_z (-P x.), D_y S_z (-P y.) + S_y D_z (-P z.)

    const int tid = threadIdx.x;
    const int nx = kp.nx, ny = kp.ny, nw = kp.nw;
    const unsigned N = (unsigned)kp.N, PS = (unsigned)kp.PS;
    const unsigned QS = (unsigned)kp.QS;
    const bool walls = kp.walls != 0;
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (bx % ntx) * TX, y0 = (bx / ntx) * TY;
    int pb, pe;
    chunk_range(kp, 0, chunk, by, pb, pe);
    if (pb >= pe) return;
    Thermo<R> th;
    th.load(kp);

    // in-plane indices of this thread's field elements (tile + halo 2)
    unsigned fidx[FE];
#pragma unroll
    for (int m = 0; m < FE; ++m) {
        int k = tid + m * NT;
        k = k < E2 ? k : E2 - 1;
        fidx[m] = (unsigned)wrapl(x0 + k % W2 - 2, nx) + (unsigned)nx * (unsigned)wrapl(y0 + k / W2 - 2, ny);
    }
    auto plane_of = [&](int q) { return walls ? (q < 0 ? 0 : (q > nw - 1 ? nw - 1 : q)) : wrapl(q, nw); };
    auto fluid = [&](int q) { return !walls || (q >= 1 && q <= nw - 2); };

    // fields of three consecutive planes in registers, plus the next plane's
    // loads in flight
    R fr[3][FE], fp[3][FE], nr[FE], np_[FE];
    auto load = [&](int q, R *dr, R *dp) {
        const unsigned base = (unsigned)plane_of(q) * PS;
#pragma unroll
        for (int m = 0; m < FE; ++m) {
            dr[m] = rho[base + fidx[m]];
            dp[m] = phi[base + fidx[m]];
        }
    };
    // -P (xx xy xz yy yz zz) and mu_phi of the thread's tile + halo 1
    // elements on three planes
    R tp[3][TE][6], tm[3][TE];

    // Field stage of plane q (fields of q - 1, q, q + 1 in fr/fp[0..2]):
    // 1/sqrt(rho) into the ring; on fluid planes grad, lap, mu and -P into
    // tp/tm[2] (after shifting the register ring down).
    auto field_stage = [&](int q) {
        __syncthreads();
        const int sq = wrapl(q, 3);
#pragma unroll
        for (int m = 0; m < FE; ++m) {
            const int k = tid + m * NT;
            if (E2 % NT == 0 || k < E2) {
                s_q[sq][k] = fdiv((R)1, fsqrt(fr[1][m]));
                s_c[0][k] = fr[1][m];
                s_c[1][k] = fp[1][m];
                s_z[0][k] = sm3(fr[0][m], fr[1][m], fr[2][m]);
                s_z[1][k] = df3(fr[0][m], fr[2][m]);
                s_z[2][k] = sm3(fp[0][m], fp[1][m], fp[2][m]);
                s_z[3][k] = df3(fp[0][m], fp[2][m]);
            }
        }
#pragma unroll
        for (int e = 0; e < TE; ++e) {
#pragma unroll
            for (int c = 0; c < 6; ++c) { tp[0][e][c] = tp[1][e][c]; tp[1][e][c] = tp[2][e][c]; }
            tm[0][e] = tm[1][e];
            tm[1][e] = tm[2][e];
        }
        if (!fluid(q)) return;  // uniform: a ghost layer has no -P
        __syncthreads();
#pragma unroll
        for (int m = 0; m < YE; ++m) {
            const int k = tid + m * NT;
            if (EY % NT == 0 || k < EY) {
                const int c = k + W2;  // centre in tile + halo 2 (rows 1 .. TY + 2)
                s_y[0][k] = sm3(s_z[0][c - W2], s_z[0][c], s_z[0][c + W2]);
                s_y[1][k] = df3(s_z[0][c - W2], s_z[0][c + W2]);
                s_y[2][k] = sm3(s_z[1][c - W2], s_z[1][c], s_z[1][c + W2]);
                s_y[3][k] = sm3(s_z[2][c - W2], s_z[2][c], s_z[2][c + W2]);
                s_y[4][k] = df3(s_z[2][c - W2], s_z[2][c + W2]);
                s_y[5][k] = sm3(s_z[3][c - W2], s_z[3][c], s_z[3][c + W2]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < TE; ++e) {
            const int k = tid + e * NT;
            if (E1 % NT != 0 && k >= E1) continue;  // only the first waves hold a halo element
            const int x1 = k % W1, y1 = k / W1;
            const int cy = y1 * W2 + x1 + 1;  // in the y-pass arrays (row y1 = halo-2 row y1 + 1)
            const int c2 = (y1 + 1) * W2 + x1 + 1;
            const R r0 = s_c[0][c2], p0 = s_c[1][c2];
            R G[3], H[3];
            G[0] = df3(s_y[0][cy - 1], s_y[0][cy + 1]);
            G[1] = sm3(s_y[1][cy - 1], s_y[1][cy], s_y[1][cy + 1]);
            G[2] = sm3(s_y[2][cy - 1], s_y[2][cy], s_y[2][cy + 1]);
            const R sr = sm3(s_y[0][cy - 1], s_y[0][cy], s_y[0][cy + 1]);
            H[0] = df3(s_y[3][cy - 1], s_y[3][cy + 1]);
            H[1] = sm3(s_y[4][cy - 1], s_y[4][cy], s_y[4][cy + 1]);
            H[2] = sm3(s_y[5][cy - 1], s_y[5][cy], s_y[5][cy + 1]);
            const R sp = sm3(s_y[3][cy - 1], s_y[3][cy], s_y[3][cy + 1]);
            const R Lr = (R)6 * (sr - r0), Lp = (R)6 * (sp - p0);
            R mur, mup, mP[6];
            thermo<3, R>(th, r0, p0, G, H, Lr, Lp, mur, mup, mP);
#pragma unroll
            for (int c = 0; c < 6; ++c) tp[2][e][c] = mP[c];
            tm[2][e] = mup;
        }
    };

    // prologue: fields of pb - 2 .. pb + 1, the field stages of pb - 1, pb,
    // and the loads of pb + 2 in flight
    load(pb - 2, fr[0], fp[0]);
    load(pb - 1, fr[1], fp[1]);
    load(pb, fr[2], fp[2]);
    load(pb + 1, nr, np_);
    field_stage(pb - 1);
#pragma unroll
    for (int m = 0; m < FE; ++m) {
        fr[0][m] = fr[1][m]; fr[1][m] = fr[2][m]; fr[2][m] = nr[m];
        fp[0][m] = fp[1][m]; fp[1][m] = fp[2][m]; fp[2][m] = np_[m];
    }
    load(pb + 2, nr, np_);
    field_stage(pb);

    const int tx = tid % TX, ty = tid / TX;
    const bool active = x0 + tx < nx && y0 + ty < ny;
    const unsigned own = (unsigned)(x0 + tx < nx ? x0 + tx : nx - 1) + (unsigned)nx * (unsigned)(y0 + ty < ny ? y0 + ty : ny - 1);
    const int oq = (ty + 2) * W2 + tx + 2;  // own node in tile + halo 2
    const int o1 = (ty + 1) * W1 + tx + 1;  // own node in tile + halo 1

    for (int p = pb; p < pe; ++p) {
        // fields of p, p + 1, p + 2 and the loads of p + 3 in flight
#pragma unroll
        for (int m = 0; m < FE; ++m) {
            fr[0][m] = fr[1][m]; fr[1][m] = fr[2][m]; fr[2][m] = nr[m];
            fp[0][m] = fp[1][m]; fp[1][m] = fp[2][m]; fp[2][m] = np_[m];
        }
        if (p + 1 < pe) load(p + 3, nr, np_);
        field_stage(p + 1);
        __syncthreads();  // the field stage's LDS becomes the force stage's
        // -P of p - 1, p, p + 1 in tp[0..2]: z factors of the divergence
        const bool first = walls && (p == 1 || p == nw - 2);
#pragma unroll
        for (int e = 0; e < TE; ++e) {
            const int k = tid + e * NT;
            if (E1 % NT == 0 || k < E1) {
                if (first) {
                    // wall rule: in-layer central differences of -P only
#pragma unroll
                    for (int c = 0; c < 5; ++c) s_w[c][k] = tp[1][e][c];
                } else {
                    s_w[0][k] = sm3(tp[0][e][0], tp[1][e][0], tp[2][e][0]);  // xx
                    s_w[1][k] = sm3(tp[0][e][1], tp[1][e][1], tp[2][e][1]);  // xy
                    s_w[2][k] = sm3(tp[0][e][2], tp[1][e][2], tp[2][e][2]);  // xz
                    s_w[3][k] = sm3(tp[0][e][3], tp[1][e][3], tp[2][e][3]);  // yy
                    s_w[4][k] = sm3(tp[0][e][4], tp[1][e][4], tp[2][e][4]);  // yz
                    s_w[5][k] = df3(tp[0][e][2], tp[2][e][2]);               // xz
                    s_w[6][k] = df3(tp[0][e][4], tp[2][e][4]);               // yz
                    s_w[7][k] = df3(tp[0][e][5], tp[2][e][5]);               // zz
                }
                s_mu[k] = tm[1][e];
            }
        }
        __syncthreads();
        if (!first) {
#pragma unroll
            for (int m = 0; m < DE; ++m) {
                const int k = tid + m * NT;
                if (ED % NT == 0 || k < ED) {
                    const int c = k + W1;
                    s_d[0][k] = sm3(s_w[0][c - W1], s_w[0][c], s_w[0][c + W1]);  // S_y S_z xx
                    s_d[1][k] = sm3(s_w[1][c - W1], s_w[1][c], s_w[1][c + W1]);  // S_y S_z xy
                    s_d[2][k] = sm3(s_w[2][c - W1], s_w[2][c], s_w[2][c + W1]);  // S_y S_z xz
                    s_d[3][k] = df3(s_w[1][c - W1], s_w[1][c + W1]) + sm3(s_w[5][c - W1], s_w[5][c], s_w[5][c + W1]);
                    s_d[4][k] = df3(s_w[3][c - W1], s_w[3][c + W1]) + sm3(s_w[6][c - W1], s_w[6][c], s_w[6][c + W1]);
                    s_d[5][k] = df3(s_w[4][c - W1], s_w[4][c + W1]) + sm3(s_w[7][c - W1], s_w[7][c], s_w[7][c + W1]);
                }
            }
            __syncthreads();
        }
        if (active) {
            R F[3];
            const int sm = wrapl(p - 1, 3), s0 = wrapl(p, 3), sp = wrapl(p + 1, 3);
            // link pressure 2 rho_x rho_y / (rho_x + rho_y + 4 sqrt(rho_x rho_y))
            // = 2 / (i_x^2 + i_y^2 + 4 i_x i_y), i = 1/sqrt(rho)
            const R i0 = s_q[s0][oq], a0 = i0 * i0, c0 = (R)4 * i0;
            auto hlink = [&](R i1) { return fdiv((R)1, i1 * (i1 + c0) + a0); };  // half the link pressure
            if (first) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    // -P_ax at x +- 1 and -P_ay at y +- 1 (sym order xx xy xz yy yz)
                    const int cx = a, cy = a == 0 ? 1 : (a == 1 ? 3 : 4);
                    F[a] = (R)0.5 * (s_w[cx][o1 + 1] - s_w[cx][o1 - 1]) + (R)0.5 * (s_w[cy][o1 + W1] - s_w[cy][o1 - W1]);
                }
                F[0] += (R)2 * (hlink(s_q[s0][oq + 1]) - hlink(s_q[s0][oq - 1]));
                F[1] += (R)2 * (hlink(s_q[s0][oq + W2]) - hlink(s_q[s0][oq - W2]));
                F[2] += (R)2 * (hlink(s_q[sp][oq]) - hlink(s_q[sm][oq]));
            } else {
                const int od = ty * W1 + tx + 1;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    F[a] = df3(s_d[a][od - 1], s_d[a][od + 1]) + sm3(s_d[3 + a][od - 1], s_d[3 + a][od], s_d[3 + a][od + 1]);
#pragma unroll
                for (int i = 0; i < 27; ++i) {
                    if (i == 13) continue;
                    const int cx = cdir(3, i, 0), cy = cdir(3, i, 1), cz = cdir(3, i, 2);
                    const int sl = cz < 0 ? sm : (cz > 0 ? sp : s0);
                    const R hl = hlink(s_q[sl][oq + cx + cy * W2]);
                    const R w12 = (R)(12.0 * wgt(3, i));
                    if (cx) F[0] += (R)cx * w12 * hl;
                    if (cy) F[1] += (R)cy * w12 * hl;
                    if (cz) F[2] += (R)cz * w12 * hl;
                }
            }
            if (walls && kp.wetting == 0 && (p == 2 || p == nw - 3)) {
                const unsigned n = (unsigned)p * PS + own;
                const R r0 = rho[n], p0 = phi[n];
                const R rrel = (r0 - (R)kp.rho_g) * th.inv_drho, prel = p0 * th.inv_chi;
                if (p == 2) F[2] -= (R)(1.0 / 6.0) * rrel * ((R)kp.kw[0][0] + prel * (R)kp.kw[0][1]);
                if (p == nw - 3) F[2] += (R)(1.0 / 6.0) * rrel * ((R)kp.kw[1][0] + prel * (R)kp.kw[1][1]);
            }
            const unsigned n = (unsigned)p * PS + own;
#pragma unroll
            for (int a = 0; a < 3; ++a) fmu[(size_t)a * QS + n] = F[a];
            fmu[(size_t)3 * QS + n] = s_mu[o1];
        }
    }
}

#define LBM3_STENCIL_ATTR __launch_bounds__(TX * TY)

template <int PREC, int TX, int TY>
__global__ void LBM3_STENCIL_ATTR
k_stencil(KParams kp, typename Ty<PREC>::R *__restrict__ rho, typename Ty<PREC>::R *__restrict__ phi,
          typename Ty<PREC>::R *__restrict__ fmu, int chunk)
{
    force_march3<PREC, TX, TY>(kp, rho, phi, fmu, chunk, blockIdx.x, blockIdx.y);
}

template <int PREC, int TX, int TY>
__global__ void LBM3_STENCIL_ATTR
k_stencil_batch(const SimDesc *__restrict__ d, const int *__restrict__ sim, int phase)
{
    using R = typename Ty<PREC>::R;
    const SimDesc &sd = d[sim[blockIdx.x]];
    const KParams &kp = sd.kp;
    const int fc = sd.fc ^ phase;
    const int local = blockIdx.x - sd.fblk0;
    force_march3<PREC, TX, TY>(kp, on_global<R>(d, sd.rho[1 - fc]), on_global<R>(d, sd.phi[1 - fc]),
                               on_global<R>(d, sd.fmu), sd.chunk, local % sd.ntiles, local / sd.ntiles);
}

// Collision and push streaming of fluid node number t (counted from the
// first fluid plane), the second kernel of the two-kernel step: F and mu_phi
// from the stencil pass, rho, phi of the node and of its push targets (for
// the FP16 offsets) from the moments pass.  The same arithmetic as the
// fused kernel, one node per thread with no LDS and no barriers, so the
// waves of a CU overlap their loads and their collisions freely.  Returns
// the alpha kind (-1: none).
//
// UNI: every wave lies in one plane of the wall axis (the plane stride is a
// multiple of 64), so the plane index is taken as wave-uniform and the
// bounce-back choice of each population is a scalar branch.  GL: whether
// the stored g is loaded (0 never: tau_g = 1 with collisions, where
// g* = g^eq; 1 always; 2 decided at run time by the same rule, for the
// batched kernel; 3 never, and g is not stored either: tau_g = 1 with
// collisions, where the post-collision g is g^eq of (a, phi, v) and the node
// stores those five values for the next moments pass).  Target addresses
// are the sum of an x, a y and a plane byte offset, shared by the f and g
// stores.
template <int D, int PREC, bool UNI, int GL>
__device__ __forceinline__ int collide_node(const KParams &kp, const typename Ty<PREC>::S *__restrict__ fin,
                                            const typename Ty<PREC>::S *__restrict__ gin,
                                            typename Ty<PREC>::S *__restrict__ fout,
                                            typename Ty<PREC>::S *__restrict__ gout,
                                            const typename Ty<PREC>::R *__restrict__ rho,
                                            const typename Ty<PREC>::R *__restrict__ phi,
                                            const typename Ty<PREC>::R *__restrict__ rprev,
                                            const typename Ty<PREC>::R *__restrict__ pprev,
                                            const typename Ty<PREC>::R *__restrict__ fmu, long long t, bool &fast)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    constexpr int Q = D == 2 ? 9 : 27;
    constexpr int WA = D - 1;
    constexpr unsigned SS = sizeof(S), SR = sizeof(R);
    const bool walls = kp.walls != 0;
    const unsigned N = (unsigned)kp.N, PS = (unsigned)kp.PS;
    const unsigned QS = (unsigned)kp.QS;
    const int nx = kp.nx, ny = kp.ny, nw = kp.nw;
    const unsigned n = (unsigned)((walls ? kp.PS : 0) + t);
    const bool collide = !(kp.flags & 1u), alpha2 = (kp.flags & 2u) != 0;
    const R itg = (R)kp.inv_tau_g;
    const bool need_g = GL == 1 || (GL == 2 && (!collide || itg != (R)1));
    static_assert(GL != 3 || D == 3, "implicit g is a 3D two-kernel path");

    S fr[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fr[i] = ld32<S>(arr(fin + (size_t)i * QS, N), n * SS);
    const R r0 = ld32<R>(arr(rho, N), n * SR), p0 = ld32<R>(arr(phi, N), n * SR);
    R F[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = ld32<R>(arr(fmu + (size_t)a * QS, N), n * SR);
    const R mup = ld32<R>(arr(fmu + (size_t)D * QS, N), n * SR);
    R rp = (R)0, pp = (R)0;
    if constexpr (PREC == P16) { rp = ld32<R>(arr(rprev, N), n * SR); pp = ld32<R>(arr(pprev, N), n * SR); }

    // the node's coordinates; byte offsets (storage type) of x - 1, x, x + 1,
    // of the rows y - 1, y, y + 1 and of the planes p - 1, p, p + 1
    const int x = (int)(n % (unsigned)nx);
    const unsigned rest = n / (unsigned)nx;
    const int y = D == 3 ? (int)(rest % (unsigned)ny) : 0;
    int p = D == 3 ? (int)(rest / (unsigned)ny) : (int)rest;
    if constexpr (UNI) p = __builtin_amdgcn_readfirstlane(p);
    const unsigned xo[3] = {(unsigned)(x == 0 ? nx - 1 : x - 1) * SS, (unsigned)x * SS,
                            (unsigned)(x == nx - 1 ? 0 : x + 1) * SS};
    unsigned yo[3] = {0, 0, 0};
    if constexpr (D == 3) {
        yo[0] = (unsigned)(y == 0 ? ny - 1 : y - 1) * (unsigned)nx * SS;
        yo[1] = (unsigned)y * (unsigned)nx * SS;
        yo[2] = (unsigned)(y == ny - 1 ? 0 : y + 1) * (unsigned)nx * SS;
    }
    const int pm = walls ? p - 1 : (p == 0 ? nw - 1 : p - 1), pq = walls ? p + 1 : (p == nw - 1 ? 0 : p + 1);
    const unsigned zo[3] = {(unsigned)pm * PS * SS, (unsigned)p * PS * SS, (unsigned)pq * PS * SS};
    // halfway bounce-back: the populations leaving toward a wall layer
    const bool low = walls && p == 1, high = walls && p == nw - 2;
    auto target = [&](int i) -> unsigned {
        return xo[cdir(D, i, 0) + 1] + yo[D == 3 ? cdir(D, i, 1) + 1 : 1] + zo[cdir(D, i, WA) + 1];
    };
    auto bounces = [&](int i) { return (cdir(D, i, WA) < 0 && low) || (cdir(D, i, WA) > 0 && high); };

    const R beta = (R)kp.beta, Gam = (R)kp.Gamma;
    R f[Q];
    R j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = dec_f<PREC, D>(fr[i], i, rp);
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (cdir(D, i, a) != 0) j[a] += (R)cdir(D, i, a) * f[i];
    }
    R u[3], du[3], v[3];
    const R ir = fdiv((R)1, r0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = j[a] * ir;
        du[a] = F[a] * ir;
        v[a] = u[a] + (R)0.5 * du[a];
    }
    int kind = -1;
    fast = collide && too_fast<D, R>(u, du);
    if (collide) kind = collide_f<D, R>(f, r0, u, du, beta, (R)kp.alpha_eps, (R)kp.alpha_tol, kp.alpha_maxit, alpha2);
    // g loads ahead of the f stores (loads and stores retire in order)
    R gg[Q];
    if constexpr (GL != 0) {
        if (need_g) {
#pragma unroll
            for (int i = 0; i < Q; ++i) gg[i] = dec_g<PREC, D>(ld32<S>(arr(gin + (size_t)i * QS, N), n * SS), i, pp);
        }
    }
    // push streaming with halfway bounce-back at the walls
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (bounces(i)) {
            st32<S>(arr(fout + (size_t)(Q - 1 - i) * QS, N), n * SS, enc_f<PREC, D>(f[i], Q - 1 - i, r0));
        } else {
            const unsigned nt = target(i);
            const R rt = PREC == P16 ? ld32<R>(arr(rho, N), nt / SS * SR) : r0;
            st32<S>(arr(fout + (size_t)i * QS, N), nt, enc_f<PREC, D>(f[i], i, rt));
        }
    }
    if constexpr (GL == 3) {
        // g* = g^eq is a function of (a, phi, v): store those five values at
        // the node instead of pushing 27 populations
        R *gp = (R *)gout;
        const R vals[5] = {geq_a<D, R>(v, p0, mup, Gam), p0, v[0], v[1], v[2]};
#pragma unroll
        for (int k = 0; k < 5; ++k) st32<R>(arr(gp + (size_t)k * QS, N), n * SR, vals[k]);
        return kind;
    }
    if (!need_g) {
        collide_g<D, R, true>(gg, v, p0, mup, Gam, itg);
    } else if constexpr (GL != 0) {
        if (collide) collide_g<D, R>(gg, v, p0, mup, Gam, itg);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (bounces(i)) {
            st32<S>(arr(gout + (size_t)(Q - 1 - i) * QS, N), n * SS, enc_g<PREC, D>(gg[i], Q - 1 - i, p0));
        } else {
            const unsigned nt = target(i);
            const R pt = (PREC == P16 && i == Q / 2) ? ld32<R>(arr(phi, N), nt / SS * SR) : p0;
            st32<S>(arr(gout + (size_t)i * QS, N), nt, enc_g<PREC, D>(gg[i], i, pt));
        }
    }
    return kind;
}

// alpha statistics of a block and its nodes with |u + du| >= 1: per wave
// counted with a ballot, summed in LDS
__device__ __forceinline__ void count_kinds(int kind, bool fast, int *s_cnt)
{
    const unsigned long long nw_ = __ballot(kind == 1), ns_ = __ballot(kind == 0), nf_ = __ballot(kind == 2);
    const unsigned long long nq_ = __ballot(fast);
    if ((threadIdx.x & 63) == 0) {
        if (nw_) atomicAdd(&s_cnt[0], __popcll(nw_));
        if (ns_) atomicAdd(&s_cnt[1], __popcll(ns_));
        if (nf_) atomicAdd(&s_cnt[2], __popcll(nf_));
        if (nq_) atomicAdd(&s_cnt[3], __popcll(nq_));
    }
}

// three waves per SIMD (168 registers) measured 19 % faster than two on a
// 256^3 grid; four spill
#define LBM3_COLLIDE_ATTR __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == P64 ? 1 : 3)))

template <int D, int PREC, bool UNI, int GL>
__global__ void LBM3_COLLIDE_ATTR
k_collide(KParams kp, const typename Ty<PREC>::S *__restrict__ fin, const typename Ty<PREC>::S *__restrict__ gin,
          typename Ty<PREC>::S *__restrict__ fout, typename Ty<PREC>::S *__restrict__ gout,
          const typename Ty<PREC>::R *__restrict__ rho, const typename Ty<PREC>::R *__restrict__ phi,
          const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
          const typename Ty<PREC>::R *__restrict__ fmu, unsigned long long *__restrict__ cnt)
{
    __shared__ int s_cnt[4];
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int kind = -1;
    bool fast = false;
    if (t < count)
        kind = collide_node<D, PREC, UNI, GL>(kp, fin, gin, fout, gout, rho, phi, rprev, pprev, fmu, t, fast);
    count_kinds(kind, fast, s_cnt);
    __syncthreads();
    if (threadIdx.x < 4 && s_cnt[threadIdx.x])
        atomicAdd(&cnt[(size_t)(blockIdx.x & (kCntSlots - 1)) * kCntStride + threadIdx.x],
                  (unsigned long long)s_cnt[threadIdx.x]);
}

// IMP: every simulation of the launch has implicit g (the batch groups them
// apart), so only that form of the node is compiled in; the kernel holding
// both forms needs registers for both and spills.
template <int D, int PREC, bool IMP>
__global__ void LBM3_COLLIDE_ATTR
k_collide_batch(const SimDesc *__restrict__ d, const int *__restrict__ sim, int phase)
{
    using R = typename Ty<PREC>::R;
    using S = typename Ty<PREC>::S;
    __shared__ int s_cnt[4];
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const SimDesc &sd = d[sim[blockIdx.x]];
    const KParams &kp = sd.kp;
    const int pc = sd.pc ^ phase, fc = sd.fc ^ phase;
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    const long long t = (long long)(blockIdx.x - sd.cblk0) * blockDim.x + threadIdx.x;
    int kind = -1;
    bool fast = false;
    // the same arithmetic either way; a plane stride that is a multiple of
    // the wave makes the bounce-back branches scalar (block-uniform test)
    // implicit g (gp set: tau_g = 1 with collisions): the five values go to gp
    auto node = [&](auto uni, auto gl) {
        S *gout = decltype(gl)::value == 3 ? on_global<S>(d, sd.gp) : on_global<S>(d, sd.g[1 - pc]);
        return collide_node<D, PREC, decltype(uni)::value, decltype(gl)::value>(
            kp, on_global<const S>(d, sd.f[pc]), on_global<const S>(d, sd.g[pc]), on_global<S>(d, sd.f[1 - pc]),
            gout, on_global<const R>(d, sd.rho[1 - fc]), on_global<const R>(d, sd.phi[1 - fc]),
            on_global<const R>(d, sd.rho[fc]), on_global<const R>(d, sd.phi[fc]), on_global<const R>(d, sd.fmu), t,
            fast);
    };
    using G2 = std::integral_constant<int, 2>;
    using G3 = std::integral_constant<int, 3>;
    if (t < count) {
        const bool uni = kp.PS % 64 == 0;
        if constexpr (IMP) {
            kind = uni ? node(std::true_type{}, G3{}) : node(std::false_type{}, G3{});
        } else {
            kind = uni ? node(std::true_type{}, G2{}) : node(std::false_type{}, G2{});
        }
    }
    count_kinds(kind, fast, s_cnt);
    __syncthreads();
    if (threadIdx.x < 4 && s_cnt[threadIdx.x])
        atomicAdd(&on_global<unsigned long long>(d, sd.counters)[(size_t)(blockIdx.x & (kCntSlots - 1)) * kCntStride +
                                                               threadIdx.x],
                  (unsigned long long)s_cnt[threadIdx.x]);
}

// ---------------------------------------------------------------- init ---
template <typename R>
__global__ void __launch_bounds__(256)
k_init_fields(long long N, const double *__restrict__ src, R *__restrict__ r0, R *__restrict__ r1)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    R v = (R)src[t];
    r0[t] = v;
    r1[t] = v;
}

// f = w rho0; g = g^eq(phi0, mu_phi, 0), mu_phi from the stencils of the
// ghost-filled initial fields.
template <int D, int PREC>
__global__ void __launch_bounds__(256)
k_init_pops(KParams kp, const typename Ty<PREC>::R *__restrict__ rho, const typename Ty<PREC>::R *__restrict__ phi,
            typename Ty<PREC>::S *__restrict__ f, typename Ty<PREC>::S *__restrict__ g)
{
    using R = typename Ty<PREC>::R;
    constexpr int Q = D == 2 ? 9 : 27;
    constexpr int WA = D - 1;
    long long first = kp.walls ? kp.PS : 0;
    long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    long long n = first + t;
    int x = (int)(n % kp.nx);
    int y = (int)((n / kp.nx) % kp.ny);
    int z = (int)(n / ((long long)kp.nx * kp.ny));
    int p = (D == 2) ? y : z;
    Thermo<R> th;
    th.load(kp);
    R r0 = rho[n], p0 = phi[n];
    R G[3] = {0, 0, 0}, H[3] = {0, 0, 0}, Lr = 0, Lp = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int q = p + cdir(D, i, WA);
        if (!kp.walls) q = wrapi(q, kp.nw);
        long long m = (long long)q * kp.PS + wrapi(x + cdir(D, i, 0), kp.nx) +
                      (D == 3 ? (long long)kp.nx * wrapi(y + cdir(D, i, 1), kp.ny) : 0);
        R rn = rho[m], pn = phi[m];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            G[a] += (R)(3.0 * wgt(D, i) * cdir(D, i, a)) * rn;
            H[a] += (R)(3.0 * wgt(D, i) * cdir(D, i, a)) * pn;
        }
        Lr += (R)(6.0 * wgt(D, i)) * (rn - r0);
        Lp += (R)(6.0 * wgt(D, i)) * (pn - p0);
    }
    R mur, mup, mP[D * (D + 1) / 2];
    thermo<D, R>(th, r0, p0, G, H, Lr, Lp, mur, mup, mP);
    R sum = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (i == Q / 2) continue;
        R gi = (R)wgt(D, i) * (R)3 * (R)kp.Gamma * mup;
        sum += gi;
        g[(long long)i * kp.QS + n] = enc_g<PREC, D>(gi, i, p0);
        f[(long long)i * kp.QS + n] = enc_f<PREC, D>((R)wgt(D, i) * r0, i, r0);
    }
    g[(long long)(Q / 2) * kp.QS + n] = enc_g<PREC, D>(p0 - sum, Q / 2, p0);
    f[(long long)(Q / 2) * kp.QS + n] = enc_f<PREC, D>((R)wgt(D, Q / 2) * r0, Q / 2, r0);
}

// ------------------------------------------------------------- observe ---
constexpr int OBS_THREADS = 256;
constexpr int NSUM = 16;

// per-block FP64 partial sums of the observables over fluid nodes
template <int D, int PREC>
__global__ void __launch_bounds__(OBS_THREADS)
k_observe(KParams kp, const typename Ty<PREC>::S *__restrict__ f, const typename Ty<PREC>::S *__restrict__ g,
          const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
          double *__restrict__ partials)
{
    using R = typename Ty<PREC>::R;
    constexpr int Q = D == 2 ? 9 : 27;
    __shared__ double s[NSUM][OBS_THREADS];
    double acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0.0;
    long long first = kp.walls ? kp.PS : 0;
    long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    for (long long t = (long long)blockIdx.x * OBS_THREADS + threadIdx.x; t < count;
         t += (long long)gridDim.x * OBS_THREADS) {
        long long n = first + t;
        R rp = 0, pp = 0;
        if constexpr (PREC == P16) { rp = rprev[n]; pp = pprev[n]; }
        double r = 0, ph = 0, j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double fi = (double)dec_f<PREC, D>(f[(long long)i * kp.QS + n], i, rp);
            r += fi;
            ph += (double)dec_g<PREC, D>(g[(long long)i * kp.QS + n], i, pp);
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (cdir(D, i, a) != 0) j[a] += cdir(D, i, a) * fi;
        }
        if (!(r > 0.0) || !isfinite(r) || !isfinite(ph)) { acc[12] += 1.0; continue; }
        double C1 = (r - kp.rho_l) / (kp.rho_g - kp.rho_l);
        double C2 = 0.5 * (1.0 + ph / kp.chi - C1);
        double C3 = 0.5 * (1.0 - ph / kp.chi - C1);
        acc[0] += C1; acc[1] += C2; acc[2] += C3;
        acc[3] += r; acc[4] += ph;
        double uu = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) { acc[5 + a] += j[a]; uu += (j[a] / r) * (j[a] / r); }
        acc[8] += 0.5 * r * uu;
        acc[9] = fmax(acc[9], sqrt(uu));
    }
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = OBS_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < NSUM; ++k) {
                if (k == 9) s[k][threadIdx.x] = fmax(s[k][threadIdx.x], s[k][threadIdx.x + w]);
                else s[k][threadIdx.x] += s[k][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NSUM) partials[(long long)blockIdx.x * NSUM + threadIdx.x] = s[threadIdx.x][0];
}

// fixed-order reduction of the block partials (slot 9 is a max)
__global__ void __launch_bounds__(NSUM)
k_reduce(const double *__restrict__ partials, int nblocks, double *__restrict__ out)
{
    int k = threadIdx.x;
    double acc = 0.0, c = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        double v = partials[(long long)b * NSUM + k];
        if (k == 9) { acc = fmax(acc, v); continue; }
        double t = acc + v;  // compensated
        c += (fabs(acc) >= fabs(v)) ? (acc - t) + v : (v - t) + acc;
        acc = t;
    }
    out[k] = acc + c;
}

// plain fixed-order compensated sum of every slot
__global__ void __launch_bounds__(NSUM)
k_reduce_sum(const double *__restrict__ partials, int nblocks, double *__restrict__ out)
{
    int k = threadIdx.x;
    double acc = 0.0, c = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        double v = partials[(long long)b * NSUM + k];
        double t = acc + v;
        c += (fabs(acc) >= fabs(v)) ? (acc - t) + v : (v - t) + acc;
        acc = t;
    }
    out[k] = acc + c;
}

template <int D, int PREC>
__global__ void __launch_bounds__(256)
k_export_pop(long long N, const typename Ty<PREC>::S *__restrict__ s /* population i */, int i,
             const typename Ty<PREC>::R *__restrict__ rprev, const typename Ty<PREC>::R *__restrict__ pprev,
             int isg, double *__restrict__ out)
{
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    using R = typename Ty<PREC>::R;
    R rp = 0, pp = 0;
    if constexpr (PREC == P16) { rp = rprev[n]; pp = pprev[n]; }
    out[n] = isg ? (double)dec_g<PREC, D>(s[n], i, pp) : (double)dec_f<PREC, D>(s[n], i, rp);
}

template <typename R>
__global__ void __launch_bounds__(256)
k_export_field(long long N, const R *__restrict__ s, double *__restrict__ out)
{
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) out[n] = (double)s[n];
}

// Kasa least squares, FP64: per iso-point (x, y[, z]) accumulate the normal
// equations of  x^2 + y^2 (+ z^2) + D x + E y (+ F z) + G = 0.
template <int D, typename R>
__global__ void __launch_bounds__(OBS_THREADS)
k_contour(KParams kp, const R *__restrict__ rho, const R *__restrict__ phi, int comp, int wall,
          double exclude, double *__restrict__ partials)
{
    __shared__ double s[NSUM][OBS_THREADS];
    double acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0.0;
    const int nw = kp.nw;
    const double wplane = wall == 0 ? 0.5 : nw - 1.5;
    auto conc = [&](long long n) {
        double r = (double)rho[n], ph = (double)phi[n];
        double C1 = (r - kp.rho_l) / (kp.rho_g - kp.rho_l);
        return comp == 2 ? 0.5 * (1.0 + ph / kp.chi - C1) : 0.5 * (1.0 - ph / kp.chi - C1);
    };
    auto add = [&](double px, double py, double pz) {
        double q[4] = {px, py, D == 3 ? pz : 1.0, 1.0};
        const int m = D == 3 ? 4 : 3;
        double rr = px * px + py * py + (D == 3 ? pz * pz : 0.0);
        int k = 0;
        for (int a = 0; a < m; ++a)
            for (int b = a; b < m; ++b) acc[k++] += q[a] * q[b];
        for (int a = 0; a < m; ++a) acc[k++] += q[a] * rr;
    };
    for (long long n = (long long)blockIdx.x * OBS_THREADS + threadIdx.x; n < kp.N;
         n += (long long)gridDim.x * OBS_THREADS) {
        int x = (int)(n % kp.nx), y = (int)((n / kp.nx) % kp.ny), z = (int)(n / ((long long)kp.nx * kp.ny));
        int p = D == 2 ? y : z;
        if (kp.walls && (p < 1 || p > nw - 2)) continue;
        double c0 = conc(n) - 0.5;
        double pos[3] = {(double)x, (double)y, (double)z};
        for (int a = 0; a < D; ++a) {
            int co = a == 0 ? x : (a == 1 ? y : z);
            int na = a == 0 ? kp.nx : (a == 1 ? kp.ny : kp.nz);
            if (co + 1 >= na) continue;
            if (a == D - 1 && kp.walls && co + 1 > nw - 2) continue;
            long long stride = a == 0 ? 1 : (a == 1 ? kp.nx : (long long)kp.nx * kp.ny);
            double c1 = conc(n + stride) - 0.5;
            double t;
            if (c0 == 0.0 && a == 0) t = 0.0;
            else if (c0 * c1 < 0.0) t = c0 / (c0 - c1);
            else continue;
            double q[3] = {pos[0], pos[1], pos[2]};
            q[a] += t;
            double hgt = D == 2 ? q[1] : q[2];
            if (fabs(hgt - wplane) <= exclude) continue;
            add(q[0], q[1], q[2]);
        }
    }
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = OBS_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < NSUM; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < NSUM) partials[(long long)blockIdx.x * NSUM + threadIdx.x] = s[threadIdx.x][0];
}

// ----------------------------------------------------------- launchers --
#define LBM3_CHECK_LAUNCH() (hipGetLastError() == hipSuccess ? 0 : -1)

template <int PREC> using SP = typename Ty<PREC>::S *;
template <int PREC> using RP = typename Ty<PREC>::R *;

static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Events of the stage a profiled step is launching: the stage's first
// kernel records `start` and its last `stop` from their own dispatch packets
// (hipExtLaunchKernelGGL), so the interval is the kernels' run time, without
// a marker packet (and the dispatch gap that comes with it) in between.
static thread_local hipEvent_t t_stage_start = nullptr, t_stage_stop = nullptr;
// within a two-kernel stage: the end of its first kernel, the start of its second
static thread_local hipEvent_t t_sub_stop = nullptr, t_sub_start = nullptr;

void set_stage_events(void *start, void *stop, void *sub_stop, void *sub_start)
{
    t_stage_start = (hipEvent_t)start;
    t_stage_stop = (hipEvent_t)stop;
    t_sub_stop = (hipEvent_t)sub_stop;
    t_sub_start = (hipEvent_t)sub_start;
}

template <typename F, typename... A>
static void stage_launch(F kernel, dim3 grid, dim3 block, hipStream_t st, bool first, bool last, A... args)
{
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, first ? t_stage_start : t_sub_start,
                          last ? t_stage_stop : t_sub_stop, 0, args...);
}

template <int D, int PREC>
// 2D: blocks of 64 threads (four per 256-thread block of moments_blocks), so
// that a small grid's few thousand threads spread over more CUs (2048 x 64:
// step 1.7 % faster); the batched launch keeps 256
static int moments_t(const KParams &kp, const Buffers &b, int pc, int fc, hipStream_t st)
{
    constexpr unsigned split = D == 2 ? 4u : 1u;
    stage_launch(k_moments<D, PREC>, dim3((unsigned)moments_blocks(kp, PREC) * split), dim3(256 / split), st, true,
                 true, kp,
                 (SP<PREC>)b.f[pc], (SP<PREC>)b.g[pc], (RP<PREC>)b.rho[fc], (RP<PREC>)b.phi[fc],
                 (RP<PREC>)b.rho[1 - fc], (RP<PREC>)b.phi[1 - fc]);
    return LBM3_CHECK_LAUNCH();
}

int launch_moments(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D == 2) {
        if (prec == P64) return moments_t<2, P64>(kp, b, pc, fc, st);
        if (prec == P32) return moments_t<2, P32>(kp, b, pc, fc, st);
        return moments_t<2, P16>(kp, b, pc, fc, st);
    }
    if (prec == P64) return moments_t<3, P64>(kp, b, pc, fc, st);
    if (prec == P32) return moments_t<3, P32>(kp, b, pc, fc, st);
    return moments_t<3, P16>(kp, b, pc, fc, st);
}

template <int PREC>
static void moments_imp_t(const KParams &kp, const Buffers &b, int pc, int fc, hipStream_t st)
{
    constexpr int TX = kImpTX, TY = kImpTY;
    const int chunk = moments_march_chunk(kp);
    const long long nb = moments_march_blocks(kp);
    stage_launch(k_moments_imp<PREC, TX, TY>, dim3((unsigned)nb), dim3(TX * TY), st, true, true, kp,
                 (SP<PREC>)b.f[pc], (RP<PREC>)b.gp, (RP<PREC>)b.rho[fc], (RP<PREC>)b.rho[1 - fc],
                 (RP<PREC>)b.phi[1 - fc], chunk);
}

int launch_moments_imp(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D != 3 || !b.gp) return -1;
    if (prec == P64) moments_imp_t<P64>(kp, b, pc, fc, st);
    else if (prec == P32) moments_imp_t<P32>(kp, b, pc, fc, st);
    else moments_imp_t<P16>(kp, b, pc, fc, st);
    return LBM3_CHECK_LAUNCH();
}

int launch_g_materialize(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D != 3 || !b.gp) return -1;
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    if (prec == P64)
        k_g_materialize<P64><<<nblk(count, 256), 256, 0, st>>>(kp, (RP<P64>)b.gp, (RP<P64>)b.phi[fc], (SP<P64>)b.g[pc]);
    else if (prec == P32)
        k_g_materialize<P32><<<nblk(count, 256), 256, 0, st>>>(kp, (RP<P32>)b.gp, (RP<P32>)b.phi[fc], (SP<P32>)b.g[pc]);
    else
        k_g_materialize<P16><<<nblk(count, 256), 256, 0, st>>>(kp, (RP<P16>)b.gp, (RP<P16>)b.phi[fc], (SP<P16>)b.g[pc]);
    return LBM3_CHECK_LAUNCH();
}

int launch_ghost(const KParams &kp, int prec, const Buffers &b, int fdst, void *stream)
{
    if (!kp.walls) return 0;
    hipStream_t st = (hipStream_t)stream;
    long long np = kp.D == 2 ? kp.nx : (long long)kp.nx * kp.ny;
    unsigned g = nblk(2 * np, 256);
    if (prec == P64) {
        if (kp.D == 2) stage_launch(k_ghost<2, double>, dim3(g), dim3(256), st, true, true, kp, (double *)b.rho[fdst], (double *)b.phi[fdst]);
        else stage_launch(k_ghost<3, double>, dim3(g), dim3(256), st, true, true, kp, (double *)b.rho[fdst], (double *)b.phi[fdst]);
    } else {
        if (kp.D == 2) stage_launch(k_ghost<2, float>, dim3(g), dim3(256), st, true, true, kp, (float *)b.rho[fdst], (float *)b.phi[fdst]);
        else stage_launch(k_ghost<3, float>, dim3(g), dim3(256), st, true, true, kp, (float *)b.rho[fdst], (float *)b.phi[fdst]);
    }
    return LBM3_CHECK_LAUNCH();
}

// chunk of march planes per block: about `target` blocks.  Measured per tile
// class: the small 2D tiles (one wave each, all resident at once) run best
// with one plane per block up to 8192 blocks (2048 x 64: 9 % faster than two
// planes); the 254-node 2D tiles with about 2048 blocks and at least two
// planes, so the ring prologue is amortised (4096 x 256: three-plane chunks
// 1.3 % faster than five, two-plane ones 2 % slower); the 3D tiles with
// 8-plane chunks on a 256^3 grid.
static int choose_chunk(int cls, long long tiles, int planes)
{
    const long long target = cls == 0 ? 8192 : (cls == 1 ? 2048 : 4096);
    const long long cmin = cls == 0 ? 1 : 2;
    long long c = (tiles * planes + target - 1) / target;
    if (c < cmin) c = cmin;
    if (c > 64) c = 64;
    if (c > planes) c = planes;
    return (int)c;
}

static void tile_of_class(int cls, int prec, int &TX, int &TY)
{
    if (cls == 0) { TX = kSmall2DTX; TY = 1; }
    else if (cls == 1) { TX = 254; TY = 1; }
    else if (cls == 2) { TX = 32; TY = prec == P64 ? 4 : 16; }
    else { TX = 32; TY = prec == P64 ? 4 : 8; }  // stencil pass: two blocks per CU
}

// 0: 2D below 2^20 nodes, 1: larger 2D, 2: 3D fused, 3: 3D two-kernel step
static int fused_class(const KParams &kp)
{
    if (kp.D == 3) return (kp.flags & kFlagFused3D) ? 2 : 3;
    return (long long)kp.nx * kp.nw < kSmall2DNodes ? 0 : 1;
}

bool two_kernel_step(const KParams &kp) { return fused_class(kp) == 3; }

FusedGeom fused_geometry(const KParams &kp, int prec)
{
    FusedGeom g;
    g.cls = fused_class(kp);
    int TX, TY;
    tile_of_class(g.cls, prec, TX, TY);
    int ntx = (kp.nx + TX - 1) / TX;
    int nty = kp.D == 3 ? (kp.ny + TY - 1) / TY : 1;
    int planes = kp.walls ? kp.nw - 2 : kp.nw;
    g.ntiles = ntx * nty;
    g.chunk = choose_chunk(g.cls, (long long)g.ntiles, planes);
    g.nchunks = chunk_count(kp, wall_edge(kp, g.cls == 0, g.chunk), g.chunk);
    return g;
}

// ONE_OK: a one-plane instantiation exists and is taken when the chunk is 1
template <int D, int PREC, int TX, int TY, int NTH, bool ONE_OK = false>
static int fused_t(const KParams &kp, const Buffers &b, int pc, int fc, hipStream_t st)
{
    FusedGeom g = fused_geometry(kp, PREC);
    dim3 grid((unsigned)g.ntiles, (unsigned)g.nchunks);
    if (ONE_OK && g.chunk == 1)
        stage_launch(k_fused<D, PREC, TX, TY, NTH, ONE_OK>, grid, dim3(NTH), st, true, true, kp, (SP<PREC>)b.f[pc],
                     (SP<PREC>)b.g[pc], (SP<PREC>)b.f[1 - pc], (SP<PREC>)b.g[1 - pc], (RP<PREC>)b.rho[1 - fc],
                     (RP<PREC>)b.phi[1 - fc], (RP<PREC>)b.rho[fc], (RP<PREC>)b.phi[fc], b.counters, g.chunk);
    else
        stage_launch(k_fused<D, PREC, TX, TY, NTH>, grid, dim3(NTH), st, true, true, kp, (SP<PREC>)b.f[pc],
                     (SP<PREC>)b.g[pc], (SP<PREC>)b.f[1 - pc], (SP<PREC>)b.g[1 - pc], (RP<PREC>)b.rho[1 - fc],
                     (RP<PREC>)b.phi[1 - fc], (RP<PREC>)b.rho[fc], (RP<PREC>)b.phi[fc], b.counters, g.chunk);
    return LBM3_CHECK_LAUNCH();
}

// two-kernel 3D step: the stencil march writes F and mu_phi, then one
// thread per fluid node collides and streams
template <int PREC, int TX, int TY, int NTH>
static int split_t(const KParams &kp, const Buffers &b, int pc, int fc, hipStream_t st)
{
    FusedGeom g = fused_geometry(kp, PREC);
    dim3 grid((unsigned)g.ntiles, (unsigned)g.nchunks);
    stage_launch(k_stencil<PREC, TX, TY>, grid, dim3(NTH), st, true, false, kp, (RP<PREC>)b.rho[1 - fc],
                 (RP<PREC>)b.phi[1 - fc], (RP<PREC>)b.fmu, g.chunk);
    int r = LBM3_CHECK_LAUNCH();
    if (r) return r;
    // the plane stride a multiple of the wave: planes are wave-uniform;
    // tau_g = 1 with collisions: the stored g is not read
    const bool uni = kp.PS % 64 == 0;
    const bool gl = (kp.flags & 1u) || kp.inv_tau_g != 1.0;
    // implicit g: the collision stores (a, phi, v) in b.gp instead of g
    const bool imp = b.gp != nullptr && !gl;
    auto go = [&](auto kern) {
        stage_launch(kern, dim3((unsigned)collide_blocks(kp)), dim3(256), st, false, true, kp, (SP<PREC>)b.f[pc],
                     (SP<PREC>)b.g[pc], (SP<PREC>)b.f[1 - pc], imp ? (SP<PREC>)b.gp : (SP<PREC>)b.g[1 - pc],
                     (RP<PREC>)b.rho[1 - fc], (RP<PREC>)b.phi[1 - fc], (RP<PREC>)b.rho[fc], (RP<PREC>)b.phi[fc],
                     (RP<PREC>)b.fmu, b.counters);
    };
    if (imp) {
        if (uni) go(k_collide<3, PREC, true, 3>);
        else go(k_collide<3, PREC, false, 3>);
        return LBM3_CHECK_LAUNCH();
    }
    if (uni) {
        if (gl) go(k_collide<3, PREC, true, 1>);
        else go(k_collide<3, PREC, true, 0>);
    } else {
        if (gl) go(k_collide<3, PREC, false, 1>);
        else go(k_collide<3, PREC, false, 0>);
    }
    return LBM3_CHECK_LAUNCH();
}

bool fused_fills_ghost(const KParams &kp) { return kp.D == 2; }

int launch_fused(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const int cls = fused_class(kp);
    if (cls == 0) {
        if (prec == P64) return fused_t<2, P64, 62, 1, 64, true>(kp, b, pc, fc, st);
        if (prec == P32) return fused_t<2, P32, 62, 1, 64, true>(kp, b, pc, fc, st);
        return fused_t<2, P16, 62, 1, 64, true>(kp, b, pc, fc, st);
    }
    if (cls == 1) {
        if (prec == P64) return fused_t<2, P64, 254, 1, 256>(kp, b, pc, fc, st);
        if (prec == P32) return fused_t<2, P32, 254, 1, 256>(kp, b, pc, fc, st);
        return fused_t<2, P16, 254, 1, 256>(kp, b, pc, fc, st);
    }
    if (cls == 3) {
        if (prec == P64) return split_t<P64, 32, 4, 128>(kp, b, pc, fc, st);
        if (prec == P32) return split_t<P32, 32, 8, 256>(kp, b, pc, fc, st);
        return split_t<P16, 32, 8, 256>(kp, b, pc, fc, st);
    }
    if (prec == P64) return fused_t<3, P64, 32, 4, 128>(kp, b, pc, fc, st);
    if (prec == P32) return fused_t<3, P32, 32, 16, 512>(kp, b, pc, fc, st);
    return fused_t<3, P16, 32, 16, 512>(kp, b, pc, fc, st);
}

long long collide_blocks(const KParams &kp)
{
    if (fused_class(kp) != 3) return 0;
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    return (count + 255) / 256;
}

// ------------------------------------------------------- batched launches
long long moments_batch_blocks(const KParams &kp, int prec, bool implicit)
{
    return kp.D == 3 && implicit ? moments_march_blocks(kp) : moments_blocks(kp, prec);
}

long long moments_blocks(const KParams &kp, int prec)
{
    const long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    const int v = mom_width(kp, prec);
    return ((count + v - 1) / v + 255) / 256;
}

long long ghost_blocks(const KParams &kp)
{
    if (!kp.walls || fused_fills_ghost(kp)) return 0;
    long long np = kp.D == 2 ? kp.nx : (long long)kp.nx * kp.ny;
    return (2 * np + 255) / 256;
}

int launch_moments_batch(int D, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                         bool first, void *stream)
{
    if (nblocks <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)nblocks);
    const int fi = first ? 1 : 0;
    if (D == 2) {
        if (prec == P64) k_moments_batch<2, P64><<<grid, 256, 0, st>>>(d, sim, phase, fi);
        else if (prec == P32) k_moments_batch<2, P32><<<grid, 256, 0, st>>>(d, sim, phase, fi);
        else k_moments_batch<2, P16><<<grid, 256, 0, st>>>(d, sim, phase, fi);
    } else {
        if (prec == P64) k_moments_batch<3, P64><<<grid, 256, 0, st>>>(d, sim, phase, fi);
        else if (prec == P32) k_moments_batch<3, P32><<<grid, 256, 0, st>>>(d, sim, phase, fi);
        else k_moments_batch<3, P16><<<grid, 256, 0, st>>>(d, sim, phase, fi);
    }
    return LBM3_CHECK_LAUNCH();
}

int launch_ghost_batch(int D, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                       void *stream)
{
    if (nblocks <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)nblocks);
    if (D == 2) {
        if (prec == P64) k_ghost_batch<2, double><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_ghost_batch<2, float><<<grid, 256, 0, st>>>(d, sim, phase);
    } else {
        if (prec == P64) k_ghost_batch<3, double><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_ghost_batch<3, float><<<grid, 256, 0, st>>>(d, sim, phase);
    }
    return LBM3_CHECK_LAUNCH();
}

int launch_fused_batch(int cls, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                       void *stream)
{
    if (nblocks <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)nblocks);
    if (cls == 0) {
        if (prec == P64) k_fused_batch<2, P64, 62, 1, 64><<<grid, 64, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_fused_batch<2, P32, 62, 1, 64><<<grid, 64, 0, st>>>(d, sim, phase);
        else k_fused_batch<2, P16, 62, 1, 64><<<grid, 64, 0, st>>>(d, sim, phase);
    } else if (cls == 1) {
        if (prec == P64) k_fused_batch<2, P64, 254, 1, 256><<<grid, 256, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_fused_batch<2, P32, 254, 1, 256><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_fused_batch<2, P16, 254, 1, 256><<<grid, 256, 0, st>>>(d, sim, phase);
    } else if (cls == 2) {
        if (prec == P64) k_fused_batch<3, P64, 32, 4, 128><<<grid, 128, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_fused_batch<3, P32, 32, 16, 512><<<grid, 512, 0, st>>>(d, sim, phase);
        else k_fused_batch<3, P16, 32, 16, 512><<<grid, 512, 0, st>>>(d, sim, phase);
    } else {
        if (prec == P64) k_stencil_batch<P64, 32, 4><<<grid, 128, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_stencil_batch<P32, 32, 8><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_stencil_batch<P16, 32, 8><<<grid, 256, 0, st>>>(d, sim, phase);
    }
    return LBM3_CHECK_LAUNCH();
}

int launch_collide_batch(int D, int prec, bool implicit, const SimDesc *d, const int *sim, long long nblocks,
                         int phase, void *stream)
{
    if (nblocks <= 0 || D != 3) return nblocks <= 0 ? 0 : 1;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)nblocks);
    if (implicit) {
        if (prec == P64) k_collide_batch<3, P64, true><<<grid, 256, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_collide_batch<3, P32, true><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_collide_batch<3, P16, true><<<grid, 256, 0, st>>>(d, sim, phase);
    } else {
        if (prec == P64) k_collide_batch<3, P64, false><<<grid, 256, 0, st>>>(d, sim, phase);
        else if (prec == P32) k_collide_batch<3, P32, false><<<grid, 256, 0, st>>>(d, sim, phase);
        else k_collide_batch<3, P16, false><<<grid, 256, 0, st>>>(d, sim, phase);
    }
    return LBM3_CHECK_LAUNCH();
}

template <int D, int PREC>
static int init_t(const KParams &kp, const Buffers &b, hipStream_t st)
{
    long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    k_init_pops<D, PREC><<<nblk(count, 256), 256, 0, st>>>(kp, (RP<PREC>)b.rho[0], (RP<PREC>)b.phi[0],
                                                            (SP<PREC>)b.f[0], (SP<PREC>)b.g[0]);
    return LBM3_CHECK_LAUNCH();
}

// upload staging -> fields: which = 0 rho, 1 phi (both field buffers)
int launch_init_field(const KParams &kp, int prec, const Buffers &b, int which, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    void **dst = which == 0 ? (void **)b.rho : (void **)b.phi;
    if (prec == P64) k_init_fields<double><<<nblk(kp.N, 256), 256, 0, st>>>(kp.N, b.scratch, (double *)dst[0], (double *)dst[1]);
    else k_init_fields<float><<<nblk(kp.N, 256), 256, 0, st>>>(kp.N, b.scratch, (float *)dst[0], (float *)dst[1]);
    return LBM3_CHECK_LAUNCH();
}

int launch_init(const KParams &kp, int prec, const Buffers &b, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D == 2) {
        if (prec == P64) return init_t<2, P64>(kp, b, st);
        if (prec == P32) return init_t<2, P32>(kp, b, st);
        return init_t<2, P16>(kp, b, st);
    }
    if (prec == P64) return init_t<3, P64>(kp, b, st);
    if (prec == P32) return init_t<3, P32>(kp, b, st);
    return init_t<3, P16>(kp, b, st);
}

int observe_blocks(const KParams &kp)
{
    long long count = kp.walls ? kp.N - 2 * kp.PS : kp.N;
    long long nb = (count + OBS_THREADS * 8 - 1) / (OBS_THREADS * 8);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return (int)nb;
}

template <int D, int PREC>
static int observe_t(const KParams &kp, const Buffers &b, int pc, int fc, hipStream_t st)
{
    int nb = observe_blocks(kp);
    k_observe<D, PREC><<<nb, OBS_THREADS, 0, st>>>(kp, (SP<PREC>)b.f[pc], (SP<PREC>)b.g[pc], (RP<PREC>)b.rho[fc],
                                                    (RP<PREC>)b.phi[fc], b.partials);
    k_reduce<<<1, NSUM, 0, st>>>(b.partials, nb, b.result);
    return LBM3_CHECK_LAUNCH();
}

int launch_observe(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D == 2) {
        if (prec == P64) return observe_t<2, P64>(kp, b, pc, fc, st);
        if (prec == P32) return observe_t<2, P32>(kp, b, pc, fc, st);
        return observe_t<2, P16>(kp, b, pc, fc, st);
    }
    if (prec == P64) return observe_t<3, P64>(kp, b, pc, fc, st);
    if (prec == P32) return observe_t<3, P32>(kp, b, pc, fc, st);
    return observe_t<3, P16>(kp, b, pc, fc, st);
}

template <int D, int PREC>
static int export_pop_t(const KParams &kp, const Buffers &b, int pc, int fc, int which, int i, hipStream_t st)
{
    const void *src = which == 0 ? b.f[pc] : b.g[pc];
    k_export_pop<D, PREC><<<nblk(kp.N, 256), 256, 0, st>>>(kp.N, (const typename Ty<PREC>::S *)src + (size_t)i * kp.QS, i,
                                                           (RP<PREC>)b.rho[fc], (RP<PREC>)b.phi[fc], which,
                                                           b.scratch);
    return LBM3_CHECK_LAUNCH();
}

int launch_export_pop(const KParams &kp, int prec, const Buffers &b, int pc, int fc, int which, int i,
                      void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (kp.D == 2) {
        if (prec == P64) return export_pop_t<2, P64>(kp, b, pc, fc, which, i, st);
        if (prec == P32) return export_pop_t<2, P32>(kp, b, pc, fc, which, i, st);
        return export_pop_t<2, P16>(kp, b, pc, fc, which, i, st);
    }
    if (prec == P64) return export_pop_t<3, P64>(kp, b, pc, fc, which, i, st);
    if (prec == P32) return export_pop_t<3, P32>(kp, b, pc, fc, which, i, st);
    return export_pop_t<3, P16>(kp, b, pc, fc, which, i, st);
}

int launch_export_field(const KParams &kp, int prec, const Buffers &b, int fsrc, int which, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const void *src = which == 0 ? b.rho[fsrc] : b.phi[fsrc];
    if (prec == P64) k_export_field<double><<<nblk(kp.N, 256), 256, 0, st>>>(kp.N, (const double *)src, b.scratch);
    else k_export_field<float><<<nblk(kp.N, 256), 256, 0, st>>>(kp.N, (const float *)src, b.scratch);
    return LBM3_CHECK_LAUNCH();
}

int launch_contour(const KParams &kp, int prec, const Buffers &b, int fsrc, int comp, int wall, double exclude,
                   void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    long long nb = (kp.N + OBS_THREADS * 8 - 1) / (OBS_THREADS * 8);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    if (prec == P64) {
        if (kp.D == 2) k_contour<2, double><<<(unsigned)nb, OBS_THREADS, 0, st>>>(kp, (const double *)b.rho[fsrc], (const double *)b.phi[fsrc], comp, wall, exclude, b.partials);
        else k_contour<3, double><<<(unsigned)nb, OBS_THREADS, 0, st>>>(kp, (const double *)b.rho[fsrc], (const double *)b.phi[fsrc], comp, wall, exclude, b.partials);
    } else {
        if (kp.D == 2) k_contour<2, float><<<(unsigned)nb, OBS_THREADS, 0, st>>>(kp, (const float *)b.rho[fsrc], (const float *)b.phi[fsrc], comp, wall, exclude, b.partials);
        else k_contour<3, float><<<(unsigned)nb, OBS_THREADS, 0, st>>>(kp, (const float *)b.rho[fsrc], (const float *)b.phi[fsrc], comp, wall, exclude, b.partials);
    }
    k_reduce_sum<<<1, NSUM, 0, st>>>(b.partials, (int)nb, b.result);
    return LBM3_CHECK_LAUNCH();
}

}  // namespace lbm3k
