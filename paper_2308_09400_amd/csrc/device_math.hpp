// Device-side geometry and barrier math for the GIPC pair kernels (gfx950,
// FP64 on the vector ALUs).
//
// Two jobs live here:
//  * classification: reduce a point-triangle / edge-edge tuple to the
//    sub-type given by the active constraints of its constrained minimum
//    (Eq. 4 / Eq. 5), flagging nearly-parallel edge pairs for the
//    mollifier (Eq. 25);
//  * evaluation of a typed pair: distance of the sub-type, gap g = f^2
//    (Eq. 9-11), barrier (Eq. 24 or Eq. 12), mollifier, gradient factors and
//    the analytically projected proxy Hessian (Eq. 18-23, 32-36).
//
// Every distance is written as |p* - q*| with p* - q* = sum_k c_k x_k over
// the stencil slots; at the constrained minimiser d(d^2)/dx_k = 2 c_k w with
// w = p* - q*, so grad f = (c (x) w) / (dhat d) for every sub-type.  The
// proxy Hessian of a non-mollified pair is kappa * lambda_1 * grad f grad f^T
// (Eq. 20-21: Q_1 = e_m e_m^T, and only J_mm varies with x).  A mollified
// pair adds the J_22 = sqrt(c) row: its 2x2 inner block
// [[lambda_g1, 4t], [4t, lambda_q1]] (Eq. 33-35) is projected onto its
// non-negative eigenspace; the remaining eigenpairs of Eq. 32 live on
// off-diagonal entries of J, which dJ/dx never touches, so they contribute
// nothing after the change of basis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gipc {

// Sub-type codes of staged pairs.  Vertex slot conventions of the staged
// stencil (v0..v3):
//   PT  [p, t0, t1, t2]    point-plane distance
//   PE  [p, e0, e1, -]     point-line distance
//   PP  [p, q, -, -]       point-point distance
//   EE  [a0, a1, b0, b1]   line-line distance
//   EEM [a0, a1, b0, b1]   line-line, mollified
//   PEM [p, o, e0, e1]     point p vs line e0e1, mollified; o = p's edge partner
//   PPM [p, o, q, r]       point p vs point q, mollified; (p,o) and (q,r) the edges
// For the mollified kinds the parallelness is always c = |(v1-v0) x (v3-v2)|^2.
enum FineType : int { FT_NONE = 0, FT_PT = 1, FT_PE = 2, FT_PP = 3, FT_EE = 4, FT_EEM = 5, FT_PEM = 6, FT_PPM = 7 };

__host__ __device__ inline int ft_nverts(int ft) {
    return ft == FT_PP ? 2 : (ft == FT_PE ? 3 : (ft == FT_NONE ? 0 : 4));
}

// Interior stationary points are used only when the Gram determinant
// exceeds this fraction of the product of squared edge lengths.
constexpr double kInteriorTol = 1e-10;

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// p*q - r*s within 1.5 ulp of the exact value (Kahan's difference of
// products; the fma recovers the rounding error of r*s).  The parallelness
// c of Eq. 25 uses it: for edges that are parallel up to the rounding of
// their coordinates the plain cross product is cancellation noise, and its
// direction sets grad sqrt(c), so n must be a function of the input alone.
__device__ __forceinline__ double diff_prod(double p, double q, double r, double s) {
    double w = __dmul_rn(r, s);
    double err = fma(-r, s, w);
    return __dadd_rn(fma(p, q, -w), err);
}
__device__ __forceinline__ d3 cross_acc(d3 a, d3 b) {
    return mk(diff_prod(a.y, b.z, a.z, b.y), diff_prod(a.z, b.x, a.x, b.z), diff_prod(a.x, b.y, a.y, b.x));
}
__device__ __forceinline__ d3 ld3(const double* __restrict__ X, int v) {
    const double* q = X + 3ll * v;
    return mk(q[0], q[1], q[2]);
}

struct DevParams {
    double dhat, kappa, dthr_ratio, epsx_ratio;
    int filter, mollify, eq12;
    // batches of independent scenes: scene id per vertex and the scenes'
    // dhat and kappa (all NULL for a single scene, which uses dhat, kappa)
    const int32_t* vscene;
    const double* dhat_s;
    const double* kappa_s;
};

// dhat and kappa of the scene that owns vertex v (every vertex of a staged
// pair belongs to the same scene)
__device__ __forceinline__ void scene_params(const DevParams& pm, int v, double& dhat, double& kappa) {
    if (pm.vscene) {
        const int s = pm.vscene[v];
        dhat = pm.dhat_s[s];
        kappa = pm.kappa_s[s];
    } else {
        dhat = pm.dhat;
        kappa = pm.kappa;
    }
}

// point P against segment AB: squared distance, clamped parameter
__device__ __forceinline__ double seg_dist2(d3 P, d3 A, d3 B, double& al) {
    d3 ab = B - A, ap = P - A;
    double l2 = dot(ab, ab);
    double a = l2 > 0.0 ? dot(ap, ab) / l2 : 0.0;
    a = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
    d3 w = ap - a * ab;
    al = a;
    return dot(w, w);
}

// ------------------------------------------------------------------------
// classification (Eq. 4 / Eq. 5): smallest of the interior stationary point
// (when it exists and is feasible) and the boundary sub-problems, in a
// fixed order; the first candidate wins ties.

struct Staged {
    int ft;
    int v[4];
};

// degen (out): the triangle has zero area (its vertices are collinear or
// coincide); its distance is then the smallest over its edges
__device__ inline Staged classify_pt(const double* __restrict__ X, int vp, int v0, int v1, int v2, double& d2,
                                     bool& degen) {
    d3 p = ld3(X, vp), t0 = ld3(X, v0), t1 = ld3(X, v1), t2 = ld3(X, v2);
    d3 e1 = t1 - t0, e2 = t2 - t0, r = p - t0;
    d3 n = cross(e1, e2);
    double nn = dot(n, n), a11 = dot(e1, e1), a22 = dot(e2, e2);
    degen = !(nn > 0.0);
    double best = INFINITY;
    Staged s{FT_NONE, {-1, -1, -1, -1}};
    if (nn > kInteriorTol * a11 * a22) {
        double a12 = dot(e1, e2), b1 = dot(e1, r), b2 = dot(e2, r);
        double be1 = (a22 * b1 - a12 * b2) / nn, be2 = (a11 * b2 - a12 * b1) / nn;
        if (be1 >= 0.0 && be2 >= 0.0 && be1 + be2 <= 1.0) {
            double h = dot(r, n);
            best = h * h / nn;
            s = Staged{FT_PT, {vp, v0, v1, v2}};
        }
    }
    const d3 T[3] = {t0, t1, t2};
    const int TV[3] = {v0, v1, v2};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        int ia = e, ib = (e + 1) % 3;
        double al;
        double dd = seg_dist2(p, T[ia], T[ib], al);
        if (dd < best) {
            best = dd;
            if (al > 0.0 && al < 1.0) s = Staged{FT_PE, {vp, TV[ia], TV[ib], -1}};
            else s = Staged{FT_PP, {vp, al <= 0.0 ? TV[ia] : TV[ib], -1, -1}};
        }
    }
    d2 = best;
    return s;
}

// degen (out): the edge has zero length (the pair is then point-point)
__device__ inline Staged classify_pe(const double* __restrict__ X, int vp, int v0, int v1, double& d2, bool& degen) {
    double al;
    const d3 a = ld3(X, v0), b = ld3(X, v1);
    const d3 e = b - a;
    degen = !(dot(e, e) > 0.0);
    d2 = seg_dist2(ld3(X, vp), a, b, al);
    if (al > 0.0 && al < 1.0) return Staged{FT_PE, {vp, v0, v1, -1}};
    return Staged{FT_PP, {vp, al <= 0.0 ? v0 : v1, -1, -1}};
}

// eps_x of Eq. 25 from the rest positions of the two edges
__device__ __forceinline__ double eps_x(const double* __restrict__ XR, int a0, int a1, int b0, int b1, double ratio) {
    d3 a = ld3(XR, a1) - ld3(XR, a0), b = ld3(XR, b1) - ld3(XR, b0);
    return ratio * dot(a, a) * dot(b, b);
}

// degen (out): an edge has zero length
__device__ inline Staged classify_ee(const double* __restrict__ X, const double* __restrict__ XR, int va0, int va1,
                                     int vb0, int vb1, const DevParams& pm, double& d2, bool& degen) {
    d3 a0 = ld3(X, va0), a1 = ld3(X, va1), b0 = ld3(X, vb0), b1 = ld3(X, vb1);
    d3 a = a1 - a0, b = b1 - b0, r = a0 - b0;
    d3 n = cross(a, b);
    double cc = dot(n, n), aa = dot(a, a), bb = dot(b, b);
    degen = !(aa > 0.0) || !(bb > 0.0);
    bool moll = pm.mollify && cc < eps_x(XR, va0, va1, vb0, vb1, pm.epsx_ratio);
    double best = INFINITY;
    Staged s{FT_NONE, {-1, -1, -1, -1}};
    if (cc > kInteriorTol * aa * bb) {
        double ab = dot(a, b), ar = dot(a, r), br = dot(b, r);
        double g1 = (ab * br - bb * ar) / cc, g2 = (aa * br - ab * ar) / cc;
        if (g1 >= 0.0 && g1 <= 1.0 && g2 >= 0.0 && g2 <= 1.0) {
            double h = dot(r, n);
            best = h * h / cc;
            s = Staged{moll ? FT_EEM : FT_EE, {va0, va1, vb0, vb1}};
        }
    }
    // an endpoint of one edge against the other edge; partner = the
    // endpoint's own edge mate
    const d3 P[4] = {a0, a1, b0, b1};
    const int PV[4] = {va0, va1, vb0, vb1}, OV[4] = {va1, va0, vb1, vb0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool onA = k < 2;
        d3 A = onA ? b0 : a0, B = onA ? b1 : a1;
        int vA = onA ? vb0 : va0, vB = onA ? vb1 : va1;
        double al;
        double dd = seg_dist2(P[k], A, B, al);
        if (dd < best) {
            best = dd;
            if (al > 0.0 && al < 1.0) {
                s = moll ? Staged{FT_PEM, {PV[k], OV[k], vA, vB}} : Staged{FT_PE, {PV[k], vA, vB, -1}};
            } else {
                int q = al <= 0.0 ? vA : vB, rr = al <= 0.0 ? vB : vA;
                s = moll ? Staged{FT_PPM, {PV[k], OV[k], q, rr}} : Staged{FT_PP, {PV[k], q, -1, -1}};
            }
        }
    }
    d2 = best;
    return s;
}

// A point-edge or point-point pair cut from a close-to-parallel edge-edge
// pair, given in the paper's encodings (Sec. 7.2, "Data structures"): point
// p of edge (p, o) against edge (e0, e1) (edge = true) or against its
// endpoint e0, whose edge is (e0, e1) (edge = false).  The distance is the
// point-segment (or point-point) sub-problem of Eq. 5; the mollifier is
// decided from both edges, as for an edge-edge pair.
// degen (out): an edge has zero length.
__device__ inline Staged classify_par(const double* __restrict__ X, const double* __restrict__ XR, int vp, int vo,
                                      int ve0, int ve1, bool edge, const DevParams& pm, double& d2, bool& degen) {
    const d3 P = ld3(X, vp), O = ld3(X, vo), E0 = ld3(X, ve0), E1 = ld3(X, ve1);
    const d3 a = O - P, b = E1 - E0;
    const d3 n = cross(a, b);
    degen = !(dot(a, a) > 0.0) || !(dot(b, b) > 0.0);
    const bool moll = pm.mollify && dot(n, n) < eps_x(XR, vp, vo, ve0, ve1, pm.epsx_ratio);
    if (!edge) {
        const d3 w = P - E0;
        d2 = dot(w, w);
        return moll ? Staged{FT_PPM, {vp, vo, ve0, ve1}} : Staged{FT_PP, {vp, ve0, -1, -1}};
    }
    double al;
    d2 = seg_dist2(P, E0, E1, al);
    if (al > 0.0 && al < 1.0)
        return moll ? Staged{FT_PEM, {vp, vo, ve0, ve1}} : Staged{FT_PE, {vp, ve0, ve1, -1}};
    const int q = al <= 0.0 ? ve0 : ve1, rr = al <= 0.0 ? ve1 : ve0;
    return moll ? Staged{FT_PPM, {vp, vo, q, rr}} : Staged{FT_PP, {vp, q, -1, -1}};
}

// ------------------------------------------------------------------------
// barrier of Eq. 24, b = dhat^4 (1-g)^2 ln^2 g, or Eq. 12,
// b = -dhat^4 (1-g)^2 ln g, with d/dg and d^2/dg^2

__device__ __forceinline__ void barrier(double g, double dhat, int eq12, double& b, double& db, double& d2b) {
    double s = (dhat * dhat) * (dhat * dhat);
    double L = log(g), u = 1.0 - g, ig = 1.0 / g;
    if (eq12) {
        b = -s * u * u * L;
        db = s * (2.0 * u * L - u * u * ig);
        d2b = s * (-2.0 * L + u * (1.0 + 3.0 * g) * ig * ig);
    } else {
        b = s * u * u * L * L;
        db = 2.0 * s * u * L * (u * ig - L);
        d2b = s * (2.0 * L * L - 8.0 * u * L * ig + 2.0 * u * u * (1.0 - L) * ig * ig);
    }
}

// Projection of the symmetric 2x2 [[A, B], [B, C]] onto its non-negative
// eigenspace (spectral projector; no eigenvector division, stable at ties).
// The entries of the mollified block differ by many orders of magnitude
// (sqrt(c) and f scale J_22 and J_33 very differently), and the small
// eigenvalue is the one that dominates after the change of basis, so both
// eigenvalues are formed without cancellation: the larger-magnitude root as
// m +- disc, the other as det / root, with det = AC - B^2 by Kahan's
// fused difference of products.
__device__ __forceinline__ void psd2(double A, double B, double C, double& P11, double& P12, double& P22) {
    double h = 0.5 * (A - C), m = 0.5 * (A + C);
    double disc = sqrt(h * h + B * B);
    double bb = B * B;
    double det = fma(A, C, -bb) + fma(-B, B, bb);
    double mup, mum;
    if (m >= 0.0) {
        mup = m + disc;
        mum = mup > 0.0 ? det / mup : m - disc;
    } else {
        mum = m - disc;
        mup = det / mum;
    }
    if (mum >= 0.0) {
        P11 = A; P12 = B; P22 = C;
        return;
    }
    if (mup <= 0.0) {
        P11 = P12 = P22 = 0.0;
        return;
    }
    // mup * (M - mum I) / (mup - mum); disc > 0 here
    double am = h + disc, cm = disc - h;
    if (h >= 0.0) cm = B * B / (disc + h);
    else am = B * B / (disc - h);
    double s = mup / (2.0 * disc);
    P11 = s * am;
    P12 = s * B;
    P22 = s * cm;
}

// Compact factors of one evaluated pair.
//   grad f   = (c_k w~)_k,        w~ = w / (dhat d)
//   grad sqrt(c) = (-u, u, -v, v) over slots (v0, v1, v2, v3)   [mollified]
//   gradient = a2 grad f + a1 grad sqrt(c)
//   Hessian  = P22 gf gf^T + P12 (gs gf^T + gf gs^T) + P11 gs gs^T
struct PairFactors {
    double E;
    double c[4];
    d3 wt;
    double P22, a2;
    int moll;
    d3 u, v;
    double P11, P12, a1;
    // the same inner coefficients before projection (kappa included):
    // H22r gf gf^T + H12r (gs gf^T + gf gs^T) + H11r gs gs^T is the proxy
    // Hessian with the unprojected inner Hessian
    double H11r, H12r, H22r;
};

// Stored main record of an evaluated pair, 8 doubles (64 B):
//   [c1, c2, w~x, w~y, w~z, P22, a2, E]
// c0 and c3 follow from the family of the sub-type: the point-first kinds
// (PT, PE, PP) have c0 = 1 and c0 + c1 + c2 + c3 = 0; the edge-edge kinds
// (EE, EEM, PEM, PPM) have c0 + c1 = 1 and c2 + c3 = -1.  The staged order
// puts the edge-edge family last, from the first EE pair on.
// Extra record of a mollified pair, 8 doubles (64 B, one line for the
// gathers of the assembly): [u, v, P11, P12]; its a1 is kept in an array of
// its own, read only by the gradient.
enum RecIdx { R_C1 = 0, R_C2 = 1, R_W = 2, R_P22 = 5, R_A2 = 6, R_E = 7 };

__device__ __forceinline__ double rec_coef(const double* m, int i, bool ee_family) {
    if (i == 1) return m[R_C1];
    if (i == 2) return m[R_C2];
    if (ee_family) return i == 0 ? 1.0 - m[R_C1] : -1.0 - m[R_C2];
    return i == 0 ? 1.0 : -((1.0 + m[R_C1]) + m[R_C2]);
}

__device__ inline void eval_typed(int ft, const int* v, const double* __restrict__ X, const double* __restrict__ XR,
                                  const DevParams& pm, PairFactors& o) {
    o.E = 0.0;
    o.c[0] = o.c[1] = o.c[2] = o.c[3] = 0.0;
    o.wt = mk(0, 0, 0);
    o.P22 = o.a2 = 0.0;
    o.moll = 0;
    o.u = o.v = mk(0, 0, 0);
    o.P11 = o.P12 = o.a1 = 0.0;
    o.H11r = o.H12r = o.H22r = 0.0;
    if (ft == FT_NONE) return;

    d3 w;
    double c0, c1, c2, c3;
    if (ft == FT_PP || ft == FT_PPM) {
        int q = ft == FT_PP ? v[1] : v[2];
        w = ld3(X, v[0]) - ld3(X, q);
        c0 = 1.0;
        if (ft == FT_PP) { c1 = -1.0; c2 = 0.0; }
        else { c1 = 0.0; c2 = -1.0; }
        c3 = 0.0;
    } else if (ft == FT_PE || ft == FT_PEM) {
        int ia = ft == FT_PE ? v[1] : v[2], ib = ft == FT_PE ? v[2] : v[3];
        d3 p = ld3(X, v[0]), e0 = ld3(X, ia), e1 = ld3(X, ib);
        d3 e = e1 - e0, r = p - e0;
        double al = dot(r, e) / dot(e, e);
        w = r - al * e;
        c0 = 1.0;
        if (ft == FT_PE) { c1 = -(1.0 - al); c2 = -al; c3 = 0.0; }
        else { c1 = 0.0; c2 = -(1.0 - al); c3 = -al; }
    } else if (ft == FT_PT) {
        d3 p = ld3(X, v[0]), t0 = ld3(X, v[1]), t1 = ld3(X, v[2]), t2 = ld3(X, v[3]);
        d3 e1 = t1 - t0, e2 = t2 - t0, r = p - t0;
        d3 n = cross(e1, e2);
        double nn = dot(n, n);
        double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2), b1 = dot(e1, r), b2 = dot(e2, r);
        double be1 = (a22 * b1 - a12 * b2) / nn, be2 = (a11 * b2 - a12 * b1) / nn;
        w = (dot(r, n) / nn) * n;
        c0 = 1.0; c1 = -(1.0 - be1 - be2); c2 = -be1; c3 = -be2;
    } else {  // FT_EE, FT_EEM: line-line
        d3 a0 = ld3(X, v[0]), a1 = ld3(X, v[1]), b0 = ld3(X, v[2]), b1 = ld3(X, v[3]);
        d3 a = a1 - a0, b = b1 - b0, r = a0 - b0;
        d3 n = cross(a, b);
        double cc = dot(n, n);
        double aa = dot(a, a), bb = dot(b, b), ab = dot(a, b), ar = dot(a, r), br = dot(b, r);
        double g1 = (ab * br - bb * ar) / cc, g2 = (aa * br - ab * ar) / cc;
        w = (dot(r, n) / cc) * n;
        c0 = 1.0 - g1; c1 = g1; c2 = -(1.0 - g2); c3 = -g2;
    }

    double dhat, kappa;
    scene_params(pm, v[0], dhat, kappa);
    double d2 = dot(w, w);
    if (!(d2 > 0.0) || !(d2 < dhat * dhat)) return;  // inactive or degenerate: no contribution
    double d = sqrt(d2), f = d / dhat, g = d2 / (dhat * dhat);
    double inv = 1.0 / (dhat * d);
    o.c[0] = c0; o.c[1] = c1; o.c[2] = c2; o.c[3] = c3;
    o.wt = inv * w;

    // mollifier (Eq. 25-28)
    double e = 1.0, de = 0.0, d2e = 0.0, cpar = 0.0, sc = 0.0;
    if (ft >= FT_EEM && pm.mollify) {
        d3 A = ld3(X, v[1]) - ld3(X, v[0]), B = ld3(X, v[3]) - ld3(X, v[2]);
        d3 n = cross_acc(A, B);
        cpar = dot(n, n);
        double ex = eps_x(XR, v[0], v[1], v[2], v[3], pm.epsx_ratio);
        if (cpar < ex) {
            o.moll = 1;
            double iex = 1.0 / ex;
            e = cpar * iex * (2.0 - cpar * iex);
            de = 2.0 * iex * (1.0 - cpar * iex);
            d2e = -2.0 * iex * iex;
            sc = sqrt(cpar);
            if (sc > 0.0) {
                double is = 1.0 / sc;
                o.u = is * cross(B, n);
                o.v = is * cross(n, A);
            }
        }
    }

    double b, db, d2b;
    barrier(g, dhat, pm.eq12, b, db, d2b);
    o.E = kappa * e * b;
    o.a2 = 2.0 * kappa * e * db * f;      // d(kappa e b)/df along grad f
    o.a1 = 2.0 * kappa * de * b * sc;     // along grad sqrt(c)

    // proxy Hessian at the filtered Jacobian (Eq. 23)
    double ff = pm.filter ? fmax(f, pm.dthr_ratio) : f;
    double gf = ff * ff;
    double bF, dbF, d2bF;
    barrier(gf, dhat, pm.eq12, bF, dbF, d2bF);
    double lam1 = 2.0 * dbF + 4.0 * gf * d2bF;   // Eq. 18
    if (!o.moll) {
        o.P22 = kappa * fmax(lam1, 0.0);
        o.H22r = kappa * lam1;
    } else {
        double lg1 = 2.0 * (de * bF + 2.0 * cpar * d2e * bF);   // lambda_gamma1
        double lq1 = e * lam1;                                  // lambda_g1
        double t = de * dbF * sc * ff;                          // Eq. 33
        double P11, P12, P22;
        psd2(lg1, 4.0 * t, lq1, P11, P12, P22);
        o.P11 = kappa * P11; o.P12 = kappa * P12; o.P22 = kappa * P22;
        o.H11r = kappa * lg1; o.H12r = kappa * 4.0 * t; o.H22r = kappa * lq1;
    }
}

}  // namespace gipc
