// The gamma search (Algorithm A1 step 4 run as Algorithm A2 step 6, "Kernel 3").
//
// One lane per reference node, in the work order the sort produced.  A wave walks the
// sorted cell table in lockstep: entry n is wave-uniform (one scalar load of a 64-byte
// row), a lane takes part while key_n^2 < gamma^2 of that lane, and the wave leaves the
// walk as soon as no lane does (ballot).  This is the paper's early break, exact because
// the key is a lower bound of every face the cell owns.
//
// Faces.  The Kuhn triangulation splits each cube along its main diagonal; its faces are
// chains q -> q+1_B1 -> q+1_B1+1_B2 -> ... with disjoint non-empty axis blocks B_j.  A
// cell owns the faces anchored at its lower corner q: 1 vertex, 7 edges, 12 triangles and
// 6 tetrahedra in 3D (1, 3, 2 in 2D), so every face of the triangulation is evaluated by
// exactly one cell, and a face owned by cell q lies inside the closed cell q.  Like the
// paper's GPU kernel (Sec. 2.2) every face is evaluated instead of Ju's branching
// recursion.
//
// Projection.  In coordinates relative to the reference node, normalised by DTA and dD,
// a face point is  x_i = s_i (a_i + t_j) for i in B_j  (s_i = h_i / DTA, a = cell offset),
// dose G = g_0 + sum_j t_j Delta_j  (g_k = (D_e(v_k) - D_r) / dD, Delta_j = g_j - g_{j-1}),
// with 1 >= t_1 >= ... >= t_k >= 0.  The Gram matrix of the chain edges is
// diag(sigma_j^2) + Delta Delta^T (sigma_j^2 = sum_{i in B_j} s_i^2), whose inverse is
// closed-form (Sherman-Morrison).  With mu_j = sum_{i in B_j} s_i^2 a_i / sigma_j^2:
//     N = g_0 - sum_j Delta_j mu_j          (value of the face's affine dose at the node)
//     Den = 1 + sum_j Delta_j^2 / sigma_j^2
//     Lambda = N / Den,   t_j = -mu_j - Delta_j Lambda / sigma_j^2
//     dist^2 = perp + N Lambda               (perp: spatial part no t can remove)
// which is the normal-equation solution w = (V^T V)^-1 V^T P of Sec. 2.1 for this edge
// basis; the projection counts when the t_j satisfy the chain inequalities (all
// barycentric weights >= 0).  No residual is formed by subtracting large squares.
#include <cfloat>
#include <type_traits>

#include "internal.hpp"

namespace gammax {

namespace {

constexpr int WAVE = 64;
constexpr int SEARCH_THREADS = 256;

template <typename T>
struct Num;
template <>
struct Num<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
    static __device__ __forceinline__ float min(float a, float b) { return __builtin_fminf(a, b); }
};
template <>
struct Num<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
    static __device__ __forceinline__ double min(double a, double b) { return __builtin_fmin(a, b); }
};

template <typename T>
__device__ __forceinline__ T vmin(T a, T b) { return Num<T>::min(a, b); }

// Fused multiply-add, written out: the projections below form every product-sum they fuse
// explicitly and the compiler contracts nothing else in them (contraction off), so each
// instantiation of a face (masked or not, in any kernel and any lane layout) computes the same
// bits whatever code surrounds it.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One chain step: Delta and w = Delta / sigma^2 (Delta^2 / sigma^2 = Delta w and Delta mu
// enter the sums below as fused products).
template <typename T>
struct Step {
    T d, w;
};
template <typename T>
__device__ __forceinline__ Step<T> mk_step(T hi, T lo, T inv_s2) {
#pragma clang fp contract(off)
    Step<T> s;
    s.d = hi - lo;
    s.w = s.d * inv_s2;
    return s;
}
// N after a step: N - Delta mu; Den after a step: Den + Delta^2 / sigma^2.
template <typename T>
__device__ __forceinline__ T n_step(T n, const Step<T>& s, T mu) { return fmadd(-s.d, mu, n); }
template <typename T>
__device__ __forceinline__ T den_step(T den, const Step<T>& s) { return fmadd(s.d, s.w, den); }
// Chain parameter of a step at Lambda: t = -mu - w Lambda.
template <typename T>
__device__ __forceinline__ T t_step(const Step<T>& s, T mu, T L) { return fmadd(-s.w, L, -mu); }

template <typename T>
__device__ __forceinline__ T face1(T g0, const Step<T>& a, T mua, T perp) {
#pragma clang fp contract(off)
    const T N = n_step(g0, a, mua);
    const T L = N * Num<T>::rcp(den_step(T(1), a));
    const T t1 = t_step(a, mua, L);
    return (t1 >= T(0) && t1 <= T(1)) ? fmadd(N, L, perp) : Num<T>::inf();
}
template <typename T>
__device__ __forceinline__ T face2(T g0, const Step<T>& a, T mua, const Step<T>& b, T mub, T perp) {
#pragma clang fp contract(off)
    const T N = n_step(n_step(g0, a, mua), b, mub);
    const T L = N * Num<T>::rcp(den_step(den_step(T(1), a), b));
    const T t1 = t_step(a, mua, L);
    const T t2 = t_step(b, mub, L);
    return (t1 <= T(1) && t1 >= t2 && t2 >= T(0)) ? fmadd(N, L, perp) : Num<T>::inf();
}
// The denominator of a tetrahedron (its guard measure) on its own.
template <typename T>
__device__ __forceinline__ T den3(const Step<T>& a, const Step<T>& b, const Step<T>& c) {
    return den_step(den_step(den_step(T(1), a), b), c);
}
template <typename T>
__device__ __forceinline__ T face3(T g0, const Step<T>& a, T mua, const Step<T>& b, T mub,
                                   const Step<T>& c, T muc, T& den_out) {
#pragma clang fp contract(off)
    const T N = n_step(n_step(n_step(g0, a, mua), b, mub), c, muc);
    const T den = den3(a, b, c);
    den_out = den;
    const T L = N * Num<T>::rcp(den);
    const T t1 = t_step(a, mua, L);
    const T t2 = t_step(b, mub, L);
    const T t3 = t_step(c, muc, L);
    return (t1 <= T(1) && t1 >= t2 && t2 >= t3 && t3 >= T(0)) ? N * L : Num<T>::inf();
}

// Spatial constants of one cell offset (uniform over the wave).
template <typename T>
struct Geo {
    T ax, ay, az, px, py, pz, vxy, vxz, vyz, vxyz, mxy, mxz, myz, mxyz;
};

__device__ __forceinline__ Geo<float> geo_from_row(const TabEntry& e) {
    Geo<float> g;
    g.ax = (float)e.ax; g.ay = (float)e.ay; g.az = (float)e.az;
    g.px = e.px; g.py = e.py; g.pz = e.pz;
    g.vxy = e.vxy; g.vxz = e.vxz; g.vyz = e.vyz; g.vxyz = e.vxyz;
    g.mxy = e.mxy; g.mxz = e.mxz; g.myz = e.myz; g.mxyz = e.mxyz;
    return g;
}

__device__ __forceinline__ Geo<double> geo_fp64(int iax, int iay, int iaz, double sx2, double sy2,
                                                double sz2) {
    Geo<double> g;
    const double ax = iax, ay = iay, az = iaz;
    g.ax = ax; g.ay = ay; g.az = az;
    g.px = sx2 * ax * ax; g.py = sy2 * ay * ay; g.pz = sz2 * az * az;
    const double dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    g.vxy = sx2 * sy2 * dxy * dxy / (sx2 + sy2);
    g.mxy = (sx2 * ax + sy2 * ay) / (sx2 + sy2);
    if (sz2 > 0.0) {
        const double s = sx2 + sy2 + sz2;
        g.vxz = sx2 * sz2 * dxz * dxz / (sx2 + sz2);
        g.vyz = sy2 * sz2 * dyz * dyz / (sy2 + sz2);
        g.vxyz = (sx2 * sy2 * dxy * dxy + sx2 * sz2 * dxz * dxz + sy2 * sz2 * dyz * dyz) / s;
        g.mxz = (sx2 * ax + sz2 * az) / (sx2 + sz2);
        g.myz = (sy2 * ay + sz2 * az) / (sy2 + sz2);
        g.mxyz = (sx2 * ax + sy2 * ay + sz2 * az) / s;
    } else {
        g.vxz = g.vyz = g.vxyz = g.mxz = g.myz = g.mxyz = 0.0;
    }
    return g;
}

// 1/sigma^2 of the chain blocks x, y, z, xy, xz, yz, xyz.
template <typename T>
struct InvS2 {
    T x, y, z, xy, xz, yz, xyz;
};
template <typename T>
__device__ __forceinline__ InvS2<T> inv_s2(T sx2, T sy2, T sz2) {
    InvS2<T> r;
    r.x = T(1) / sx2;
    r.y = T(1) / sy2;
    r.z = sz2 > T(0) ? T(1) / sz2 : T(0);
    r.xy = T(1) / (sx2 + sy2);
    r.xz = sz2 > T(0) ? T(1) / (sx2 + sz2) : T(0);
    r.yz = sz2 > T(0) ? T(1) / (sy2 + sz2) : T(0);
    r.xyz = T(1) / (sx2 + sy2 + sz2);
    return r;
}

// The FP32 reciprocals as the host formed them for the search arguments (the same IEEE
// divisions as inv_s2<float>, once per map instead of once per lane).
__device__ __forceinline__ InvS2<float> inv_s2_of(const SearchArgs& a) {
    InvS2<float> r;
    r.x = a.inv_s2[0];
    r.y = a.inv_s2[1];
    r.z = a.inv_s2[2];
    r.xy = a.inv_s2[3];
    r.xz = a.inv_s2[4];
    r.yz = a.inv_s2[5];
    r.xyz = a.inv_s2[6];
    return r;
}

// Tetrahedron of a 3D cell redone in FP64 (the precision guard).  The four corner doses
// are re-read from memory so that the common FP32 path keeps no extra registers alive.
// perm: 0 xyz, 1 xzy, 2 yxz, 3 yzx, 4 zxy, 5 zyx (order in which the axes are stepped).
struct GuardCtx {
    const float* ev;
    int base, ox, oy, oz;
    float dr;
    double inv_dd;
    int ax, ay, az;
    double sx2, sy2, sz2;
};

template <typename V>
__device__ __forceinline__ V pick3(int i, V x, V y, V z) {
    return i == 0 ? x : (i == 1 ? y : z);
}

__device__ __forceinline__ double tet_fp64(const GuardCtx& c, int perm) {
    // perm -> stepping order: first axis perm/2, then the other two ascending (even perm)
    // or descending (odd perm)
    const int first = perm >> 1;
    int r0 = first == 0 ? 1 : 0, r1 = first == 2 ? 1 : 2;
    if (perm & 1) {
        const int t = r0;
        r0 = r1;
        r1 = t;
    }
    const double dr = (double)c.dr;
    int idx = c.base;
    double gprev = ((double)c.ev[idx] - dr) * c.inv_dd;
    double N = gprev, den = 1.0;
    double tw0 = 0.0, tw1 = 0.0, tw2 = 0.0, mu0 = 0.0, mu1 = 0.0, mu2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int ax = j == 0 ? first : (j == 1 ? r0 : r1);
        idx += pick3(ax, c.ox, c.oy, c.oz);
        const double s2 = pick3(ax, c.sx2, c.sy2, c.sz2);
        const double aa = (double)pick3(ax, c.ax, c.ay, c.az);
        const double gnext = ((double)c.ev[idx] - dr) * c.inv_dd;
        const double d = gnext - gprev;
        N -= d * aa;
        den += d * d / s2;
        const double tw = d / s2;
        if (j == 0) { tw0 = tw; mu0 = aa; }
        if (j == 1) { tw1 = tw; mu1 = aa; }
        if (j == 2) { tw2 = tw; mu2 = aa; }
        gprev = gnext;
    }
    const double L = N / den;
    const double t1 = -mu0 - tw0 * L, t2 = -mu1 - tw1 * L, t3 = -mu2 - tw2 * L;
    return (t1 <= 1.0 && t1 >= t2 && t2 >= t3 && t3 >= 0.0) ? N * L : __builtin_huge_val();
}

// Normalised dose difference of a cell vertex, rounded as its own product: the walks of
// every tail layout feed the projections the same values, whatever the compiler fuses
// around them.
template <typename T>
__device__ __forceinline__ T dose_norm(T v, T dr, T inv) {
#pragma clang fp contract(off)
    return (v - dr) * inv;
}

// Whether any of the six tetrahedra of a 3D cell has a normal-equation denominator above
// den_guard: the test cell3 applies (GMODE 1), with its chain steps and its summation order.
__device__ __forceinline__ bool tets_ill(const float* g, const InvS2<float>& is, float den_guard) {
#pragma clang fp contract(off)
    const Step<float> s0x = mk_step(g[1], g[0], is.x), s0y = mk_step(g[2], g[0], is.y);
    const Step<float> s0z = mk_step(g[4], g[0], is.z);
    const Step<float> s1y = mk_step(g[3], g[1], is.y), s1z = mk_step(g[5], g[1], is.z);
    const Step<float> s2x = mk_step(g[3], g[2], is.x), s2z = mk_step(g[6], g[2], is.z);
    const Step<float> s4x = mk_step(g[5], g[4], is.x), s4y = mk_step(g[6], g[4], is.y);
    const Step<float> s3z = mk_step(g[7], g[3], is.z), s5y = mk_step(g[7], g[5], is.y);
    const Step<float> s6x = mk_step(g[7], g[6], is.x);
    bool ill = den3(s0x, s1y, s3z) > den_guard;
    ill = ill || den3(s0x, s1z, s5y) > den_guard;
    ill = ill || den3(s0y, s2x, s3z) > den_guard;
    ill = ill || den3(s0y, s2z, s6x) > den_guard;
    ill = ill || den3(s0z, s4x, s5y) > den_guard;
    ill = ill || den3(s0z, s4y, s6x) > den_guard;
    return ill;
}

// All faces owned by one 3D cell; returns the smallest dist^2 (or +inf).
// ok_*: the cell extends along that axis inside the grid (MASKED only).
// GMODE 0: no guard; 1: flag an ill-conditioned tetrahedron (ill = true); 2: project it
// again in FP64.
template <typename T, bool MASKED, int GMODE>
__device__ __forceinline__ T cell3(const T* g, const Geo<T>& G, const InvS2<T>& is, bool okx, bool oky,
                                   bool okz, T den_guard, const GuardCtx& gc, uint32_t& n_fp64,
                                   bool& ill) {
#pragma clang fp contract(off)
    const T INF = Num<T>::inf();
    const T g0 = g[0];
    // chain steps, named by start vertex bits and block (x = bit0, y = bit1, z = bit2)
    const Step<T> s0x = mk_step(g[1], g[0], is.x);
    const Step<T> s0y = mk_step(g[2], g[0], is.y);
    const Step<T> s0z = mk_step(g[4], g[0], is.z);
    const Step<T> s0xy = mk_step(g[3], g[0], is.xy);
    const Step<T> s0xz = mk_step(g[5], g[0], is.xz);
    const Step<T> s0yz = mk_step(g[6], g[0], is.yz);
    const Step<T> s0xyz = mk_step(g[7], g[0], is.xyz);
    const Step<T> s1y = mk_step(g[3], g[1], is.y);
    const Step<T> s1z = mk_step(g[5], g[1], is.z);
    const Step<T> s1yz = mk_step(g[7], g[1], is.yz);
    const Step<T> s2x = mk_step(g[3], g[2], is.x);
    const Step<T> s2z = mk_step(g[6], g[2], is.z);
    const Step<T> s2xz = mk_step(g[7], g[2], is.xz);
    const Step<T> s4x = mk_step(g[5], g[4], is.x);
    const Step<T> s4y = mk_step(g[6], g[4], is.y);
    const Step<T> s4xy = mk_step(g[7], g[4], is.xy);
    const Step<T> s3z = mk_step(g[7], g[3], is.z);
    const Step<T> s5y = mk_step(g[7], g[5], is.y);
    const Step<T> s6x = mk_step(g[7], g[6], is.x);
    // vertex q
    T best = fmadd(g0, g0, (G.px + G.py) + G.pz);
    // edges
    T e;
    e = face1(g0, s0x, G.ax, G.py + G.pz);
    best = vmin<T>(best, (!MASKED || okx) ? e : INF);
    e = face1(g0, s0y, G.ay, G.px + G.pz);
    best = vmin<T>(best, (!MASKED || oky) ? e : INF);
    e = face1(g0, s0z, G.az, G.px + G.py);
    best = vmin<T>(best, (!MASKED || okz) ? e : INF);
    e = face1(g0, s0xy, G.mxy, G.pz + G.vxy);
    best = vmin<T>(best, (!MASKED || (okx && oky)) ? e : INF);
    e = face1(g0, s0xz, G.mxz, G.py + G.vxz);
    best = vmin<T>(best, (!MASKED || (okx && okz)) ? e : INF);
    e = face1(g0, s0yz, G.myz, G.px + G.vyz);
    best = vmin<T>(best, (!MASKED || (oky && okz)) ? e : INF);
    const bool all = !MASKED || (okx && oky && okz);
    e = face1(g0, s0xyz, G.mxyz, G.vxyz);
    best = vmin<T>(best, all ? e : INF);
    // triangles in the cube faces through q
    T tri = vmin<T>(face2(g0, s0x, G.ax, s1y, G.ay, G.pz), face2(g0, s0y, G.ay, s2x, G.ax, G.pz));
    best = vmin<T>(best, (!MASKED || (okx && oky)) ? tri : INF);
    tri = vmin<T>(face2(g0, s0x, G.ax, s1z, G.az, G.py), face2(g0, s0z, G.az, s4x, G.ax, G.py));
    best = vmin<T>(best, (!MASKED || (okx && okz)) ? tri : INF);
    tri = vmin<T>(face2(g0, s0y, G.ay, s2z, G.az, G.px), face2(g0, s0z, G.az, s4y, G.ay, G.px));
    best = vmin<T>(best, (!MASKED || (oky && okz)) ? tri : INF);
    // triangles through the main diagonal
    T diag = vmin<T>(face2(g0, s0x, G.ax, s1yz, G.myz, G.vyz), face2(g0, s0yz, G.myz, s6x, G.ax, G.vyz));
    diag = vmin<T>(diag, vmin<T>(face2(g0, s0y, G.ay, s2xz, G.mxz, G.vxz), face2(g0, s0xz, G.mxz, s5y, G.ay, G.vxz)));
    diag = vmin<T>(diag, vmin<T>(face2(g0, s0z, G.az, s4xy, G.mxy, G.vxy), face2(g0, s0xy, G.mxy, s3z, G.az, G.vxy)));
    // tetrahedra
    T den[6], tv[6];
    tv[0] = face3(g0, s0x, G.ax, s1y, G.ay, s3z, G.az, den[0]);
    tv[1] = face3(g0, s0x, G.ax, s1z, G.az, s5y, G.ay, den[1]);
    tv[2] = face3(g0, s0y, G.ay, s2x, G.ax, s3z, G.az, den[2]);
    tv[3] = face3(g0, s0y, G.ay, s2z, G.az, s6x, G.ax, den[3]);
    tv[4] = face3(g0, s0z, G.az, s4x, G.ax, s5y, G.ay, den[4]);
    tv[5] = face3(g0, s0z, G.az, s4y, G.ay, s6x, G.ax, den[5]);
    uint32_t gmask = 0u;
    if (GMODE != 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) gmask |= (den[k] > den_guard) ? (1u << k) : 0u;
    }
    if (GMODE == 1) ill = ill || (all && gmask != 0u);
    if (GMODE == 2) {
#pragma unroll
        for (int k = 0; k < 6; ++k) tv[k] = ((gmask >> k) & 1u) ? INF : tv[k];
    }
    T tet = vmin<T>(vmin<T>(vmin<T>(tv[0], tv[1]), vmin<T>(tv[2], tv[3])), vmin<T>(tv[4], tv[5]));
    if (GMODE == 2 && all && gmask) {
        // rare: ill-conditioned tetrahedra are projected again in FP64
#pragma nounroll
        for (int k = 0; k < 6; ++k) {
            if ((gmask >> k) & 1u) {
                tet = vmin<T>(tet, (T)tet_fp64(gc, k));
                ++n_fp64;
            }
        }
    }
    diag = vmin<T>(diag, tet);
    best = vmin<T>(best, all ? diag : INF);
    return best;
}


// ---- Ju et al.'s recursion (Sec. 2.1: the branching form of the A1 distance) -------------
//
// The same closed-form chain projections as cell3, organised as the recursion of the
// sequential algorithm: each of the six Kuhn tetrahedra of a cell is projected first, and
// only where a barycentric weight is negative are the facets opposite those vertices
// projected, then their edges, then vertices.  It covers every face of the cell (not only
// the faces the cell owns), so it serves interior cells; cells at the grid faces keep
// cell3.  A chain starts at cube vertex U (bit i: +1 along axis i, x = bit 0) and steps
// through disjoint axis blocks S1, S2, ... that do not meet U.
struct JuCell {
    float g[8];
    float a[3], p[3], p1[3];   // per axis: offset, s^2 a^2, s^2 (a + 1)^2
    Geo<float> G;
    InvS2<float> is;
};
template <int S>
__device__ __forceinline__ float ju_mu(const JuCell& K) {
    static_assert(S >= 1 && S <= 7, "block");
    if constexpr (S == 1) return K.a[0];
    else if constexpr (S == 2) return K.a[1];
    else if constexpr (S == 4) return K.a[2];
    else if constexpr (S == 3) return K.G.mxy;
    else if constexpr (S == 5) return K.G.mxz;
    else if constexpr (S == 6) return K.G.myz;
    else return K.G.mxyz;
}
template <int S>
__device__ __forceinline__ float ju_inv(const JuCell& K) {
    if constexpr (S == 1) return K.is.x;
    else if constexpr (S == 2) return K.is.y;
    else if constexpr (S == 4) return K.is.z;
    else if constexpr (S == 3) return K.is.xy;
    else if constexpr (S == 5) return K.is.xz;
    else if constexpr (S == 6) return K.is.yz;
    else return K.is.xyz;
}
template <int S>
__device__ __forceinline__ float ju_res(const JuCell& K) {
    if constexpr (S == 1 || S == 2 || S == 4) return 0.0f;
    else if constexpr (S == 3) return K.G.vxy;
    else if constexpr (S == 5) return K.G.vxz;
    else if constexpr (S == 6) return K.G.vyz;
    else return K.G.vxyz;
}
// sum of the squared spatial components of vertex U over the axes outside mask S
template <int U, int S>
__device__ __forceinline__ float ju_perp(const JuCell& K) {
    float r = 0.0f;
    if constexpr (!(S & 1)) r += (U & 1) ? K.p1[0] : K.p[0];
    if constexpr (!(S & 2)) r += (U & 2) ? K.p1[1] : K.p[1];
    if constexpr (!(S & 4)) r += (U & 4) ? K.p1[2] : K.p[2];
    return r;
}
template <int U>
__device__ __forceinline__ float ju_vertex(const JuCell& K) {
#pragma clang fp contract(off)
    return fmadd(K.g[U], K.g[U], ju_perp<U, 0>(K));
}
template <int U, int S>
__device__ __forceinline__ Step<float> ju_step(const JuCell& K) {
    static_assert((U & S) == 0, "a chain steps away from its start");
    return mk_step(K.g[U | S], K.g[U], ju_inv<S>(K));
}
// edge from U along block S
template <int U, int S>
__device__ __forceinline__ float ju_edge(const JuCell& K) {
#pragma clang fp contract(off)
    const Step<float> a = ju_step<U, S>(K);
    const float N = n_step(K.g[U], a, ju_mu<S>(K));
    const float L = N * Num<float>::rcp(den_step(1.0f, a));
    const float t = t_step(a, ju_mu<S>(K), L);
    if (t >= 0.0f && t <= 1.0f) return fmadd(N, L, ju_perp<U, S>(K) + ju_res<S>(K));
    return t < 0.0f ? ju_vertex<U>(K) : ju_vertex<U | S>(K);
}
// triangle from U through blocks S1 then S2
template <int U, int S1, int S2>
__device__ __forceinline__ float ju_tri(const JuCell& K) {
#pragma clang fp contract(off)
    const Step<float> a = ju_step<U, S1>(K);
    const Step<float> b = ju_step<U | S1, S2>(K);
    const float N = n_step(n_step(K.g[U], a, ju_mu<S1>(K)), b, ju_mu<S2>(K));
    const float L = N * Num<float>::rcp(den_step(den_step(1.0f, a), b));
    const float t1 = t_step(a, ju_mu<S1>(K), L);
    const float t2 = t_step(b, ju_mu<S2>(K), L);
    const float w0 = 1.0f - t1, w1 = t1 - t2, w2 = t2;
    if (w0 >= 0.0f && w1 >= 0.0f && w2 >= 0.0f)
        return fmadd(N, L, (ju_perp<U, S1 | S2>(K) + ju_res<S1>(K)) + ju_res<S2>(K));
    float best = Num<float>::inf();
    if (w0 < 0.0f) best = vmin<float>(best, ju_edge<U | S1, S2>(K));
    if (w1 < 0.0f) best = vmin<float>(best, ju_edge<U, S1 | S2>(K));
    if (w2 < 0.0f) best = vmin<float>(best, ju_edge<U, S1>(K));
    return best;
}
// tetrahedron v0 -> A -> A+B -> A+B+C (axis masks A, B, C); den: its normal-equation
// denominator (the guard's measure)
template <int A, int B, int C>
__device__ __forceinline__ float ju_tet(const JuCell& K, float& den) {
#pragma clang fp contract(off)
    const Step<float> a = ju_step<0, A>(K);
    const Step<float> b = ju_step<A, B>(K);
    const Step<float> c = ju_step<A | B, C>(K);
    const float N = n_step(n_step(n_step(K.g[0], a, ju_mu<A>(K)), b, ju_mu<B>(K)), c, ju_mu<C>(K));
    den = den3(a, b, c);
    const float L = N * Num<float>::rcp(den);
    const float t1 = t_step(a, ju_mu<A>(K), L);
    const float t2 = t_step(b, ju_mu<B>(K), L);
    const float t3 = t_step(c, ju_mu<C>(K), L);
    const float w0 = 1.0f - t1, w1 = t1 - t2, w2 = t2 - t3, w3 = t3;
    if (w0 >= 0.0f && w1 >= 0.0f && w2 >= 0.0f && w3 >= 0.0f) return N * L;
    float best = Num<float>::inf();
    if (w0 < 0.0f) best = vmin<float>(best, ju_tri<A, B, C>(K));          // drop v0
    if (w1 < 0.0f) best = vmin<float>(best, ju_tri<0, A | B, C>(K));      // drop v0+A
    if (w2 < 0.0f) best = vmin<float>(best, ju_tri<0, A, B | C>(K));      // drop v0+A+B
    if (w3 < 0.0f) best = vmin<float>(best, ju_tri<0, A, B>(K));          // drop v0+A+B+C
    return best;
}
// Interior 3D cell by Ju's recursion: the smallest dist^2 over its six tetrahedra.
// GMODE 1 flags a tetrahedron whose denominator exceeds den_guard (as cell3 does).
template <int GMODE>
__device__ __forceinline__ float cell3_ju(const float* g, const Geo<float>& G, const InvS2<float>& is, float s2x,
                                          float s2y, float s2z, float den_guard, bool& ill) {
    JuCell K;
#pragma unroll
    for (int b = 0; b < 8; ++b) K.g[b] = g[b];
    K.a[0] = G.ax;
    K.a[1] = G.ay;
    K.a[2] = G.az;
    K.p[0] = G.px;
    K.p[1] = G.py;
    K.p[2] = G.pz;
    K.p1[0] = s2x * (G.ax + 1.0f) * (G.ax + 1.0f);
    K.p1[1] = s2y * (G.ay + 1.0f) * (G.ay + 1.0f);
    K.p1[2] = s2z * (G.az + 1.0f) * (G.az + 1.0f);
    K.G = G;
    K.is = is;
    float den = 0.0f;
    bool flag = false;
    float best = ju_tet<1, 2, 4>(K, den);
    flag = flag || den > den_guard;
    best = vmin<float>(best, ju_tet<1, 4, 2>(K, den));
    flag = flag || den > den_guard;
    best = vmin<float>(best, ju_tet<2, 1, 4>(K, den));
    flag = flag || den > den_guard;
    best = vmin<float>(best, ju_tet<2, 4, 1>(K, den));
    flag = flag || den > den_guard;
    best = vmin<float>(best, ju_tet<4, 1, 2>(K, den));
    flag = flag || den > den_guard;
    best = vmin<float>(best, ju_tet<4, 2, 1>(K, den));
    flag = flag || den > den_guard;
    if constexpr (GMODE == 1) ill = ill || flag;
    return best;
}

template <typename T, bool MASKED>
__device__ __forceinline__ T cell2(const T* g, const Geo<T>& G, const InvS2<T>& is, bool okx, bool oky) {
#pragma clang fp contract(off)
    const T INF = Num<T>::inf();
    const T g0 = g[0];
    const Step<T> s0x = mk_step(g[1], g[0], is.x);
    const Step<T> s0y = mk_step(g[2], g[0], is.y);
    const Step<T> s0xy = mk_step(g[3], g[0], is.xy);
    const Step<T> s1y = mk_step(g[3], g[1], is.y);
    const Step<T> s2x = mk_step(g[3], g[2], is.x);
    T best = fmadd(g0, g0, G.px + G.py);
    T e = face1(g0, s0x, G.ax, G.py);
    best = vmin<T>(best, (!MASKED || okx) ? e : INF);
    e = face1(g0, s0y, G.ay, G.px);
    best = vmin<T>(best, (!MASKED || oky) ? e : INF);
    const bool both = !MASKED || (okx && oky);
    e = face1(g0, s0xy, G.mxy, G.vxy);
    e = vmin<T>(e, face2(g0, s0x, G.ax, s1y, G.ay, T(0)));
    e = vmin<T>(e, face2(g0, s0y, G.ay, s2x, G.ax, T(0)));
    best = vmin<T>(best, both ? e : INF);
    return best;
}

// ---------------------------------------------------------------------------------------
// Work passes.
//
// Pass A (zero-key cells, all M nodes in grid order): the 2^d cells with key 0 surround
// every node, so every lane runs the same work and neighbouring lanes read neighbouring
// doses.  The 3^d dose neighbourhood is loaded once (all loads issued before the first
// use) and shared by the 2^d cells.  A node whose bound after these cells is <= the next
// key^2 is finished (the walk would break there); the others are queued for pass B.
//
// Pass B (tail): the queued nodes, sorted by the chosen key (the paper's DD sort:
// gamma0; or the bound after pass A), walk the table from the first non-zero key in
// wave lockstep.
//
// Guard pass (guarded precision): nodes that met an ill-conditioned tetrahedron in A or
// B are redone from the start with those tetrahedra projected in FP64.
// ---------------------------------------------------------------------------------------

// Per-block reduction of the counts, added into one of SUM_BINS partial slots (blocks
// spread over the slots, so no address sees more than a few hundred atomics).
// bins == nullptr: add straight into the map's scalars (`direct`).
__device__ __forceinline__ void block_sums(BlockSums* bins, uint32_t vb, uint32_t npass, uint32_t nborder,
                                           uint32_t nfp64, uint32_t ncells, uint32_t gm,
                                           Scalars* direct = nullptr) {
    __shared__ uint32_t s[5][SEARCH_THREADS / WAVE];
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        npass += (uint32_t)__shfl_xor((int)npass, o);
        nborder += (uint32_t)__shfl_xor((int)nborder, o);
        nfp64 += (uint32_t)__shfl_xor((int)nfp64, o);
        ncells += (uint32_t)__shfl_xor((int)ncells, o);
        gm = max(gm, (uint32_t)__shfl_xor((int)gm, o));
    }
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s[0][w] = npass;
        s[1][w] = nborder;
        s[2][w] = nfp64;
        s[3][w] = ncells;
        s[4][w] = gm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long p = 0, b = 0, f = 0, c = 0;
        uint32_t m = 0;
        for (int j = 0; j < SEARCH_THREADS / WAVE; ++j) {
            p += s[0][j];
            b += s[1][j];
            f += s[2][j];
            c += s[3][j];
            m = max(m, s[4][j]);
        }
        if (bins) {
            BlockSums* out = &bins[vb & (SUM_BINS - 1)];
            if (p) atomicAdd(&out->pass, p);
            if (b) atomicAdd(&out->border, b);
            if (f) atomicAdd(&out->fp64, f);
            if (c) atomicAdd(&out->cells, c);
            if (m) atomicMax(&out->maxg2, m);
        } else {
            if (p) atomicAdd(&direct->n_pass, p);
            if (b) atomicAdd(&direct->n_border, b);
            if (f) atomicAdd(&direct->n_fp64, f);
            if (c) atomicAdd(&direct->n_cells, c);
            if (m) atomicMax(&direct->maxg2_bits, m);
        }
    }
}

// Block-aggregated append to a device list: one atomic per block.  Returns the slot of
// this lane (valid where `want`).  All threads of the block must call it.
__device__ __forceinline__ uint32_t block_append(bool want, uint32_t* counter) {
    __shared__ uint32_t s_cnt[SEARCH_THREADS / WAVE];
    __shared__ uint32_t s_base;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const unsigned long long bal = __ballot(want);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    if (lane == 0) s_cnt[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0u;
        for (int j = 0; j < SEARCH_THREADS / WAVE; ++j) tot += s_cnt[j];
        s_base = tot ? atomicAdd(counter, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = s_base;
    for (int j = 0; j < w; ++j) off += s_cnt[j];
    __syncthreads();   // s_cnt/s_base may be reused by the next call
    return off + (uint32_t)__popcll(bal & lt);
}

// Finished node: write gamma, update the per-lane counts.
__device__ __forceinline__ void finish_node(const SearchArgs& a, int node, float F, uint32_t& npass,
                                            uint32_t& nborder, uint32_t& gm) {
    const float gam = sqrtf(F);
    a.gamma[node] = gam;
    npass += gam <= 1.0f;
    nborder += fabsf(gam - 1.0f) <= 1e-5f;
    gm = max(gm, f2u(gam * gam));
}

// Learned radius.  gamma_hat = max(exp(y) - 0.01, 0) from the CNN output y of a tail item;
// the speculative walk takes the bound min(gamma^2, (f * gamma_hat)^2).  The same float
// expression serves the speculative walk and the fallback, so both see the same bound.
__device__ __forceinline__ float pred_gamma(const SearchArgs& a, uint32_t item) {
    return fmaxf(expf(a.yhat[item]) - 0.01f, 0.0f);
}
__device__ __forceinline__ float spec_bound2(const SearchArgs& a, uint32_t item) {
    const float r = a.spec_factor * pred_gamma(a, item);
    return r * r;
}
// Sort key of a queued tail node: gamma0^2 (DD sort) or the bound after the key-0 cells
// (non-negative floats: bit order = numeric order).  The predicted order's keys are
// written afterwards by the network at the tail nodes.
__device__ __forceinline__ uint32_t tail_sort_key(const SearchArgs& a, int node, float F0, float F) {
    (void)node;
    return a.tail_key == 1 ? f2u(F) : f2u(F0);
}
// First table row with key^2 >= r2 (rows are in ascending key order), at least `first`.
// Rows before it either were evaluated by the speculative walk or could not improve it.
__device__ __forceinline__ int resume_row(const TabEntry* tab, int n, int first, float r2) {
    int lo = first, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid].key2 < r2) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Pass A in 3D.  MODE 0: FP32; MODE 1: FP32 and flag ill-conditioned tetrahedra.
// vb: the block's index in the node list (256 nodes each).
template <int MODE, bool JU = false>
__device__ __forceinline__ void zero3_body(const SearchArgs& a, const ZeroGeo& zg, BlockSums* sums, uint32_t vb) {
    constexpr int GMODE = MODE == 1 ? 1 : 0;
    const uint32_t M = a.sc->n_masked;
    if (vb * SEARCH_THREADS >= M) {   // grids are sized for every grid node; M is on the device
        return;
    }
    const uint32_t i = vb * SEARCH_THREADS + threadIdx.x;
    const bool live = i < M;
    const int nx = a.nx, ny = a.ny, nz = a.nz, sxy = nx * ny;
    const int node = live ? (int)a.nodes[i] : 0;
    const int x = node % nx, y = (node / nx) % ny, z = node / sxy;
    const float dr = a.ref[node];
    const float inv_dd = node_inv_dd(dr, a.sc->inv_dd, a.dd, a.local);
    const float F0 = live ? gamma0_sq(a.ev[node], dr, inv_dd) : 0.0f;
    // neighbourhood offsets, clamped at the grid faces (clamped values feed only cells
    // that do not exist or faces that are masked out)
    const int oxm = x > 0 ? -1 : 0, oxp = x + 1 < nx ? 1 : 0;
    const int oym = y > 0 ? -nx : 0, oyp = y + 1 < ny ? nx : 0;
    const int ozm = z > 0 ? -sxy : 0, ozp = z + 1 < nz ? sxy : 0;
    const int ox[3] = {oxm, 0, oxp}, oy[3] = {oym, 0, oyp}, oz[3] = {ozm, 0, ozp};
    float g27[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) g27[k] = a.ev[node + oz[k / 9] + oy[(k / 3) % 3] + ox[k % 3]];
#pragma unroll
    for (int k = 0; k < 27; ++k) g27[k] = (g27[k] - dr) * inv_dd;

    const InvS2<float> is = inv_s2_of(a);
    const bool bnd = x == 0 || x + 1 == nx || y == 0 || y + 1 == ny || z == 0 || z + 1 == nz;
    const bool wave_masked = __ballot(live && bnd) != 0ull;
    float F = F0;
    uint32_t cells = 0, n_fp64 = 0;
    bool ill = false;
    GuardCtx gc{};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        // table order of the zero-key cells: (az, ay, ax) in {-1,0}^3, lexicographic
        const int az = (c >> 2) - 1, ay = ((c >> 1) & 1) - 1, ax = (c & 1) - 1;
        float g[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            g[b] = g27[(az + 1 + ((b >> 2) & 1)) * 9 + (ay + 1 + ((b >> 1) & 1)) * 3 + (ax + 1 + (b & 1))];
        const Geo<float> G = geo_from_row(zg.row[c]);
        float v;
        if (wave_masked) {
            const bool exists = (ax == 0 || x > 0) && (ay == 0 || y > 0) && (az == 0 || z > 0);
            const bool okx = ax < 0 || x + 1 < nx, oky = ay < 0 || y + 1 < ny, okz = az < 0 || z + 1 < nz;
            v = cell3<float, true, GMODE>(g, G, is, okx, oky, okz, a.den_guard, gc, n_fp64, ill);
            v = exists ? v : Num<float>::inf();
            cells += (F > 0.0f && exists && okx && oky && okz) ? 1u : 0u;
        } else {
            if constexpr (JU)
                v = cell3_ju<GMODE>(g, G, is, a.s2x, a.s2y, a.s2z, a.den_guard, ill);
            else
                v = cell3<float, false, GMODE>(g, G, is, true, true, true, a.den_guard, gc, n_fp64, ill);
            cells += F > 0.0f ? 1u : 0u;
        }
        F = F0 > 0.0f ? vmin<float>(F, v) : F;
    }
    ill = ill && live && F0 > 0.0f;
    const bool to_guard = MODE == 1 && ill;
    const bool to_tail = live && !to_guard && F > a.k1;
    uint32_t npass = 0, nborder = 0, gm = 0, ncells = 0;
    if (live && !to_guard && !to_tail) {
        finish_node(a, node, F, npass, nborder, gm);
        ncells = cells;
    }
    // queue the tail (one atomic per block), then the guard list
    const uint32_t pos = block_append(to_tail, &a.sc->n_tail);
    if (to_tail) {
        a.tail_node[pos] = (uint32_t)node;
        a.tail_f[pos] = f2u(F);
        a.tail_key_arr[pos] = tail_sort_key(a, node, F0, F);
        a.tail_pos[pos] = pos;
    }
    if (MODE == 1) {
        const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
        if (to_guard) a.guard_list[gpos] = (uint32_t)node;
    }
    block_sums(sums, vb, npass, nborder, 0u, ncells, gm);
}

template <int MODE, bool JU = false>
__global__ __launch_bounds__(SEARCH_THREADS) void k_zero3(SearchArgs a, ZeroGeo zg, BlockSums* sums) {
    zero3_body<MODE, JU>(a, zg, sums, blockIdx.x);
}

// Pass A in 2D (4 zero-key cells, 3x3 neighbourhood).
__device__ __forceinline__ void zero2_body(const SearchArgs& a, const ZeroGeo& zg, BlockSums* sums, uint32_t vb) {
    const uint32_t M = a.sc->n_masked;
    if (vb * SEARCH_THREADS >= M) {
        return;
    }
    const uint32_t i = vb * SEARCH_THREADS + threadIdx.x;
    const bool live = i < M;
    const int nx = a.nx, ny = a.ny;
    const int node = live ? (int)a.nodes[i] : 0;
    const int x = node % nx, y = node / nx;
    const float dr = a.ref[node];
    const float inv_dd = node_inv_dd(dr, a.sc->inv_dd, a.dd, a.local);
    const float F0 = live ? gamma0_sq(a.ev[node], dr, inv_dd) : 0.0f;
    const int ox[3] = {x > 0 ? -1 : 0, 0, x + 1 < nx ? 1 : 0};
    const int oy[3] = {y > 0 ? -nx : 0, 0, y + 1 < ny ? nx : 0};
    float g9[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) g9[k] = a.ev[node + oy[k / 3] + ox[k % 3]];
#pragma unroll
    for (int k = 0; k < 9; ++k) g9[k] = (g9[k] - dr) * inv_dd;
    const InvS2<float> is = inv_s2_of(a);
    const bool bnd = x == 0 || x + 1 == nx || y == 0 || y + 1 == ny;
    const bool wave_masked = __ballot(live && bnd) != 0ull;
    float F = F0;
    uint32_t cells = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int ay = (c >> 1) - 1, ax = (c & 1) - 1;
        float g[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) g[b] = g9[(ay + 1 + ((b >> 1) & 1)) * 3 + (ax + 1 + (b & 1))];
        const Geo<float> G = geo_from_row(zg.row[c]);
        float v;
        if (wave_masked) {
            const bool exists = (ax == 0 || x > 0) && (ay == 0 || y > 0);
            const bool okx = ax < 0 || x + 1 < nx, oky = ay < 0 || y + 1 < ny;
            v = cell2<float, true>(g, G, is, okx, oky);
            v = exists ? v : Num<float>::inf();
            cells += (F > 0.0f && exists && okx && oky) ? 1u : 0u;
        } else {
            v = cell2<float, false>(g, G, is, true, true);
            cells += F > 0.0f ? 1u : 0u;
        }
        F = F0 > 0.0f ? vmin<float>(F, v) : F;
    }
    const bool to_tail = live && F > a.k1;
    uint32_t npass = 0, nborder = 0, gm = 0, ncells = 0;
    if (live && !to_tail) {
        finish_node(a, node, F, npass, nborder, gm);
        ncells = cells;
    }
    const uint32_t pos = block_append(to_tail, &a.sc->n_tail);
    if (to_tail) {
        a.tail_node[pos] = (uint32_t)node;
        a.tail_f[pos] = f2u(F);
        a.tail_key_arr[pos] = tail_sort_key(a, node, F0, F);
        a.tail_pos[pos] = pos;
    }
    block_sums(sums, vb, npass, nborder, 0u, ncells, gm);
}

template <int MODE>
__global__ __launch_bounds__(SEARCH_THREADS) void k_zero2(SearchArgs a, ZeroGeo zg, BlockSums* sums) {
    zero2_body(a, zg, sums, blockIdx.x);
    (void)MODE;
}

// Full cells among the zero-key cells of a node (every one is evaluated for a tail node).
__device__ __forceinline__ uint32_t zero_cells(int DIM, int x, int y, int z, int nx, int ny, int nz) {
    const uint32_t cx = (x > 0) + (x + 1 < nx), cy = (y > 0) + (y + 1 < ny);
    const uint32_t cz = DIM == 3 ? (uint32_t)((z > 0) + (z + 1 < nz)) : 1u;
    return cx * cy * cz;
}

// Pass A with one lane per cell: the 2^d lanes of a group share one node (grid order) and
// each takes one of its zero-key cells (table rows 0 .. 2^d-1), then the group takes the
// minimum with shuffles.  Lighter waves than one lane per node (more of them resident, no
// wave-quantisation tail).  Grid-stride over the nodes; MODE 0: FP32, 1: FP32 + flag.
template <int DIM, int MODE>
__global__ __launch_bounds__(SEARCH_THREADS) void k_zero_group(SearchArgs a, ZeroGeo zg, BlockSums* sums) {
    constexpr int G = 1 << DIM;
    constexpr int GROUPS = SEARCH_THREADS / G;
    constexpr int GMODE = (DIM == 3 && MODE == 1) ? 1 : 0;
    const uint32_t M = a.sc->n_masked;
    const int gl = threadIdx.x % G;
    const int nx = a.nx, ny = a.ny, nz = a.nz, sxy = nx * ny;
    const float inv_dd_g = a.sc->inv_dd;
    const InvS2<float> is = inv_s2_of(a);
    const TabEntry row = zg.row[gl];            // this lane's zero-key cell
    const Geo<float> Gm = geo_from_row(row);
    GuardCtx gc{};
    uint32_t dummy_fp64 = 0, cells = 0, gm = 0, npass = 0, nborder = 0;

    for (uint32_t base = blockIdx.x * GROUPS; base < M; base += gridDim.x * GROUPS) {
        const uint32_t i = base + threadIdx.x / G;
        const bool live = i < M;
        const int node = live ? (int)a.nodes[i] : 0;
        const int x = node % nx, y = (node / nx) % ny, z = DIM == 3 ? node / sxy : 0;
        const float dr = a.ref[node];
        const float inv_dd = node_inv_dd(dr, inv_dd_g, a.dd, a.local);
        const float F0 = live ? gamma0_sq(a.ev[node], dr, inv_dd) : 0.0f;
        const int qx = x + row.ax, qy = y + row.ay, qz = z + row.az;
        const bool cin = (unsigned)qx < (unsigned)nx && (unsigned)qy < (unsigned)ny &&
                         (DIM == 2 || (unsigned)qz < (unsigned)nz);
        const bool okx = qx + 1 < nx, oky = qy + 1 < ny, okz = DIM == 2 || qz + 1 < nz;
        const bool work = F0 > 0.0f && cin;
        const bool edge = !(okx && oky && okz);
        const bool wave_masked = __ballot(work && edge) != 0ull;
        float c = Num<float>::inf();
        bool ill = false;
        if (work) {
            const int b0 = (DIM == 3 ? qz * sxy : 0) + qy * nx + qx;
            const int ox = okx ? 1 : 0, oy = oky ? nx : 0, oz = (DIM == 3 && okz) ? sxy : 0;
            if constexpr (DIM == 3) {
                float g[8];
                g[0] = a.ev[b0];
                g[1] = a.ev[b0 + ox];
                g[2] = a.ev[b0 + oy];
                g[3] = a.ev[b0 + oy + ox];
                g[4] = a.ev[b0 + oz];
                g[5] = a.ev[b0 + oz + ox];
                g[6] = a.ev[b0 + oz + oy];
                g[7] = a.ev[b0 + oz + oy + ox];
#pragma unroll
                for (int b = 0; b < 8; ++b) g[b] = (g[b] - dr) * inv_dd;
                if (wave_masked)
                    c = cell3<float, true, GMODE>(g, Gm, is, okx, oky, okz, a.den_guard, gc, dummy_fp64, ill);
                else
                    c = cell3<float, false, GMODE>(g, Gm, is, true, true, true, a.den_guard, gc, dummy_fp64, ill);
            } else {
                float g[4];
                g[0] = a.ev[b0];
                g[1] = a.ev[b0 + ox];
                g[2] = a.ev[b0 + oy];
                g[3] = a.ev[b0 + oy + ox];
#pragma unroll
                for (int b = 0; b < 4; ++b) g[b] = (g[b] - dr) * inv_dd;
                if (wave_masked)
                    c = cell2<float, true>(g, Gm, is, okx, oky);
                else
                    c = cell2<float, false>(g, Gm, is, true, true);
            }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            c = vmin<float>(c, __shfl_xor(c, o));
            ill = (__shfl_xor((int)ill, o) != 0) || ill;
        }
        // every lane of the group now holds the same F0, minimum and flag
        const float F = vmin<float>(F0, c);
        const bool node_guard = MODE == 1 && live && ill;
        const bool node_tail = live && !node_guard && F > a.k1;
        // cells are counted by the pass that finishes the node
        if (live && !node_guard && !node_tail && work && !edge) ++cells;
        const bool leader = gl == 0;
        const bool to_guard = leader && node_guard;
        const bool to_tail = leader && node_tail;
        if (leader && live && !node_guard && !node_tail) finish_node(a, node, F, npass, nborder, gm);
        const uint32_t pos = block_append(to_tail, &a.sc->n_tail);
        if (to_tail) {
            a.tail_node[pos] = (uint32_t)node;
            a.tail_f[pos] = f2u(F);
            a.tail_key_arr[pos] = tail_sort_key(a, node, F0, F);
            a.tail_pos[pos] = pos;
        }
        if (MODE == 1) {
            const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
            if (to_guard) a.guard_list[gpos] = (uint32_t)node;
        }
    }
    block_sums(sums, blockIdx.x, npass, nborder, 0u, cells, gm);
}

// The walk.  TAIL: items are tail positions, the walk starts at row `first` with the bound
// left by pass A; otherwise items are node indices and the walk starts at row 0 with
// gamma0.  MODE 0: FP32; 1: FP32 + flag; 2: FP32 with FP64 re-projection; 3: FP64.
// spec (TAIL only): 0 plain; 1 speculative (bound min(gamma^2, (f gamma_hat)^2); a node
// whose gamma^2 stays above (f gamma_hat)^2 is queued on the fallback list instead of
// finished); 2 fallback (the plain walk from the first row at or beyond f gamma_hat).
// vb / vgrid: the block's index and the number of blocks striding over the list.
template <int DIM, int MODE, bool TAIL>
__device__ __forceinline__ void walk_body(const SearchArgs& a, const TabEntry* __restrict__ tab,
                                          const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                                          int first, int spec, BlockSums* sums, uint32_t vb, uint32_t vgrid) {
    using T = typename std::conditional<MODE == 3, double, float>::type;
    constexpr int GMODE = DIM == 3 ? (MODE == 1 ? 1 : (MODE == 2 ? 2 : 0)) : 0;
    const uint32_t M = *count;
    const int lane = threadIdx.x & (WAVE - 1);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int sxy = nx * ny;
    const float inv_dd_g = a.sc->inv_dd;
    const double dmax = (double)ord_to_float(a.sc->dmax_ord);
    const InvS2<T> is = inv_s2<T>(MODE == 3 ? (T)(a.sx * a.sx) : (T)a.s2x,
                                  MODE == 3 ? (T)(a.sy * a.sy) : (T)a.s2y,
                                  DIM == 3 ? (MODE == 3 ? (T)(a.sz * a.sz) : (T)a.s2z) : T(0));
    const double sx2d = a.sx * a.sx, sy2d = a.sy * a.sy, sz2d = a.sz * a.sz;
    const uint32_t stride = vgrid * SEARCH_THREADS;
    uint32_t cells = 0, n_fp64 = 0, gm = 0, npass = 0, nborder = 0;

    // the loop bound is uniform per wave, so every lane reaches the block-wide calls below
    const uint32_t wave0 = vb * SEARCH_THREADS + (threadIdx.x & ~(WAVE - 1));
    const uint32_t iters = wave0 < M ? (M - wave0 + stride - 1) / stride : 0u;
    uint32_t it_max = iters;
    // block-uniform trip count (all waves of a block take part in block_append)
    {
        __shared__ uint32_t s_it[SEARCH_THREADS / WAVE];
        if (lane == 0) s_it[threadIdx.x / WAVE] = iters;
        __syncthreads();
        it_max = 0u;
        for (int j = 0; j < SEARCH_THREADS / WAVE; ++j) it_max = max(it_max, s_it[j]);
        __syncthreads();
    }
    for (uint32_t it = 0; it < it_max; ++it) {
        const uint32_t i = wave0 + it * stride + lane;
        const bool live = i < M;
        const uint32_t item = live ? order[i] : 0u;
        const int node = TAIL ? (live ? (int)a.tail_node[item] : 0) : (int)item;
        const int x = node % nx;
        const int y = (node / nx) % ny;
        const int z = DIM == 3 ? node / sxy : 0;
        const float dr = a.ref[node];
        const float inv_dd = node_inv_dd(dr, inv_dd_g, a.dd, a.local);
        const double inv_dd64 = a.local ? 1.0 / (a.dd64 * (double)dr) : 1.0 / (a.dd64 * dmax);
        T F;
        if constexpr (MODE == 3) {
            const double g0 = ((double)a.ev[node] - (double)dr) * inv_dd64;
            F = g0 * g0;
        } else {
            F = TAIL ? u2f(live ? a.tail_f[item] : 0u) : gamma0_sq(a.ev[node], dr, inv_dd);
        }
        if (!live) F = T(0);
        const T invdd = MODE == 3 ? (T)inv_dd64 : (T)inv_dd;
        const T drT = (T)dr;
        uint32_t lane_cells = 0, lane_fp64 = 0;
        bool ill = false;
        // learned radius: the speculative bound, and the fallback's first row
        const float r2s = (TAIL && spec && live) ? spec_bound2(a, item) : Num<float>::inf();
        int lstart = first;
        if (TAIL && spec == 2 && live) lstart = resume_row(tab, a.tab_len, first, r2s);
        int wstart = lstart;
        if (TAIL && spec == 2) {
            // the wave starts at its smallest row (the rows are wave-uniform loads)
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) wstart = min(wstart, __shfl_xor(wstart, o));
        }

        for (int n = wstart; n < a.tab_len; ++n) {
            const TabEntry e = tab[n];
            const T bound = (TAIL && spec == 1) ? vmin<T>(F, (T)r2s) : F;
            const bool act = live && n >= lstart && ((T)e.key2 < bound);
            if (__ballot(live && ((T)e.key2 < bound)) == 0ull) break;
            const int qx = x + e.ax, qy = y + e.ay, qz = z + e.az;
            const bool cin = (unsigned)qx < (unsigned)nx && (unsigned)qy < (unsigned)ny &&
                             (DIM == 2 || (unsigned)qz < (unsigned)nz);
            const bool okx = qx + 1 < nx, oky = qy + 1 < ny, okz = DIM == 2 || qz + 1 < nz;
            const bool work = act && cin;
            const bool edge = !(okx && oky && okz);
            const bool wave_masked = __ballot(work && edge) != 0ull;
            if (!work) continue;
            lane_cells += edge ? 0u : 1u;   // full grid cells, the unit of the work count
            const int base = (DIM == 3 ? qz * sxy : 0) + qy * nx + qx;
            const int ox = okx ? 1 : 0, oy = oky ? nx : 0, oz = (DIM == 3 && okz) ? sxy : 0;
            Geo<T> G;
            if constexpr (MODE == 3) {
                G = geo_fp64(e.ax, e.ay, e.az, sx2d, sy2d, DIM == 3 ? sz2d : 0.0);
            } else {
                G = geo_from_row(e);
            }
            if constexpr (DIM == 3) {
                float v[8];
                v[0] = a.ev[base];
                v[1] = a.ev[base + ox];
                v[2] = a.ev[base + oy];
                v[3] = a.ev[base + oy + ox];
                v[4] = a.ev[base + oz];
                v[5] = a.ev[base + oz + ox];
                v[6] = a.ev[base + oz + oy];
                v[7] = a.ev[base + oz + oy + ox];
                T g[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) g[b] = dose_norm<T>((T)v[b], drT, invdd);
                GuardCtx gc{};
                if constexpr (GMODE == 2) {
                    gc = GuardCtx{a.ev, base, ox, oy, oz, dr, inv_dd64, e.ax, e.ay, e.az, sx2d, sy2d, sz2d};
                }
                T c;
                if (wave_masked)
                    c = cell3<T, true, GMODE>(g, G, is, okx, oky, okz, (T)a.den_guard, gc, lane_fp64, ill);
                else
                    c = cell3<T, false, GMODE>(g, G, is, true, true, true, (T)a.den_guard, gc, lane_fp64, ill);
                F = vmin<T>(F, c);
            } else {
                float v[4];
                v[0] = a.ev[base];
                v[1] = a.ev[base + ox];
                v[2] = a.ev[base + oy];
                v[3] = a.ev[base + oy + ox];
                T g[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) g[b] = dose_norm<T>((T)v[b], drT, invdd);
                T c;
                if (wave_masked)
                    c = cell2<T, true>(g, G, is, okx, oky);
                else
                    c = cell2<T, false>(g, G, is, true, true);
                F = vmin<T>(F, c);
            }
        }

        const bool to_guard = MODE == 1 && live && ill;
        const bool to_fb = TAIL && spec == 1 && live && !to_guard && (float)F > r2s;
        if (live && !to_guard && !to_fb) {
            finish_node(a, node, (float)F, npass, nborder, gm);
            cells += lane_cells + (TAIL ? zero_cells(DIM, x, y, z, nx, ny, nz) : 0u);
            n_fp64 += lane_fp64;
        }
        if (to_fb) cells += lane_cells;
        if (MODE == 1) {
            const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
            if (to_guard) a.guard_list[gpos] = (uint32_t)node;
        }
        if (TAIL && spec == 1) {
            const uint32_t fpos = block_append(to_fb, &a.sc->n_fallback);
            if (to_fb) {
                a.fb_list[fpos] = item;
                a.tail_f[item] = f2u((float)F);
            }
        }
    }
    block_sums(sums, vb, npass, nborder, n_fp64, cells, gm, a.sc);
}

template <int DIM, int MODE, bool TAIL>
__global__ __launch_bounds__(SEARCH_THREADS) void k_walk(SearchArgs a, const TabEntry* __restrict__ tab,
                                                         const uint32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ count, int first,
                                                         int spec, BlockSums* sums) {
    walk_body<DIM, MODE, TAIL>(a, tab, order, count, first, spec, sums, blockIdx.x, gridDim.x);
}

// Pass B with G lanes per node: the G lanes of a group take G consecutive table rows of
// one node at once (independent loads, so the gathers of G cells overlap instead of
// forming one dependent chain), then take the minimum over the group and move to the next
// G rows while the first of them still has key^2 < gamma^2.  Every row the sequential walk
// would evaluate is evaluated; up to G-1 rows past its break may be too.
// MODE 0: FP32; 1: FP32 + flag ill-conditioned tetrahedra (3D).
// g_req: lanes per node (8..64), or <= 0 to pick it from the tail length on the device:
// about 2^19 lanes in flight fill the GPU, so a short tail gets wide groups (latency) and a
// long one narrow groups (fewer rows past the break), but never fewer than -g_req (when
// negative) lanes: a tail whose longest walks are long needs wide groups whatever its
// length, since the kernel lasts as long as its longest walk.
// spec: as in k_walk (1 speculative, 2 fallback from the first row at or beyond f gamma_hat).
template <int DIM, int MODE>
__device__ __forceinline__ void tail_group_body(const SearchArgs& a, const TabEntry* __restrict__ tab,
                                                const uint32_t* __restrict__ order,
                                                const uint32_t* __restrict__ count, int first, int g_req,
                                                int spec, BlockSums* sums, uint32_t vb, uint32_t vgrid) {
    constexpr int GMODE = (DIM == 3 && MODE == 1) ? 1 : 0;
    const uint32_t M = *count;
    int G = g_req;
    if (G <= 0) {
        // automatic: -g_req (if given) is the least width, raised for lists whose longest
        // walks would otherwise take many dependent steps
        const int gmin = G < 0 ? -G : 8;
        G = 64;
        while (G > gmin && (uint64_t)M * (uint64_t)G > (1ull << 19)) G >>= 1;
    }
    const int GROUPS = SEARCH_THREADS / G;
    const int gl = threadIdx.x % G;               // lane within the group
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int sxy = nx * ny;
    const float inv_dd_g = a.sc->inv_dd;
    const InvS2<float> is = inv_s2_of(a);
    uint32_t cells = 0, gm = 0, npass = 0, nborder = 0, nfb = 0;
    GuardCtx gc{};
    uint32_t dummy_fp64 = 0;

    // block-uniform trip count
    for (uint64_t base = (uint64_t)vb * GROUPS; base < M; base += (uint64_t)vgrid * GROUPS) {
        const uint32_t i = (uint32_t)base + threadIdx.x / G;
        const bool live = i < M;
        const uint32_t item = live ? order[i] : 0u;
        const int node = live ? (int)a.tail_node[item] : 0;
        const int x = node % nx;
        const int y = (node / nx) % ny;
        const int z = DIM == 3 ? node / sxy : 0;
        const float dr = a.ref[node];
        const float inv_dd = node_inv_dd(dr, inv_dd_g, a.dd, a.local);
        float F = live ? u2f(a.tail_f[item]) : 0.0f;
        uint32_t lane_cells = 0;
        bool ill = false;
        const float r2s = (spec && live) ? spec_bound2(a, item) : Num<float>::inf();
        // the fallback resumes at the first row the speculative bound cut off, which the
        // speculative launch stored in the (by then unused) sort-key slot of the item
        const int start = (spec == 2 && live) ? (int)a.tail_key_arr[item] : first;
        uint32_t steps = 0;   // batches of G rows this group walked
        int last_n0 = -1;     // first row of the group's last batch (speculative walk)

        for (int n0 = start; n0 < a.tab_len; n0 += G) {
            const float k_first = tab[n0].key2;       // uniform per group
            const float bound = spec == 1 ? vmin<float>(F, r2s) : F;
            const bool grp_act = live && k_first < bound;
            if (__ballot(grp_act) == 0ull) break;
            steps += grp_act ? 1u : 0u;
            last_n0 = grp_act ? n0 : last_n0;
            const int n = n0 + gl;
            TabEntry e;
            bool act = false;
            if (grp_act && n < a.tab_len) {
                e = tab[n];
                act = e.key2 < bound;
            }
            int qx = 0, qy = 0, qz = 0;
            if (act) {
                qx = x + e.ax;
                qy = y + e.ay;
                qz = z + e.az;
            }
            const bool cin = (unsigned)qx < (unsigned)nx && (unsigned)qy < (unsigned)ny &&
                             (DIM == 2 || (unsigned)qz < (unsigned)nz);
            const bool okx = qx + 1 < nx, oky = qy + 1 < ny, okz = DIM == 2 || qz + 1 < nz;
            const bool work = act && cin;
            const bool edge = !(okx && oky && okz);
            const bool wave_masked = __ballot(work && edge) != 0ull;
            float c = Num<float>::inf();
            constexpr int NV = DIM == 3 ? 8 : 4;
            float g[NV];
            // Dose bound: the PL dose inside the cell lies between its vertex values, so a
            // cell whose vertex differences share a sign is at least key^2 + (smallest
            // |difference|)^2 from the node; at or above F it cannot lower F and is skipped
            // (still counted as visited).  A lane's decision is its own, so the result does
            // not depend on which nodes share the wave.
            bool need = false;
            if (work) {
                lane_cells += edge ? 0u : 1u;
                const int base_i = (DIM == 3 ? qz * sxy : 0) + qy * nx + qx;
                const int ox = okx ? 1 : 0, oy = oky ? nx : 0, oz = (DIM == 3 && okz) ? sxy : 0;
                g[0] = a.ev[base_i];
                g[1] = a.ev[base_i + ox];
                g[2] = a.ev[base_i + oy];
                g[3] = a.ev[base_i + oy + ox];
                if constexpr (DIM == 3) {
                    g[4] = a.ev[base_i + oz];
                    g[5] = a.ev[base_i + oz + ox];
                    g[6] = a.ev[base_i + oz + oy];
                    g[7] = a.ev[base_i + oz + oy + ox];
                }
                float gmin = Num<float>::inf(), gmax = -Num<float>::inf();
#pragma unroll
                for (int b = 0; b < NV; ++b) {
                    g[b] = dose_norm<float>(g[b], dr, inv_dd);
                    gmin = vmin<float>(gmin, g[b]);
                    gmax = __builtin_fmaxf(gmax, g[b]);
                }
                const float m = gmin > 0.0f ? gmin : (gmax < 0.0f ? -gmax : 0.0f);
                // margin 2^-8 F: far above the rounding of the projections, so a skipped
                // cell's projected value could not have been below F either, and F, the
                // walk and the result are bit for bit those of the unpruned walk
                need = e.key2 + m * m < F + F * 0x1p-8f;
                // the guard still judges a skipped cell's tetrahedra (whether a node is
                // redone in FP64 must not depend on the pruning)
                if constexpr (GMODE == 1)
                    if (!need && okx && oky && okz) ill = ill || tets_ill(g, is, a.den_guard);
            }
            // the whole projection only where some lane of the wave needs it
            if (__ballot(need) != 0ull && need) {
                const Geo<float> Gm = geo_from_row(e);
                if constexpr (DIM == 3) {
                    if (wave_masked)
                        c = cell3<float, true, GMODE>(g, Gm, is, okx, oky, okz, a.den_guard, gc, dummy_fp64, ill);
                    else
                        c = cell3<float, false, GMODE>(g, Gm, is, true, true, true, a.den_guard, gc, dummy_fp64,
                                                       ill);
                } else {
                    if (wave_masked)
                        c = cell2<float, true>(g, Gm, is, okx, oky);
                    else
                        c = cell2<float, false>(g, Gm, is, true, true);
                }
            }
            // group minimum (the group is G consecutive lanes of the wave)
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) c = vmin<float>(c, __shfl_xor(c, o));
            F = vmin<float>(F, c);
        }
        // reduce the group's flags and cell counts onto its first lane
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            lane_cells += (uint32_t)__shfl_xor((int)lane_cells, o);
            ill = (__shfl_xor((int)ill, o) != 0) || ill;
        }
        // record a long walk (rare): the next map of this context widens its groups
        {
            uint32_t rows = (live && gl == 0) ? steps * (uint32_t)G : 0u;
            if (__ballot(rows > LONG_WALK_ROWS) != 0ull) {
                for (int o = WAVE / 2; o > 0; o >>= 1) rows = max(rows, (uint32_t)__shfl_xor((int)rows, o));
                if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(&a.sc->long_rows, rows);
            }
        }
        const bool leader = live && gl == 0;
        const bool to_guard = MODE == 1 && leader && ill;
        const bool to_fb = spec == 1 && leader && !to_guard && F > r2s;
        // a short tail walks with the plain bound; the nodes the prediction would not have
        // certified (F above its bound) are counted as its fallbacks, except those the guard
        // redoes (as the speculative walk does)
        if (spec == 3) nfb += (leader && !to_guard && F > r2s) ? 1u : 0u;
        if (leader && !to_guard && !to_fb) {
            finish_node(a, node, F, npass, nborder, gm);
            cells += lane_cells + zero_cells(DIM, x, y, z, nx, ny, nz);
        }
        if (to_fb) cells += lane_cells;
        if (MODE == 1) {
            const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
            if (to_guard) a.guard_list[gpos] = (uint32_t)node;
        }
        if (spec == 1) {
            // the first row the speculative bound cut off.  A node sent to the fallback kept
            // F above r2s, so its bound was r2s throughout: it walked every row before its
            // last batch and, in that batch, the rows below r2s (a prefix: rows are in key
            // order); with no batch walked it is the first row
            const int rr = last_n0 + gl;
            const bool below = last_n0 >= 0 && rr < a.tab_len && tab[rr].key2 < r2s;
            const unsigned long long bm = __ballot(below);
            const int lane = (int)(threadIdx.x & (WAVE - 1));
            const unsigned long long gmask = G >= WAVE ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
            const int cut = last_n0 < 0 ? start : last_n0 + (int)__popcll(bm & gmask);
            const uint32_t fpos = block_append(to_fb, &a.sc->n_fallback);
            if (to_fb) {
                a.fb_list[fpos] = item;
                a.tail_f[item] = f2u(F);
                a.tail_key_arr[item] = (uint32_t)cut;
            }
        }
    }
    if (spec == 3) {
        // one atomic per block (one per wave on a single address serialises)
        __shared__ uint32_t s_fb[SEARCH_THREADS / WAVE];
        for (int o = WAVE / 2; o > 0; o >>= 1) nfb += (uint32_t)__shfl_xor((int)nfb, o);
        if ((threadIdx.x & (WAVE - 1)) == 0) s_fb[threadIdx.x / WAVE] = nfb;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0u;
            for (int j = 0; j < SEARCH_THREADS / WAVE; ++j) t += s_fb[j];
            if (t) atomicAdd(&a.sc->n_fallback_inline, t);
        }
    }
    block_sums(sums, vb, npass, nborder, 0u, cells, gm);
}

template <int DIM, int MODE>
__global__ __launch_bounds__(SEARCH_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_tail_group(SearchArgs a, const TabEntry* __restrict__ tab,
                                                               const uint32_t* __restrict__ order,
                                                               const uint32_t* __restrict__ count, int first,
                                                               int g_req, int spec, BlockSums* sums) {
    tail_group_body<DIM, MODE>(a, tab, order, count, first, g_req, spec, sums, blockIdx.x, gridDim.x);
}

// One block: sum the per-block partial counts into the scalars, and flag a cell table
// that does not reach the search radius (the host then rebuilds it and runs again).
// ADD: add the sums into the scalars (which the prep zeroed) instead of storing them, so
// that other blocks may add theirs at the same time.
template <bool ADD = false>
__device__ __forceinline__ void finalize_body(const BlockSums* __restrict__ sums, int n, Scalars* sc,
                                              float r2_cap) {
    if (threadIdx.x == 0 && u2f(sc->r2_bits) > r2_cap && sc->n_masked > 0) sc->flags |= FLAG_TABLE_SHORT;
    unsigned long long p = 0, b = 0, f = 0, c = 0;
    uint32_t m = 0;
    for (int j = threadIdx.x; j < n; j += SEARCH_THREADS) {
        p += sums[j].pass;
        b += sums[j].border;
        f += sums[j].fp64;
        c += sums[j].cells;
        m = max(m, sums[j].maxg2);
    }
    __shared__ unsigned long long s[4][SEARCH_THREADS];
    __shared__ uint32_t sm[SEARCH_THREADS];
    s[0][threadIdx.x] = p;
    s[1][threadIdx.x] = b;
    s[2][threadIdx.x] = f;
    s[3][threadIdx.x] = c;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int h = SEARCH_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int k = 0; k < 4; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (ADD) {
            if (s[0][0]) atomicAdd(&sc->n_pass, s[0][0]);
            if (s[1][0]) atomicAdd(&sc->n_border, s[1][0]);
            if (s[2][0]) atomicAdd(&sc->n_fp64, s[2][0]);
            if (s[3][0]) atomicAdd(&sc->n_cells, s[3][0]);
            if (sm[0]) atomicMax(&sc->maxg2_bits, sm[0]);
        } else {
            sc->n_pass = s[0][0];
            sc->n_border = s[1][0];
            sc->n_fp64 = s[2][0];
            sc->n_cells = s[3][0];
            sc->maxg2_bits = sm[0];
        }
    }
}

__global__ __launch_bounds__(SEARCH_THREADS) void k_finalize(const BlockSums* __restrict__ sums, int n,
                                                             Scalars* sc, float r2_cap) {
    finalize_body(sums, n, sc, r2_cap);
}

// The guard pass and the count reduction in one launch (guarded precision, 3D): block 0
// first adds the partial slots of the earlier passes into the scalars, then every block
// redoes its share of the guard list in FP64-guarded precision and adds its own counts
// straight into the scalars (a block with no guard nodes adds nothing).
__global__ __launch_bounds__(SEARCH_THREADS) void k_guard_finalize(SearchArgs a, const TabEntry* __restrict__ tab,
                                                                   const BlockSums* __restrict__ sums) {
    if (blockIdx.x == 0) finalize_body<true>(sums, SUM_BINS, a.sc, a.r2_cap);
    walk_body<3, 2, false>(a, tab, a.guard_list, &a.sc->n_guard, 0, 0, nullptr, blockIdx.x, gridDim.x);
}

constexpr unsigned kTailBlocks = 1024;   // grid-stride blocks of the tail walk
constexpr unsigned kGuardBlocks = 64;    // grid-stride blocks of the guard pass
constexpr unsigned kZeroGroupBlocks = 8192;   // grid-stride blocks of pass A, one lane per cell

unsigned blocks_for(uint32_t m) { return (m + SEARCH_THREADS - 1) / SEARCH_THREADS; }

template <int DIM, int MODE, bool TAIL>
void walk(const SearchArgs& a, const uint32_t* order, const uint32_t* count, int first, unsigned blocks,
          BlockSums* sums, hipStream_t s, int spec = 0) {
    hipLaunchKernelGGL((k_walk<DIM, MODE, TAIL>), dim3(blocks), dim3(SEARCH_THREADS), 0, s, a, a.tab, order,
                       count, first, spec, sums);
}

template <int DIM, int MODE>
void tail_group_g(const SearchArgs& a, const uint32_t* order, const uint32_t* count, int G, int first,
                  unsigned blocks, int spec, BlockSums* sums, hipStream_t s) {
    hipLaunchKernelGGL((k_tail_group<DIM, MODE>), dim3(blocks), dim3(SEARCH_THREADS), 0, s, a, a.tab, order, count,
                       first, G, spec, sums);
}

void tail_group(const SearchArgs& a, const uint32_t* order, const uint32_t* count, int ndim, int mode, int G,
                int first, unsigned blocks, int spec, BlockSums* sums, hipStream_t s) {
    if (ndim == 3) {
        if (mode == 1) tail_group_g<3, 1>(a, order, count, G, first, blocks, spec, sums, s);
        else tail_group_g<3, 0>(a, order, count, G, first, blocks, spec, sums, s);
    } else {
        tail_group_g<2, 0>(a, order, count, G, first, blocks, spec, sums, s);
    }
}

// Pass B over `order` (count on the device): one lane per node (G == 1) or G lanes.
unsigned tail_pass(const SearchArgs& a, const SearchPlan& p, const uint32_t* order, const uint32_t* count,
                   int first, bool guarded, int spec, unsigned tb, BlockSums* sums, hipStream_t s) {
    // 0: chosen on the device from the list length; negative: the same with a least width
    const int G = p.tail_lanes ? p.tail_lanes : -(p.tail_min_lanes > 8 ? p.tail_min_lanes : 8);
    if (G == 1) {
        if (p.ndim == 3) {
            if (guarded) walk<3, 1, true>(a, order, count, first, tb, sums, s, spec);
            else walk<3, 0, true>(a, order, count, first, tb, sums, s, spec);
        } else {
            walk<2, 0, true>(a, order, count, first, tb, sums, s, spec);
        }
        return tb;
    }
    const unsigned groups = SEARCH_THREADS / (unsigned)(G > 0 ? G : -G);
    unsigned gb = (p.M + groups - 1) / groups;
    if (gb > kTailBlocks) gb = kTailBlocks;
    tail_group(a, order, count, p.ndim, guarded ? 1 : 0, G, first, gb, spec, sums, s);
    return gb;
}

// ---- batches ------------------------------------------------------------------------

// The key-0 pass of every pair of a batch: block b takes item b = (pair, block of 256 nodes)
// and runs that pair's pass over those nodes, as the pair's own kernel would (a block past
// the pair's M returns at once).
__global__ __launch_bounds__(SEARCH_THREADS) void k_batch_key0(const BatchPair* __restrict__ pairs,
                                                               const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    if (P.ndim == 3) {
        if (P.guarded) zero3_body<1>(P.sa, P.zg, P.sa.sums, w.y);
        else zero3_body<0>(P.sa, P.zg, P.sa.sums, w.y);
    } else {
        zero2_body(P.sa, P.zg, P.sa.sums, w.y);
    }
}

// The tail walk of every pair (no sort, plain radius): block b takes item (pair, tail block).
__global__ __launch_bounds__(SEARCH_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_tail(
    const BatchPair* __restrict__ pairs, const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    if (P.ndim == 3) {
        if (P.guarded)
            tail_group_body<3, 1>(P.sa, P.sa.tab, P.sa.tail_pos, &P.sa.sc->n_tail, P.first, P.g_req, 0, P.sa.sums,
                                  w.y, (uint32_t)P.tail_blocks);
        else
            tail_group_body<3, 0>(P.sa, P.sa.tab, P.sa.tail_pos, &P.sa.sc->n_tail, P.first, P.g_req, 0, P.sa.sums,
                                  w.y, (uint32_t)P.tail_blocks);
    } else {
        tail_group_body<2, 0>(P.sa, P.sa.tab, P.sa.tail_pos, &P.sa.sc->n_tail, P.first, P.g_req, 0, P.sa.sums, w.y,
                              (uint32_t)P.tail_blocks);
    }
}

// Every pair's guard pass with its count reduction (as k_guard_finalize), or the count
// reduction alone (as k_finalize); block 0 of each pair then stamps its completion.
__global__ __launch_bounds__(SEARCH_THREADS) void k_batch_finish(const BatchPair* __restrict__ pairs,
                                                                 const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    if (P.guarded) {
        if (w.y == 0) finalize_body<true>(P.sa.sums, SUM_BINS, P.sa.sc, P.sa.r2_cap);
        walk_body<3, 2, false>(P.sa, P.sa.tab, P.sa.guard_list, &P.sa.sc->n_guard, 0, 0, nullptr, w.y, kGuardBlocks);
    } else {
        finalize_body(P.sa.sums, SUM_BINS, P.sa.sc, P.sa.r2_cap);
    }
    if (w.y == 0 && threadIdx.x == 0) *P.done = wall_clock64();
}

__global__ void k_stamp(unsigned long long* t) {
    if (threadIdx.x == 0) *t = wall_clock64();
}

// ---- two grids (the evaluation dose on a grid of its own, 3D) ---------------------------

// Evaluation-grid position of reference node r: u = (k * rh - eo) / eh per axis (z, y, x).
__device__ __forceinline__ void grids_pos(const GridsArgs& a, int r, double u[3], bool& inside) {
    const int x = r % a.rn[2], y = (r / a.rn[2]) % a.rn[1], z = r / (a.rn[2] * a.rn[1]);
    const int k[3] = {z, y, x};
    inside = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        u[i] = ((double)k[i] * a.rh[i] - a.eo[i]) / a.eh[i];
        inside = inside && u[i] >= 0.0 && u[i] <= (double)(a.en[i] - 1);
    }
}

// Holding cell (lower corner c0, clamped so that the cell exists) and the node's position f
// inside it, in [0, 1] per axis.
template <typename T>
__device__ __forceinline__ void grids_cell(const GridsArgs& a, const double u[3], int c0[3], T f[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        int c = (int)floor(u[i]);
        c = c > a.en[i] - 2 ? a.en[i] - 2 : (c < 0 ? 0 : c);
        c0[i] = c;
        f[i] = (T)(u[i] - (double)c);
    }
}

// Spatial constants of the cell at offset (a - f) from the node, in evaluation-grid units
// (the per-row constants of the one-grid table, for a node off the grid's nodes).
// (is: the reciprocals of the block sums of s^2, so no division per cell)
template <typename T>
__device__ __forceinline__ Geo<T> geo_frac(T ax, T ay, T az, T sx2, T sy2, T sz2, const InvS2<T>& is) {
    Geo<T> g;
    g.ax = ax; g.ay = ay; g.az = az;
    g.px = sx2 * ax * ax; g.py = sy2 * ay * ay; g.pz = sz2 * az * az;
    const T dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    g.vxy = sx2 * sy2 * dxy * dxy * is.xy;
    g.vxz = sx2 * sz2 * dxz * dxz * is.xz;
    g.vyz = sy2 * sz2 * dyz * dyz * is.yz;
    g.vxyz = (sx2 * sy2 * dxy * dxy + sx2 * sz2 * dxz * dxz + sy2 * sz2 * dyz * dyz) * is.xyz;
    g.mxy = (sx2 * ax + sy2 * ay) * is.xy;
    g.mxz = (sx2 * ax + sz2 * az) * is.xz;
    g.myz = (sy2 * ay + sz2 * az) * is.yz;
    g.mxyz = (sx2 * ax + sy2 * ay + sz2 * az) * is.xyz;
    return g;
}

__device__ __forceinline__ float grids_thr(const GridsArgs& a, float dmax) { return a.thr * dmax; }

// First bound of a node: the nearest of the 8 vertices of its holding cell.
template <typename T>
__device__ __forceinline__ T grids_f0(const GridsArgs& a, const int c0[3], const T f[3], T dr, T inv_dd) {
    const T s2[3] = {(T)(a.eh[0] / a.dta) * (T)(a.eh[0] / a.dta), (T)(a.eh[1] / a.dta) * (T)(a.eh[1] / a.dta),
                     (T)(a.eh[2] / a.dta) * (T)(a.eh[2] / a.dta)};
    T best = Num<T>::inf();
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bz = (b >> 2) & 1, by = (b >> 1) & 1, bx = b & 1;
        const T dz = (T)bz - f[0], dy = (T)by - f[1], dx = (T)bx - f[2];
        const int64_t j = ((int64_t)(c0[0] + bz) * a.en[1] + (c0[1] + by)) * a.en[2] + (c0[2] + bx);
        const T gv = ((T)a.ev[j] - dr) * inv_dd;
        best = vmin<T>(best, s2[0] * dz * dz + s2[1] * dy * dy + s2[2] * dx * dx + gv * gv);
    }
    return best;
}

constexpr int GRIDS_MAX_ITEMS = 8;
__global__ __launch_bounds__(256) void k_grids_max(GridsArgs a, int64_t nr, int64_t ne) {
    float m = -Num<float>::inf();
    bool bad = false;
    const int64_t n = nr > ne ? nr : ne;
    // GRIDS_MAX_ITEMS nodes of each volume per thread and step, every load of a step issued
    // before the first use (indices clamped to the last node: the copies change neither the
    // maximum nor the finiteness check)
    constexpr int K = GRIDS_MAX_ITEMS;
    const int64_t step = (int64_t)gridDim.x * 256 * K;
    for (int64_t b0 = (int64_t)blockIdx.x * 256 * K; b0 < n; b0 += step) {
        float r[K], e[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t i = b0 + (int64_t)k * 256 + threadIdx.x;
            r[k] = a.ref[i < nr ? i : nr - 1];
            e[k] = a.ev[i < ne ? i : ne - 1];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            bad = bad || !isfinite(r[k]) || !isfinite(e[k]);
            m = fmaxf(m, r[k]);
        }
    }
    // one partial per block (an atomic maximum per wave on one address serialises: it took
    // 30-80 us); the listing kernel reduces the partials
    __shared__ uint32_t s_m[4];
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m > -Num<float>::inf() ? float_to_ord(m) : 0u;
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&a.sc->flags, FLAG_NONFINITE);
    __syncthreads();
    if (threadIdx.x == 0) a.part[blockIdx.x] = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
}

// Listing in chunks of 16 nodes per thread (4096 per block): one atomic per chunk on the
// list counter (one per 256 nodes would serialise on that address).
constexpr int GRIDS_PER_THREAD = 16;
__global__ __launch_bounds__(256) void k_grids_list(GridsArgs a, int64_t nr, int nb_max) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_base;
    // the dose maximum from k_grids_max's partials (every block reduces them itself)
    uint32_t dm = 0u;
    for (int j = threadIdx.x; j < nb_max; j += 256) dm = max(dm, a.part[j]);
    for (int o = 32; o > 0; o >>= 1) dm = max(dm, (uint32_t)__shfl_xor((int)dm, o));
    if ((threadIdx.x & 63) == 0) s_wsum[threadIdx.x >> 6] = dm;
    __syncthreads();
    dm = max(max(s_wsum[0], s_wsum[1]), max(s_wsum[2], s_wsum[3]));
    __syncthreads();   // s_wsum is reused below
    const float dmax = ord_to_float(dm);
    const float thr_val = grids_thr(a, dmax);
    const float inv_dd_g = 1.0f / ((float)a.dd * dmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.sc->dmax_ord = dm;
        a.sc->thr_val = thr_val;
        a.sc->inv_dd = inv_dd_g;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t chunk = 256 * GRIDS_PER_THREAD;
    // block-uniform trip count, so that every thread reaches the barriers
    for (int64_t b0 = (int64_t)blockIdx.x * chunk; b0 < nr; b0 += (int64_t)gridDim.x * chunk) {
        float F0[GRIDS_PER_THREAD], drs[GRIDS_PER_THREAD];
        uint32_t takes = 0u, cnt = 0u;
        // every reference load first, and the gamma = -1 stores after the chunk's loads: a
        // store between them (gamma may alias the doses, as far as the compiler knows) kept
        // each node's loads waiting for the previous node's
#pragma unroll
        for (int k = 0; k < GRIDS_PER_THREAD; ++k) {
            const int64_t r = b0 + threadIdx.x + 256 * k;
            drs[k] = a.ref[r < nr ? r : nr - 1];
        }
#pragma unroll
        for (int k = 0; k < GRIDS_PER_THREAD; ++k) {
            const int64_t r = b0 + threadIdx.x + 256 * k;
            F0[k] = 0.0f;
            if (r < nr) {
                const float dr = drs[k];
                double u[3];
                bool inside;
                grids_pos(a, (int)r, u, inside);
                if (dr >= thr_val && (!a.local || dr > 0.0f) && inside) {
                    int c0[3];
                    float f[3];
                    grids_cell<float>(a, u, c0, f);
                    F0[k] = grids_f0<float>(a, c0, f, dr, node_inv_dd(dr, inv_dd_g, (float)a.dd, a.local));
                    takes |= 1u << k;
                    ++cnt;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < GRIDS_PER_THREAD; ++k) {
            const int64_t r = b0 + threadIdx.x + 256 * k;
            if (r < nr) a.gamma[r] = -1.0f;
        }
        // exclusive prefix of the per-thread counts over the block
        uint32_t incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wsum[w] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t tot = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
            s_base = tot ? atomicAdd(&a.sc->n_masked, tot) : 0u;
        }
        __syncthreads();
        uint32_t pos = s_base + incl - cnt;
        for (int j2 = 0; j2 < w; ++j2) pos += s_wsum[j2];
        __syncthreads();   // s_wsum / s_base are reused by the next chunk
        uint32_t fb = 0u;
#pragma unroll
        for (int k = 0; k < GRIDS_PER_THREAD; ++k) {
            if ((takes >> k) & 1u) {
                a.list[pos] = (uint32_t)(b0 + threadIdx.x + 256 * k);
                a.f0[pos] = F0[k];
                fb = max(fb, f2u(F0[k]));
                ++pos;
            }
        }
        // the largest first bound: one atomic per block and chunk, only while it can raise it
        for (int o = 32; o > 0; o >>= 1) fb = max(fb, (uint32_t)__shfl_xor((int)fb, o));
        if (lane == 0) s_wsum[w] = fb;
        __syncthreads();
        if (threadIdx.x == 0) {
            fb = max(max(s_wsum[0], s_wsum[1]), max(s_wsum[2], s_wsum[3]));
            if (fb > __atomic_load_n(&a.sc->r2_bits, __ATOMIC_RELAXED)) atomicMax(&a.sc->r2_bits, fb);
        }
        __syncthreads();   // s_wsum is reused by the next chunk
    }
}

// G lanes per node walk the lower-key table of the evaluation grid from row 0.
// Whether the cell at offset (ax, ay, az) from the holding cell can still lower F.  The node
// (at f inside the holding cell) is at least the cell's geometric distance from it, and the
// PL dose inside the cell lies between its vertex values, so when those share a sign the
// cell is at least dist^2 + (smallest |g|)^2 away.  A cell at or above F (1 + 2^-8) is
// skipped: the margin is far above the rounding of the projections, so it could not have
// lowered F either.  The bound needs no projection, so the guard judges only the cells that
// are projected: a skipped cell's conditioning cannot change the result.
__device__ __forceinline__ bool grids_need(const float* g, float ax, float ay, float az, const float* f, float sx2,
                                           float sy2, float sz2, float F) {
    float gmin = g[0], gmax = g[0];
#pragma unroll
    for (int b = 1; b < 8; ++b) {
        gmin = vmin<float>(gmin, g[b]);
        gmax = __builtin_fmaxf(gmax, g[b]);
    }
    const float m = gmin > 0.0f ? gmin : (gmax < 0.0f ? -gmax : 0.0f);
    // distance from f to the interval [a, a + 1], per axis
    const float dx = __builtin_fmaxf(__builtin_fmaxf(0.0f, ax - f[2]), f[2] - ax - 1.0f);
    const float dy = __builtin_fmaxf(__builtin_fmaxf(0.0f, ay - f[1]), f[1] - ay - 1.0f);
    const float dz = __builtin_fmaxf(__builtin_fmaxf(0.0f, az - f[0]), f[0] - az - 1.0f);
    const float lb = ((sx2 * dx * dx + sy2 * dy * dy) + sz2 * dz * dz) + m * m;
    return lb < F + F * 0x1p-8f;
}

// The counts of a block of 256 threads (every thread calls): summed over its waves in LDS and
// added with one atomic per count.  An atomic per wave on these few addresses serialises.
__device__ __forceinline__ void grids_counts(Scalars* sc, uint32_t npass, uint32_t nborder, unsigned long long cells,
                                             uint32_t gm) {
    __shared__ unsigned long long s_c[4];
    __shared__ uint32_t s_p[4], s_b[4], s_g[4];
    for (int o = 32; o > 0; o >>= 1) {
        npass += (uint32_t)__shfl_xor((int)npass, o);
        nborder += (uint32_t)__shfl_xor((int)nborder, o);
        gm = max(gm, (uint32_t)__shfl_xor((int)gm, o));
        cells += (unsigned long long)__shfl_xor((long long)cells, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_p[w] = npass;
        s_b[w] = nborder;
        s_g[w] = gm;
        s_c[w] = cells;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        npass = s_p[0] + s_p[1] + s_p[2] + s_p[3];
        nborder = s_b[0] + s_b[1] + s_b[2] + s_b[3];
        gm = max(max(s_g[0], s_g[1]), max(s_g[2], s_g[3]));
        cells = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (npass) atomicAdd(&sc->n_pass, (unsigned long long)npass);
        if (nborder) atomicAdd(&sc->n_border, (unsigned long long)nborder);
        if (cells) atomicAdd(&sc->n_cells, cells);
        if (gm) atomicMax(&sc->maxg2_bits, gm);
    }
}

// The 27 key-0 cells (offsets a in {-1,0,1}^3 from the holding cell) of every listed node,
// one lane per node, from the 4x4x4 evaluation neighbourhood loaded one z-pair of planes at
// a time (clamped at the grid faces; cells that do not exist are skipped).  A node whose
// bound is at most k1 is finished; the others go to the tail list.
template <int GMODE>
__global__ __launch_bounds__(256) void k_grids_zero(GridsArgs a) {
    const uint32_t M = a.sc->n_masked;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x * 256 >= M) return;   // uniform
    const bool live = i < M;
    const int r = live ? (int)a.list[i] : (int)a.list[0];
    double u[3];
    bool inside;
    grids_pos(a, r, u, inside);
    int c0[3];
    float f[3];
    grids_cell<float>(a, u, c0, f);
    const float dr = a.ref[r];
    const float inv_dd = node_inv_dd(dr, a.sc->inv_dd, (float)a.dd, a.local);
    const float sx2 = (float)((a.eh[2] / a.dta) * (a.eh[2] / a.dta)), sy2 = (float)((a.eh[1] / a.dta) * (a.eh[1] / a.dta)),
                sz2 = (float)((a.eh[0] / a.dta) * (a.eh[0] / a.dta));
    const InvS2<float> is = inv_s2<float>(sx2, sy2, sz2);
    const int enx = a.en[2], eny = a.en[1], enz = a.en[0];
    // per axis: does the cell at -1 exist, is the cell at +1 whole
    const bool lox = c0[2] > 0, loy = c0[1] > 0, loz = c0[0] > 0;
    const bool hix = c0[2] + 2 < enx, hiy = c0[1] + 2 < eny, hiz = c0[0] + 2 < enz;
    const bool bnd = !(lox && loy && loz && hix && hiy && hiz);
    const bool wave_masked = __ballot(live && bnd) != 0ull;
    auto cl = [](int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); };
    int ix[4], iy[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        ix[d] = cl(c0[2] - 1 + d, enx);
        iy[d] = cl(c0[1] - 1 + d, eny);
    }
    float F = live ? a.f0[i] : 0.0f;
    uint32_t cells = 0, n_fp64 = 0;
    bool ill = false;
    GuardCtx gc{};
#pragma unroll 1
    for (int az = -1; az <= 1; ++az) {
        // the two planes of this slab of cells
        float pl[2][16];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int64_t zb = (int64_t)cl(c0[0] + az + p, enz) * eny;
#pragma unroll
            for (int dy = 0; dy < 4; ++dy)
#pragma unroll
                for (int dx = 0; dx < 4; ++dx)
                    pl[p][dy * 4 + dx] = a.ev[(zb + iy[dy]) * enx + ix[dx]];
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int k = 0; k < 16; ++k) pl[p][k] = dose_norm<float>(pl[p][k], dr, inv_dd);
        const bool ez = az < 0 ? loz : true, okz = az > 0 ? hiz : true;
#pragma unroll
        for (int ay = -1; ay <= 1; ++ay)
#pragma unroll
            for (int ax = -1; ax <= 1; ++ax) {
                float g[8];
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    g[b] = pl[(b >> 2) & 1][(ay + 1 + ((b >> 1) & 1)) * 4 + (ax + 1 + (b & 1))];
                const bool ey = ay < 0 ? loy : true, oky = ay > 0 ? hiy : true;
                const bool ex = ax < 0 ? lox : true, okx = ax > 0 ? hix : true;
                const bool exists = live && ex && ey && ez;
                const bool whole = okx && oky && okz;
                cells += (exists && (whole || !wave_masked)) ? 1u : 0u;
                const bool need = exists && grids_need(g, (float)ax, (float)ay, (float)az, f, sx2, sy2, sz2, F);
                float v = Num<float>::inf();
                if (__ballot(need) != 0ull && need) {
                    const Geo<float> G = geo_frac<float>((float)ax - f[2], (float)ay - f[1], (float)az - f[0], sx2,
                                                         sy2, sz2, is);
                    if (wave_masked)
                        v = cell3<float, true, GMODE>(g, G, is, okx, oky, okz, a.den_guard, gc, n_fp64, ill);
                    else
                        v = cell3<float, false, GMODE>(g, G, is, true, true, true, a.den_guard, gc, n_fp64, ill);
                }
                F = vmin<float>(F, v);
            }
    }
    ill = ill && live;
    const bool to_guard = GMODE == 1 && ill;
    const bool to_tail = live && !to_guard && F > a.k1;
    uint32_t npass = 0, nborder = 0, gm = 0;
    unsigned long long ncells = 0;
    if (live && !to_guard && !to_tail) {
        const float gam = sqrtf(F);
        a.gamma[r] = gam;
        npass = gam <= 1.0f;
        nborder = fabsf(gam - 1.0f) <= 1e-5f;
        gm = f2u(gam * gam);
        ncells = cells;
    }
    const uint32_t tpos = block_append(to_tail, &a.sc->n_tail);
    if (to_tail) {
        a.tail_list[tpos] = (uint32_t)r;
        a.tail_f[tpos] = F;
    }
    if (GMODE == 1) {
        const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
        if (to_guard) a.guard_list[gpos] = (uint32_t)r;
    }
    // tail nodes count their key-0 cells in the walk's total: add them here
    if (to_tail) ncells = cells;
    grids_counts(a.sc, npass, nborder, ncells, gm);
}

// LIST 0: the listed nodes from row 0; 1: the guard list (FP64) from row 0; 2: the tail
// list of the key-0 pass from the first row past the key-0 cells.
template <typename T, int GMODE, int LIST>
__global__ __launch_bounds__(256) void k_grids_walk(GridsArgs a, int G) {
    constexpr bool GUARD = LIST == 1;
    const uint32_t M = LIST == 1 ? a.sc->n_guard : (LIST == 2 ? a.sc->n_tail : a.sc->n_masked);
    const uint32_t* list = LIST == 1 ? a.guard_list : (LIST == 2 ? a.tail_list : a.list);
    const int first = LIST == 2 ? 27 : 0;
    const int GROUPS = 256 / G;
    const int gl = threadIdx.x % G;
    const double dmax = (double)ord_to_float(a.sc->dmax_ord);
    const float inv_dd_g = a.sc->inv_dd;
    const T sx2 = (T)((a.eh[2] / a.dta) * (a.eh[2] / a.dta)), sy2 = (T)((a.eh[1] / a.dta) * (a.eh[1] / a.dta)),
            sz2 = (T)((a.eh[0] / a.dta) * (a.eh[0] / a.dta));
    const InvS2<T> is = inv_s2<T>(sx2, sy2, sz2);
    const int enx = a.en[2], eny = a.en[1], enz = a.en[0], esxy = enx * eny;
    uint32_t npass = 0, nborder = 0, gm = 0, n_fp64 = 0;
    unsigned long long cells = 0;
    GuardCtx gc{};
    for (uint64_t base = (uint64_t)blockIdx.x * GROUPS; base < M; base += (uint64_t)gridDim.x * GROUPS) {
        const uint32_t i = (uint32_t)base + threadIdx.x / G;
        const bool live = i < M;
        const int r = live ? (int)list[i] : 0;
        double u[3];
        bool inside;
        grids_pos(a, r, u, inside);
        int c0[3];
        T f[3];
        grids_cell<T>(a, u, c0, f);
        const float dr32 = a.ref[r];
        const T dr = (T)dr32;
        T inv_dd;
        if constexpr (sizeof(T) == 8)
            inv_dd = a.local ? (T)(1.0 / (a.dd * (double)dr32)) : (T)(1.0 / (a.dd * dmax));
        else
            inv_dd = (T)node_inv_dd(dr32, inv_dd_g, (float)a.dd, a.local);
        T F = T(0);
        if (live) {
            if constexpr (LIST == 2) F = (T)a.tail_f[i];
            else if (GUARD || sizeof(T) == 8) F = grids_f0<T>(a, c0, f, dr, inv_dd);
            else F = (T)a.f0[i];
        }
        uint32_t lane_cells = 0;
        bool ill = false;
        for (int n0 = first; n0 < a.tab_len; n0 += G) {
            const bool grp_act = live && (T)a.tab[n0].key2 < F;
            if (__ballot(grp_act) == 0ull) break;
            const int n = n0 + gl;
            TabEntry e;
            bool act = false;
            if (grp_act && n < a.tab_len) {
                e = a.tab[n];
                act = (T)e.key2 < F;
            }
            int cz = 0, cy = 0, cx = 0;
            if (act) {
                cz = c0[0] + e.az;
                cy = c0[1] + e.ay;
                cx = c0[2] + e.ax;
            }
            const bool cin = (unsigned)cx < (unsigned)enx && (unsigned)cy < (unsigned)eny && (unsigned)cz < (unsigned)enz;
            const bool okx = cx + 1 < enx, oky = cy + 1 < eny, okz = cz + 1 < enz;
            const bool work = act && cin;
            const bool edge = !(okx && oky && okz);
            const bool wave_masked = __ballot(work && edge) != 0ull;
            T c = Num<T>::inf();
            T g[8];
            bool need = false;
            if (work) {
                lane_cells += edge ? 0u : 1u;
                const int64_t b = (int64_t)cz * esxy + (int64_t)cy * enx + cx;
                const int ox = okx ? 1 : 0, oy = oky ? enx : 0, oz = okz ? esxy : 0;
                g[0] = dose_norm<T>((T)a.ev[b], dr, inv_dd);
                g[1] = dose_norm<T>((T)a.ev[b + ox], dr, inv_dd);
                g[2] = dose_norm<T>((T)a.ev[b + oy], dr, inv_dd);
                g[3] = dose_norm<T>((T)a.ev[b + oy + ox], dr, inv_dd);
                g[4] = dose_norm<T>((T)a.ev[b + oz], dr, inv_dd);
                g[5] = dose_norm<T>((T)a.ev[b + oz + ox], dr, inv_dd);
                g[6] = dose_norm<T>((T)a.ev[b + oz + oy], dr, inv_dd);
                g[7] = dose_norm<T>((T)a.ev[b + oz + oy + ox], dr, inv_dd);
                need = true;
                if constexpr (sizeof(T) == 4) need = grids_need(g, (float)e.ax, (float)e.ay, (float)e.az, f, sx2, sy2, sz2, F);
            }
            if (__ballot(need) != 0ull && need) {
                const Geo<T> Gm = geo_frac<T>((T)e.ax - f[2], (T)e.ay - f[1], (T)e.az - f[0], sx2, sy2, sz2, is);
                if (wave_masked)
                    c = cell3<T, true, GMODE>(g, Gm, is, okx, oky, okz, (T)a.den_guard, gc, n_fp64, ill);
                else
                    c = cell3<T, false, GMODE>(g, Gm, is, true, true, true, (T)a.den_guard, gc, n_fp64, ill);
            }
            for (int o = G / 2; o > 0; o >>= 1) c = vmin<T>(c, __shfl_xor(c, o));
            F = vmin<T>(F, c);
        }
        for (int o = G / 2; o > 0; o >>= 1) {
            lane_cells += (uint32_t)__shfl_xor((int)lane_cells, o);
            ill = (__shfl_xor((int)ill, o) != 0) || ill;
        }
        const bool leader = live && gl == 0;
        const bool to_guard = GMODE == 1 && leader && ill;
        if (leader && !to_guard) {
            const float gam = (float)sqrt((double)F);
            a.gamma[r] = gam;
            npass += gam <= 1.0f;
            nborder += fabsf(gam - 1.0f) <= 1e-5f;
            gm = max(gm, f2u(gam * gam));
            cells += lane_cells;
        }
        if (GMODE == 1) {
            const uint32_t gpos = block_append(to_guard, &a.sc->n_guard);
            if (to_guard) a.guard_list[gpos] = (uint32_t)r;
        }
    }
    grids_counts(a.sc, npass, nborder, cells, gm);
}

}  // namespace

hipError_t launch_batch_key0(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s) {
    if (n_items > 0)
        hipLaunchKernelGGL(k_batch_key0, dim3((unsigned)n_items), dim3(SEARCH_THREADS), 0, s, pairs, items);
    return hipGetLastError();
}

hipError_t launch_batch_tail(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s) {
    if (n_items > 0)
        hipLaunchKernelGGL(k_batch_tail, dim3((unsigned)n_items), dim3(SEARCH_THREADS), 0, s, pairs, items);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s) {
    if (n_items > 0)
        hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)n_items), dim3(SEARCH_THREADS), 0, s, pairs, items);
    return hipGetLastError();
}

unsigned tail_grid_blocks(uint32_t m_bound, int g) {
    // as tail_pass: groups of |g| lanes (automatic: the least width), at most kTailBlocks
    const unsigned groups = SEARCH_THREADS / (unsigned)(g > 0 ? g : -g);
    unsigned gb = (m_bound + groups - 1) / groups;
    return gb > kTailBlocks ? kTailBlocks : gb;
}

unsigned guard_grid_blocks() { return kGuardBlocks; }

hipError_t launch_stamp(unsigned long long* t, hipStream_t s) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, t);
    return hipGetLastError();
}

int64_t search_sums_needed(uint32_t) { return SUM_BINS; }

hipError_t launch_search(const SearchArgs& a, const SearchPlan& p, hipStream_t s) {
    const unsigned nb = blocks_for(p.M);
    if (nb == 0) return hipSuccess;
    const unsigned tb = nb < kTailBlocks ? nb : kTailBlocks;
    BlockSums* sums = a.sums;
    int used = 0;
    if (p.precision == 2) {
        // FP64 throughout: one walk over all nodes from the first row
        if (p.ndim == 3) walk<3, 3, false>(a, a.nodes, &a.sc->n_masked, 0, nb, sums, s);
        else walk<2, 3, false>(a, a.nodes, &a.sc->n_masked, 0, nb, sums, s);
        used = (int)nb;
        if (p.ev_shell_end) (void)hipEventRecord(p.ev_shell_end, s);
        if (p.ev_sort_end) (void)hipEventRecord(p.ev_sort_end, s);
        if (p.ev_tail_end) (void)hipEventRecord(p.ev_tail_end, s);
    } else {
        const bool guarded = p.precision == 1 && p.ndim == 3;
        const int first = p.ndim == 3 ? 8 : 4;
        // pass A (unless a batch queued it for every pair in one launch)
        if (p.skip_zero) {
        } else if (p.zero_lanes) {
            // one lane per zero-key cell, grid-stride over the nodes
            const unsigned lanes = p.ndim == 3 ? 8u : 4u;
            uint64_t want = ((uint64_t)p.M * lanes + SEARCH_THREADS - 1) / SEARCH_THREADS;
            const unsigned zb = (unsigned)(want < kZeroGroupBlocks ? want : kZeroGroupBlocks);
            if (p.ndim == 3) {
                if (guarded) hipLaunchKernelGGL((k_zero_group<3, 1>), dim3(zb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
                else hipLaunchKernelGGL((k_zero_group<3, 0>), dim3(zb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
            } else {
                hipLaunchKernelGGL((k_zero_group<2, 0>), dim3(zb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
            }
        } else if (p.ndim == 3 && p.projection == 1) {
            // Ju's recursion in the key-0 pass (interior cells)
            if (guarded) hipLaunchKernelGGL((k_zero3<1, true>), dim3(nb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
            else hipLaunchKernelGGL((k_zero3<0, true>), dim3(nb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
        } else if (p.ndim == 3) {
            if (guarded) hipLaunchKernelGGL(k_zero3<1>, dim3(nb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
            else hipLaunchKernelGGL(k_zero3<0>, dim3(nb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
        } else {
            hipLaunchKernelGGL(k_zero2<0>, dim3(nb), dim3(SEARCH_THREADS), 0, s, a, p.zero, sums);
        }
        used += (int)nb;
        if (p.ev_shell_end) (void)hipEventRecord(p.ev_shell_end, s);
        if (p.after_zero) {
            hipError_t e = p.after_zero(p.after_zero_user, s);
            if (e != hipSuccess) return e;
        }
        // tail sort (count read on the device).  The order only groups similar walks into a
        // wave (every order gives the same map), so long tails are sorted by the keys' top 16
        // bits: two radix passes instead of four
        if (p.hist) {
            hipError_t e = p.small_sort
                               ? sort_order_small(a.tail_key_arr, a.tail_pos, &a.sc->n_tail, &a.sc->sort_overflow, s)
                               : radix_sort_pairs(a.tail_key_arr, a.tail_pos, p.tmp_keys, p.tmp_vals, p.M,
                                                  &a.sc->n_tail, p.hist, s, 16);
            if (e != hipSuccess) return e;
        }
        if (p.ev_sort_end) (void)hipEventRecord(p.ev_sort_end, s);
        // pass B (with the learned radius: the speculative walk, then the plain walk of the
        // nodes it could not certify, resumed where the speculative bound cut them off)
        if (a.tab_len > first) {
            const int spec = p.spec;
            used += (int)tail_pass(a, p, a.tail_pos, &a.sc->n_tail, first, guarded, spec, tb, sums, s);
            if (spec == 1)
                used += (int)tail_pass(a, p, a.fb_list, &a.sc->n_fallback, first, guarded, 2, tb, sums, s);
        }
        if (p.ev_tail_end) (void)hipEventRecord(p.ev_tail_end, s);
        // guard pass, with the count reduction in the same launch
        if (guarded) {
            hipLaunchKernelGGL(k_guard_finalize, dim3(kGuardBlocks), dim3(SEARCH_THREADS), 0, s, a, a.tab, sums);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(SEARCH_THREADS), 0, s, sums, SUM_BINS, a.sc, a.r2_cap);
    return hipGetLastError();
}


hipError_t launch_grids_prep(const GridsArgs& a, hipStream_t s) {
    const int64_t nr = (int64_t)a.rn[0] * a.rn[1] * a.rn[2];
    const int64_t ne = (int64_t)a.en[0] * a.en[1] * a.en[2];
    const int64_t n = nr > ne ? nr : ne;
    constexpr int64_t kMaxBlocks = 512;   // partials each listing block reduces (<= MAX_BLOCKS)
    static_assert(kMaxBlocks <= MAX_BLOCKS, "the partials buffer holds MAX_BLOCKS words");
    const int64_t nb1 = (n + 256 * GRIDS_MAX_ITEMS - 1) / (256 * GRIDS_MAX_ITEMS);
    const unsigned b1 = (unsigned)(nb1 < kMaxBlocks ? nb1 : kMaxBlocks);
    hipLaunchKernelGGL(k_grids_max, dim3(b1), dim3(256), 0, s, a, nr, ne);
    const int64_t chunks = (nr + 256 * GRIDS_PER_THREAD - 1) / (256 * GRIDS_PER_THREAD);
    const unsigned b2 = (unsigned)(chunks < 4096 ? chunks : 4096);
    hipLaunchKernelGGL(k_grids_list, dim3(b2), dim3(256), 0, s, a, nr, (int)b1);
    return hipGetLastError();
}

hipError_t launch_grids_walk(const GridsArgs& a, int precision, bool guard, int lanes, hipStream_t s) {
    const int G = lanes;
    const dim3 grid(2048), block(256);
    if (guard) hipLaunchKernelGGL((k_grids_walk<double, 0, 1>), grid, block, 0, s, a, G);
    else if (precision == 2) hipLaunchKernelGGL((k_grids_walk<double, 0, 0>), grid, block, 0, s, a, G);
    else if (precision == 1) hipLaunchKernelGGL((k_grids_walk<float, 1, 0>), grid, block, 0, s, a, G);
    else hipLaunchKernelGGL((k_grids_walk<float, 0, 0>), grid, block, 0, s, a, G);
    return hipGetLastError();
}

hipError_t launch_grids_zero(const GridsArgs& a, int precision, hipStream_t s) {
    const int64_t nr = (int64_t)a.rn[0] * a.rn[1] * a.rn[2];   // the list holds at most nr nodes
    const unsigned nb = (unsigned)((nr + 255) / 256);
    if (precision == 1) hipLaunchKernelGGL(k_grids_zero<1>, dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_grids_zero<0>, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_grids_tail(const GridsArgs& a, int precision, int lanes, hipStream_t s) {
    const dim3 grid(2048), block(256);
    if (precision == 1) hipLaunchKernelGGL((k_grids_walk<float, 1, 2>), grid, block, 0, s, a, lanes);
    else hipLaunchKernelGGL((k_grids_walk<float, 0, 2>), grid, block, 0, s, a, lanes);
    return hipGetLastError();
}

}  // namespace gammax
