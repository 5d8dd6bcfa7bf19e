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

// One chain step: Delta, w = Delta / sigma^2, p = Delta^2 / sigma^2, m = Delta * mu.
template <typename T>
struct Step {
    T d, w, p, m;
};
template <typename T>
__device__ __forceinline__ Step<T> mk_step(T hi, T lo, T mu, T inv_s2) {
    Step<T> s;
    s.d = hi - lo;
    s.w = s.d * inv_s2;
    s.p = s.d * s.w;
    s.m = s.d * mu;
    return s;
}

template <typename T>
__device__ __forceinline__ T face1(T g0, const Step<T>& a, T mua, T perp) {
    const T N = g0 - a.m;
    const T L = N * Num<T>::rcp(T(1) + a.p);
    const T t1 = -mua - a.w * L;
    return (t1 >= T(0) && t1 <= T(1)) ? perp + N * L : Num<T>::inf();
}
template <typename T>
__device__ __forceinline__ T face2(T g0, const Step<T>& a, T mua, const Step<T>& b, T mub, T perp) {
    const T N = (g0 - a.m) - b.m;
    const T L = N * Num<T>::rcp((T(1) + a.p) + b.p);
    const T t1 = -mua - a.w * L;
    const T t2 = -mub - b.w * L;
    return (t1 <= T(1) && t1 >= t2 && t2 >= T(0)) ? perp + N * L : Num<T>::inf();
}
template <typename T>
__device__ __forceinline__ T face3(T g0, const Step<T>& a, T mua, const Step<T>& b, T mub,
                                   const Step<T>& c, T muc, T& den_out) {
    const T N = ((g0 - a.m) - b.m) - c.m;
    const T den = ((T(1) + a.p) + b.p) + c.p;
    den_out = den;
    const T L = N * Num<T>::rcp(den);
    const T t1 = -mua - a.w * L;
    const T t2 = -mub - b.w * L;
    const T t3 = -muc - c.w * L;
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

// All faces owned by one 3D cell; returns the smallest dist^2 (or +inf).
// ok_*: the cell extends along that axis inside the grid (MASKED only).
// GMODE 0: no guard; 1: flag an ill-conditioned tetrahedron (ill = true); 2: project it
// again in FP64.
template <typename T, bool MASKED, int GMODE>
__device__ __forceinline__ T cell3(const T* g, const Geo<T>& G, const InvS2<T>& is, bool okx, bool oky,
                                   bool okz, T den_guard, const GuardCtx& gc, uint32_t& n_fp64,
                                   bool& ill) {
    const T INF = Num<T>::inf();
    const T g0 = g[0];
    // chain steps, named by start vertex bits and block (x = bit0, y = bit1, z = bit2)
    const Step<T> s0x = mk_step(g[1], g[0], G.ax, is.x);
    const Step<T> s0y = mk_step(g[2], g[0], G.ay, is.y);
    const Step<T> s0z = mk_step(g[4], g[0], G.az, is.z);
    const Step<T> s0xy = mk_step(g[3], g[0], G.mxy, is.xy);
    const Step<T> s0xz = mk_step(g[5], g[0], G.mxz, is.xz);
    const Step<T> s0yz = mk_step(g[6], g[0], G.myz, is.yz);
    const Step<T> s0xyz = mk_step(g[7], g[0], G.mxyz, is.xyz);
    const Step<T> s1y = mk_step(g[3], g[1], G.ay, is.y);
    const Step<T> s1z = mk_step(g[5], g[1], G.az, is.z);
    const Step<T> s1yz = mk_step(g[7], g[1], G.myz, is.yz);
    const Step<T> s2x = mk_step(g[3], g[2], G.ax, is.x);
    const Step<T> s2z = mk_step(g[6], g[2], G.az, is.z);
    const Step<T> s2xz = mk_step(g[7], g[2], G.mxz, is.xz);
    const Step<T> s4x = mk_step(g[5], g[4], G.ax, is.x);
    const Step<T> s4y = mk_step(g[6], g[4], G.ay, is.y);
    const Step<T> s4xy = mk_step(g[7], g[4], G.mxy, is.xy);
    const Step<T> s3z = mk_step(g[7], g[3], G.az, is.z);
    const Step<T> s5y = mk_step(g[7], g[5], G.ay, is.y);
    const Step<T> s6x = mk_step(g[7], g[6], G.ax, is.x);

    // vertex q
    T best = (G.px + G.py + G.pz) + g0 * g0;
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

template <typename T, bool MASKED>
__device__ __forceinline__ T cell2(const T* g, const Geo<T>& G, const InvS2<T>& is, bool okx, bool oky) {
    const T INF = Num<T>::inf();
    const T g0 = g[0];
    const Step<T> s0x = mk_step(g[1], g[0], G.ax, is.x);
    const Step<T> s0y = mk_step(g[2], g[0], G.ay, is.y);
    const Step<T> s0xy = mk_step(g[3], g[0], G.mxy, is.xy);
    const Step<T> s1y = mk_step(g[3], g[1], G.ay, is.y);
    const Step<T> s2x = mk_step(g[3], g[2], G.ax, is.x);
    T best = (G.px + G.py) + g0 * g0;
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

// MODE 0: FP32.  MODE 1: FP32; a node that meets an ill-conditioned tetrahedron is not
// written but appended to the guard list.  MODE 2: FP32 with FP64 re-projection of the
// ill-conditioned tetrahedra (run over the guard list).  MODE 3: FP64 throughout.
template <int DIM, int MODE>
__global__ __launch_bounds__(SEARCH_THREADS) void k_search(SearchArgs a, const TabEntry* __restrict__ tab,
                                                           const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ count) {
    using T = typename std::conditional<MODE == 3, double, float>::type;
    constexpr int GMODE = DIM == 3 ? (MODE == 1 ? 1 : (MODE == 2 ? 2 : 0)) : 0;
    const uint32_t M = *count;
    const int lane = threadIdx.x & (WAVE - 1);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int sxy = nx * ny;
    const float inv_dd_g = a.sc_in->inv_dd;
    const double dmax = (double)ord_to_float(a.sc_in->dmax_ord);
    const InvS2<T> is = inv_s2<T>(MODE == 3 ? (T)(a.sx * a.sx) : (T)a.s2x,
                                  MODE == 3 ? (T)(a.sy * a.sy) : (T)a.s2y,
                                  DIM == 3 ? (MODE == 3 ? (T)(a.sz * a.sz) : (T)a.s2z) : T(0));
    const double sx2d = a.sx * a.sx, sy2d = a.sy * a.sy, sz2d = a.sz * a.sz;
    const uint32_t stride = gridDim.x * SEARCH_THREADS;
    uint32_t cells = 0, n_fp64 = 0, gm = 0, npass = 0, nborder = 0;

    for (uint32_t wbase = blockIdx.x * SEARCH_THREADS + (threadIdx.x & ~(WAVE - 1)); wbase < M;
         wbase += stride) {
        const uint32_t i = wbase + lane;
        const bool live = i < M;
        const int node = live ? (int)order[i] : 0;
        const int x = node % nx;
        const int y = (node / nx) % ny;
        const int z = DIM == 3 ? node / sxy : 0;
        const float dr = a.ref[node];
        const float de0 = a.ev[node];
        const float inv_dd = node_inv_dd(dr, inv_dd_g, a.dd, a.local);
        const double inv_dd64 = a.local ? 1.0 / (a.dd64 * (double)dr) : 1.0 / (a.dd64 * dmax);
        T F;
        if constexpr (MODE == 3) {
            const double g0 = ((double)de0 - (double)dr) * inv_dd64;
            F = g0 * g0;
        } else {
            F = gamma0_sq(de0, dr, inv_dd);
        }
        if (!live) F = T(0);
        const T invdd = MODE == 3 ? (T)inv_dd64 : (T)inv_dd;
        const T drT = (T)dr;
        uint32_t lane_cells = 0, lane_fp64 = 0;
        bool ill = false;

        for (int n = 0; n < a.tab_len; ++n) {
            const TabEntry e = tab[n];
            const bool act = live && ((T)e.key2 < F);
            if (__ballot(act) == 0ull) break;
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
                for (int b = 0; b < 8; ++b) g[b] = ((T)v[b] - drT) * invdd;
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
                for (int b = 0; b < 4; ++b) g[b] = ((T)v[b] - drT) * invdd;
                T c;
                if (wave_masked)
                    c = cell2<T, true>(g, G, is, okx, oky);
                else
                    c = cell2<T, false>(g, G, is, true, true);
                F = vmin<T>(F, c);
            }
        }

        if (MODE == 1 && live && ill) {
            // redone by the guarded pass; nothing of this node is written or counted here
            const uint32_t pos = atomicAdd(&a.sc->n_guard, 1u);
            a.guard_list[pos] = (uint32_t)node;
        } else if (live) {
            const float gam = (float)sqrt(F);
            a.gamma[node] = gam;
            npass += gam <= 1.0f;
            nborder += fabsf(gam - 1.0f) <= 1e-5f;
            gm = max(gm, __float_as_uint(gam * gam));
            cells += lane_cells;
            n_fp64 += lane_fp64;
        }
    }

    // counters: one atomic per wave
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        cells += (uint32_t)__shfl_xor((int)cells, o);
        n_fp64 += (uint32_t)__shfl_xor((int)n_fp64, o);
        npass += (uint32_t)__shfl_xor((int)npass, o);
        nborder += (uint32_t)__shfl_xor((int)nborder, o);
        gm = max(gm, (uint32_t)__shfl_xor((int)gm, o));
    }
    if (lane == 0) {
        if (npass) atomicAdd(&a.sc->n_pass, (unsigned long long)npass);
        if (nborder) atomicAdd(&a.sc->n_border, (unsigned long long)nborder);
        if (cells) atomicAdd(&a.sc->n_cells, (unsigned long long)cells);
        if (n_fp64) atomicAdd(&a.sc->n_fp64, (unsigned long long)n_fp64);
        if (gm) atomicMax(&a.sc->maxg2_bits, gm);
    }
}

template <int DIM, int MODE>
hipError_t launch_one(const SearchArgs& a, const uint32_t* order, const uint32_t* count, unsigned blocks,
                      hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_search<DIM, MODE>), dim3(blocks), dim3(SEARCH_THREADS), 0, s, a, a.tab, order, count);
    return hipGetLastError();
}

// Blocks of the pass over the guard list (grid-stride; the list is almost always empty).
constexpr unsigned kGuardBlocks = 64;

}  // namespace

hipError_t launch_search(const SearchArgs& a, int ndim, int precision, uint32_t max_items, hipStream_t s) {
    const unsigned blocks = (max_items + SEARCH_THREADS - 1) / SEARCH_THREADS;
    const uint32_t* cnt = &a.sc_in->n_masked;
    if (ndim == 3) {
        if (precision == 0) return launch_one<3, 0>(a, a.order, cnt, blocks, s);
        if (precision == 2) return launch_one<3, 3>(a, a.order, cnt, blocks, s);
        return launch_one<3, 1>(a, a.order, cnt, blocks, s);
    }
    if (precision == 2) return launch_one<2, 3>(a, a.order, cnt, blocks, s);
    return launch_one<2, 0>(a, a.order, cnt, blocks, s);
}

hipError_t launch_search_guard(const SearchArgs& a, int ndim, int precision, hipStream_t s) {
    if (ndim != 3 || precision != 1) return hipSuccess;
    return launch_one<3, 2>(a, a.guard_list, &a.sc_in->n_guard, kGuardBlocks, s);
}

}  // namespace gammax
