// Radially sorted cell table (Algorithm A1 steps 2-3; Algorithm A2 steps 4-5, "Kernel 2").
//
// One thread per candidate cell offset in the box that the radius allows: the key
// (minimum distance from the reference node to the closed cell, over DTA) is computed
// in FP64 and rounded toward -inf to float, so a float comparison never skips a cell
// that could hold a closer simplex.  Candidates are then sorted by the radix sort and
// the kept prefix is expanded into 64-byte rows with the per-offset spatial constants
// the search needs.
#include <cmath>

#include "internal.hpp"

namespace gammax {

namespace {

__device__ __forceinline__ void decode_box(const TableGeom& g, uint32_t j, int64_t a[3]) {
    int64_t rem = j;
    for (int i = g.ndim - 1; i >= 0; --i) {
        a[i] = g.lo[i] + rem % g.ext[i];
        rem /= g.ext[i];
    }
}

__device__ __forceinline__ double key2_of(const TableGeom& g, const int64_t a[3]) {
    double k2 = 0.0;
    for (int i = 0; i < g.ndim; ++i) {
        int64_t m;
        if (g.lower) m = a[i] > 1 ? a[i] - 1 : (a[i] < -1 ? -a[i] - 1 : 0);
        else m = a[i] > 0 ? a[i] : (a[i] < -1 ? -a[i] - 1 : 0);
        double d = g.s[i] * (double)m;
        k2 += d * d;
    }
    return k2;
}

__global__ __launch_bounds__(256) void k_table_gen(TableGeom g, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ count) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    if (j < g.box) {
        int64_t a[3] = {0, 0, 0};
        decode_box(g, (uint32_t)j, a);
        double k2 = key2_of(g, a);
        keep = k2 < g.r2_cap;
        keys[j] = keep ? __float_as_uint(__double2float_rd(k2)) : 0xFFFFFFFFu;
        vals[j] = (uint32_t)j;
    }
    unsigned long long b = __ballot(keep);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (uint32_t)__popcll(b));
}

// Spatial constants of the row for offset a (slowest axis first), in double, rounded to
// float; key2 is filled by the caller.
__host__ __device__ inline void fill_row(int ndim, const double* s, const int64_t* a, TabEntry& e) {
    // axis letters: x = fastest, y, z = slowest
    double ax, ay, az, sx2, sy2, sz2;
    if (ndim == 3) {
        az = (double)a[0]; ay = (double)a[1]; ax = (double)a[2];
        sz2 = s[0] * s[0]; sy2 = s[1] * s[1]; sx2 = s[2] * s[2];
    } else {
        az = 0.0; ay = (double)a[0]; ax = (double)a[1];
        sz2 = 0.0; sy2 = s[0] * s[0]; sx2 = s[1] * s[1];
    }
    e.ax = (int32_t)ax;
    e.ay = (int32_t)ay;
    e.az = (int32_t)az;
    e.px = (float)(sx2 * ax * ax);
    e.py = (float)(sy2 * ay * ay);
    e.pz = (float)(sz2 * az * az);
    const double dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    e.vxy = (float)(sx2 * sy2 * dxy * dxy / (sx2 + sy2));
    e.mxy = (float)((sx2 * ax + sy2 * ay) / (sx2 + sy2));
    if (ndim == 3) {
        const double sxyz = sx2 + sy2 + sz2;
        e.vxz = (float)(sx2 * sz2 * dxz * dxz / (sx2 + sz2));
        e.vyz = (float)(sy2 * sz2 * dyz * dyz / (sy2 + sz2));
        e.vxyz = (float)((sx2 * sy2 * dxy * dxy + sx2 * sz2 * dxz * dxz + sy2 * sz2 * dyz * dyz) / sxyz);
        e.mxz = (float)((sx2 * ax + sz2 * az) / (sx2 + sz2));
        e.myz = (float)((sy2 * ay + sz2 * az) / (sy2 + sz2));
        e.mxyz = (float)((sx2 * ax + sy2 * ay + sz2 * az) / sxyz);
    } else {
        e.vxz = e.vyz = e.vxyz = 0.0f;
        e.mxz = e.myz = e.mxyz = 0.0f;
    }
    e.pad = 0.0f;
}

__global__ __launch_bounds__(256) void k_table_rows(TableGeom g, const uint32_t* __restrict__ vals,
                                                    int64_t n, TabEntry* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t a[3] = {0, 0, 0};
    decode_box(g, vals[i], a);
    TabEntry e;
    fill_row(g.ndim, g.s, a, e);
    e.key2 = __double2float_rd(key2_of(g, a));
    rows[i] = e;
}

__global__ __launch_bounds__(256) void k_table_export(const TabEntry* __restrict__ rows, int64_t n,
                                                      float* __restrict__ key2,
                                                      int32_t* __restrict__ offs, int ndim) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    TabEntry e = rows[i];
    key2[i] = e.key2;
    if (ndim == 3) {
        offs[3 * i + 0] = e.az;
        offs[3 * i + 1] = e.ay;
        offs[3 * i + 2] = e.ax;
    } else {
        offs[3 * i + 0] = e.ay;
        offs[3 * i + 1] = e.ax;
        offs[3 * i + 2] = 0;
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void table_row_host(int ndim, const double s[3], int az, int ay, int ax, TabEntry* out) {
    int64_t a[3];
    if (ndim == 3) {
        a[0] = az; a[1] = ay; a[2] = ax;
    } else {
        a[0] = ay; a[1] = ax; a[2] = 0;
    }
    fill_row(ndim, s, a, *out);
    double k2 = 0.0;
    for (int i = 0; i < ndim; ++i) {
        const int64_t m = a[i] > 0 ? a[i] : (a[i] < -1 ? -a[i] - 1 : 0);
        const double d = s[i] * (double)m;
        k2 += d * d;
    }
    float f = (float)k2;                       // nearest, then step down if above
    if ((double)f > k2) f = std::nextafter(f, -INFINITY);
    out->key2 = f;
}

void table_box(TableGeom& g) {
    const double r = std::sqrt(g.r2_cap);
    g.box = 1;
    for (int i = 0; i < 3; ++i) {
        if (i >= g.ndim) {
            g.lo[i] = 0;
            g.ext[i] = 1;
            continue;
        }
        // max(0, a, -a-1) < r / s_i  =>  a in [-(c+1), c] with c = ceil(r / s_i)
        double c = std::ceil(r / g.s[i]);
        int64_t lim = (c > (double)g.shape[i]) ? g.shape[i] : (int64_t)c;
        int64_t lo = -lim - 1, hi = g.lower ? lim + 1 : lim;
        if (lo < -(g.shape[i] - 1)) lo = -(g.shape[i] - 1);
        if (hi > g.shape[i] - 1) hi = g.shape[i] - 1;
        g.lo[i] = lo;
        g.ext[i] = hi - lo + 1;
        g.box *= g.ext[i];
    }
}

hipError_t launch_table_gen(const TableGeom& g, uint32_t* keys, uint32_t* vals, uint32_t* count,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_table_gen, dim3(blocks_for(g.box)), dim3(256), 0, s, g, keys, vals, count);
    return hipGetLastError();
}

hipError_t launch_table_rows(const TableGeom& g, const uint32_t* vals, int64_t n, TabEntry* rows,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_rows, dim3(blocks_for(n)), dim3(256), 0, s, g, vals, n, rows);
    return hipGetLastError();
}

hipError_t launch_table_export(const TabEntry* rows, int64_t n, int ndim, float* key2, int32_t* offs,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_export, dim3(blocks_for(n)), dim3(256), 0, s, rows, n, key2, offs, ndim);
    return hipGetLastError();
}

}  // namespace gammax
