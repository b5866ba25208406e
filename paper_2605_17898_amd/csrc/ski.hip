// Structured kernel interpolation (SKI / KISS-GP; LightGP Sec. 2 "Structured
// kernel interpolation", Sec. 3 "Inference": SKI with FFT for O(N log N)
// products).  Following Wilson & Nickisch (2015):
//   K_XX ~ W K_UU W^T,   K_y V ~ W K_UU W^T V + sigma^2 V,
// U a regular grid of m_0 x .. x m_{D-1} points (D <= 3), W the local cubic
// convolution interpolation of Keys (1981, a = -1/2): 4 nodes per dimension.
//
// Grid (per dimension k): data range [min_k, max_k] (from the points, or the
// caller's), r_k = max_k - min_k (1 if zero), spacing h_k = r_k / (m_k - 4),
// first node lo_k = min_k - h_k, so a point's stencil b - 1 .. b + 2 of its
// cell b lies on the grid; nodes off the grid (points outside the range)
// are skipped.
//
// K_UU is multilevel Toeplitz for a stationary kernel; its product is taken
// through the D-dimensional circulant embedding of size L_k = 2 m_k: the
// first column holds k(o h) at offsets o_k = j_k (j_k < m_k), L_k - j_k
// (j_k > m_k) and 0 at j_k = m_k; its FFT (FP64, hipFFT D2Z) is the
// spectrum.  The training points are bucketed once by the cell of their
// stencil (counting sort).  One product: form the padded grid [t][L] =
// W^T V without atomics (each grid entry sums over the points of the 4^D
// cells that reach it, FP64), FFT, multiply by the spectrum / prod L,
// inverse FFT, gather W (.) in FP64 and round once.
#include "internal.hpp"

#include <hipfft/hipfft.h>

#include <cmath>
#include <map>
#include <tuple>
#include <vector>

namespace mfgp {

namespace {

constexpr int kBoundBlocks = 256;

using SkiGeom = SkiGeomH;

struct KParams {
    int family;
    double inv_l[3];
    double s2;
    double period;
};

__device__ __forceinline__ void keys4(double f, double w[4]) {
    // distances 1 + f, f, 1 - f, 2 - f of nodes b - 1 .. b + 2 (a = -1/2)
    const double s0 = 1.0 + f, s1 = f, s2 = 1.0 - f, s3 = 2.0 - f;
    w[0] = ((-0.5 * s0 + 2.5) * s0 - 4.0) * s0 + 2.0;
    w[1] = (1.5 * s1 - 2.5) * s1 * s1 + 1.0;
    w[2] = (1.5 * s2 - 2.5) * s2 * s2 + 1.0;
    w[3] = ((-0.5 * s3 + 2.5) * s3 - 4.0) * s3 + 2.0;
}

// Stencil of a point: base node per dimension (b - 1) and the 4 weights;
// false for a non-finite coordinate.
__device__ __forceinline__ bool stencil(const float* __restrict__ x, const double* __restrict__ geo,
                                        const SkiGeom& g, int base[3], double w[3][4]) {
    for (int k = 0; k < g.d; ++k) {
        double t = (static_cast<double>(x[k]) - geo[k]) / geo[3 + k];
        if (!(t == t) || isinf(t)) return false;
        t = fmin(fmax(t, -4.0), static_cast<double>(g.m[k]) + 4.0);
        const double b = floor(t);
        base[k] = static_cast<int>(b) - 1;
        keys4(t - b, w[k]);
    }
    return true;
}

__global__ void ski_bounds_stage1(const float* __restrict__ X, int64_t n, const float* __restrict__ Xs, int64_t ms,
                                  int d, float* __restrict__ part) {
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t total = n + ms;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float* x = i < n ? X + i * d : Xs + (i - n) * d;
        for (int k = 0; k < d; ++k) {
            mn[k] = fminf(mn[k], x[k]);
            mx[k] = fmaxf(mx[k], x[k]);
        }
    }
    __shared__ float smn[3][256], smx[3][256];
    for (int k = 0; k < 3; ++k) {
        smn[k][threadIdx.x] = mn[k];
        smx[k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 3; ++k) {
                smn[k][threadIdx.x] = fminf(smn[k][threadIdx.x], smn[k][threadIdx.x + off]);
                smx[k][threadIdx.x] = fmaxf(smx[k][threadIdx.x], smx[k][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        part[blockIdx.x * 6 + threadIdx.x] = smn[threadIdx.x][0];
        part[blockIdx.x * 6 + 3 + threadIdx.x] = smx[threadIdx.x][0];
    }
}

// geo[k] = lo_k, geo[3 + k] = h_k from the block minima / maxima (auto) or the
// caller's range (explicit: lo/hi arguments).
__global__ void ski_geo_kernel(const float* __restrict__ part, int nb, int explicit_range, SkiGeom g, float lo0,
                               float lo1, float lo2, float hi0, float hi1, float hi2, double* __restrict__ geo) {
    const int k = threadIdx.x;
    if (k >= g.d) return;
    float mn, mx;
    if (explicit_range) {
        mn = k == 0 ? lo0 : (k == 1 ? lo1 : lo2);
        mx = k == 0 ? hi0 : (k == 1 ? hi1 : hi2);
    } else {
        mn = INFINITY;
        mx = -INFINITY;
        for (int b = 0; b < nb; ++b) {
            mn = fminf(mn, part[b * 6 + k]);
            mx = fmaxf(mx, part[b * 6 + 3 + k]);
        }
    }
    double r = static_cast<double>(mx) - static_cast<double>(mn);
    if (!(r > 0.0)) r = 1.0;
    const double h = r / static_cast<double>(g.m[k] - 4);
    geo[k] = static_cast<double>(mn) - h;
    geo[3 + k] = h;
}

// First column of the circulant embedding (s2 k at the wrapped offsets).
__global__ void ski_column_kernel(SkiGeom g, const double* __restrict__ geo, KParams kp, double* __restrict__ c) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= g.Lr) return;
    int64_t rest = q;
    double r2 = 0.0, sp = 0.0;
    for (int k = 0; k < 3; ++k) {
        const int j = static_cast<int>(rest % g.L[k]);
        rest /= g.L[k];
        if (k >= g.d) continue;
        int o;
        if (j < g.m[k]) {
            o = j;
        } else if (j == g.m[k]) {
            c[q] = 0.0;
            return;
        } else {
            o = g.L[k] - j;
        }
        const double delta = o * geo[3 + k];
        const double u = delta * kp.inv_l[k];
        r2 += u * u;
        if (kp.family == MFGP_PERIODIC) {
            const double sn = sin(3.14159265358979323846 * delta / kp.period) * kp.inv_l[k];
            sp += 2.0 * sn * sn;
        }
    }
    double v;
    const double r = sqrt(r2);
    switch (kp.family) {
        case MFGP_RBF: v = exp(-0.5 * r2); break;
        case MFGP_MATERN12: v = exp(-r); break;
        case MFGP_MATERN32: v = (1.0 + sqrt(3.0) * r) * exp(-sqrt(3.0) * r); break;
        case MFGP_MATERN52: v = (1.0 + sqrt(5.0) * r + 5.0 * r2 / 3.0) * exp(-sqrt(5.0) * r); break;
        default: v = exp(-sp); break;
    }
    c[q] = kp.s2 * v;
}

// d c / d theta at the wrapped offsets for parameter `which` of the kernel's
// gradient order without sigma^2: the lengthscales (one per dimension when
// ard, else one shared), the period (periodic family), s2.  With u_k = D_k / l_k:
//   RBF         d/dl_k = s2 exp(-r^2/2) u_k^2 / l_k
//   Matern-1/2  d/dl_k = s2 exp(-r) u_k^2 / (r l_k)          (0 at r = 0)
//   Matern-3/2  d/dl_k = s2 3 exp(-sqrt3 r) u_k^2 / l_k
//   Matern-5/2  d/dl_k = s2 (5/3) (1 + sqrt5 r) exp(-sqrt5 r) u_k^2 / l_k
//   Periodic    d/dl_k = s2 exp(-S) 4 sin^2(pi D_k / p) / l_k^3,
//               d/dp   = s2 exp(-S) sum_k 2 pi D_k sin(2 pi D_k / p) / (p^2 l_k^2)
//   d/ds2 = the unit-scale kernel.
__global__ void ski_dcolumn_kernel(SkiGeom g, const double* __restrict__ geo, KParams kp, int ard, int which,
                                   double* __restrict__ c) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= g.Lr) return;
    const double pi = 3.14159265358979323846;
    int64_t rest = q;
    double delta[3] = {0, 0, 0}, u2[3] = {0, 0, 0};
    double r2 = 0.0, sp = 0.0;
    for (int k = 0; k < 3; ++k) {
        const int j = static_cast<int>(rest % g.L[k]);
        rest /= g.L[k];
        if (k >= g.d) continue;
        int o;
        if (j < g.m[k]) {
            o = j;
        } else if (j == g.m[k]) {
            c[q] = 0.0;
            return;
        } else {
            o = g.L[k] - j;
        }
        delta[k] = o * geo[3 + k];
        const double u = delta[k] * kp.inv_l[k];
        u2[k] = u * u;
        r2 += u2[k];
        if (kp.family == MFGP_PERIODIC) {
            const double sn = sin(pi * delta[k] / kp.period) * kp.inv_l[k];
            sp += 2.0 * sn * sn;
        }
    }
    const double r = sqrt(r2);
    const int nl = ard ? g.d : 1;
    double v = 0.0;
    if (which < nl) {
        for (int k = 0; k < g.d; ++k) {
            if (ard && k != which) continue;
            double f;
            switch (kp.family) {
                case MFGP_RBF: f = exp(-0.5 * r2) * u2[k]; break;
                case MFGP_MATERN12: f = r > 0.0 ? exp(-r) * u2[k] / r : 0.0; break;
                case MFGP_MATERN32: f = 3.0 * exp(-sqrt(3.0) * r) * u2[k]; break;
                case MFGP_MATERN52: f = (5.0 / 3.0) * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r) * u2[k]; break;
                default: {
                    const double sn = sin(pi * delta[k] / kp.period);
                    f = exp(-sp) * 4.0 * sn * sn * kp.inv_l[k] * kp.inv_l[k];
                }
            }
            v += f * kp.inv_l[k];
        }
        v *= kp.s2;
    } else if (kp.family == MFGP_PERIODIC && which == nl) {
        double a = 0.0;
        for (int k = 0; k < g.d; ++k)
            a += 2.0 * pi * delta[k] * sin(2.0 * pi * delta[k] / kp.period) * kp.inv_l[k] * kp.inv_l[k];
        v = kp.s2 * exp(-sp) * a / (kp.period * kp.period);
    } else {
        switch (kp.family) {
            case MFGP_RBF: v = exp(-0.5 * r2); break;
            case MFGP_MATERN12: v = exp(-r); break;
            case MFGP_MATERN32: v = (1.0 + sqrt(3.0) * r) * exp(-sqrt(3.0) * r); break;
            case MFGP_MATERN52: v = (1.0 + sqrt(5.0) * r + 5.0 * r2 / 3.0) * exp(-sqrt(5.0) * r); break;
            default: v = exp(-sp); break;
        }
    }
    c[q] = v;
}

// out[c] = sum_q a[c][q] b[c][q] (FP64, one block per column, fixed order)
__global__ void ski_dot_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t len,
                               double* __restrict__ out) {
    const int64_t off = static_cast<int64_t>(blockIdx.x) * len;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < len; q += blockDim.x) acc = fma(a[off + q], b[off + q], acc);
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Cell of a point's stencil: b_k + 2 per dimension (b_k the floor of its
// grid coordinate), flattened with dimension 0 fastest over m_k + 3 values;
// -1 for a non-finite point or one whose stencil misses the grid.
__device__ __forceinline__ int64_t point_cell(const float* __restrict__ x, const double* __restrict__ geo,
                                              const SkiGeom& g) {
    int64_t cell = 0, stride = 1;
    for (int k = 0; k < g.d; ++k) {
        double t = (static_cast<double>(x[k]) - geo[k]) / geo[3 + k];
        if (!(t == t) || isinf(t)) return -1;
        t = fmin(fmax(t, -4.0), static_cast<double>(g.m[k]) + 4.0);
        const int b = static_cast<int>(floor(t));
        if (b < -2 || b > g.m[k]) return -1;
        cell += (b + 2) * stride;
        stride *= g.m[k] + 3;
    }
    return cell;
}

__global__ void ski_count_kernel(const float* __restrict__ X, int64_t n, SkiGeom g, const double* __restrict__ geo,
                                 int* __restrict__ counts) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = point_cell(X + i * g.d, geo, g);
    if (c >= 0) atomicAdd(counts + c, 1);
}

// offsets = exclusive prefix sum of counts [len], offsets[len] = total, in
// three passes over tiles of kScanTile counts (tile sums; their prefix in one
// block; each tile's prefix plus its offset); counts is cleared for use as
// the placement cursor.
constexpr int kScanTile = 1024;

__global__ void ski_tile_sum_kernel(const int* __restrict__ counts, int64_t len, int* __restrict__ tsum) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int v = 0;
    for (int q = threadIdx.x; q < kScanTile; q += blockDim.x)
        if (base + q < len) v += counts[base + q];
    __shared__ int red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int sft = 128; sft > 0; sft >>= 1) {
        if (threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = red[0];
}

__global__ void ski_tile_prefix_kernel(int* __restrict__ tsum, int64_t ntile, int* __restrict__ offsets, int64_t len) {
    if (threadIdx.x != 0) return;
    int run = 0;
    for (int64_t b = 0; b < ntile; ++b) {
        const int v = tsum[b];
        tsum[b] = run;
        run += v;
    }
    offsets[len] = run;
}

__global__ void ski_tile_scan_kernel(int* __restrict__ counts, int64_t len, const int* __restrict__ tsum,
                                     int* __restrict__ offsets) {
    // thread q holds entries base + 4 q .. base + 4 q + 3 (256 threads x 4 = one tile)
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + 4 * threadIdx.x;
    int v[4], loc = 0;
    for (int e = 0; e < 4; ++e) {
        v[e] = base + e < len ? counts[base + e] : 0;
        loc += v[e];
    }
    __shared__ int sc[256];
    sc[threadIdx.x] = loc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan
        const int add = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    int run = tsum[blockIdx.x] + sc[threadIdx.x] - loc;
    for (int e = 0; e < 4; ++e) {
        if (base + e < len) {
            offsets[base + e] = run;
            counts[base + e] = 0;
        }
        run += v[e];
    }
}

// perm[pos] = i and frac[pos][k] = the fractional grid coordinate of point i
// (t_k - floor t_k) at its place pos in its cell's range.
__global__ void ski_place_kernel(const float* __restrict__ X, int64_t n, SkiGeom g, const double* __restrict__ geo,
                                 const int* __restrict__ offsets, int* __restrict__ cursor, int* __restrict__ perm,
                                 double* __restrict__ frac, int* __restrict__ pcell) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = point_cell(X + i * g.d, geo, g);
    if (c < 0) return;
    const int64_t pos = offsets[c] + atomicAdd(cursor + c, 1);
    perm[pos] = static_cast<int>(i);
    pcell[pos] = static_cast<int>(c);
    for (int k = 0; k < g.d; ++k) {
        double t = (static_cast<double>(X[i * g.d + k]) - geo[k]) / geo[3 + k];
        t = fmin(fmax(t, -4.0), static_cast<double>(g.m[k]) + 4.0);
        frac[pos * g.d + k] = t - floor(t);
    }
}

// Weight of stencil entry e (node b - 1 + e) at fractional coordinate f.
__device__ __forceinline__ double keys1(double f, int e) {
    double w[4];
    keys4(f, w);
    return w[e];
}

// The padded grid [t][Lr] = W^T V without atomics: thread per (grid entry,
// column); an entry inside the node box sums w V[p, c] over the points p of
// the 4^D cells whose stencils reach it (cells b_k + 2 = j_k .. j_k + 3), the
// weight recomputed from the point exactly as in the gather; padding gets 0.
template <typename T>
__global__ void ski_transpose_kernel(SkiGeom g, const T* __restrict__ V, int t, const int* __restrict__ offsets,
                                     const int* __restrict__ perm, const double* __restrict__ frac,
                                     double* __restrict__ grid) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= g.Lr * t) return;
    const int c = static_cast<int>(idx / g.Lr);
    int64_t rest = idx - static_cast<int64_t>(c) * g.Lr;
    int j[3];
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        j[k] = static_cast<int>(rest % g.L[k]);
        rest /= g.L[k];
        if (k < g.d && j[k] >= g.m[k]) inside = false;
    }
    double acc = 0.0;
    if (inside) {
        const int n1 = g.d > 1 ? 4 : 1, n2 = g.d > 2 ? 4 : 1;
        const int64_t s1 = g.m[0] + 3, s2 = s1 * (g.d > 1 ? g.m[1] + 3 : 1);
        for (int a2 = 0; a2 < n2; ++a2)
            for (int a1 = 0; a1 < n1; ++a1)
                for (int a0 = 0; a0 < 4; ++a0) {
                    // cell with b_k + 2 = j_k + a_k, i.e. node j_k is its stencil's entry 3 - a_k
                    const int64_t cell = (j[0] + a0) + (g.d > 1 ? (j[1] + a1) * s1 : 0) +
                                         (g.d > 2 ? (j[2] + a2) * s2 : 0);
                    const int q0 = offsets[cell], q1 = offsets[cell + 1];
                    for (int q = q0; q < q1; ++q) {
                        const int pnt = perm[q];
                        const double* fq = frac + static_cast<int64_t>(q) * g.d;
                        double wt = keys1(fq[0], 3 - a0);
                        if (g.d > 1) wt *= keys1(fq[1], 3 - a1);
                        if (g.d > 2) wt *= keys1(fq[2], 3 - a2);
                        acc = fma(wt, static_cast<double>(V[static_cast<int64_t>(pnt) * t + c]), acc);
                    }
                }
    }
    grid[idx] = acc;
}

// The same transpose with one wave per node entry and column (for launches
// with few entries): the lanes stride over the points of each of the 4^(D-1)
// cell rows (4 consecutive cells along dimension 0 each, one contiguous range
// of perm), and a fixed butterfly sums the lanes.  Padding entries get 0.
template <typename T>
__global__ void ski_transpose_wave_kernel(SkiGeom g, const T* __restrict__ V, int t, const int* __restrict__ offsets,
                                          const int* __restrict__ perm, const double* __restrict__ frac,
                                          const int* __restrict__ pcell, double* __restrict__ grid) {
    const int64_t idx = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (idx >= g.Lr * t) return;
    const int c = static_cast<int>(idx / g.Lr);
    int64_t rest = idx - static_cast<int64_t>(c) * g.Lr;
    int j[3];
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        j[k] = static_cast<int>(rest % g.L[k]);
        rest /= g.L[k];
        if (k < g.d && j[k] >= g.m[k]) inside = false;
    }
    double acc = 0.0;
    if (inside) {
        const int n1 = g.d > 1 ? 4 : 1, n2 = g.d > 2 ? 4 : 1;
        const int64_t s1 = g.m[0] + 3, s2 = s1 * (g.d > 1 ? g.m[1] + 3 : 1);
        for (int a2 = 0; a2 < n2; ++a2)
            for (int a1 = 0; a1 < n1; ++a1) {
                // cells (j0 + a0, j1 + a1, j2 + a2), a0 = 0..3: one contiguous range
                const int64_t c0 = j[0] + (g.d > 1 ? (j[1] + a1) * s1 : 0) + (g.d > 2 ? (j[2] + a2) * s2 : 0);
                const int q0 = offsets[c0], q1 = offsets[c0 + 4];
                for (int q = q0 + lane; q < q1; q += 64) {
                    const int a0 = static_cast<int>(pcell[q] - c0);   // 0..3 by construction
                    const int pnt = perm[q];
                    const double* fq = frac + static_cast<int64_t>(q) * g.d;
                    double wt = keys1(fq[0], 3 - a0);
                    if (g.d > 1) wt *= keys1(fq[1], 3 - a1);
                    if (g.d > 2) wt *= keys1(fq[2], 3 - a2);
                    acc = fma(wt, static_cast<double>(V[static_cast<int64_t>(pnt) * t + c]), acc);
                }
            }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) grid[idx] = acc;
}

__global__ void fill0i_kernel(int* __restrict__ a, int64_t total) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < total) a[idx] = 0;
}

// out = sum over the stencil of w grid[c][node] (FP64); then either
// OUT float: out[i, c] = that + sig2 Vself[i, c] (Vself may be null), or
// residual:  R[i, c] = B[i, c] - (that + sig2 X64[i, c]).
__global__ void ski_gather_kernel(const float* __restrict__ X, int64_t n, SkiGeom g, const double* __restrict__ geo,
                                  const double* __restrict__ grid, int t, double sig2, const float* __restrict__ Vself,
                                  float* __restrict__ out, const float* __restrict__ B,
                                  const double* __restrict__ X64, double* __restrict__ R) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * t) return;
    const int64_t i = idx / t;
    const int c = static_cast<int>(idx - i * t);
    int base[3] = {0, 0, 0};
    double w[3][4] = {{1, 0, 0, 0}, {1, 0, 0, 0}, {1, 0, 0, 0}};
    double acc = 0.0;
    if (stencil(X + i * g.d, geo, g, base, w)) {
        const double* gc = grid + static_cast<int64_t>(c) * g.Lr;
        const int n1 = g.d > 1 ? 4 : 1, n2 = g.d > 2 ? 4 : 1;
        for (int a2 = 0; a2 < n2; ++a2) {
            const int j2 = base[2] + a2;
            if (g.d > 2 && (j2 < 0 || j2 >= g.m[2])) continue;
            for (int a1 = 0; a1 < n1; ++a1) {
                const int j1 = base[1] + a1;
                if (g.d > 1 && (j1 < 0 || j1 >= g.m[1])) continue;
                const double w12 = (g.d > 2 ? w[2][a2] : 1.0) * (g.d > 1 ? w[1][a1] : 1.0);
                const int64_t row = (g.d > 1 ? j1 : 0) * static_cast<int64_t>(g.L[0]) +
                                    (g.d > 2 ? j2 : 0) * static_cast<int64_t>(g.L[0]) * g.L[1];
                for (int a0 = 0; a0 < 4; ++a0) {
                    const int j0 = base[0] + a0;
                    if (j0 < 0 || j0 >= g.m[0]) continue;
                    acc = fma(w12 * w[0][a0], gc[row + j0], acc);
                }
            }
        }
    }
    if (R) {
        R[idx] = static_cast<double>(B[idx]) - (acc + sig2 * X64[idx]);
    } else {
        if (Vself) acc += sig2 * static_cast<double>(Vself[idx]);
        out[idx] = static_cast<float>(acc);
    }
}

__global__ void ski_spectral_mul_kernel(hipfftDoubleComplex* __restrict__ spec, const hipfftDoubleComplex* __restrict__ lam,
                                        int64_t Lc, int t, double scale) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= Lc * t) return;
    const hipfftDoubleComplex a = spec[idx];
    const hipfftDoubleComplex b = lam[idx % Lc];
    spec[idx] = make_hipDoubleComplex((a.x * b.x - a.y * b.y) * scale, (a.x * b.y + a.y * b.x) * scale);
}

inline unsigned nblk(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

SkiGeom make_geom(int d, const int32_t* m) {
    SkiGeom g{};
    g.d = d;
    g.Lr = 1;
    for (int k = 0; k < 3; ++k) {
        g.m[k] = k < d ? m[k] : 1;
        g.L[k] = k < d ? 2 * m[k] : 1;
        g.Lr *= g.L[k];
    }
    g.Lc = static_cast<int64_t>(g.L[0] / 2 + 1) * g.L[1] * g.L[2];
    return g;
}

// hipFFT plans by (device, rank, sizes, batch, direction), kept per host
// thread until it releases them (release_fft_plans) or ends.  hipFFT places
// a plan's tables and work area in device memory when it creates it.
using PlanKey = std::tuple<int, int, int, int, int, int, int>;
thread_local std::map<PlanKey, hipfftHandle> plans;

hipfftHandle fft_plan(const SkiGeom& g, int batch, bool forward, hipError_t& err) {
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    const auto key = std::make_tuple(dev, g.d, g.L[0], g.L[1], g.L[2], batch, forward ? 1 : 0);
    auto it = plans.find(key);
    if (it != plans.end()) return it->second;
    int nn[3];
    for (int k = 0; k < g.d; ++k) nn[k] = g.L[g.d - 1 - k];   // slowest first
    hipfftHandle p = nullptr;
    if (hipfftPlanMany(&p, g.d, nn, nullptr, 1, static_cast<int>(g.Lr), nullptr, 1, static_cast<int>(g.Lc),
                       forward ? HIPFFT_D2Z : HIPFFT_Z2D, batch) != HIPFFT_SUCCESS) {
        err = hipErrorUnknown;
        return nullptr;
    }
    plans.emplace(key, p);
    return p;
}

}  // namespace

// Destroys the calling thread's cached plans, each with its device current.
hipError_t release_fft_plans() {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    for (auto& kv : plans) {
        if (hipSetDevice(std::get<0>(kv.first)) == hipSuccess) (void)hipfftDestroy(kv.second);
    }
    plans.clear();
    return hipSetDevice(cur);
}

static int64_t cell_count(const SkiGeom& g) {
    int64_t c = 1;
    for (int k = 0; k < g.d; ++k) c *= g.m[k] + 3;
    return c;
}

static int64_t tile_count(int64_t ncell) { return (ncell + kScanTile - 1) / kScanTile; }

size_t ski_scratch_bytes(int d, const int32_t* m, int t, int64_t n) {
    const SkiGeom g = make_geom(d, m);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t nc = static_cast<size_t>(cell_count(g)) + 1;
    return al(6 * sizeof(double)) + al(g.Lc * sizeof(hipfftDoubleComplex)) +
           al(static_cast<size_t>(t) * g.Lr * sizeof(double)) +
           al(static_cast<size_t>(t) * g.Lc * sizeof(hipfftDoubleComplex)) + al(kBoundBlocks * 6 * sizeof(float)) +
           2 * al(nc * sizeof(int)) + al(static_cast<size_t>(tile_count(nc)) * sizeof(int)) +
           al(static_cast<size_t>(n) * sizeof(int)) +
           al(static_cast<size_t>(n) * d * sizeof(double)) + al(static_cast<size_t>(n) * sizeof(int)) + 256;
}

// Grid geometry and spectrum for the kernel: the range from X (and Xs) or the
// caller's lo / hi; t the column count of the products that follow.
hipError_t ski_setup(SkiOp& op, const mfgp_kernel& k, const float* X, int64_t n, const float* Xs, int64_t ms,
                     const int32_t* m, const float* lo, const float* hi, int t, void* scratch, hipStream_t s) {
    op.g = make_geom(k.d, m);
    op.t = t;
    char* p = static_cast<char*>(scratch);
    auto take = [&](size_t b) {
        char* r = p;
        p += (b + 255) / 256 * 256;
        return r;
    };
    op.geo = reinterpret_cast<double*>(take(6 * sizeof(double)));
    op.lam = take(op.g.Lc * sizeof(hipfftDoubleComplex));
    op.grid = reinterpret_cast<double*>(take(static_cast<size_t>(t) * op.g.Lr * sizeof(double)));
    op.spec = take(static_cast<size_t>(t) * op.g.Lc * sizeof(hipfftDoubleComplex));
    op.part = reinterpret_cast<float*>(take(kBoundBlocks * 6 * sizeof(float)));
    op.ncell = cell_count(op.g);
    op.counts = reinterpret_cast<int*>(take((op.ncell + 1) * sizeof(int)));
    op.offsets = reinterpret_cast<int*>(take((op.ncell + 1) * sizeof(int)));
    int* tsum = reinterpret_cast<int*>(take(static_cast<size_t>(tile_count(op.ncell + 1)) * sizeof(int)));
    op.perm = reinterpret_cast<int*>(take(static_cast<size_t>(n) * sizeof(int)));
    op.frac = reinterpret_cast<double*>(take(static_cast<size_t>(n) * k.d * sizeof(double)));
    op.pcell = reinterpret_cast<int*>(take(static_cast<size_t>(n) * sizeof(int)));
    const bool expl = lo && hi;
    if (!expl) {
        hipLaunchKernelGGL(ski_bounds_stage1, dim3(kBoundBlocks), dim3(256), 0, s, X, n, Xs, Xs ? ms : 0, k.d, op.part);
    }
    float l3[3] = {0, 0, 0}, h3[3] = {0, 0, 0};
    for (int q = 0; q < k.d && expl; ++q) {
        l3[q] = lo[q];
        h3[q] = hi[q];
    }
    hipLaunchKernelGGL(ski_geo_kernel, dim3(1), dim3(64), 0, s, op.part, kBoundBlocks, expl ? 1 : 0, op.g, l3[0],
                       l3[1], l3[2], h3[0], h3[1], h3[2], op.geo);
    // bucket the training points by stencil cell (counting sort)
    hipLaunchKernelGGL(fill0i_kernel, dim3(nblk(op.ncell + 1)), dim3(256), 0, s, op.counts, op.ncell + 1);
    hipLaunchKernelGGL(ski_count_kernel, dim3(nblk(n)), dim3(256), 0, s, X, n, op.g, op.geo, op.counts);
    const int64_t ntile = tile_count(op.ncell);
    hipLaunchKernelGGL(ski_tile_sum_kernel, dim3(static_cast<unsigned>(ntile)), dim3(256), 0, s, op.counts, op.ncell,
                       tsum);
    hipLaunchKernelGGL(ski_tile_prefix_kernel, dim3(1), dim3(64), 0, s, tsum, ntile, op.offsets, op.ncell);
    hipLaunchKernelGGL(ski_tile_scan_kernel, dim3(static_cast<unsigned>(ntile)), dim3(256), 0, s, op.counts, op.ncell,
                       tsum, op.offsets);
    hipLaunchKernelGGL(ski_place_kernel, dim3(nblk(n)), dim3(256), 0, s, X, n, op.g, op.geo, op.offsets, op.counts,
                       op.perm, op.frac, op.pcell);
    KParams kp{};
    kp.family = k.family;
    kp.s2 = k.outputscale;
    kp.period = k.period;
    for (int q = 0; q < 3; ++q) kp.inv_l[q] = q < k.d ? 1.0 / (k.ard ? k.lengthscale[q] : k.lengthscale[0]) : 0.0;
    // the column in grid slot 0, its transform in lam
    hipLaunchKernelGGL(ski_column_kernel, dim3(nblk(op.g.Lr)), dim3(256), 0, s, op.g, op.geo, kp, op.grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipfftHandle f1 = fft_plan(op.g, 1, true, e);
    if (!f1) return e;
    if (hipfftSetStream(f1, s) != HIPFFT_SUCCESS ||
        hipfftExecD2Z(f1, op.grid, static_cast<hipfftDoubleComplex*>(op.lam)) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    return hipGetLastError();
}

// W^T V into the padded grid: a wave per entry while the launch is small
// (few entries, many points each), else a thread per entry.
constexpr int64_t kWaveEntries = int64_t(1) << 17;

template <typename T>
static hipError_t launch_transpose(const SkiOp& op, const T* V, int t, double* out, hipStream_t s) {
    const int64_t tot = op.g.Lr * t;
    if (tot <= kWaveEntries)
        hipLaunchKernelGGL((ski_transpose_wave_kernel<T>), dim3(nblk(tot * 64)), dim3(256), 0, s, op.g, V, t,
                           op.offsets, op.perm, op.frac, op.pcell, out);
    else
        hipLaunchKernelGGL((ski_transpose_kernel<T>), dim3(nblk(tot)), dim3(256), 0, s, op.g, V, t, op.offsets,
                           op.perm, op.frac, out);
    return hipGetLastError();
}

// One SKI product W_r K_UU W_c^T V over the columns' points Xc [nc] and the
// rows' points Xr [nr]; writes out (float, + sig2 Vself) or the FP64
// residual R = B - (product + sig2 X64) when R is non-null (then V = X64).
template <typename T>
static hipError_t ski_product(const SkiOp& op, const float* Xc, int64_t nc, const float* Xr, int64_t nr,
                              const T* V, int t, double sig2, const float* Vself, float* out, const float* B,
                              const double* X64, double* R, hipStream_t s) {
    if (t > op.t) return hipErrorInvalidValue;
    (void)Xc;   // the columns' points are the bucketed training points
    (void)nc;
    hipError_t e = launch_transpose<T>(op, V, t, op.grid, s);
    if (e != hipSuccess) return e;
    hipfftHandle fwd = fft_plan(op.g, t, true, e);
    if (!fwd) return e;
    hipfftHandle inv = fft_plan(op.g, t, false, e);
    if (!inv) return e;
    auto* spec = static_cast<hipfftDoubleComplex*>(op.spec);
    if (hipfftSetStream(fwd, s) != HIPFFT_SUCCESS || hipfftExecD2Z(fwd, op.grid, spec) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    hipLaunchKernelGGL(ski_spectral_mul_kernel, dim3(nblk(op.g.Lc * t)), dim3(256), 0, s, spec,
                       static_cast<const hipfftDoubleComplex*>(op.lam), op.g.Lc, t, 1.0 / static_cast<double>(op.g.Lr));
    if (hipfftSetStream(inv, s) != HIPFFT_SUCCESS || hipfftExecZ2D(inv, spec, op.grid) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    hipLaunchKernelGGL(ski_gather_kernel, dim3(nblk(nr * t)), dim3(256), 0, s, Xr, nr, op.g, op.geo, op.grid, t, sig2,
                       Vself, out, B, X64, R);
    return hipGetLastError();
}

hipError_t ski_apply(const SkiOp& op, const float* Xc, int64_t nc, const float* Xr, int64_t nr, const float* V, int t,
                     float* out, bool with_noise, float sig2, const float* Vself, hipStream_t s) {
    return ski_product<float>(op, Xc, nc, Xr, nr, V, t, with_noise ? static_cast<double>(sig2) : 0.0,
                              with_noise ? Vself : nullptr, out, nullptr, nullptr, nullptr, s);
}

hipError_t ski_residual(const SkiOp& op, const float* X, int64_t n, const float* B, const double* X64, int t,
                        float sig2, double* R, hipStream_t s) {
    return ski_product<double>(op, X, n, X, n, X64, t, static_cast<double>(sig2), nullptr, nullptr, B, X64, R, s);
}

size_t ski_grad_scratch_bytes(int d, const int32_t* m, int t) {
    const SkiGeom g = make_geom(d, m);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return al(static_cast<size_t>(t) * g.Lr * sizeof(double)) +
           al(static_cast<size_t>(t) * g.Lc * sizeof(hipfftDoubleComplex)) + al(g.Lc * sizeof(hipfftDoubleComplex)) +
           al(static_cast<size_t>(t) * sizeof(double)) + 256;
}

// grad[j] = sum_c w_c (W^T A_c)^T (dK_UU / dtheta_j) (W^T B_c) for the
// kernel's parameters without sigma^2 (W^T A in the product grid, W^T B
// transformed once, one spectral product per parameter).
hipError_t ski_gradient(const SkiOp& op, const mfgp_kernel& k, const float* X, int64_t n, const float* A,
                        const float* B, int t, const double* colw, double* grad, void* gscratch, hipStream_t s) {
    if (t > op.t) return hipErrorInvalidValue;
    const SkiGeom& g = op.g;
    char* p = static_cast<char*>(gscratch);
    auto take = [&](size_t b) {
        char* r = p;
        p += (b + 255) / 256 * 256;
        return r;
    };
    double* grid2 = reinterpret_cast<double*>(take(static_cast<size_t>(t) * g.Lr * sizeof(double)));
    auto* spec2 = reinterpret_cast<hipfftDoubleComplex*>(take(static_cast<size_t>(t) * g.Lc * sizeof(hipfftDoubleComplex)));
    auto* lamj = reinterpret_cast<hipfftDoubleComplex*>(take(g.Lc * sizeof(hipfftDoubleComplex)));
    double* dots = reinterpret_cast<double*>(take(static_cast<size_t>(t) * sizeof(double)));
    auto* spec = static_cast<hipfftDoubleComplex*>(op.spec);
    (void)n;
    hipError_t e = launch_transpose<float>(op, A, t, op.grid, s);
    if (e == hipSuccess) e = launch_transpose<float>(op, B, t, grid2, s);
    if (e != hipSuccess) return e;
    hipfftHandle fwd = fft_plan(g, t, true, e);
    if (!fwd) return e;
    hipfftHandle inv = fft_plan(g, t, false, e);
    if (!inv) return e;
    hipfftHandle f1 = fft_plan(g, 1, true, e);
    if (!f1) return e;
    if (hipfftSetStream(fwd, s) != HIPFFT_SUCCESS || hipfftExecD2Z(fwd, grid2, spec) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    KParams kp{};
    kp.family = k.family;
    kp.s2 = k.outputscale;
    kp.period = k.period;
    for (int q = 0; q < 3; ++q) kp.inv_l[q] = q < k.d ? 1.0 / (k.ard ? k.lengthscale[q] : k.lengthscale[0]) : 0.0;
    const int np = (k.ard ? k.d : 1) + (k.family == MFGP_PERIODIC ? 1 : 0) + 1;
    std::vector<double> h(t);
    for (int j = 0; j < np; ++j) {
        // the derivative column into grid2 slot 0, its spectrum into lamj
        hipLaunchKernelGGL(ski_dcolumn_kernel, dim3(nblk(g.Lr)), dim3(256), 0, s, g, op.geo, kp, k.ard ? 1 : 0, j,
                           grid2);
        if (hipfftSetStream(f1, s) != HIPFFT_SUCCESS || hipfftExecD2Z(f1, grid2, lamj) != HIPFFT_SUCCESS)
            return hipErrorUnknown;
        e = hipMemcpyAsync(spec2, spec, static_cast<size_t>(t) * g.Lc * sizeof(hipfftDoubleComplex),
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ski_spectral_mul_kernel, dim3(nblk(g.Lc * t)), dim3(256), 0, s, spec2, lamj, g.Lc, t,
                           1.0 / static_cast<double>(g.Lr));
        if (hipfftSetStream(inv, s) != HIPFFT_SUCCESS || hipfftExecZ2D(inv, spec2, grid2) != HIPFFT_SUCCESS)
            return hipErrorUnknown;
        hipLaunchKernelGGL(ski_dot_kernel, dim3(t), dim3(256), 0, s, op.grid, grid2, g.Lr, dots);
        e = hipMemcpyAsync(h.data(), dots, t * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        double gj = 0.0;
        for (int c = 0; c < t; ++c) gj += colw[c] * h[c];
        grad[j] = gj;
    }
    return hipGetLastError();
}

}  // namespace mfgp
