// images.hip -- brute-force image search on the triangulated grid and the
// image-plane chi^2 (paper Sec. 2.3 and Fig. 4: unlens a triangulated
// image-plane grid and test every triangle for the source; Sec. 4.2, Fig. 7:
// found images are stored, assigned to their closest constraint, then Eq. (6)).
//
// Compiled with -ffp-contract=off: every product and sum here is rounded on
// its own, so a vertex u = v - f alpha, an orientation and an interpolated
// image position are the exactly-specified FP64 expressions, bit-identical to
// any other evaluation of the same expressions.
//
// Design (gfx950): the grid is cut into tiles of 8 x 8 cells.  A first pass
// reads the deflection grid once and writes each tile's deflection bounds; a
// second pass gives each lane a tile and bounds the tile in the source plane
// for each source, so almost every (tile, source) pair is rejected without
// touching the tile's cells.  A wave then visits only tiles with surviving
// sources (lane = cell) and tests those sources exactly: corners unlensed with the source's own Dls/Ds, an exact
// bounding-box test per triangle, and only then the orientation tests (a
// floating-point filter with an exact expansion fallback).  Found images are appended to per-source slots
// with one atomic each; a second pass orders each slot list by triangle id.
#include <math.h>

#include "chi2_launch.h"

namespace lens {

// ---------------------------------------------------------------------------
// Exact orientation sign.
// orient(a, b, p) = (bx-ax)(py-ay) - (by-ay)(px-ax).  A filter answers when
// the FP64 value is far from zero (error below ~3.3e-16 (|l| + |r|), Shewchuk
// 1997); otherwise the six products of the expanded form are made exact with
// an FMA error term each and summed into a nonoverlapping expansion
// (Shewchuk's Grow-Expansion); the sign of its largest nonzero component is
// the sign of the exact value.  Exact for finite inputs whose nonzero
// magnitudes lie in [2^-400, 2^400] (every product and its error term is then
// a normal number); an expansion that meets any other input sets ST_DOMAIN in
// the status word, which the entry points turn into an argument error.  (The
// filter is valid for any finite inputs whose product sum lies in its range.)
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ bool exact_domain(double v) {
    const double a = fabs(v);
    return a == 0.0 || (a >= 0x1p-400 && a <= 0x1p400);
}

__device__ __noinline__ int orient_sign_expansion(double ax, double ay, double bx, double by,
                                                  double px, double py, int *status) {
    if (!(exact_domain(ax) & exact_domain(ay) & exact_domain(bx) & exact_domain(by) &
          exact_domain(px) & exact_domain(py)))
        atomicOr(status, ST_DOMAIN);
    const double u[6] = {bx, -bx, -ax, -by, by, ay};
    const double w[6] = {py, ay, py, px, ax, px};
    double h[12];
    int hn = 0;
    for (int t = 0; t < 6; ++t) {
        const double p = u[t] * w[t];
        const double e = fma(u[t], w[t], -p);
        const double terms[2] = {e, p};
        for (int r = 0; r < 2; ++r) {
            double q = terms[r];
            for (int i = 0; i < hn; ++i) {
                double s, err;
                two_sum(q, h[i], s, err);
                h[i] = err;
                q = s;
            }
            h[hn++] = q;
        }
    }
    for (int i = hn - 1; i >= 0; --i)
        if (h[i] != 0.0) return h[i] > 0.0 ? 1 : -1;
    return 0;
}

__device__ __forceinline__ int orient_sign(double ax, double ay, double bx, double by, double px,
                                           double py, int *status) {
    const double l = (bx - ax) * (py - ay);
    const double r = (by - ay) * (px - ax);
    const double det = l - r;
    const double sum = fabs(l) + fabs(r);
    if (sum > 1e-280 && sum < 1e280 && fabs(det) > 1e-15 * sum) return det > 0.0 ? 1 : -1;
    return orient_sign_expansion(ax, ay, bx, by, px, py, status);
}

// Sign of orient(a, b, p + (d, d^2)), d -> 0+.
__device__ __forceinline__ int orient_perturbed(double ax, double ay, double bx, double by,
                                                double px, double py, int *status) {
    const int s = orient_sign(ax, ay, bx, by, px, py, status);
    if (s) return s;
    if (by != ay) return by < ay ? 1 : -1;
    if (bx != ax) return bx > ax ? 1 : -1;
    return 0;
}

// Triangle (u0, u1, u2) holds p (perturbed), non-degenerate.  Caller has
// already checked the exact bounding box.
__device__ __noinline__ bool tri_contains(double u0x, double u0y, double u1x, double u1y,
                                          double u2x, double u2y, double px, double py,
                                          int *status) {
    if (orient_sign(u0x, u0y, u1x, u1y, u2x, u2y, status) == 0) return false;
    const int s0 = orient_perturbed(u0x, u0y, u1x, u1y, px, py, status);
    const int s1 = orient_perturbed(u1x, u1y, u2x, u2y, px, py, status);
    if (s0 != s1) return false;
    const int s2 = orient_perturbed(u2x, u2y, u0x, u0y, px, py, status);
    return s1 == s2 && s0 != 0;
}

// p + (d, d^2) can only be strictly inside when min x <= px < max x and
// min y <= py < max y (exact comparisons).
__device__ __forceinline__ bool box_may_hold(double ax, double ay, double bx, double by, double cx,
                                             double cy, double px, double py) {
    const double x0 = fmin(ax, fmin(bx, cx)), x1 = fmax(ax, fmax(bx, cx));
    const double y0 = fmin(ay, fmin(by, cy)), y1 = fmax(ay, fmax(by, cy));
    return (px >= x0) & (px < x1) & (py >= y0) & (py < y1);
}

__device__ void store_image(const ImgLaunch &L, size_t q, long long tri, double u0x, double u0y,
                            double u1x, double u1y, double u2x, double u2y, double v0x,
                            double v0y, double v1x, double v1y, double v2x, double v2y, double px,
                            double py) {
    const int slot = atomicAdd(&L.count[q], 1);
    if (slot >= L.kmax) return;
    const double oa = (u2x - u1x) * (py - u1y) - (u2y - u1y) * (px - u1x);
    const double ob = (u0x - u2x) * (py - u2y) - (u0y - u2y) * (px - u2x);
    const double oc = (u1x - u0x) * (py - u0y) - (u1y - u0y) * (px - u0x);
    const double den = (oa + ob) + oc;
    double ix, iy;
    if (den != 0.0) {
        ix = ((oa * v0x + ob * v1x) + oc * v2x) / den;
        iy = ((oa * v0y + ob * v1y) + oc * v2y) / den;
    } else {
        ix = ((v0x + v1x) + v2x) / 3.0;
        iy = ((v0y + v1y) + v2y) / 3.0;
    }
    const size_t at = q * L.kmax + slot;
    L.tri[at] = tri;
    L.ix[at] = ix;
    L.iy[at] = iy;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmin(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

constexpr int SRC_CHUNK = 256;  // sources staged in LDS per round (= block size)
constexpr int TILE = 8;         // image-search tiles of TILE x TILE cells

// ---------------------------------------------------------------------------
// Pass 1: deflection bounds of every tile of TILE x TILE cells, i.e. of its
// (TILE+1) x (TILE+1) vertices (fewer at the grid's last row and column):
// tb[((g*nty + ty)*ntx + tx)*4 + {0,1,2,3}] = min ax, max ax, min ay, max ay.
// A tile holding a NaN deflection gets infinite bounds (it is never culled).
// A block takes one row of tiles and TB_TILES consecutive tiles of it: each
// thread reduces one vertex column over the tile row's TILE+1 vertex rows
// (coalesced loads), then one thread per tile combines its TILE+1 columns.
constexpr int TB_TILES = 32;
constexpr int TB_COLS = TB_TILES * TILE + 1;

__global__ void __launch_bounds__(256) tile_bounds_kernel(ImgLaunch L) {
    __shared__ double s_b[4][TB_COLS];
    __shared__ int s_bad[TB_COLS];
    const int nx = L.grid.nx, ny = L.grid.ny;
    const int tid = threadIdx.x;
    const int tx0 = blockIdx.x * TB_TILES, ty = blockIdx.y, g = blockIdx.z;
    const size_t nv = (size_t)nx * ny;
    const double *ax = L.alpha + (size_t)g * 2 * nv;
    const double *ay = ax + nv;
    const double inf = __builtin_inf();
    const int c0 = tx0 * TILE, j0 = ty * TILE, j1 = min(j0 + TILE, ny - 1);
    for (int k = tid; k < TB_COLS; k += 256) {
        const int c = c0 + k;
        double xl = inf, xh = -inf, yl = inf, yh = -inf;
        bool bad = false;
        if (c < nx) {
#pragma unroll
            for (int r = 0; r <= TILE; ++r) {
                const int j = j0 + r;
                if (j > j1) break;
                const size_t v = (size_t)j * nx + c;
                const double a = ax[v], b = ay[v];
                bad |= (a != a) | (b != b);
                xl = fmin(xl, a);
                xh = fmax(xh, a);
                yl = fmin(yl, b);
                yh = fmax(yh, b);
            }
        }
        s_b[0][k] = xl;
        s_b[1][k] = xh;
        s_b[2][k] = yl;
        s_b[3][k] = yh;
        s_bad[k] = bad;
    }
    __syncthreads();
    const int tx = tx0 + tid;
    if (tid < TB_TILES && tx < L.ntx) {
        double xl = inf, xh = -inf, yl = inf, yh = -inf;
        bool bad = false;
        for (int k = tid * TILE; k <= tid * TILE + TILE; ++k) {
            xl = fmin(xl, s_b[0][k]);
            xh = fmax(xh, s_b[1][k]);
            yl = fmin(yl, s_b[2][k]);
            yh = fmax(yh, s_b[3][k]);
            bad |= s_bad[k] != 0;
        }
        double *r = L.tb + (((size_t)g * L.nty + ty) * L.ntx + tx) * 4;
        r[0] = bad ? -inf : xl;
        r[1] = bad ? inf : xh;
        r[2] = bad ? -inf : yl;
        r[3] = bad ? inf : yh;
    }
}

// Pass 2.  Lane t of a wave owns tile t of a run of 64 tiles and tests 64
// sources at a time against its tile's box in the source plane: with vertex
// coordinates in [vl, vh] (monotone in the index) and deflections in
// [al, ah], rounding is monotone, so for Dls/Ds f > 0 every unlensed vertex
// fl(v - fl(f a)) of the tile lies in [fl(vl - fl(f ah)), fl(vh - fl(f al))].
// A source outside that box (by the half-open rule of the per-triangle box)
// cannot be inside any of the tile's triangles.  The wave then visits only
// tiles with surviving sources: lane = cell, corners loaded once, each
// surviving source unlensed with its own f and both triangles tested exactly.
__global__ void __launch_bounds__(256) find_images_kernel(ImgLaunch L) {
    __shared__ double s_px[SRC_CHUNK], s_py[SRC_CHUNK], s_f[SRC_CHUNK];
    const int nx = L.grid.nx, ny = L.grid.ny;
    const int tid = threadIdx.x, lane = tid & 63;
    const int g = blockIdx.y;
    const int ntile = L.ntx * L.nty;
    const int T = (blockIdx.x * 4 + (tid >> 6)) * 64 + lane;
    const bool tile_ok = T < ntile;
    const int tx = tile_ok ? T % L.ntx : 0, ty = tile_ok ? T / L.ntx : 0;
    const double inf = __builtin_inf();
    double axl = inf, axh = -inf, ayl = inf, ayh = -inf;
    if (tile_ok) {
        const double *r = L.tb + (((size_t)g * L.nty + ty) * L.ntx + tx) * 4;
        axl = r[0];
        axh = r[1];
        ayl = r[2];
        ayh = r[3];
    }
    const double vxl = grid_coord(L.grid.x0, tx * TILE, L.grid.dx);
    const double vxh = grid_coord(L.grid.x0, min(tx * TILE + TILE, nx - 1), L.grid.dx);
    const double vyl = grid_coord(L.grid.y0, ty * TILE, L.grid.dy);
    const double vyh = grid_coord(L.grid.y0, min(ty * TILE + TILE, ny - 1), L.grid.dy);
    const size_t nv = (size_t)nx * ny;
    const double *ax = L.alpha + (size_t)g * 2 * nv;
    const double *ay = ax + nv;

    for (int q0 = 0; q0 < L.nq; q0 += SRC_CHUNK) {
        const int nqc = min(SRC_CHUNK, L.nq - q0);
        __syncthreads();
        if (tid < nqc) {
            const size_t gq = (size_t)g * L.nq + q0 + tid;
            s_px[tid] = L.sx[gq];
            s_py[tid] = L.sy[gq];
            // the tile cull holds for 0 < f; a source with f outside (0, 1]
            // is flagged and gets no images (NaN fails every box test)
            const double fv = L.f[q0 + tid];
            const bool f_ok = fv > 0.0 && fv <= 1.0;
            if (!f_ok) atomicOr(L.status, ST_BAD_F);
            s_f[tid] = f_ok ? fv : __builtin_nan("");
        }
        __syncthreads();
        for (int b0 = 0; b0 < nqc; b0 += 64) {
            const int nb = min(64, nqc - b0);
            unsigned long long mask = 0;
            for (int k = 0; k < nb; ++k) {
                const double f = s_f[b0 + k], px = s_px[b0 + k], py = s_py[b0 + k];
                const double lx = vxl - f * axh, hx = vxh - f * axl;
                const double ly = vyl - f * ayh, hy = vyh - f * ayl;
                if ((px >= lx) & (px < hx) & (py >= ly) & (py < hy)) mask |= 1ull << k;
            }
            unsigned long long busy = __ballot(mask != 0ull);
            while (busy) {
                const int owner = __builtin_ctzll(busy);
                busy &= busy - 1;
                const unsigned lo = __builtin_amdgcn_readlane((unsigned)mask, owner);
                const unsigned hi = __builtin_amdgcn_readlane((unsigned)(mask >> 32), owner);
                unsigned long long srcs = ((unsigned long long)hi << 32) | lo;
                const int T2 = (blockIdx.x * 4 + (tid >> 6)) * 64 + owner;
                const int cx = T2 % L.ntx, cy = T2 / L.ntx;
                const int i_raw = cx * TILE + (lane & (TILE - 1)), j_raw = cy * TILE + lane / TILE;
                const bool valid = (i_raw + 1 < nx) && (j_raw + 1 < ny);
                const int i = min(i_raw, nx - 2), j = min(j_raw, ny - 2);
                const size_t i00 = (size_t)j * nx + i, i10 = i00 + 1, i01 = i00 + nx,
                             i11 = i01 + 1;
                const double a00x = ax[i00], a00y = ay[i00], a10x = ax[i10], a10y = ay[i10];
                const double a01x = ax[i01], a01y = ay[i01], a11x = ax[i11], a11y = ay[i11];
                const double x0 = grid_coord(L.grid.x0, i, L.grid.dx);
                const double x1 = grid_coord(L.grid.x0, i + 1, L.grid.dx);
                const double y0 = grid_coord(L.grid.y0, j, L.grid.dy);
                const double y1 = grid_coord(L.grid.y0, j + 1, L.grid.dy);
                const long long t0 = 2LL * ((long long)j * (nx - 1) + i);
                while (srcs) {
                    const int qq = b0 + __builtin_ctzll(srcs);
                    srcs &= srcs - 1;
                    if (!valid) continue;
                    const double px = s_px[qq], py = s_py[qq], f = s_f[qq];
                    const size_t gq = (size_t)g * L.nq + q0 + qq;
                    const double u00x = x0 - f * a00x, u00y = y0 - f * a00y;
                    const double u10x = x1 - f * a10x, u10y = y0 - f * a10y;
                    const double u01x = x0 - f * a01x, u01y = y1 - f * a01y;
                    const double u11x = x1 - f * a11x, u11y = y1 - f * a11y;
                    // T0 = (v[i,j], v[i+1,j], v[i,j+1])
                    if (box_may_hold(u00x, u00y, u10x, u10y, u01x, u01y, px, py) &&
                        tri_contains(u00x, u00y, u10x, u10y, u01x, u01y, px, py, L.status))
                        store_image(L, gq, t0, u00x, u00y, u10x, u10y, u01x, u01y, x0, y0, x1,
                                    y0, x0, y1, px, py);
                    // T1 = (v[i+1,j+1], v[i,j+1], v[i+1,j])
                    if (box_may_hold(u11x, u11y, u01x, u01y, u10x, u10y, px, py) &&
                        tri_contains(u11x, u11y, u01x, u01y, u10x, u10y, px, py, L.status))
                        store_image(L, gq, t0 + 1, u11x, u11y, u01x, u01y, u10x, u10y, x1, y1,
                                    x0, y1, x1, y0, px, py);
                }
            }
        }
    }
}

void image_tiles(int nx, int ny, int &ntx, int &nty) {
    ntx = (nx - 1 + TILE - 1) / TILE;
    nty = (ny - 1 + TILE - 1) / TILE;
}

hipError_t launch_find_images(const ImgLaunch &L0, hipStream_t st) {
    if (L0.grid.nx < 2 || L0.grid.ny < 2 || L0.n_grids <= 0 || L0.nq <= 0) return hipSuccess;
    ImgLaunch L = L0;
    image_tiles(L.grid.nx, L.grid.ny, L.ntx, L.nty);
    const long long ntile = (long long)L.ntx * L.nty;
    if (L.n_grids > 65535) return hipErrorInvalidConfiguration;
    if (L.nty > 65535) return hipErrorInvalidConfiguration;
    dim3 g1((unsigned)((L.ntx + TB_TILES - 1) / TB_TILES), L.nty, L.n_grids);
    hipLaunchKernelGGL(tile_bounds_kernel, g1, dim3(256), 0, st, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((unsigned)((ntile + 255) / 256), L.n_grids);
    hipLaunchKernelGGL(find_images_kernel, g2, dim3(256), 0, st, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Order each slot list by triangle id (insertion sort; lists hold <= kmax).
__global__ void sort_images_kernel(int n, int kmax, const int *__restrict__ count,
                                   long long *__restrict__ tri, double *__restrict__ ix,
                                   double *__restrict__ iy) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int c = min(count[q], kmax);
    long long *T = tri + (size_t)q * kmax;
    double *X = ix + (size_t)q * kmax, *Y = iy + (size_t)q * kmax;
    for (int a = 1; a < c; ++a) {
        const long long t = T[a];
        const double x = X[a], y = Y[a];
        int b = a - 1;
        while (b >= 0 && T[b] > t) {
            T[b + 1] = T[b];
            X[b + 1] = X[b];
            Y[b + 1] = Y[b];
            --b;
        }
        T[b + 1] = t;
        X[b + 1] = x;
        Y[b + 1] = y;
    }
}

hipError_t launch_sort_images(int n, int kmax, const int *count, long long *tri, double *ix,
                              double *iy, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sort_images_kernel, dim3((n + 127) / 128), dim3(128), 0, st, n, kmax,
                       count, tri, ix, iy);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Assignment and chi^2 (Sec. 4.2: found images go to their closest
// constraint; Eq. (6)).  Pass 1: one thread per (sample, system).
__global__ void assign_kernel(AssignLaunch a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nsamp * a.nsys) return;
    const int s = q / a.nsys, i = q - s * a.nsys;
    const int m = a.m0 + s;
    const int cnt = a.count[q];
    const int n = min(cnt, a.kmax);
    if (cnt > a.kmax) atomicOr(a.status, ST_OVERFLOW);
    const double *X = a.ix + (size_t)q * a.kmax, *Y = a.iy + (size_t)q * a.kmax;
    const int o = min(max(a.img_off[i], 0), a.nimg_total);
    const int M = min(max(a.img_off[i + 1], o), a.nimg_total) - o;
    // nearest constraint of each image (ties: lower index); <= 64 images
    int pick[64];
    for (int k = 0; k < n; ++k) {
        double best = 0.0;
        int bj = -1;
        for (int c = 0; c < M; ++c) {
            const double ex = X[k] - a.x[o + c], ey = Y[k] - a.y[o + c];
            const double d2 = ex * ex + ey * ey;
            if (bj < 0 || d2 < best) {
                best = d2;
                bj = c;
            }
        }
        pick[k] = bj;
    }
    double part = 0.0;
    int miss = 0;
    for (int c = 0; c < M; ++c) {
        double best = 0.0;
        bool found = false;
        for (int k = 0; k < n; ++k) {
            if (pick[k] != c) continue;
            const double ex = X[k] - a.x[o + c], ey = Y[k] - a.y[o + c];
            const double d2 = ex * ex + ey * ey;
            if (!found || d2 < best) {
                best = d2;
                found = true;
            }
        }
        if (found) {
            part += best / (a.sig[o + c] * a.sig[o + c]);
        } else {
            part += a.penalty;
            ++miss;
        }
    }
    a.part[q] = part;
    a.miss[q] = miss;
    const size_t out_q = (size_t)m * a.nsys + i;
    if (a.nimg) a.nimg[out_q] = cnt;
    if (a.img_xy) {
        for (int k = 0; k < a.kmax; ++k) {
            const bool have = k < n;
            a.img_xy[(out_q * a.kmax + k) * 2 + 0] = have ? X[k] : NAN;
            a.img_xy[(out_q * a.kmax + k) * 2 + 1] = have ? Y[k] : NAN;
        }
    }
}

// Pass 2: one thread per sample sums its systems in index order.
__global__ void assign_reduce_kernel(AssignLaunch a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.nsamp) return;
    double total = 0.0;
    int miss = 0;
    for (int i = 0; i < a.nsys; ++i) {
        total += a.part[(size_t)s * a.nsys + i];
        miss += a.miss[(size_t)s * a.nsys + i];
    }
    a.chi2[a.m0 + s] = total;
    if (a.nmissing) a.nmissing[a.m0 + s] = miss;
}

hipError_t launch_assign(const AssignLaunch &L, hipStream_t st) {
    const int nq = L.nsamp * L.nsys;
    if (nq > 0)
        hipLaunchKernelGGL(assign_kernel, dim3((nq + 63) / 64), dim3(64), 0, st, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.nsamp > 0)
        hipLaunchKernelGGL(assign_reduce_kernel, dim3((L.nsamp + 63) / 64), dim3(64), 0, st, L);
    return hipGetLastError();
}

}  // namespace lens
