// chi2_launch.h -- launch descriptions of the chi^2 and image-search kernels
// (source plane, image plane, refinement, assignment), shared by their
// translation units and the host side.  Not part of the ABI.
#pragma once

#include "lens_internal.h"

namespace lens {

// A Metropolis step fused into the source-plane chi^2 (one wave per walker):
// walker m's free potentials are its 7 nfree physical parameters (x0, y0,
// sigma, e, phi, rcore, rcut per potential), converted and run through the
// parameter prologue by the wave itself.
struct McmcFused {
    int mode = 0;                   // 1: chi^2 of the current state; 2: one step
    int nfree = 0;
    double *params = nullptr;       // [W][7 nfree], updated on acceptance
    double *chi2 = nullptr;         // [W] chi^2 of the current state
    int *accepted = nullptr;        // [W] accepted moves
    const double *lo = nullptr, *hi = nullptr, *step = nullptr;  // [7 nfree]
    const double *u = nullptr;      // [W][7 nfree + 1] uniforms of this step
    double bK = 6.0;                // sigma -> b0: 6 (dPIE) or 4 (SIS) times pi (sigma/c)^2
    int *status = nullptr;          // status word (invalid parameters)
};

// Rows of the per-image constants written by the prep kernel.
constexpr int CHI2_REC_ROWS = 4;

// Source-plane chi^2
struct Chi2SrcLaunch {
    Derived freet;            // derived free potentials of all samples
    const int *free_off;      // [S+1]
    int n_samples;
    int sample0;              // first sample of this launch (per-sample path)
    int nsys, nimg;
    const int *img_off;
    const double *x, *y, *sig, *f;
    Derived fixedt;           // derived fixed potentials (shared by all samples)
    int nimg_pad;
    double *chi2;             // [S] or NULL
    double *src_x, *src_y;    // [S*nsys] barycentric sources, or NULL
    double *rec;              // [CHI2_REC_ROWS][nimg_pad]: fixed deflection x, y, Dls/Ds
                              // and 1/sigma^2 per image
    int persistent;           // 1: stride over the batch by the grid size
    int grid_blocks;
    int prec;
    int chunk;                // potentials per LDS stage (set by the launch wrapper)
    int stage_sig = 0;        // 1: each image's 1/sigma^2 staged in LDS (set by the wrapper)
    Series S;                 // filled by the launch wrapper
    McmcFused mc;             // the sampler's step (mode 0: a plain chi^2 batch)
    // prep with inline fixed prologue (inline_fixed = 1): the fixed potentials'
    // amplitude table (nfixed entries) instead of fixedt, and with
    // free_prologue = 1 the free table's prologue (free_amp -> freet) in the
    // same launch; status receives ST_INVALID_TABLE
    int inline_fixed = 0, free_prologue = 0, nfixed = 0;
    PotSoA fixed_amp = {}, free_amp = {};
    int *status = nullptr;
    // per-sample kernel with derive_free = 1: each wave forms its sample's
    // free potentials' derived constants from free_amp itself (no free table
    // prologue launch; freet is not read)
    int derive_free = 0;
};
hipError_t launch_chi2_prep(const Chi2SrcLaunch &c, hipStream_t st);
hipError_t launch_chi2_src(const Chi2SrcLaunch &c, hipStream_t st);
// The sampler's chi^2 (FP64, one wave per walker, c.n_samples walkers): c.mc.mode 1 or 2.
hipError_t launch_mcmc_chi2(const Chi2SrcLaunch &c, hipStream_t st);

// Image plane
// Image search: n_grids deflection grids (grid g at alpha + g*2*nv: x plane
// then y plane, Dls/Ds = 1), nq sources per grid: source q of grid g at
// (sx[g*nq+q], sy[g*nq+q]) with Dls/Ds f[q].  Outputs per (g, q).
struct ImgLaunch {
    const double *alpha;
    GridArgs grid;
    int n_grids, nq;
    const double *sx, *sy, *f;
    int kmax;
    int *count;                // [n_grids*nq]
    long long *tri;            // [n_grids*nq*kmax]
    double *ix, *iy;           // [n_grids*nq*kmax]
    double *tb;                // [n_grids*ntx*nty*4] tile deflection bounds (scratch)
    int ntx, nty;              // tiles per row / column (set by the launcher)
    int *status;               // ST_DOMAIN / ST_BAD_F bits (atomic or)
};
void image_tiles(int nx, int ny, int &ntx, int &nty);
hipError_t launch_find_images(const ImgLaunch &L, hipStream_t st);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_i64(long long *p, size_t n, long long v, hipStream_t st);
hipError_t launch_sort_images(int n, int kmax, const int *count, long long *tri, double *ix,
                              double *iy, hipStream_t st);

// Vertex deflection grids for a chunk of samples: out[(s)*2*nv + {0,nv} + v]
struct AlphaGridLaunch {
    Derived freet;
    const int *free_off;
    int m0, nsamp;             // samples m0 .. m0+nsamp-1
    GridArgs grid;
    const double *afix_x, *afix_y; // fixed-potential deflection (nv each) or NULL
    double *out;
    int prec;
    Series S;                  // filled by the launch wrapper
};
hipError_t launch_alpha_grid(const AlphaGridLaunch &L, hipStream_t st);

// Newton refinement of the stored images of samples m0 .. m0+nsamp-1 (in place).
struct RefineLaunch {
    Derived fixedt, freet;
    const int *free_off;
    int m0, nsamp, nsys, kmax;
    const int *count;          // [nsamp*nsys] image counts (may exceed kmax)
    double *ix, *iy;           // [nsamp*nsys*kmax] positions, refined in place
    const double *sx, *sy;     // [nsamp*nsys] the chunk's sources
    const double *f;           // [nsys] Dls/Ds
    int max_iter;
    double tol, max_shift;
    Series S;                  // filled by the launch wrapper
};
hipError_t launch_refine_images(const RefineLaunch &L, hipStream_t st);

struct AssignLaunch {
    int nsamp, nsys, kmax;     // samples m0 .. m0+nsamp-1 of this chunk
    const int *count;          // [nsamp*nsys]
    const double *ix, *iy;     // [(s*nsys+i)*kmax + k]
    const int *img_off;
    int nimg_total;            // catalogue images (offset clamp)
    const double *x, *y, *sig;
    double penalty;
    int m0;                    // offset of these samples in the outputs
    double *chi2;              // [S]
    int *nimg;                 // [S*nsys] or NULL
    int *nmissing;             // [S] or NULL
    double *img_xy;            // [S*nsys*kmax*2] or NULL
    double *part;              // scratch [nsamp*nsys]
    int *miss;                 // scratch [nsamp*nsys]
    int *status;
};
hipError_t launch_assign(const AssignLaunch &L, hipStream_t st);

}  // namespace lens
