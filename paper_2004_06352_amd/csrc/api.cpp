// api.cpp -- the C ABI of include/lenshpc.h: argument validation, context
// scratch, and the launch sequences of the map and chi^2 calls.
//
// Every argument error is found before the first launch (and leaves outputs
// untouched); device arrays are checked against the allocation they lie in.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "chi2_launch.h"
#include "potential_launch.h"

using namespace lens;

static thread_local std::string g_err;

static lens_status_t fail(lens_status_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(LENS_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                        __FILE__, __LINE__);                                                \
    } while (0)

#define TRY(expr)                          \
    do {                                   \
        lens_status_t s_ = (expr);         \
        if (s_ != LENS_OK) return s_;      \
    } while (0)

struct lens_ctx {
    int device = 0;
    uint64_t scratch_max = 0;
    uint32_t flags = 0;
    void *scratch = nullptr;
    size_t scratch_size = 0;
    int *small = nullptr;        // device: [0] status, [2] overflow word, others spare
    int *host_small = nullptr;   // pinned mirror
    int num_cu = 256;
    lens_map_tuning_t tune[3];
    int chi2_blocks_per_cu = 16;  // persistent chi^2 waves (one-wave blocks) per CU
};

struct lens_mcmc {
    lens_ctx_t *ctx = nullptr;
    void *mem = nullptr;  // fixed potentials' derived table and per-image constants
    lens::Chi2SrcLaunch step;  // the fused step launch (mode 2)
};

struct lens_chi2_plan {
    lens_ctx_t *ctx = nullptr;
    void *mem = nullptr;  // the plan's own scratch (derived tables, per-image constants)
    // image mode: the captured sequence; source mode: the recorded launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int *status = nullptr;  // image mode: the search's status word, in mem
    bool direct = false;
    bool has_prep = false, has_src = false;
    lens::Chi2SrcLaunch prep, src;
};

// Device memory of the allocation-free map call: the derived constants of at
// most LENS_NOALLOC_MAX_POT potentials, laid out as a context's derived table
// of that many entries.  Each device holds its own copy for the life of the
// process.  Host code never passes `scratch` itself (its host-side name is
// not a device address): the address of each device's copy is looked up once
// per device when a context is created there, and only that address is used.
constexpr size_t kNoallocBytes =
    (size_t)LENS_NOALLOC_MAX_POT * (lens::NDER * sizeof(double) + lens::NDERF * sizeof(float));
static_assert(LENS_NOALLOC_MAX_POT % 64 == 0, "a derived table's stride is a multiple of 64");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kMaxDevices] = {};

namespace {

const lens_map_tuning_t kDefaultMapTuning = {64, 4, 1, 1, 64};

// Keep the caller's current device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool is_fin(double v) { return std::isfinite(v); }

// The byte range [p, p + bytes) must lie inside one device allocation.
lens_status_t check_range(const void *p, size_t bytes, const char *name) {
    if (bytes == 0) return LENS_OK;
    if (!p) return fail(LENS_EINVAL, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess || base == nullptr) {
        (void)hipGetLastError();
        return fail(LENS_EINVAL, "%s (%p) is not a device allocation", name, p);
    }
    const char *b = (const char *)base, *q = (const char *)p;
    if (q < b || (size_t)(q - b) + bytes > size)
        return fail(LENS_EINVAL, "%s: %zu bytes at %p exceed its allocation (%zu bytes at %p)",
                    name, bytes, p, size, (const void *)base);
    return LENS_OK;
}

lens_status_t check_table(const lens_pot_table_t *t, const char *name) {
    if (!t) return fail(LENS_EINVAL, "%s is NULL", name);
    if (t->n < 0) return fail(LENS_EINVAL, "%s.n = %d < 0", name, t->n);
    const size_t b = (size_t)t->n * sizeof(double);
    const void *ps[7] = {t->x0, t->y0, t->b0, t->eps, t->phi, t->rcore, t->rcut};
    const char *nm[7] = {"x0", "y0", "b0", "eps", "phi", "rcore", "rcut"};
    for (int i = 0; i < 7; ++i) {
        char full[96];
        snprintf(full, sizeof full, "%s.%s", name, nm[i]);
        TRY(check_range(ps[i], b, full));
    }
    return LENS_OK;
}

lens_status_t check_grid(const lens_grid_t *g) {
    if (!g) return fail(LENS_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) return fail(LENS_EINVAL, "grid %d x %d", g->nx, g->ny);
    if ((long long)g->nx * g->ny > (1LL << 31))
        return fail(LENS_EINVAL, "grid of %lld points exceeds 2^31", (long long)g->nx * g->ny);
    if (!is_fin(g->x0) || !is_fin(g->y0) || !is_fin(g->dx) || !is_fin(g->dy) || !(g->dx > 0) ||
        !(g->dy > 0))
        return fail(LENS_EINVAL, "grid origin/spacing not finite and positive");
    return LENS_OK;
}

lens_status_t check_prec(lens_precision_t p) {
    if (p != LENS_FP64 && p != LENS_FP32_ACC64 && p != LENS_FP32_COMP32)
        return fail(LENS_EINVAL, "unknown precision %d", p);
    return LENS_OK;
}

// Bump allocator over the context scratch.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    }
};

lens_status_t ensure_scratch(lens_ctx_t *ctx, size_t bytes) {
    if (bytes <= ctx->scratch_size) return LENS_OK;
    if (bytes > ctx->scratch_max)
        return fail(LENS_ENOMEM, "needs %zu bytes of scratch, context limit is %llu", bytes,
                    (unsigned long long)ctx->scratch_max);
    if (ctx->scratch) {
        HIP_TRY(hipFree(ctx->scratch));  // waits for work still using it
        ctx->scratch = nullptr;
        ctx->scratch_size = 0;
    }
    size_t sz = std::max(bytes, (size_t)1 << 20);
    sz = std::min<size_t>(std::max(sz, bytes), std::max<size_t>(bytes, ctx->scratch_max));
    hipError_t e = hipMalloc(&ctx->scratch, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->scratch = nullptr;
        return fail(LENS_ENOMEM, "hipMalloc(%zu) failed: %s", sz, hipGetErrorString(e));
    }
    ctx->scratch_size = sz;
    return LENS_OK;
}

char *sc(lens_ctx_t *ctx, size_t off) { return (char *)ctx->scratch + off; }

PotSoA soa(const lens_pot_table_t *t) {
    return PotSoA{t->x0, t->y0, t->b0, t->eps, t->phi, t->rcore, t->rcut};
}

Derived derived_in(char *base, size_t off, int n) {
    const int st = derived_stride(n);
    double *d = (double *)(base + off);
    float *f = (float *)(d + (size_t)NDER * st);
    return Derived{d, f, n, st};
}

Derived derived_at(lens_ctx_t *ctx, size_t off, int n) { return derived_in(sc(ctx, off), 0, n); }

// The table prologue; parts: PRO_F32 / PRO_LOG, what the consumer reads
// besides the FP64 block.
lens_status_t run_prologue(lens_ctx_t *ctx, const lens_pot_table_t *t, const Derived &D,
                           int parts, hipStream_t st) {
    HIP_TRY(launch_prologue(soa(t), t->n, const_cast<double *>(D.d), const_cast<float *>(D.f),
                            D.stride, ctx->small, parts, st));
    return LENS_OK;
}

bool checked(const lens_ctx_t *ctx) { return (ctx->flags & LENS_CTX_CHECK_TABLES) != 0; }

// In checked contexts: clear the status word before the prologues.
lens_status_t status_reset(lens_ctx_t *ctx, hipStream_t st) {
    if (!checked(ctx)) return LENS_OK;
    HIP_TRY(launch_zero_i32(ctx->small, 1, st));
    return LENS_OK;
}

// In checked contexts: wait for the prologues and report invalid content.
lens_status_t status_check(lens_ctx_t *ctx, hipStream_t st) {
    if (!checked(ctx)) return LENS_OK;
    HIP_TRY(hipMemcpyAsync(ctx->host_small, ctx->small, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctx->host_small[0] & ST_INVALID_TABLE)
        return fail(LENS_EINVAL, "a potential table holds invalid parameters");
    return LENS_OK;
}

// Address of this device's copy of `scratch`, looked up once per device with
// the device current (context creation calls this).
lens_status_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return fail(LENS_EUNSUPPORTED, "device %d: the allocation-free call supports devices "
                    "0..%d", device, kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return LENS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return fail(LENS_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                    hipGetErrorString(e));
    }
    g_noalloc_ptr[device] = p;
    return LENS_OK;
}

// The map calls.  `fixed_scratch` (the allocation-free call): the derived
// table goes to that device memory, sized for LENS_NOALLOC_MAX_POT entries,
// instead of the context's scratch.
lens_status_t map_common(lens_ctx_t *ctx, const lens_pot_table_t *table, const lens_grid_t *grid,
                         double dlsds, lens_precision_t prec, void *out[5], bool grad, bool hess,
                         hipStream_t st, void *const *dout = nullptr,
                         char *fixed_scratch = nullptr) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    TRY(check_prec(prec));
    TRY(check_table(table, "table"));
    TRY(check_grid(grid));
    if (!is_fin(dlsds) || dlsds < 0) return fail(LENS_EINVAL, "dlsds = %g", dlsds);
    const size_t np = (size_t)grid->nx * grid->ny;
    const size_t esz = prec == LENS_FP64 ? sizeof(double) : sizeof(float);
    const char *names[5] = {"ax", "ay", "hxx", "hxy", "hyy"};
    for (int c = 0; c < 5; ++c)
        if (out[c]) TRY(check_range(out[c], np * esz, names[c]));
    const char *dnames[6] = {"kappa", "gamma1", "gamma2", "gamma", "mu", "det"};
    if (dout)
        for (int c = 0; c < 6; ++c)
            if (dout[c]) TRY(check_range(dout[c], np * esz, dnames[c]));
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    Derived D;
    if (fixed_scratch) {
        if (table->n > LENS_NOALLOC_MAX_POT)
            return fail(LENS_ENOMEM, "table of %d potentials: the allocation-free call holds at "
                        "most %d", table->n, LENS_NOALLOC_MAX_POT);
        // the same layout as a context table of n entries (stride from n),
        // which fits in the space of LENS_NOALLOC_MAX_POT entries
        D = derived_in(fixed_scratch, 0, table->n);
    } else {
        Carve cv;
        const size_t o_tab = cv.take(derived_bytes(table->n));
        TRY(ensure_scratch(ctx, cv.off));
        D = derived_at(ctx, o_tab, table->n);
    }
    TRY(status_reset(ctx, st));
    TRY(run_prologue(ctx, table, D, prec == LENS_FP64 ? 0 : PRO_F32, st));
    TRY(status_check(ctx, st));
    MapLaunch m;
    m.tab = D;
    m.grid = GridArgs{grid->nx, grid->ny, grid->x0, grid->y0, grid->dx, grid->dy};
    m.dlsds = dlsds;
    for (int c = 0; c < 5; ++c) m.out[c] = out[c];
    if (dout) {
        m.derived = true;
        for (int c = 0; c < 6; ++c) m.dout[c] = dout[c];
    }
    m.prec = prec;
    m.grad = grad;
    m.hess = hess;
    m.tune = ctx->tune[prec];
    HIP_TRY(launch_map(m, st));
    return LENS_OK;
}

// ------------------------- chi^2 ---------------------------------------------
lens_status_t check_batch(const lens_model_batch_t *b) {
    if (!b) return fail(LENS_EINVAL, "batch is NULL");
    if (b->n_samples < 0) return fail(LENS_EINVAL, "n_samples < 0");
    TRY(check_range(b->free_offset, ((size_t)b->n_samples + 1) * sizeof(int32_t),
                    "batch.free_offset"));
    TRY(check_table(&b->free, "batch.free"));
    TRY(check_table(&b->fixed, "batch.fixed"));
    return LENS_OK;
}

lens_status_t check_catalog(const lens_catalog_t *c) {
    if (!c) return fail(LENS_EINVAL, "catalog is NULL");
    if (c->n_sys < 1) return fail(LENS_EINVAL, "catalog.n_sys = %d", c->n_sys);
    if (c->n_img < 1 || c->n_img > 4000)
        return fail(LENS_EINVAL, "catalog.n_img = %d (1..4000)", c->n_img);
    TRY(check_range(c->img_offset, ((size_t)c->n_sys + 1) * sizeof(int32_t),
                    "catalog.img_offset"));
    const size_t b = (size_t)c->n_img * sizeof(double);
    TRY(check_range(c->x, b, "catalog.x"));
    TRY(check_range(c->y, b, "catalog.y"));
    TRY(check_range(c->sigma, b, "catalog.sigma"));
    TRY(check_range(c->dlsds, (size_t)c->n_sys * sizeof(double), "catalog.dlsds"));
    return LENS_OK;
}

// Checked contexts: the offset arrays and catalogue values, read back.
// In checked contexts: the catalogue's offsets, errors, Dls/Ds and positions.
lens_status_t check_catalog_contents(lens_ctx_t *ctx, const lens_catalog_t *c, hipStream_t st) {
    if (!checked(ctx)) return LENS_OK;
    std::vector<int32_t> io(c->n_sys + 1);
    std::vector<double> sig(c->n_img), f(c->n_sys), x(c->n_img), y(c->n_img);
    HIP_TRY(hipMemcpyAsync(io.data(), c->img_offset, io.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(sig.data(), c->sigma, sig.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(f.data(), c->dlsds, f.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(x.data(), c->x, x.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(y.data(), c->y, y.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (io[0] != 0 || io[c->n_sys] != c->n_img)
        return fail(LENS_EINVAL, "img_offset must run from 0 to n_img = %d", c->n_img);
    for (int i = 0; i < c->n_sys; ++i) {
        if (io[i + 1] < io[i]) return fail(LENS_EINVAL, "img_offset decreases at %d", i);
        if (!(f[i] > 0.0 && f[i] <= 1.0)) return fail(LENS_EINVAL, "dlsds[%d] = %g", i, f[i]);
    }
    for (int t = 0; t < c->n_img; ++t)
        if (!(sig[t] > 0.0) || !is_fin(sig[t]) || !is_fin(x[t]) || !is_fin(y[t]))
            return fail(LENS_EINVAL, "catalog image %d: bad position or sigma", t);
    return LENS_OK;
}

// In checked contexts: the batch's sample offsets, then the catalogue.
lens_status_t check_contents(lens_ctx_t *ctx, const lens_model_batch_t *b,
                             const lens_catalog_t *c, hipStream_t st) {
    if (!checked(ctx)) return LENS_OK;
    std::vector<int32_t> fo(b->n_samples + 1);
    HIP_TRY(hipMemcpyAsync(fo.data(), b->free_offset, fo.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (fo[0] != 0 || fo[b->n_samples] != b->free.n)
        return fail(LENS_EINVAL, "free_offset must run from 0 to free.n = %d", b->free.n);
    for (int m = 0; m < b->n_samples; ++m)
        if (fo[m + 1] < fo[m]) return fail(LENS_EINVAL, "free_offset decreases at %d", m);
    return check_catalog_contents(ctx, c, st);
}

struct SrcPlan {
    size_t o_fix, o_free, o_rec, o_src;
    int nimg_pad;
    char *base = nullptr;  // scratch the offsets refer to (the context's, or a plan's own)
};

SrcPlan plan_src(Carve &cv, const lens_model_batch_t *b, const lens_catalog_t *c, bool sources) {
    SrcPlan p;
    p.nimg_pad = (c->n_img + 63) / 64 * 64;
    p.o_fix = cv.take(derived_bytes(b->fixed.n));
    p.o_free = cv.take(derived_bytes(b->free.n));
    p.o_rec = cv.take((size_t)CHI2_REC_ROWS * p.nimg_pad * sizeof(double));
    p.o_src = sources ? cv.take((size_t)std::max(b->n_samples, 1) * c->n_sys * 2 * sizeof(double))
                      : 0;
    return p;
}

int batched_blocks(const lens_ctx_t *ctx, int S) {
    return std::max(1, std::min(S, ctx->num_cu * ctx->chi2_blocks_per_cu));
}

// Which parts of the source-plane sequence to issue: everything; only what
// depends on the fixed potentials and the catalogue (the per-image
// constants); only what depends on the free potentials (their prologue and
// the per-sample kernel, the per-image constants being ready); only the
// per-sample kernel (the free derived table written elsewhere); or
// everything and the fixed potentials' derived table too (for callers that
// evaluate the fixed potentials again, the image plane).  Without the last,
// the fixed potentials' constants are formed inside the per-image launch and
// no table of them is written.
// SRC_SAMPLES_DERIVE: the per-sample kernel alone, forming the free
// potentials' derived constants itself from their amplitude table (one
// launch; the per-image constants being ready).
enum SrcParts {
    SRC_ALL, SRC_FIXED_ONLY, SRC_FREE_ONLY, SRC_SAMPLES_ONLY, SRC_ALL_TABLES, SRC_SAMPLES_DERIVE
};

// Prologues, fixed deflection at the constraints, then the per-sample kernel.
// The launches a source-mode plan replays: the sequence's prep and
// per-sample kernels, described once (arguments, shapes, buffers) and issued
// as plain launches on each replay.
struct SrcRecord {
    bool has_prep = false, has_src = false;
    Chi2SrcLaunch prep, src;
};

// rec: record the prep and per-sample launches there instead of issuing them
// (batched path, no table prologue of its own, unchecked).
lens_status_t src_sequence(lens_ctx_t *ctx, const lens_model_batch_t *b, const lens_catalog_t *c,
                           lens_precision_t prec, lens_chi2_path_t path, const SrcPlan &p,
                           double *chi2, bool sources, hipStream_t st, bool with_check,
                           SrcParts parts = SRC_ALL, SrcRecord *rec = nullptr) {
    if (rec && (with_check || path != LENS_CHI2_PATH_BATCHED || parts == SRC_ALL_TABLES ||
                parts == SRC_FREE_ONLY))
        return fail(LENS_EUNSUPPORTED, "this source-plane sequence cannot be recorded");
    char *base = p.base ? p.base : sc(ctx, 0);
    const Derived DF = derived_in(base, p.o_fix, b->fixed.n);
    const Derived DV = derived_in(base, p.o_free, b->free.n);
    const int f32 = prec == LENS_FP64 ? 0 : PRO_F32;
    if (with_check) TRY(status_reset(ctx, st));
    if (parts == SRC_ALL_TABLES)
        HIP_TRY(launch_prologue2(soa(&b->fixed), b->fixed.n, const_cast<double *>(DF.d),
                                 const_cast<float *>(DF.f), DF.stride, soa(&b->free), b->free.n,
                                 const_cast<double *>(DV.d), const_cast<float *>(DV.f),
                                 DV.stride, ctx->small, f32, st));
    else if (parts == SRC_SAMPLES_DERIVE)
        ;  // the per-sample kernel derives the free constants itself
    else if (parts == SRC_FREE_ONLY)
        TRY(run_prologue(ctx, &b->free, DV, f32, st));
    Chi2SrcLaunch L;
    L.freet = DV;
    L.free_off = b->free_offset;
    L.n_samples = b->n_samples;
    L.sample0 = 0;
    L.nsys = c->n_sys;
    L.nimg = c->n_img;
    L.img_off = c->img_offset;
    L.x = c->x;
    L.y = c->y;
    L.sig = c->sigma;
    L.f = c->dlsds;
    L.fixedt = DF;
    L.rec = (double *)(base + p.o_rec);
    L.nimg_pad = p.nimg_pad;
    L.chi2 = chi2;
    L.src_x = sources ? (double *)(base + p.o_src) : nullptr;
    L.src_y = sources ? L.src_x + (size_t)b->n_samples * c->n_sys : nullptr;
    const bool batched = path == LENS_CHI2_PATH_BATCHED;
    L.prec = prec == LENS_FP64 ? 0 : 1;
    if (parts == SRC_ALL || parts == SRC_FIXED_ONLY) {
        L.inline_fixed = 1;
        L.free_prologue = parts == SRC_ALL ? 1 : 0;
        L.nfixed = b->fixed.n;
        L.fixed_amp = soa(&b->fixed);
        L.free_amp = soa(&b->free);
        L.status = ctx->small;
    }
    if (parts == SRC_ALL || parts == SRC_FIXED_ONLY || parts == SRC_ALL_TABLES) {
        if (rec) {
            rec->prep = L;
            rec->has_prep = true;
        } else {
            HIP_TRY(launch_chi2_prep(L, st));
        }
    }
    if (with_check) TRY(status_check(ctx, st));
    if (parts == SRC_FIXED_ONLY || b->n_samples == 0) return LENS_OK;
    if (parts == SRC_SAMPLES_DERIVE) {
        L.derive_free = 1;
        L.free_amp = soa(&b->free);
        L.status = ctx->small;
    }
    if (batched) {
        L.persistent = 1;
        L.grid_blocks = batched_blocks(ctx, b->n_samples);
        if (rec) {
            rec->src = L;
            rec->has_src = true;
        } else {
            HIP_TRY(launch_chi2_src(L, st));
        }
    } else {
        L.persistent = 0;
        L.grid_blocks = 1;
        for (int m = 0; m < b->n_samples; ++m) {
            L.sample0 = m;
            HIP_TRY(launch_chi2_src(L, st));
        }
    }
    return LENS_OK;
}

// Image-plane scratch after the source-plane part: the fixed potentials'
// deflection grid, then per chunk of samples the deflection grids, slot
// arrays and tile bounds.  The chunk is 128 samples (1 on the per-sample
// path), fewer when the context's scratch limit does not hold that many.
struct ImgPlan {
    size_t o_afix, o_alpha, o_count, o_tri, o_ix, o_iy, o_part, o_miss, o_tb;
    int chunk;
};

ImgPlan plan_img(Carve &cv, int nx, int ny, int n_sys, int kmax, int S, bool one_at_a_time,
                 uint64_t scratch_max) {
    ImgPlan p;
    const size_t nv = (size_t)nx * ny;
    p.o_afix = cv.take(2 * nv * sizeof(double));
    const size_t fixed_bytes = cv.off;
    int ntx, nty;
    image_tiles(nx, ny, ntx, nty);
    const size_t per_sample = 2 * nv * sizeof(double) + (size_t)ntx * nty * 4 * sizeof(double) +
                              (size_t)n_sys * (sizeof(int) + 2 * sizeof(double) + sizeof(int) +
                                               (size_t)kmax * (sizeof(long long) + 2 * sizeof(double))) +
                              4096;
    int chunk = one_at_a_time ? 1 : 128;
    if (scratch_max > fixed_bytes) {
        const size_t fit = (scratch_max - fixed_bytes) / per_sample;
        chunk = (int)std::min<size_t>(chunk, std::max<size_t>(fit, 1));
    }
    chunk = std::max(1, std::min(chunk, std::max(S, 1)));
    p.chunk = chunk;
    p.o_alpha = cv.take((size_t)chunk * 2 * nv * sizeof(double));
    p.o_count = cv.take((size_t)chunk * n_sys * sizeof(int));
    p.o_tri = cv.take((size_t)chunk * n_sys * kmax * sizeof(long long));
    p.o_ix = cv.take((size_t)chunk * n_sys * kmax * sizeof(double));
    p.o_iy = cv.take((size_t)chunk * n_sys * kmax * sizeof(double));
    p.o_part = cv.take((size_t)chunk * n_sys * sizeof(double));
    p.o_miss = cv.take((size_t)chunk * n_sys * sizeof(int));
    p.o_tb = cv.take((size_t)chunk * ntx * nty * 4 * sizeof(double));
    return p;
}

// Outputs of the image-plane sequence and the word its search reports to.
struct ImgOut {
    double *chi2;
    int32_t *nimg, *nmissing;
    double *img_xy;
    int *status;  // device: ST_OVERFLOW | ST_DOMAIN | ST_BAD_F bits of this call
};

// Which parts of the image-plane sequence to issue: everything; only what
// depends on the fixed potentials and the catalogue (their derived table,
// the per-image constants and the fixed potentials' deflection at the grid
// vertices); only what depends on the free potentials (their prologue, the
// sources, then per chunk the search and the assignment), the fixed part
// being ready.
enum ImgParts { IMG_ALL, IMG_FIXED_ONLY, IMG_FREE_ONLY };

// The launches of the image-plane chi^2 (Sec. 4.2, Fig. 7), with no
// synchronisation: sources (the source-plane kernels), the fixed potentials'
// deflection at the grid vertices, then per chunk of samples the vertex
// deflections, the triangle search, the slot order, the optional Newton
// refinement and the assignment.  Offsets of sp and ip refer to sp.base (the
// context's scratch when NULL).
lens_status_t img_sequence(lens_ctx_t *ctx, const lens_model_batch_t *b, const lens_catalog_t *c,
                           const lens_chi2_opts_t *o, const SrcPlan &sp, const ImgPlan &ip,
                           const ImgOut &out, hipStream_t st, bool with_check, ImgParts parts) {
    char *base = sp.base ? sp.base : sc(ctx, 0);
    const int S = b->n_samples;
    const int kmax = o->max_img_per_sys;
    const GridArgs G{o->grid.nx, o->grid.ny, o->grid.x0, o->grid.y0, o->grid.dx, o->grid.dy};
    const size_t nv = (size_t)G.nx * G.ny;
    const int chunk = ip.chunk;
    const Derived DF = derived_in(base, sp.o_fix, b->fixed.n);
    const Derived DV = derived_in(base, sp.o_free, b->free.n);
    double *afx = (double *)(base + ip.o_afix), *afy = afx + nv;
    if (parts != IMG_FIXED_ONLY) HIP_TRY(launch_zero_i32(out.status, 1, st));
    if (parts == IMG_ALL) {
        TRY(src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, nullptr, true, st,
                         with_check, SRC_ALL_TABLES));
    } else if (parts == IMG_FIXED_ONLY) {
        TRY(run_prologue(ctx, &b->fixed, DF, 0, st));
        TRY(src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, nullptr, true, st,
                         with_check, SRC_FIXED_ONLY));
    } else {
        TRY(run_prologue(ctx, &b->free, DV, o->prec == LENS_FP64 ? 0 : PRO_F32, st));
        TRY(src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, nullptr, true, st,
                         false, SRC_SAMPLES_ONLY));
    }
    if (parts != IMG_FREE_ONLY && b->fixed.n > 0) {
        MapLaunch m;
        m.tab = DF;
        m.grid = G;
        m.dlsds = 1.0;
        m.out[0] = afx;
        m.out[1] = afy;
        m.out[2] = m.out[3] = m.out[4] = nullptr;
        m.prec = 0;
        m.grad = true;
        m.hess = false;
        m.tune = ctx->tune[0];
        HIP_TRY(launch_map(m, st));
    }
    if (parts == IMG_FIXED_ONLY) return LENS_OK;
    const double *srcx = (const double *)(base + sp.o_src);
    const double *srcy = srcx + (size_t)S * c->n_sys;
    double *alpha = (double *)(base + ip.o_alpha);
    int *count = (int *)(base + ip.o_count);
    long long *tri = (long long *)(base + ip.o_tri);
    double *ix = (double *)(base + ip.o_ix), *iy = (double *)(base + ip.o_iy);
    for (int m0 = 0; m0 < S; m0 += chunk) {
        const int ns = std::min(chunk, S - m0);
        AlphaGridLaunch A;
        A.freet = DV;
        A.free_off = b->free_offset;
        A.m0 = m0;
        A.nsamp = ns;
        A.grid = G;
        A.afix_x = b->fixed.n > 0 ? afx : nullptr;
        A.afix_y = b->fixed.n > 0 ? afy : nullptr;
        A.out = alpha;
        A.prec = o->prec == LENS_FP64 ? 0 : 1;
        HIP_TRY(launch_alpha_grid(A, st));
        HIP_TRY(launch_zero_i32(count, ns * c->n_sys, st));
        ImgLaunch I;
        I.alpha = alpha;
        I.grid = G;
        I.n_grids = ns;
        I.nq = c->n_sys;
        I.sx = srcx + (size_t)m0 * c->n_sys;
        I.sy = srcy + (size_t)m0 * c->n_sys;
        I.f = c->dlsds;
        I.kmax = kmax;
        I.count = count;
        I.tri = tri;
        I.ix = ix;
        I.iy = iy;
        I.tb = (double *)(base + ip.o_tb);
        I.status = out.status;
        HIP_TRY(launch_find_images(I, st));
        HIP_TRY(launch_sort_images(ns * c->n_sys, kmax, count, tri, ix, iy, st));
        if (o->refine_max_iter > 0) {
            RefineLaunch F;
            F.fixedt = DF;
            F.freet = DV;
            F.free_off = b->free_offset;
            F.m0 = m0;
            F.nsamp = ns;
            F.nsys = c->n_sys;
            F.kmax = kmax;
            F.count = count;
            F.ix = ix;
            F.iy = iy;
            F.sx = I.sx;
            F.sy = I.sy;
            F.f = c->dlsds;
            F.max_iter = o->refine_max_iter;
            F.tol = o->refine_tol;
            F.max_shift = 2.0 * std::max(G.dx, G.dy);
            HIP_TRY(launch_refine_images(F, st));
        }
        AssignLaunch Q;
        Q.nsamp = ns;
        Q.nsys = c->n_sys;
        Q.kmax = kmax;
        Q.count = count;
        Q.ix = ix;
        Q.iy = iy;
        Q.img_off = c->img_offset;
        Q.nimg_total = c->n_img;
        Q.x = c->x;
        Q.y = c->y;
        Q.sig = c->sigma;
        Q.penalty = o->missing_penalty;
        Q.m0 = m0;
        Q.chi2 = out.chi2;
        Q.nimg = out.nimg;
        Q.nmissing = out.nmissing;
        Q.img_xy = out.img_xy;
        Q.part = (double *)(base + ip.o_part);
        Q.miss = (int *)(base + ip.o_miss);
        Q.status = out.status;
        HIP_TRY(launch_assign(Q, st));
    }
    return LENS_OK;
}

// The image search's device-side findings (read back after the call).
lens_status_t search_status(int bits) {
    if (bits & ST_BAD_F)
        return fail(LENS_EINVAL, "a source's Dls/Ds lies outside (0, 1]");
    if (bits & ST_DOMAIN)
        return fail(LENS_EINVAL,
                    "an orientation test met a coordinate outside the exact domain "
                    "(nonzero magnitudes in [2^-400, 2^400], finite)");
    return LENS_OK;
}

// Outcome of the image search from its status bits (read back after a call).
lens_status_t search_outcome(int bits) {
    TRY(search_status(bits));
    if (bits & ST_OVERFLOW)
        return fail(LENS_EOVERFLOW, "more images than max_img_per_sys in some (sample, system)");
    return LENS_OK;
}


lens_status_t check_chi2_args(lens_ctx_t *ctx, const lens_model_batch_t *b,
                              const lens_catalog_t *c, const lens_chi2_opts_t *o) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    if (!o) return fail(LENS_EINVAL, "opts is NULL");
    TRY(check_batch(b));
    TRY(check_catalog(c));
    TRY(check_prec(o->prec));
    if (o->path != LENS_CHI2_PATH_BATCHED && o->path != LENS_CHI2_PATH_PER_SAMPLE)
        return fail(LENS_EINVAL, "unknown path %d", o->path);
    if (o->mode != LENS_CHI2_SOURCE && o->mode != LENS_CHI2_IMAGE)
        return fail(LENS_EINVAL, "unknown mode %d", o->mode);
    if (o->mode == LENS_CHI2_IMAGE) {
        TRY(check_grid(&o->grid));
        if (o->grid.nx < 2 || o->grid.ny < 2)
            return fail(LENS_EINVAL, "image mode needs a grid of at least 2 x 2");
        if (o->max_img_per_sys < 1 || o->max_img_per_sys > 64)
            return fail(LENS_EINVAL, "max_img_per_sys = %d (1..64)", o->max_img_per_sys);
        if (!is_fin(o->missing_penalty))
            return fail(LENS_EINVAL, "missing_penalty is not finite");
        if (o->refine_max_iter < 0 || o->refine_max_iter > 64)
            return fail(LENS_EINVAL, "refine_max_iter = %d (0..64)", o->refine_max_iter);
        if (o->refine_max_iter > 0 && !(o->refine_tol > 0.0 && is_fin(o->refine_tol)))
            return fail(LENS_EINVAL, "refine_tol = %g (> 0)", o->refine_tol);
    }
    return LENS_OK;
}

// A plan: its own scratch, the fixed part computed once when resident, and
// the rest of one lens_chi2_batch call (batched path) captured into a graph.
lens_status_t plan_create(lens_ctx_t *ctx, const lens_model_batch_t *b, const lens_catalog_t *c,
                          const lens_chi2_opts_t *o, double *chi2, int32_t *nimg,
                          int32_t *nmissing, double *img_xy, uint32_t flags, void *stream,
                          lens_chi2_plan_t **out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(check_chi2_args(ctx, b, c, o));
    if (flags & ~LENS_PLAN_FIXED_RESIDENT)
        return fail(LENS_EINVAL, "unknown plan flags %u", (unsigned)flags);
    const bool resident = (flags & LENS_PLAN_FIXED_RESIDENT) != 0;
    const bool img = o->mode == LENS_CHI2_IMAGE;
    const int S = b->n_samples;
    TRY(check_range(chi2, (size_t)S * sizeof(double), "chi2"));
    if (img) {
        const int kmax = o->max_img_per_sys;
        if (nimg) TRY(check_range(nimg, (size_t)S * c->n_sys * sizeof(int32_t), "nimg"));
        if (nmissing) TRY(check_range(nmissing, (size_t)S * sizeof(int32_t), "nmissing"));
        if (img_xy)
            TRY(check_range(img_xy, (size_t)S * c->n_sys * kmax * 2 * sizeof(double), "img_xy"));
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Carve cv;
    SrcPlan sp = plan_src(cv, b, c, img);
    ImgPlan ip{};
    if (img)
        ip = plan_img(cv, o->grid.nx, o->grid.ny, c->n_sys, o->max_img_per_sys, S, false,
                      ctx->scratch_max);
    const size_t o_status = cv.take(sizeof(int));
    TRY(check_contents(ctx, b, c, st));
    lens_chi2_plan_t *p = new lens_chi2_plan_t();
    p->ctx = ctx;
    hipError_t e = hipMalloc(&p->mem, std::max<size_t>(cv.off, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(LENS_ENOMEM, "hipMalloc(%zu) for the plan failed", cv.off);
    }
    sp.base = (char *)p->mem;
    p->status = (int *)(sp.base + o_status);
    auto bail = [&](lens_status_t s) {
        (void)hipStreamSynchronize(st);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        (void)hipFree(p->mem);
        delete p;
        return s;
    };
    // validate the tables once, outside the capture (checked contexts), and
    // with LENS_PLAN_FIXED_RESIDENT compute the fixed part now
    const ImgOut io{chi2, nimg, nmissing, img_xy, p->status};
    lens_status_t s = LENS_OK;
    if (img) {
        if (resident || checked(ctx))
            s = img_sequence(ctx, b, c, o, sp, ip, io, st, checked(ctx), IMG_FIXED_ONLY);
    } else {
        s = src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, nullptr, false, st,
                         checked(ctx), SRC_FIXED_ONLY);
    }
    if (s == LENS_OK && checked(ctx)) {
        s = status_reset(ctx, st);
        const Derived DV = derived_in(sp.base, sp.o_free, b->free.n);
        if (s == LENS_OK)
            s = run_prologue(ctx, &b->free, DV, o->prec == LENS_FP64 ? 0 : PRO_F32, st);
        if (s == LENS_OK) s = status_check(ctx, st);
    }
    if (s != LENS_OK) return bail(s);
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(LENS_EDEVICE, "%s", hipGetErrorString(e)));
    if (!img) {
        // one or two kernels: replayed as plain launches of their recorded
        // descriptions (a graph launch costs more here than the launches it
        // would save)
        SrcRecord r;
        s = src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, chi2, false, st, false,
                         resident ? SRC_SAMPLES_DERIVE : SRC_ALL, &r);
        if (s != LENS_OK) return bail(s);
        p->direct = true;
        p->has_prep = r.has_prep;
        p->has_src = r.has_src;
        p->prep = r.prep;
        p->src = r.src;
        p->status = nullptr;
        *out = p;
        return LENS_OK;
    }
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return bail(fail(LENS_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e)));
    if (img)
        s = img_sequence(ctx, b, c, o, sp, ip, io, st, false,
                         resident ? IMG_FREE_ONLY : IMG_ALL);
    else
        s = src_sequence(ctx, b, c, o->prec, LENS_CHI2_PATH_BATCHED, sp, chi2, false, st, false,
                         resident ? SRC_SAMPLES_DERIVE : SRC_ALL);
    e = hipStreamEndCapture(st, &p->graph);
    if (s != LENS_OK) return bail(s);
    if (e != hipSuccess)
        return bail(fail(LENS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e)));
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return bail(fail(LENS_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)));
    // the executable graph's resources go to the device now, not at the
    // first launch
    e = hipGraphUpload(p->exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(p->exec);
        return bail(fail(LENS_EDEVICE, "hipGraphUpload: %s", hipGetErrorString(e)));
    }
    if (!img) p->status = nullptr;
    *out = p;
    return LENS_OK;
}

}  // namespace

// =============================================================================
extern "C" {

const char *lens_last_error(void) { return g_err.c_str(); }
int32_t lens_abi_version(void) { return LENSHPC_ABI_VERSION; }

lens_status_t lens_ctx_create(int32_t device, uint64_t scratch_bytes_max, uint32_t flags,
                              lens_ctx_t **out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(LENS_EDEVICE, "no HIP device");
    }
    if (device < 0 || device >= ndev) return fail(LENS_EINVAL, "device %d of %d", device, ndev);
    if (flags & ~LENS_CTX_CHECK_TABLES) return fail(LENS_EINVAL, "unknown flags 0x%x", flags);
    DeviceGuard dg(device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", device);
    TRY(noalloc_setup(device));
    lens_ctx_t *c = new lens_ctx_t();
    c->device = device;
    c->scratch_max = scratch_bytes_max;
    c->flags = flags;
    for (int p = 0; p < 3; ++p) c->tune[p] = kDefaultMapTuning;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&c->small, 64 * sizeof(int)) != hipSuccess ||
        hipHostMalloc(&c->host_small, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (c->small) (void)hipFree(c->small);
        delete c;
        return fail(LENS_ENOMEM, "context allocation failed");
    }
    if (hipMemset(c->small, 0, 64 * sizeof(int)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->small);
        (void)hipHostFree(c->host_small);
        delete c;
        return fail(LENS_EDEVICE, "context initialisation failed");
    }
    *out = c;
    return LENS_OK;
}

lens_status_t lens_ctx_destroy(lens_ctx_t *ctx) {
    if (!ctx) return LENS_OK;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->small) (void)hipFree(ctx->small);
    if (ctx->host_small) (void)hipHostFree(ctx->host_small);
    delete ctx;
    return LENS_OK;
}

lens_status_t lens_ctx_status(lens_ctx_t *ctx) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(ctx->host_small, ctx->small, sizeof(int), hipMemcpyDeviceToHost));
    const int s = ctx->host_small[0];
    HIP_TRY(hipMemset(ctx->small, 0, sizeof(int)));
    if (s & ST_INVALID_TABLE) return fail(LENS_EINVAL, "a table held invalid parameters");
    if (s & ST_OVERFLOW) return fail(LENS_EOVERFLOW, "image slots overflowed");
    return LENS_OK;
}

lens_status_t lens_set_map_tuning(lens_ctx_t *ctx, lens_precision_t prec,
                                  const lens_map_tuning_t *t) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    TRY(check_prec(prec));
    if (!t) {
        ctx->tune[prec] = kDefaultMapTuning;
        return LENS_OK;
    }
    if (!map_tuning_valid(*t))
        return fail(LENS_EINVAL, "invalid map tuning {%d,%d,%d,%d,%d}", t->block_x, t->block_y,
                    t->pix_per_thread, t->stage, t->lds_chunk);
    ctx->tune[prec] = *t;
    return LENS_OK;
}

lens_status_t lens_get_map_tuning(lens_ctx_t *ctx, lens_precision_t prec, lens_map_tuning_t *out) {
    if (!ctx || !out) return fail(LENS_EINVAL, "NULL argument");
    TRY(check_prec(prec));
    *out = ctx->tune[prec];
    return LENS_OK;
}

lens_status_t lens_set_chi2_tuning(lens_ctx_t *ctx, int32_t blocks_per_cu) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    if (blocks_per_cu < 1 || blocks_per_cu > 64)
        return fail(LENS_EINVAL, "waves_per_cu = %d (1..64)", blocks_per_cu);
    ctx->chi2_blocks_per_cu = blocks_per_cu;
    return LENS_OK;
}

lens_status_t lens_get_chi2_tuning(lens_ctx_t *ctx, int32_t *blocks_per_cu) {
    if (!ctx || !blocks_per_cu) return fail(LENS_EINVAL, "NULL argument");
    *blocks_per_cu = ctx->chi2_blocks_per_cu;
    return LENS_OK;
}

lens_status_t lens_table_from_physical(lens_ctx_t *ctx, const lens_phys_table_t *phys,
                                       int32_t convention, double *out_b0, double *out_eps,
                                       void *stream) {
    if (!ctx || !phys) return fail(LENS_EINVAL, "NULL argument");
    if (phys->n < 0) return fail(LENS_EINVAL, "n < 0");
    if (convention != 0 && convention != 1) return fail(LENS_EINVAL, "convention %d", convention);
    const size_t b = (size_t)phys->n * sizeof(double);
    TRY(check_range(phys->sigma, b, "phys.sigma"));
    TRY(check_range(phys->e, b, "phys.e"));
    TRY(check_range(out_b0, b, "out_b0"));
    TRY(check_range(out_eps, b, "out_eps"));
    DeviceGuard dg(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    TRY(status_reset(ctx, st));
    HIP_TRY(launch_phys_to_amp(phys->sigma, phys->e, phys->n, convention, out_b0, out_eps,
                               ctx->small, st));
    TRY(status_check(ctx, st));
    return LENS_OK;
}

lens_status_t lens_grad_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                            const lens_grid_t *grid, double dlsds, lens_precision_t prec, void *ax,
                            void *ay, void *stream) {
    if (!ax || !ay) return fail(LENS_EINVAL, "ax and ay are required");
    void *out[5] = {ax, ay, nullptr, nullptr, nullptr};
    return map_common(ctx, table, grid, dlsds, prec, out, true, false, (hipStream_t)stream);
}

lens_status_t lens_hessian_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                               const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                               void *hxx, void *hxy, void *hyy, void *ax, void *ay, void *stream) {
    if (!hxx || !hxy || !hyy) return fail(LENS_EINVAL, "hxx, hxy and hyy are required");
    if ((ax == nullptr) != (ay == nullptr))
        return fail(LENS_EINVAL, "ax and ay must both be given or both be NULL");
    void *out[5] = {ax, ay, hxx, hxy, hyy};
    return map_common(ctx, table, grid, dlsds, prec, out, ax != nullptr, true,
                      (hipStream_t)stream);
}

lens_status_t lens_hessian_map_noalloc(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                       const lens_grid_t *grid, double dlsds,
                                       lens_precision_t prec, void *hxx, void *hxy, void *hyy,
                                       void *ax, void *ay, void *stream) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    if (!hxx || !hxy || !hyy) return fail(LENS_EINVAL, "hxx, hxy and hyy are required");
    if ((ax == nullptr) != (ay == nullptr))
        return fail(LENS_EINVAL, "ax and ay must both be given or both be NULL");
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices)
            base = static_cast<char *>(g_noalloc_ptr[ctx->device]);
    }
    if (!base) return fail(LENS_EDEVICE, "no fixed scratch on device %d", ctx->device);
    void *out[5] = {ax, ay, hxx, hxy, hyy};
    return map_common(ctx, table, grid, dlsds, prec, out, ax != nullptr, true,
                      (hipStream_t)stream, nullptr, base);
}

// Potential (td = 0) or time-delay (td = 1) map: validation, prologue, kernel.
lens_status_t psi_common(lens_ctx_t *ctx, const lens_pot_table_t *table, const lens_grid_t *grid,
                         double dlsds, int td, double bx, double by, double scale, double *out,
                         hipStream_t st) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    TRY(check_table(table, "table"));
    TRY(check_grid(grid));
    if (!is_fin(dlsds) || dlsds < 0) return fail(LENS_EINVAL, "dlsds = %g", dlsds);
    if (td && (!is_fin(bx) || !is_fin(by) || !is_fin(scale)))
        return fail(LENS_EINVAL, "beta and scale must be finite");
    TRY(check_range(out, (size_t)grid->nx * grid->ny * sizeof(double), td ? "t" : "psi"));
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    Carve cv;
    const size_t o_tab = cv.take(derived_bytes(table->n));
    TRY(ensure_scratch(ctx, cv.off));
    const Derived D = derived_at(ctx, o_tab, table->n);
    TRY(status_reset(ctx, st));
    TRY(run_prologue(ctx, table, D, PRO_LOG, st));
    TRY(status_check(ctx, st));
    const GridArgs G{grid->nx, grid->ny, grid->x0, grid->y0, grid->dx, grid->dy};
    HIP_TRY(launch_potential_map(D, G, dlsds, out, td, bx, by, scale, st));
    return LENS_OK;
}

lens_status_t lens_potential_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                 const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                                 double *psi, void *stream) {
    if (prec != LENS_FP64)
        return fail(LENS_EUNSUPPORTED, "the potential map is computed in FP64 only");
    return psi_common(ctx, table, grid, dlsds, 0, 0.0, 0.0, 0.0, psi, (hipStream_t)stream);
}

lens_status_t lens_time_delay_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                  const lens_grid_t *grid, double dlsds, double beta_x,
                                  double beta_y, double scale, double *t, void *stream) {
    return psi_common(ctx, table, grid, dlsds, 1, beta_x, beta_y, scale, t, (hipStream_t)stream);
}

lens_status_t lens_derived_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                               const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                               void *kappa, void *gamma1, void *gamma2, void *gamma, void *mu,
                               void *det, void *stream) {
    void *dout[6] = {kappa, gamma1, gamma2, gamma, mu, det};
    bool any = false;
    for (int c = 0; c < 6; ++c) any |= dout[c] != nullptr;
    if (!any) return fail(LENS_EINVAL, "no output requested");
    void *out[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    return map_common(ctx, table, grid, dlsds, prec, out, false, true, (hipStream_t)stream, dout);
}

lens_status_t lens_chi2_batch(lens_ctx_t *ctx, const lens_model_batch_t *b,
                              const lens_catalog_t *c, const lens_chi2_opts_t *o, double *chi2,
                              int32_t *nimg, int32_t *nmissing, double *img_xy, void *stream) {
    TRY(check_chi2_args(ctx, b, c, o));
    const int S = b->n_samples;
    TRY(check_range(chi2, (size_t)S * sizeof(double), "chi2"));
    const bool img = o->mode == LENS_CHI2_IMAGE;
    const int kmax = img ? o->max_img_per_sys : 0;
    if (img) {
        if (nimg) TRY(check_range(nimg, (size_t)S * c->n_sys * sizeof(int32_t), "nimg"));
        if (nmissing) TRY(check_range(nmissing, (size_t)S * sizeof(int32_t), "nmissing"));
        if (img_xy)
            TRY(check_range(img_xy, (size_t)S * c->n_sys * kmax * 2 * sizeof(double), "img_xy"));
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Carve cv;
    SrcPlan sp = plan_src(cv, b, c, img);
    if (!img) {
        TRY(ensure_scratch(ctx, cv.off));
        TRY(check_contents(ctx, b, c, st));
        return src_sequence(ctx, b, c, o->prec, o->path, sp, chi2, false, st, true);
    }
    // ---- image plane ----
    const ImgPlan ip = plan_img(cv, o->grid.nx, o->grid.ny, c->n_sys, kmax, S,
                                o->path == LENS_CHI2_PATH_PER_SAMPLE, ctx->scratch_max);
    TRY(ensure_scratch(ctx, cv.off));
    TRY(check_contents(ctx, b, c, st));
    const ImgOut out{chi2, nimg, nmissing, img_xy, ctx->small + 2};
    TRY(img_sequence(ctx, b, c, o, sp, ip, out, st, true, IMG_ALL));
    HIP_TRY(hipMemcpyAsync(ctx->host_small + 2, ctx->small + 2, sizeof(int),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return search_outcome(ctx->host_small[2]);
}

lens_status_t lens_find_images(lens_ctx_t *ctx, const double *ax, const double *ay,
                               const lens_grid_t *grid, int32_t n_src, const double *src_x,
                               const double *src_y, const double *f, int32_t kmax, int32_t *nimg,
                               int64_t *img_tri, double *img_x, double *img_y, void *stream) {
    if (!ctx) return fail(LENS_EINVAL, "ctx is NULL");
    TRY(check_grid(grid));
    if (grid->nx < 2 || grid->ny < 2) return fail(LENS_EINVAL, "grid must be at least 2 x 2");
    if (n_src < 0) return fail(LENS_EINVAL, "n_src < 0");
    if (kmax < 1 || kmax > 64) return fail(LENS_EINVAL, "kmax = %d (1..64)", kmax);
    const size_t nv = (size_t)grid->nx * grid->ny;
    if (ay != ax + nv)
        return fail(LENS_EINVAL, "ay must follow ax in one buffer (ay == ax + nx*ny)");
    TRY(check_range(ax, 2 * nv * sizeof(double), "ax/ay"));
    TRY(check_range(src_x, (size_t)n_src * 8, "src_x"));
    TRY(check_range(src_y, (size_t)n_src * 8, "src_y"));
    TRY(check_range(f, (size_t)n_src * 8, "f"));
    TRY(check_range(nimg, (size_t)n_src * 4, "nimg"));
    TRY(check_range(img_tri, (size_t)n_src * kmax * 8, "img_tri"));
    TRY(check_range(img_x, (size_t)n_src * kmax * 8, "img_x"));
    TRY(check_range(img_y, (size_t)n_src * kmax * 8, "img_y"));
    if (n_src == 0) return LENS_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    int ntx, nty;
    image_tiles(grid->nx, grid->ny, ntx, nty);
    Carve cv;
    const size_t o_tb = cv.take((size_t)ntx * nty * 4 * sizeof(double));
    TRY(ensure_scratch(ctx, cv.off));
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_zero_i32(nimg, n_src, st));
    HIP_TRY(launch_zero_i32(ctx->small + 2, 1, st));  // search status word
    HIP_TRY(launch_fill_i64((long long *)img_tri, (size_t)n_src * kmax, -1, st));
    HIP_TRY(launch_fill_f64(img_x, (size_t)n_src * kmax, NAN, st));
    HIP_TRY(launch_fill_f64(img_y, (size_t)n_src * kmax, NAN, st));
    ImgLaunch I;
    I.alpha = ax;
    I.grid = GridArgs{grid->nx, grid->ny, grid->x0, grid->y0, grid->dx, grid->dy};
    I.n_grids = 1;
    I.nq = n_src;
    I.sx = src_x;
    I.sy = src_y;
    I.f = f;
    I.kmax = kmax;
    I.count = nimg;
    I.tri = (long long *)img_tri;
    I.ix = img_x;
    I.iy = img_y;
    I.tb = (double *)sc(ctx, o_tb);
    I.status = ctx->small + 2;
    HIP_TRY(launch_find_images(I, st));
    HIP_TRY(launch_sort_images(n_src, kmax, nimg, (long long *)img_tri, img_x, img_y, st));
    std::vector<int32_t> cnt(n_src);
    HIP_TRY(hipMemcpyAsync(cnt.data(), nimg, (size_t)n_src * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ctx->host_small + 2, ctx->small + 2, sizeof(int),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    TRY(search_status(ctx->host_small[2]));
    for (int s = 0; s < n_src; ++s)
        if (cnt[s] > kmax) return fail(LENS_EOVERFLOW, "source %d has %d images > kmax", s, cnt[s]);
    return LENS_OK;
}

// ---------------------------------------------------------------------------
lens_status_t lens_chi2_plan_create_ex(lens_ctx_t *ctx, const lens_model_batch_t *b,
                                       const lens_catalog_t *c, const lens_chi2_opts_t *o,
                                       double *chi2, uint32_t flags, void *stream,
                                       lens_chi2_plan_t **out) {
    if (o && o->mode != LENS_CHI2_SOURCE) {
        if (out) *out = nullptr;
        return fail(LENS_EUNSUPPORTED, "image-mode plans are created by lens_chi2_plan_create2");
    }
    return plan_create(ctx, b, c, o, chi2, nullptr, nullptr, nullptr, flags, stream, out);
}

lens_status_t lens_chi2_plan_create2(lens_ctx_t *ctx, const lens_model_batch_t *b,
                                     const lens_catalog_t *c, const lens_chi2_opts_t *o,
                                     double *chi2, int32_t *nimg, int32_t *nmissing,
                                     double *img_xy, uint32_t flags, void *stream,
                                     lens_chi2_plan_t **out) {
    return plan_create(ctx, b, c, o, chi2, nimg, nmissing, img_xy, flags, stream, out);
}

lens_status_t lens_chi2_plan_status(lens_chi2_plan_t *p, void *stream) {
    if (!p) return fail(LENS_EINVAL, "plan is NULL");
    if (!p->status) return LENS_OK;
    DeviceGuard dg(p->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    int bits = 0;
    HIP_TRY(hipMemcpyAsync(p->ctx->host_small + 3, p->status, sizeof(int),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bits = p->ctx->host_small[3];
    return search_outcome(bits);
}

lens_status_t lens_chi2_plan_create(lens_ctx_t *ctx, const lens_model_batch_t *b,
                                    const lens_catalog_t *c, const lens_chi2_opts_t *o,
                                    double *chi2, void *stream, lens_chi2_plan_t **out) {
    return lens_chi2_plan_create_ex(ctx, b, c, o, chi2, 0u, stream, out);
}

// ---------------------------------------------------------------------------
// Metropolis sampler: the fixed part's per-image constants are computed once;
// a step is one launch of the source-plane chi^2 kernel in its sampler form
// (each wave proposes for its walker, derives the proposal's potentials,
// evaluates its chi^2 and takes the decision).
lens_status_t lens_mcmc_create(lens_ctx_t *ctx, const lens_pot_table_t *fixed,
                               const lens_catalog_t *c, const lens_mcmc_desc_t *d, void *stream,
                               lens_mcmc_t **out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !d) return fail(LENS_EINVAL, "ctx or desc is NULL");
    TRY(check_table(fixed, "fixed"));
    TRY(check_catalog(c));
    const int W = d->n_walkers, nf = d->n_free;
    if (W < 1 || nf < 1 || (long long)W * nf > (1LL << 28))
        return fail(LENS_EINVAL, "n_walkers = %d, n_free = %d", W, nf);
    if (d->convention != 0 && d->convention != 1)
        return fail(LENS_EINVAL, "convention = %d", d->convention);
    const int P = 7 * nf;
    TRY(check_range(d->params, (size_t)W * P * sizeof(double), "params"));
    TRY(check_range(d->chi2, (size_t)W * sizeof(double), "chi2"));
    TRY(check_range(d->accepted, (size_t)W * sizeof(int32_t), "accepted"));
    TRY(check_range(d->lo, (size_t)P * sizeof(double), "lo"));
    TRY(check_range(d->hi, (size_t)P * sizeof(double), "hi"));
    TRY(check_range(d->step, (size_t)P * sizeof(double), "step"));
    TRY(check_range(d->u, (size_t)W * (P + 1) * sizeof(double), "u"));
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(LENS_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // the prior box must lie inside the valid parameter domain, and the
    // walkers inside the box (read back once)
    std::vector<double> lo(P), hi(P), step(P), th((size_t)W * P);
    HIP_TRY(hipMemcpyAsync(lo.data(), d->lo, P * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hi.data(), d->hi, P * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(step.data(), d->step, P * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(th.data(), d->params, th.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < nf; ++k) {
        const double *l = &lo[7 * k], *h = &hi[7 * k];
        for (int j = 0; j < 7; ++j)
            if (!(l[j] <= h[j]) || !is_fin(l[j]) || (j != 6 && !is_fin(h[j])) ||
                !(step[7 * k + j] >= 0.0) || !is_fin(step[7 * k + j]))
                return fail(LENS_EINVAL, "prior box or step of potential %d, parameter %d", k, j);
        if (!(l[2] >= 0.0) || !(l[3] >= 0.0) || !(h[3] < 1.0) || !(l[5] >= 0.0) || !(h[5] < l[6]))
            return fail(LENS_EINVAL,
                        "prior box of potential %d leaves the valid domain (sigma >= 0, "
                        "0 <= e < 1, 0 <= rcore < rcut)", k);
    }
    for (int w = 0; w < W; ++w)
        for (int i = 0; i < P; ++i) {
            const double v = th[(size_t)w * P + i];
            if (!(v >= lo[i] && v <= hi[i]))
                return fail(LENS_EINVAL, "walker %d parameter %d = %g outside the prior box", w,
                            i, v);
        }
    // own memory: the fixed potentials' derived table and per-image constants
    Carve cv;
    SrcPlan sp;
    sp.nimg_pad = (c->n_img + 63) / 64 * 64;
    sp.o_fix = cv.take(derived_bytes(fixed->n));
    sp.o_free = cv.take(derived_bytes(0));
    sp.o_rec = cv.take((size_t)CHI2_REC_ROWS * sp.nimg_pad * sizeof(double));
    sp.o_src = 0;
    lens_mcmc_t *m = new lens_mcmc_t();
    m->ctx = ctx;
    hipError_t e = hipMalloc(&m->mem, cv.off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return fail(LENS_ENOMEM, "hipMalloc(%zu) for the sampler failed", cv.off);
    }
    sp.base = (char *)m->mem;
    auto bail = [&](lens_status_t s) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(m->mem);
        delete m;
        return s;
    };
    // the fixed part once (its prologue and the per-image constants); the
    // walkers' potentials are derived by the chi^2 waves themselves
    lens_model_batch_t b;
    b.n_samples = W;
    b.free_offset = nullptr;
    b.free = lens_pot_table_t{0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    b.fixed = *fixed;
    lens_status_t s = check_catalog_contents(ctx, c, st);
    if (s != LENS_OK) return bail(s);
    s = src_sequence(ctx, &b, c, LENS_FP64, LENS_CHI2_PATH_BATCHED, sp, nullptr,
                                   false, st, checked(ctx), SRC_FIXED_ONLY);
    if (s != LENS_OK) return bail(s);
    Chi2SrcLaunch &L = m->step;
    L.freet = derived_in(sp.base, sp.o_free, 0);
    L.fixedt = derived_in(sp.base, sp.o_fix, fixed->n);
    L.free_off = nullptr;
    L.n_samples = W;
    L.sample0 = 0;
    L.nsys = c->n_sys;
    L.nimg = c->n_img;
    L.img_off = c->img_offset;
    L.x = c->x;
    L.y = c->y;
    L.sig = c->sigma;
    L.f = c->dlsds;
    L.nimg_pad = sp.nimg_pad;
    L.chi2 = nullptr;
    L.src_x = L.src_y = nullptr;
    L.rec = (double *)(sp.base + sp.o_rec);
    // (batch-shaped blocks sharing the staged catalogue; the launch takes one
    // wave per walker)
    L.persistent = 1;
    L.grid_blocks = W;
    L.prec = 0;
    L.mc.nfree = nf;
    L.mc.params = d->params;
    L.mc.chi2 = d->chi2;
    L.mc.accepted = d->accepted;
    L.mc.lo = d->lo;
    L.mc.hi = d->hi;
    L.mc.step = d->step;
    L.mc.u = d->u;
    L.mc.bK = d->convention == 1 ? 4.0 : 6.0;
    L.mc.status = ctx->small;
    // chi^2 of the initial state
    L.mc.mode = 1;
    e = launch_mcmc_chi2(L, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(LENS_EDEVICE, "%s", hipGetErrorString(e)));
    L.mc.mode = 2;
    *out = m;
    return LENS_OK;
}

lens_status_t lens_mcmc_step(lens_mcmc_t *m, void *stream) {
    if (!m) return fail(LENS_EINVAL, "sampler is NULL");
    DeviceGuard dg(m->ctx->device);
    HIP_TRY(launch_mcmc_chi2(m->step, (hipStream_t)stream));
    return LENS_OK;
}

lens_status_t lens_mcmc_destroy(lens_mcmc_t *m) {
    if (!m) return LENS_OK;
    DeviceGuard dg(m->ctx->device);
    if (m->mem) (void)hipFree(m->mem);
    delete m;
    return LENS_OK;
}

lens_status_t lens_chi2_plan_launch(lens_chi2_plan_t *p, void *stream) {
    if (!p) return fail(LENS_EINVAL, "plan is NULL");
    DeviceGuard dg(p->ctx->device);
    const hipStream_t st = (hipStream_t)stream;
    if (p->direct) {
        if (p->has_prep) HIP_TRY(launch_chi2_prep(p->prep, st));
        if (p->has_src) HIP_TRY(launch_chi2_src(p->src, st));
        return LENS_OK;
    }
    HIP_TRY(hipGraphLaunch(p->exec, st));
    return LENS_OK;
}

lens_status_t lens_chi2_plan_destroy(lens_chi2_plan_t *p) {
    if (!p) return LENS_OK;
    DeviceGuard dg(p->ctx->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->mem) (void)hipFree(p->mem);  // waits for launches still using it
    delete p;
    return LENS_OK;
}

// ---------------------------------------------------------------------------
// Scratch sizing (host arithmetic only): the same carve the calls make.
lens_status_t lens_map_scratch_bytes(int32_t n_pot, uint64_t *out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    if (n_pot < 0) return fail(LENS_EINVAL, "n_pot < 0");
    Carve cv;
    cv.take(derived_bytes(n_pot));
    *out = cv.off;
    return LENS_OK;
}

lens_status_t lens_chi2_scratch_bytes(int32_t n_fixed, int32_t n_free, int32_t n_samples,
                                      int32_t n_sys, int32_t n_img, const lens_chi2_opts_t *o,
                                      uint64_t *out) {
    if (!out || !o) return fail(LENS_EINVAL, "out or opts is NULL");
    if (n_fixed < 0 || n_free < 0 || n_samples < 0 || n_sys < 1 || n_img < 1)
        return fail(LENS_EINVAL, "sizes out of range");
    const bool img = o->mode == LENS_CHI2_IMAGE;
    if (img && (o->grid.nx < 2 || o->grid.ny < 2 || o->max_img_per_sys < 1 ||
                o->max_img_per_sys > 64))
        return fail(LENS_EINVAL, "image mode: grid of at least 2 x 2, max_img_per_sys 1..64");
    lens_model_batch_t b{};
    b.n_samples = n_samples;
    b.fixed.n = n_fixed;
    b.free.n = n_free;
    lens_catalog_t c{};
    c.n_sys = n_sys;
    c.n_img = n_img;
    Carve cv;
    plan_src(cv, &b, &c, img);
    if (img)
        plan_img(cv, o->grid.nx, o->grid.ny, n_sys, o->max_img_per_sys, n_samples,
                 o->path == LENS_CHI2_PATH_PER_SAMPLE, UINT64_MAX);
    *out = cv.off;
    return LENS_OK;
}

// ---------------------------------------------------------------------------
// Host helpers.
// Dls/Ds = 1 - chi(zl)/chi(zs), chi(z) = int_0^z dz'/sqrt(om (1+z')^3 + ol),
// by 5-point Gauss-Legendre on 512 equal panels.
static double comoving_gl(double z, double om, double ol) {
    static const double xg[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                                 0.5384693101056831, 0.9061798459386640};
    static const double wg[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                 0.4786286704993665, 0.2369268850561891};
    const int panels = 512;
    const double h = z / panels;
    double s = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double mid = (p + 0.5) * h;
        for (int g = 0; g < 5; ++g) {
            const double zz = mid + 0.5 * h * xg[g];
            const double a = 1.0 + zz;
            s += wg[g] / sqrt(om * a * a * a + ol);
        }
    }
    return 0.5 * h * s;
}

lens_status_t lens_dlsds(double zl, double zs, double om, double ol, double *out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    if (!(zl >= 0.0) || !(zs > zl) || !is_fin(zs) || !(om >= 0.0) || !(ol >= 0.0) ||
        fabs(om + ol - 1.0) > 1e-9)
        return fail(LENS_EINVAL, "need 0 <= zl < zs and a flat cosmology (om + ol = 1)");
    *out = 1.0 - comoving_gl(zl, om, ol) / comoving_gl(zs, om, ol);
    return LENS_OK;
}

lens_status_t lens_time_delay_scale(double zl, double zs, double h0, double om, double ol,
                                    double *out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    if (!(zl > 0.0) || !(zs > zl) || !is_fin(zs) || !(h0 > 0.0) || !is_fin(h0) ||
        !(om >= 0.0) || !(ol >= 0.0) || fabs(om + ol - 1.0) > 1e-9)
        return fail(LENS_EINVAL, "need 0 < zl < zs, H0 > 0 and a flat cosmology");
    const double cl = comoving_gl(zl, om, ol), cs = comoving_gl(zs, om, ol);
    const double h0_si = h0 * 1000.0 / 3.0856775814913673e22;  // km/s/Mpc -> 1/s
    const double rad = M_PI / 648000.0;                          // arcsec -> rad
    *out = cl * cs / ((cs - cl) * h0_si) * rad * rad / 86400.0;
    return LENS_OK;
}

lens_status_t lens_b0_from_sigma(double sigma_kms, int32_t convention, double *out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    if (!(sigma_kms >= 0.0) || !is_fin(sigma_kms) || (convention != 0 && convention != 1))
        return fail(LENS_EINVAL, "sigma %g, convention %d", sigma_kms, convention);
    const double v = sigma_kms / 299792.458;
    *out = (convention == 1 ? 4.0 : 6.0) * M_PI * v * v * (648000.0 / M_PI);
    return LENS_OK;
}

lens_status_t lens_eps_from_e(double e, double *out) {
    if (!out) return fail(LENS_EINVAL, "out is NULL");
    if (!(e >= 0.0 && e < 1.0)) return fail(LENS_EINVAL, "e = %g outside [0, 1)", e);
    *out = e / (1.0 + sqrt(1.0 - e * e));
    return LENS_OK;
}

}  // extern "C"
