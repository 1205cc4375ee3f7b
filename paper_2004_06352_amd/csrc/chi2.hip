// chi2.hip -- deflections at the constraint positions, the batched
// source-plane chi^2 (paper Sec. 2.2, Fig. 3 and Eq. (6): unlens every image
// with the lens equation of Sec. 2.1 Eq. (1), take each system's barycentre,
// sum the scatter over sigma^2) and the per-sample vertex deflection grids of
// the image-plane chi^2 (Sec. 4.2, stage 1).
//
// Design (gfx950): one wave per model sample.  What all samples share (the
// fixed potentials' deflection at each image, each image's Dls/Ds) is
// computed once per call, one block per image; a sample then costs its free
// potentials at its images, staged through LDS and evaluated for several
// images per lane.
// Unlensed positions go to LDS, lanes take one system each and the sums are
// combined by a shuffle reduction in a fixed order.  The batched path
// launches a few waves per SIMD that stride over the batch (a shared work
// counter would serialise every wave on one L2 atomic); the per-sample path
// launches the same kernel once per sample.  Both produce bit-identical
// results.
#include <math.h>

#include <algorithm>

#include "prologue.h"

#include "chi2_launch.h"
#include "eval.h"

namespace lens {

// ---------------------------------------------------------------------------
__device__ __forceinline__ int system_of(const int *__restrict__ off, int nsys, int t) {
    int lo = 0, hi = nsys;  // off[lo] <= t < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
// Two sums at once, step by step (the same additions as wave_sum on each, the
// two shuffles of a step in flight together)
__device__ __forceinline__ void wave_sum2(double &u, double &v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double su = __shfl_down(u, o, 64), sv = __shfl_down(v, o, 64);
        u += su;
        v += sv;
    }
}

// Per-image constants that every sample shares, computed once per call:
// rec[0][t], rec[1][t] = the fixed potentials' deflection at image t,
// rec[2][t] = the image's Dls/Ds (its system's: with at most 64 systems found
// by one ballot over their first images, else by bisection over the image
// offsets staged in LDS) and rec[3][t] = 1/sigma_t^2, the weight of its
// term in Eq. (6).  One block per image, of as many threads as
// there are fixed potentials (rounded up to whole waves, at most
// PREP_MAX_BLOCK): thread l evaluates the fixed potentials l, l + blockDim,
// ... in that order (lanes hold different potentials, so the kind branches
// may diverge), then a shuffle tree per wave and the wave sums in order.
// The block size depends only on the number of fixed potentials, so the
// summation order is that of the table, not of the call.
constexpr int PREP_OFF_MAX = 4097;
constexpr int PREP_MAX_BLOCK = 1024;
constexpr int PREP_FREE_BLOCK = 256;  // the free table's prologue blocks

// Threads of a per-image block for nfix fixed potentials.
__host__ __device__ inline int prep_threads(int nfix) {
    const int w = ((nfix > 1 ? nfix : 1) + 63) / 64;
    return 64 * (w < PREP_MAX_BLOCK / 64 ? w : PREP_MAX_BLOCK / 64);
}

// One fixed potential's deflection at a constraint (each lane its own
// potential): the usual kind through the full-range form, which these points
// near the mass need in most waves, the others through the general form.
__device__ __forceinline__ void prep_eval_f64(const ConstD c, double x, double y, double acc[5],
                                              const Series &S) {
    const int kind = kind_bits(c[D_KIND]);
    if ((kind & (K_CUT | K_ELL | K_SING)) == (K_CUT | K_ELL)) {
        double pa[1][5] = {{acc[0], acc[1], 0.0, 0.0, 0.0}};
        grad_cut_ell_full<1>(c, &x, &y, pa, S);
        acc[0] = pa[0][0];
        acc[1] = pa[0][1];
    } else {
        eval_pot_f64<true, false, false>(c, x, y, acc, S);
    }
}

// INLINE: the fixed potentials' derived constants are not read from a table
// but formed by each thread from the amplitude table (the table prologue's
// arithmetic, into registers), so no prologue launch of the fixed table
// precedes this one; blocks beyond the images then run the free table's
// prologue, which the per-sample kernel reads.  One launch instead of two.
template <int PREC, bool INLINE = false>
__global__ void __launch_bounds__(PREP_MAX_BLOCK) chi2_prep_kernel(Chi2SrcLaunch a) {
    __shared__ int s_off[PREP_OFF_MAX];
    __shared__ double s_red[2][PREP_MAX_BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthr = blockDim.x;
    const int t = blockIdx.x;
    if (INLINE && t >= a.nimg) {
        // PREP_FREE_BLOCK potentials per block (the threads beyond idle)
        const int k = (t - a.nimg) * PREP_FREE_BLOCK + tid;
        if (tid >= PREP_FREE_BLOCK) return;
        if (k < a.freet.n) {
            const PotSoA &F = a.free_amp;
            prologue_values<PREC != 0, false>(F.x0[k], F.y0[k], F.b0[k], F.eps[k], F.phi[k],
                                              F.rcore[k], F.rcut[k],
                            k, const_cast<double *>(a.freet.d), const_cast<float *>(a.freet.f),
                            a.freet.stride, a.status);
        }
        return;  // uniform per block
    }
    const bool staged = a.nsys + 1 <= PREP_OFF_MAX;
    if (staged)
        for (int i = tid; i <= a.nsys; i += nthr) s_off[i] = a.img_off[i];
    // Wave 0 loads, while the potentials are evaluated, what the block's last
    // step needs: the image's sigma and, lane l, system l's first image and
    // Dls/Ds (with at most 64 systems the image's system is then one ballot,
    // not a bisection and a load after the reduction).
    const bool wide = a.nsys > 64;
    int o_lo = 0;
    double f_l = 0.0, sg = 1.0;
    if (wave == 0) {
        const int l = min(lane, max(a.nsys - 1, 0));
        if (!wide) {
            o_lo = a.img_off[l];
            f_l = a.f[l];
        }
        sg = a.sig[t];
    }
    double acc[5] = {0, 0, 0, 0, 0};
    const double x = a.x[t], y = a.y[t];
    const int st = a.fixedt.stride;
    const int nfix = INLINE ? a.nfixed : a.fixedt.n;
    // the image role's threads (the launch may have more, for the free blocks)
    const int nimt = prep_threads(nfix);
    for (int k = tid; k < nfix && tid < nimt; k += nimt) {
        if (INLINE) {
            double v[NDER];
            float vf[NDERF];
            const PotSoA &T = a.fixed_amp;
            prologue_values<PREC != 0, false>(T.x0[k], T.y0[k], T.b0[k], T.eps[k], T.phi[k],
                                              T.rcore[k],
                                       T.rcut[k], 0, v, vf, 1, a.status);
            if (PREC == 0) {
                prep_eval_f64(ConstD{v, 1}, x, y, acc, a.S);
            } else {
                float o[5];
                eval_pot_f32<true, false, false>(ConstD{v, 1}, ConstF{vf, 1}, x, y, o, a.S);
                acc[0] += (double)o[0];
                acc[1] += (double)o[1];
            }
        } else if (PREC == 0) {
            prep_eval_f64(ConstD{a.fixedt.d + k, st}, x, y, acc, a.S);
        } else {
            float o[5];
            eval_pot_f32<true, false, false>(ConstD{a.fixedt.d + k, st},
                                             ConstF{a.fixedt.f + k, st}, x, y, o, a.S);
            acc[0] += (double)o[0];
            acc[1] += (double)o[1];
        }
    }
    // the image's system: the last one whose first image is at most t (the
    // bisection's answer for ordered offsets)
    double f_t = 0.0;
    if (wave == 0 && !wide) {
        const unsigned long long hit = __ballot(lane < a.nsys && o_lo <= t);
        f_t = __shfl(f_l, hit ? 63 - __clzll(hit) : 0, 64);
    }
    double ax = acc[0], ay = acc[1];
    wave_sum2(ax, ay);
    if (lane == 0) {
        s_red[0][wave] = ax;
        s_red[1][wave] = ay;
    }
    __syncthreads();
    if (tid == 0) {
        double sx = s_red[0][0], sy = s_red[1][0];
        for (int w = 1; w < nimt / 64; ++w) {
            sx += s_red[0][w];
            sy += s_red[1][w];
        }
        if (wide) f_t = a.f[system_of(staged ? s_off : a.img_off, a.nsys, t)];
        a.rec[t] = sx;
        a.rec[(size_t)a.nimg_pad + t] = sy;
        a.rec[2 * (size_t)a.nimg_pad + t] = f_t;
        a.rec[3 * (size_t)a.nimg_pad + t] = 1.0 / (sg * sg);
    }
}

// One wave per sample.  Lane l owns images l, l+64, ... in groups of
// SRC_IPL slots; the sample's free potentials are staged through LDS in
// chunks and each staged potential is evaluated for all of the lane's slots
// (the same potential order for every image).  Unlensed positions go to LDS,
// then lanes take one system each; the per-lane sums are combined by a
// shuffle reduction in a fixed order, so a sample's chi^2 does not depend on
// the batch it is evaluated in, on the path or on the launch shape.
constexpr int SRC_IPL = 4;
// Potentials staged in LDS at a time (at most), and the loads per lane that
// stage them.
constexpr int SRC_CHUNK_MAX = 8;
constexpr int SRC_STAGE_LOADS = (SRC_CHUNK_MAX * NDER + 63) / 64;
// Staged per-image constants and image offsets: at most this many per thread
// of a one-wave block (the staging is used only when nimg and nsys + 1 fit).
constexpr int SRC_SIG_LOADS = 4;
// Waves (samples at a time) per block of the per-sample kernel, at most.
constexpr int SRC_MAX_WPB = 4;
// LDS of the block-shared region (six per-image rows and the image offsets,
// in doubles) and of one wave's region (unlensed x, y and a chunk of staged
// potentials).
__host__ __device__ inline size_t src_shared_doubles(int nimg, int nsys) {
    return 6 * (size_t)nimg + ((size_t)nsys + 2) / 2;
}
__host__ __device__ inline size_t src_wave_doubles(int nimg, int chunk, int prec) {
    return 2 * (size_t)nimg + (size_t)chunk * NDER + (prec ? ((size_t)chunk * NDERF + 1) / 2 : 0);
}
// The launch's arguments read through an opaque pointer into the kernel
// argument segment (the kernel's one argument sits at its start).  Each section
// of the per-sample kernel takes a fresh one, so that the fields it needs are
// reloaded there by scalar loads instead of held from the kernel's entry: held
// across the potential loop they did not fit the scalar registers beside the
// loop's own and were parked in vector-register lanes (v_writelane and
// v_readlane, vector instructions) and spilled.
typedef const __attribute__((address_space(4))) Chi2SrcLaunch *ArgsPtr;
__device__ __forceinline__ ArgsPtr launch_args() {
    ArgsPtr p = (ArgsPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}

// The block-shared region: thread tid stages entries tid, tid + nthr, ...
// (N of them cover the at most 64 SRC_SIG_LOADS entries staging admits), all
// its loads issued before its LDS writes.
template <int N>
__device__ __forceinline__ void src_stage_images(ArgsPtr A, double *shw, int tid, int nthr) {
    const auto &a = *A;
    const size_t pad = a.nimg_pad;
    int *offw = reinterpret_cast<int *>(shw + 6 * (size_t)a.nimg);
    const int tmax = max(a.nimg - 1, 0);
    int sto[N];
#pragma unroll
    for (int i = 0; i < N; ++i) sto[i] = a.img_off[min(tid + nthr * i, a.nsys)];
    if (a.nimg > 0) {
        double v[N][6];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int t = min(tid + nthr * i, tmax);
            v[i][0] = a.x[t];
            v[i][1] = a.y[t];
            v[i][2] = a.rec[t];
            v[i][3] = a.rec[pad + t];
            v[i][4] = a.rec[3 * pad + t];
            v[i][5] = a.rec[2 * pad + t];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int t = tid + nthr * i;
            if (t < a.nimg) {
#pragma unroll
                for (int r = 0; r < 6; ++r) shw[(size_t)r * a.nimg + t] = v[i][r];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int t = tid + nthr * i;
        if (t <= a.nsys) offw[t] = min(max(sto[i], 0), a.nimg);
    }
}

// Orders one wave's LDS writes before its later reads by other lanes (the
// per-wave regions need no block barrier, and the waves of a block may run
// different numbers of samples and chunks).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The sampler's walker: physical parameters of its potential k (the proposal
// theta + step (2u - 1) when `in`, else the current state; the same rounded
// operations as the acceptance's copy) -> amplitude form (sigma [km/s] -> b0
// [arcsec] = K pi (sigma/c)^2 rad, e -> eps = e/(1 + sqrt(1 - e^2)), as the
// table conversion) -> derived constants at dst (stride 1, FP64 only).
__device__ __forceinline__ void mcmc_derive(const double *step, double bK, int *status,
                                            const double *th, const double *uw, bool in, int k,
                                            double *dst) {
    // (all 21 loads issued before the first use: one memory latency, not seven)
    double t[7], s[7], u[7], q[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int i = 7 * k + j;
        t[j] = th[i];
        s[j] = step[i];
        u[j] = uw[i];
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) q[j] = in ? t[j] + s[j] * (2.0 * u[j] - 1.0) : t[j];
    const double c_kms = 299792.458;
    const double arcsec_per_rad = 648000.0 / M_PI;
    const double v = q[2] / c_kms;
    const double b0 = bK * M_PI * v * v * arcsec_per_rad;
    const double eps = q[3] / (1.0 + sqrt(1.0 - q[3] * q[3]));
    prologue_values<false, false>(q[0], q[1], b0, eps, q[4], q[5], q[6], 0, dst, nullptr, 1,
                                  status);
}

// MCMC: the sampler form.  Walker m's free potentials are derived by the wave
// itself (lanes over the staged potentials), and after the chi^2 the wave
// takes the Metropolis decision: accept iff the proposal is inside the prior
// box and (chi2' <= chi2 or -2 ln u_last > chi2' - chi2), copying the
// proposal into the walker's parameters.
// At least four waves per SIMD, so that a 4096-sample batch is one round of
// waves.  The sampler form takes one walker per wave and has no sample loop
// (with one, the constants of the walker's logarithm and prologue were held
// in registers across it: 158 VGPRs, 134 without); with the arguments
// reloaded per section it fits four waves too (twelve bytes of scratch per
// lane outside the potential loop; 4096-walker step 37.3 -> 35.0 us in a
// same-box comparison, three waves 36.5).
// DERIVE: the sample's free constants formed by the wave from the amplitude
// table (a.derive_free), a variant of its own so that the usual batch keeps
// its register allocation.
template <int PREC, bool MCMC = false, bool DERIVE = false>
__global__ void __launch_bounds__(64 * SRC_MAX_WPB, ((DERIVE && PREC != 0) ? 3 : 4))
    chi2_src_kernel(Chi2SrcLaunch a) {
    // A block holds blockDim.x / 64 waves, each on its own samples.  LDS: when
    // the catalogue is small enough (stage_sig), a region the block's waves
    // share, staged once: each image's x, y, fixed deflection x, y, 1/sigma^2
    // and Dls/Ds [6][nimg] and the nsys + 1 image offsets; then per wave
    // [2][nimg] unlensed x, y and the staged potentials (FP64, then FP32).
    extern __shared__ double sh[];
    const ArgsPtr A0 = launch_args();
    // (the wave index is uniform across the wave: in a scalar register, the
    // per-wave LDS region's base is too)
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const size_t shared_d = A0->stage_sig ? src_shared_doubles(A0->nimg, A0->nsys) : 0;
    const double *ix = sh, *iy = sh + A0->nimg, *ir0 = sh + 2 * (size_t)A0->nimg,
                 *ir1 = sh + 3 * (size_t)A0->nimg;
    const double *sw = sh + 4 * (size_t)A0->nimg, *sf = sh + 5 * (size_t)A0->nimg;
    const int *soff = reinterpret_cast<const int *>(sh + 6 * (size_t)A0->nimg);
    double *own = sh + shared_d + (size_t)wv * src_wave_doubles(A0->nimg, A0->chunk, PREC);
    double *sx = own, *sy = own + A0->nimg;
    double *pd = own + 2 * (size_t)A0->nimg;
    float *pf = reinterpret_cast<float *>(pd + (size_t)A0->chunk * NDER);
    const int pad = A0->nimg_pad, st = A0->freet.stride, nf = A0->freet.n;
    // The first sample's range of free potentials (each next one is fetched
    // during the current sample's reduction; DERIVE, whose registers are
    // fuller, reads it at the top of the sample).
    const int mstride = gridDim.x * nw;
    int m = A0->sample0 + blockIdx.x * nw + wv;
    int fo0 = 0, fo1 = 0;
    if (!MCMC && !DERIVE && m < A0->n_samples) {
        fo0 = A0->free_off[m];
        fo1 = A0->free_off[m + 1];
    }
    // What does not depend on the sample is staged once per block, by all its
    // threads, before one block barrier: then the waves read it from LDS, not
    // each from L2 (the same few cache lines read by every wave at once had
    // their L2 channels serialise the requests), and the reduction reads LDS
    // only.  Every load of a thread is issued, unconditionally (indices
    // clamped into the arrays), before its first LDS write.
    if (A0->stage_sig) {
        if (nthr >= 256)
            src_stage_images<1>(A0, sh, tid, nthr);
        else if (nthr >= 128)
            src_stage_images<2>(A0, sh, tid, nthr);
        else
            src_stage_images<4>(A0, sh, tid, nthr);
    }
    __syncthreads();  // (the only block barrier: below, each wave on its own)
    for (; m < a.n_samples; m += mstride) {
        const ArgsPtr A1 = launch_args();
        int k0 = 0, k1 = 0;
        bool in = false;
        const int P = 7 * A1->mc.nfree;
        const double *th = nullptr, *uw = nullptr;
        if (MCMC) {
            th = A1->mc.params + (size_t)m * P;
            uw = A1->mc.u + (size_t)m * (P + 1);
            k0 = 0;
            k1 = A1->mc.nfree;
            if (A1->mc.mode == 2) {
                int out = 0;
                for (int i = lane; i < P; i += 64) {
                    const double v = th[i] + A1->mc.step[i] * (2.0 * uw[i] - 1.0);
                    if (!(v >= A1->mc.lo[i] && v <= A1->mc.hi[i])) out = 1;
                }
                in = __ballot(out) == 0;
            }
        } else {
            if (DERIVE) {
                fo0 = A1->free_off[m];
                fo1 = A1->free_off[m + 1];
            }
            k0 = __builtin_amdgcn_readfirstlane(min(max(fo0, 0), nf));
            k1 = __builtin_amdgcn_readfirstlane(min(max(fo1, k0), nf));
        }
        for (int g0 = 0; g0 < A1->nimg; g0 += 64 * SRC_IPL) {
            // (lanes past the last image load its data, unconditionally so
            // that the loads need no wait between them, and store nothing)
            double x[SRC_IPL], y[SRC_IPL], acc[SRC_IPL][5];
#pragma unroll
            for (int j = 0; j < SRC_IPL; ++j) {
                const int t = min(g0 + j * 64 + lane, A1->nimg - 1);
                if (A1->stage_sig) {
                    x[j] = ix[t];
                    y[j] = iy[t];
                    acc[j][0] = ir0[t];
                    acc[j][1] = ir1[t];
                } else {
                    x[j] = A1->x[t];
                    y[j] = A1->y[t];
                    acc[j][0] = A1->rec[t];
                    acc[j][1] = A1->rec[pad + t];
                }
                acc[j][2] = acc[j][3] = acc[j][4] = 0.0;
            }

            for (int kc = k0; kc < k1; kc += a.chunk) {
                const ArgsPtr A2 = launch_args();
                const int cnt = min(A2->chunk, k1 - kc);
                wave_lds_sync();
                if (MCMC) {
                    if (lane < cnt)
                        mcmc_derive(A2->mc.step, A2->mc.bK, A2->mc.status, th, uw, in, kc + lane,
                                    pd + lane * NDER);
                } else if (DERIVE) {
                    // the free potentials' derived constants formed here from
                    // the amplitude table (lane per potential) instead of read
                    // from a table a prologue launch wrote
                    if (lane < cnt) {
                        const int k = kc + lane;
                        prologue_values<PREC != 0, false>(
                            A2->free_amp.x0[k], A2->free_amp.y0[k], A2->free_amp.b0[k],
                            A2->free_amp.eps[k], A2->free_amp.phi[k], A2->free_amp.rcore[k],
                            A2->free_amp.rcut[k], 0, pd + lane * NDER, pf + lane * NDERF, 1,
                            A2->status);
                    }
                } else {
                    // every lane's loads in flight at once, then the stores
                    // (LDS entry e = potential e / NDER, constant e % NDER).
                    // The lane index passes through an empty asm so that the
                    // index arithmetic is formed here: hoisted out of the
                    // sample loop it would hold registers for the whole kernel.
                    int l0 = lane;
                    asm volatile("" : "+v"(l0));
                    double v[SRC_STAGE_LOADS];
#pragma unroll
                    for (int i = 0; i < SRC_STAGE_LOADS; ++i) {
                        const int e = l0 + 64 * i;
                        const int kk = e / NDER, ci = e - kk * NDER;
                        v[i] = kk < cnt ? A2->freet.d[(size_t)ci * st + kc + kk] : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < SRC_STAGE_LOADS; ++i) {
                        const int e = l0 + 64 * i;
                        if (e < cnt * NDER) pd[e] = v[i];
                    }
                }
                if (PREC != 0 && !MCMC && !DERIVE) {
                    for (int e = lane; e < cnt * NDERF; e += 64) {
                        const int ci = e / cnt, kk = e - ci * cnt;
                        pf[kk * NDERF + ci] = A2->freet.f[(size_t)ci * st + kc + kk];
                    }
                }
                wave_lds_sync();
                for (int kk = 0; kk < cnt; ++kk) {
                    const ConstD cd{pd + kk * NDER, 1};
                    if (PREC == 0) {
                        // the usual kind (two cores, elliptical, rcore > 0):
                        // full-range evaluation, slots in interleaved pairs
                        const int kind = uniform_kind(cd[D_KIND]);
                        if ((kind & (K_CUT | K_ELL | K_SING)) == (K_CUT | K_ELL)) {
#pragma unroll
                            for (int j = 0; j < SRC_IPL; j += 2) {
                                if (g0 + j * 64 >= A2->nimg) break;  // uniform
                                grad_cut_ell_full<2>(cd, x + j, y + j, acc + j, a.S);
                            }
                            continue;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < SRC_IPL; ++j) {
                        if (g0 + j * 64 >= A2->nimg) break;  // uniform: no image in this slot
                        if (PREC == 0) {
                            eval_pot_f64<true, false>(cd, x[j], y[j], acc[j], a.S);
                        } else {
                            float o[5];
                            eval_pot_f32<true, false>(cd, ConstF{pf + kk * NDERF, 1}, x[j], y[j],
                                                      o, a.S);
                            acc[j][0] += (double)o[0];
                            acc[j][1] += (double)o[1];
                        }
                    }
                }
            }
            const ArgsPtr A3 = launch_args();
            if (A3->stage_sig) {
#pragma unroll
                for (int j = 0; j < SRC_IPL; ++j) {
                    const int t = g0 + j * 64 + lane;
                    if (t < A3->nimg) {
                        const double f = sf[t];
                        sx[t] = x[j] - f * acc[j][0];
                        sy[t] = y[j] - f * acc[j][1];
                    }
                }
            } else {
                double f[SRC_IPL];
#pragma unroll
                for (int j = 0; j < SRC_IPL; ++j) {
                    const int t = g0 + j * 64 + lane;
                    f[j] = t < A3->nimg ? A3->rec[2 * (size_t)pad + t] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < SRC_IPL; ++j) {
                    const int t = g0 + j * 64 + lane;
                    if (t < A3->nimg) {
                        sx[t] = x[j] - f[j] * acc[j][0];
                        sy[t] = y[j] - f[j] * acc[j][1];
                    }
                }
            }
        }
        const ArgsPtr A4 = launch_args();
        if (!MCMC && !DERIVE && A4->persistent && m + mstride < A4->n_samples) {
            fo0 = A4->free_off[m + mstride];
            fo1 = A4->free_off[m + mstride + 1];
        }
        wave_lds_sync();
        double part = 0.0;
        for (int i = lane; i < A4->nsys; i += 64) {
            int o0, o1;
            if (A4->stage_sig) {
                o0 = soff[i];
                o1 = max(soff[i + 1], o0);
            } else {
                o0 = min(max(A4->img_off[i], 0), A4->nimg);
                o1 = min(max(A4->img_off[i + 1], o0), A4->nimg);
            }
            const int M = o1 - o0;
            double mx = 0.0, my = 0.0;
            for (int t = o0; t < o1; ++t) {
                mx += sx[t];
                my += sy[t];
            }
            if (M > 0) {
                const double im = 1.0 / M;
                mx *= im;
                my *= im;
            }
            double s = 0.0;
            if (A4->stage_sig) {
                for (int t = o0; t < o1; ++t) {
                    const double ex = sx[t] - mx, ey = sy[t] - my;
                    s = fma(ex * ex + ey * ey, sw[t], s);
                }
            } else {
                for (int t = o0; t < o1; ++t) {
                    const double ex = sx[t] - mx, ey = sy[t] - my;
                    s = fma(ex * ex + ey * ey, A4->rec[3 * (size_t)pad + t], s);
                }
            }
            part += s;
            if (A4->src_x) {
                A4->src_x[(size_t)m * A4->nsys + i] = mx;
                A4->src_y[(size_t)m * A4->nsys + i] = my;
            }
        }
        part = wave_sum(part);
        if (MCMC) {
            // the shuffle tree leaves the total in lane 0: every lane takes
            // the decision on lane 0's value
            part = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(part)),
                                    __builtin_amdgcn_readfirstlane(__double2loint(part)));
            if (A4->mc.mode == 1) {
                if (lane == 0) A4->mc.chi2[m] = part;
            } else {
                const double d = part - A4->mc.chi2[m];
                const double ul = uw[P];
                if (in && (d <= 0.0 || -2.0 * log(ul) > d)) {
                    for (int i = lane; i < P; i += 64)
                        A4->mc.params[(size_t)m * P + i] =
                            th[i] + A4->mc.step[i] * (2.0 * uw[i] - 1.0);
                    if (lane == 0) {
                        A4->mc.chi2[m] = part;
                        A4->mc.accepted[m] += 1;
                    }
                }
            }
        } else if (lane == 0 && A4->chi2) {
            A4->chi2[m] = part;
        }
        wave_lds_sync();  // sx, sy are rewritten by the next sample
        if (MCMC || !a.persistent) break;
    }
}

// LDS of a block of nw waves of the per-sample kernel: with the staging, the
// block-shared region, then per wave the unlensed positions and a chunk of
// staged potentials.  A batch stages when that fits a budget that keeps 16
// waves on a CU (160 KiB of LDS) with a full chunk; the per-sample path (one
// block) when it fits 64 KiB.
constexpr size_t SRC_LDS_BUDGET = 10240;  // per wave
static size_t src_lds(int nimg, int nsys, int prec, int chunk, bool staged, int nw) {
    return sizeof(double) * ((staged ? src_shared_doubles(nimg, nsys) : 0) +
                             (size_t)nw * src_wave_doubles(nimg, chunk, prec));
}
static bool src_staged(int nimg, int nsys, int prec, int nw, size_t budget) {
    return nimg <= 64 * SRC_SIG_LOADS && nsys + 1 <= 64 * SRC_SIG_LOADS &&
           src_lds(nimg, nsys, prec, SRC_CHUNK_MAX, true, nw) <= budget;
}
static int src_chunk(int nimg, int prec) {
    const size_t per = NDER * sizeof(double) + (prec ? NDERF * sizeof(float) : 0);
    const size_t avail = 65536 - 2 * (size_t)nimg * sizeof(double);
    return (int)std::max<size_t>(1, std::min<size_t>(SRC_CHUNK_MAX, avail / per));
}

hipError_t launch_chi2_prep(const Chi2SrcLaunch &c0, hipStream_t st) {
    Chi2SrcLaunch c = c0;
    c.S = make_series();
    if (c.inline_fixed) {
        const long long free_blocks =
            c.free_prologue ? ((long long)c.freet.n + PREP_FREE_BLOCK - 1) / PREP_FREE_BLOCK : 0;
        const long long blocks = (long long)std::max(c.nimg, 0) + free_blocks;
        if (blocks == 0) return hipSuccess;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        if (!c.free_prologue) c.freet.n = 0;
        // at least PREP_FREE_BLOCK threads, for the free table's blocks
        const int nt = std::max(prep_threads(c.nfixed), free_blocks ? PREP_FREE_BLOCK : 64);
        if (c.prec == 0)
            hipLaunchKernelGGL((chi2_prep_kernel<0, true>), dim3((unsigned)blocks), dim3(nt), 0, st,
                               c);
        else
            hipLaunchKernelGGL((chi2_prep_kernel<1, true>), dim3((unsigned)blocks), dim3(nt), 0, st,
                               c);
        return hipGetLastError();
    }
    if (c0.nimg <= 0) return hipSuccess;
    const int nt = prep_threads(c.fixedt.n);
    if (c.prec == 0)
        hipLaunchKernelGGL(chi2_prep_kernel<0>, dim3(c.nimg), dim3(nt), 0, st, c);
    else
        hipLaunchKernelGGL(chi2_prep_kernel<1>, dim3(c.nimg), dim3(nt), 0, st, c);
    return hipGetLastError();
}

// Waves per block, staging and chunk of a launch of the per-sample kernel
// (c.grid_blocks waves): a batch takes blocks of SRC_MAX_WPB waves (else 2,
// else 1) that share the staged catalogue; the per-sample path one wave.
static int src_shape(Chi2SrcLaunch &c, int prec) {
    int nw = 1;
    bool staged = false;
    if (c.persistent && c.grid_blocks > 1) {
        for (int w = SRC_MAX_WPB; w >= 1 && !staged; w /= 2)
            if (src_staged(c.nimg, c.nsys, prec, w, SRC_LDS_BUDGET * w)) {
                nw = w;
                staged = true;
            }
    } else {
        staged = src_staged(c.nimg, c.nsys, prec, 1, 65536);
    }
    c.stage_sig = staged ? 1 : 0;
    c.chunk = staged ? SRC_CHUNK_MAX : src_chunk(c.nimg, prec);
    return nw;
}

hipError_t launch_chi2_src(const Chi2SrcLaunch &c0, hipStream_t st) {
    Chi2SrcLaunch c = c0;
    c.S = make_series();
    const int nw = src_shape(c, c.prec);
    const size_t shmem = src_lds(c.nimg, c.nsys, c.prec, c.chunk, c.stage_sig, nw);
    if (shmem > 65536) return hipErrorInvalidValue;
    const dim3 grid((c.grid_blocks + nw - 1) / nw), block(64 * nw);
    if (c.prec == 0 && c.derive_free)
        hipLaunchKernelGGL((chi2_src_kernel<0, false, true>), grid, block, shmem, st, c);
    else if (c.prec == 0)
        hipLaunchKernelGGL((chi2_src_kernel<0>), grid, block, shmem, st, c);
    else if (c.derive_free)
        hipLaunchKernelGGL((chi2_src_kernel<1, false, true>), grid, block, shmem, st, c);
    else
        hipLaunchKernelGGL((chi2_src_kernel<1>), grid, block, shmem, st, c);
    return hipGetLastError();
}

hipError_t launch_mcmc_chi2(const Chi2SrcLaunch &c0, hipStream_t st) {
    Chi2SrcLaunch c = c0;
    if (c.mc.mode != 1 && c.mc.mode != 2) return hipErrorInvalidValue;
    if (c.n_samples <= 0) return hipSuccess;
    c.S = make_series();
    c.prec = 0;
    // one walker per wave (a kernel without a sample loop keeps the constants
    // of the walker's own arithmetic out of the registers of the potential loop)
    c.grid_blocks = c.n_samples;
    const int nw = src_shape(c, 0);
    const size_t shmem = src_lds(c.nimg, c.nsys, 0, c.chunk, c.stage_sig, nw);
    if (shmem > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL((chi2_src_kernel<0, true>), dim3((c.grid_blocks + nw - 1) / nw),
                       dim3(64 * nw), shmem, st, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vertex deflection (Dls/Ds = 1) of samples m0 .. m0+nsamp-1: the fixed part
// (given) plus the sample's free potentials in index order.  A block covers
// 256 vertices of AG_SPB consecutive samples, whose free potentials are
// contiguous in the table: they are staged in LDS (chunks of AG_CHUNK, read by
// broadcast) once for the group, and each vertex's fixed deflection is read
// once for the group.  Walking the staged potentials in order, a thread
// finishes a sample when the next potential belongs to a later one (the
// boundaries are uniform), so every sample sums fixed then free in index
// order, as the one-sample-per-block form did.
constexpr int AG_CHUNK = 32;
constexpr int AG_SPB = 4;

template <int PREC>
__global__ void __launch_bounds__(256, 6) alpha_grid_kernel(AlphaGridLaunch a) {
    __shared__ double pd[AG_CHUNK * NDER];
    __shared__ float pf[AG_CHUNK * NDERF];
    const size_t nv = (size_t)a.grid.nx * a.grid.ny;
    const int tid = threadIdx.x;
    const size_t v = (size_t)blockIdx.x * 256 + tid;
    const int s0 = blockIdx.y * AG_SPB;
    const int ns = min(AG_SPB, a.nsamp - s0);
    const int nf = a.freet.n, st = a.freet.stride;
    const int i = (int)(v % a.grid.nx), j = (int)(v / a.grid.nx);
    const double x = grid_coord(a.grid.x0, i, a.grid.dx);
    const double y = grid_coord(a.grid.y0, j, a.grid.dy);
    double fx = 0.0, fy = 0.0;
    if (a.afix_x && v < nv) {
        fx = a.afix_x[v];
        fy = a.afix_y[v];
    }
    // sample s of the group owns potentials [kb, ke) (offsets clamped to the
    // table and made non-decreasing)
    const int *off = a.free_off + a.m0 + s0;
    const int K0 = min(max(off[0], 0), nf);
    int kb = K0;
    int K1 = K0;
    for (int q = 1; q <= ns; ++q) K1 = min(max(off[q], K1), nf);
    int s = 0;
    int ke = min(max(off[1], kb), nf);
    double acc[5] = {fx, fy, 0, 0, 0};
    // the polynomials' leading coefficients in vector registers (each first
    // Horner step reads two coefficients; one may come from a scalar register)
    Series S = a.S;
    if (PREC == 0) {
        S.at[0] = vgpr_f64(a.S.at[0]);
        S.ah[0] = vgpr_f64(a.S.ah[0]);
    }
    auto finish = [&]() {
        if (v < nv) {
            a.out[(size_t)(s0 + s) * 2 * nv + v] = acc[0];
            a.out[(size_t)(s0 + s) * 2 * nv + nv + v] = acc[1];
        }
        acc[0] = fx;
        acc[1] = fy;
        ++s;
        kb = ke;
        if (s < ns) ke = min(max(off[s + 1], kb), nf);
    };
    // staging: wave w copies the constants w, w + 4, ... of the chunk's
    // potentials, its lanes consecutive potentials (AG_CHUNK <= 64)
    static_assert(AG_CHUNK <= 64, "a chunk's potentials fit one wave's lanes");
    const int lane = tid & 63, wv = tid >> 6;
    for (int kc = K0; kc < K1; kc += AG_CHUNK) {
        const int cnt = min(AG_CHUNK, K1 - kc);
        __syncthreads();
        if (lane < cnt) {
            for (int ci = wv; ci < NDER; ci += 4)
                pd[lane * NDER + ci] = a.freet.d[(size_t)ci * st + kc + lane];
            if (PREC != 0)
                for (int ci = wv; ci < NDERF; ci += 4)
                    pf[lane * NDERF + ci] = a.freet.f[(size_t)ci * st + kc + lane];
        }
        __syncthreads();
        // the chunk's kinds in scalar registers, and its entries addressed
        // from one vector register
        const KindMasks km = kind_masks(lane < cnt ? kind_bits(pd[lane * NDER + D_KIND]) : 0);
        const double *row = lds_entry(pd, 0);
        for (int kk = 0; kk < cnt; ++kk) {
            while (s < ns && kc + kk >= ke) finish();
            if (PREC == 0) {
                eval_pot_f64_kind<true, false>(ConstD{row + kk * NDER, 1}, km.kind(kk), x, y, acc,
                                               S);
            } else {
                float o[5];
                eval_pot_f32_kind<true, false>(ConstD{row + kk * NDER, 1},
                                               ConstF{pf + kk * NDERF, 1}, km.kind(kk), x, y, o,
                                               a.S);
                acc[0] += (double)o[0];
                acc[1] += (double)o[1];
            }
        }
    }
    while (s < ns) finish();
}

hipError_t launch_alpha_grid(const AlphaGridLaunch &L0, hipStream_t st) {
    AlphaGridLaunch L = L0;
    L.S = make_series();
    const size_t nv = (size_t)L.grid.nx * L.grid.ny;
    if (nv == 0 || L.nsamp <= 0) return hipSuccess;
    dim3 grid((unsigned)((nv + 255) / 256), (unsigned)((L.nsamp + AG_SPB - 1) / AG_SPB));
    if (grid.y > 65535u) return hipErrorInvalidConfiguration;
    if (L.prec == 0)
        hipLaunchKernelGGL(alpha_grid_kernel<0>, grid, dim3(256), 0, st, L);
    else
        hipLaunchKernelGGL(alpha_grid_kernel<1>, grid, dim3(256), 0, st, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Newton refinement of found images (the refinement of a found image, Sec.
// 2.3, done by Newton's method on the lens equation of Sec. 2.1, Eq. (1),
// with the analytic second derivatives of Sec. 2.4):
//   r = beta - (theta - f alpha(theta)),  A = I - f H(theta),
//   theta <- theta + A^-1 r  until |step| < tol;
// an image whose iterate leaves the box |theta - theta0| <= max_shift or
// does not converge within max_iter keeps its grid estimate.
//
// Design: a block of RF_WAVES waves takes 64 images of one sample (lane l of
// every wave holds image l); the potentials (fixed then the sample's free
// ones) are staged in LDS in chunks and wave w evaluates every RF_WAVES-th of
// them, so one image's 300-odd potentials are spread over the block.  The
// wave partial sums are combined in wave order by every wave, which then
// takes the same Newton step.
constexpr int RF_WAVES = 8;
constexpr int RF_THREADS = 64 * RF_WAVES;
constexpr int RF_CHUNK = 64;

__global__ void __launch_bounds__(RF_THREADS) refine_images_kernel(RefineLaunch a) {
    __shared__ double pd[RF_CHUNK * NDER];
    __shared__ double red[RF_WAVES][5][64];
    __shared__ int s_pre[RF_THREADS + 1];
    __shared__ int s_sys[64], s_k[64];
    __shared__ int s_total;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s = blockIdx.x, g = blockIdx.y, m = a.m0 + s;
    // locate image t = 64 g + lane of this sample: scan the systems' stored
    // counts in windows of RF_THREADS systems
    if (tid < 64) s_sys[tid] = -1;
    int base = 0;
    for (int sys0 = 0; sys0 < a.nsys; sys0 += RF_THREADS) {
        const int i = sys0 + tid;
        const int n = i < a.nsys ? min(max(a.count[(size_t)s * a.nsys + i], 0), a.kmax) : 0;
        __syncthreads();
        if (tid == 0) s_pre[0] = 0;
        s_pre[tid + 1] = n;
        __syncthreads();
        for (int d = 1; d < RF_THREADS; d <<= 1) {
            const int v = tid >= d ? s_pre[tid + 1 - d] : 0;
            __syncthreads();
            s_pre[tid + 1] += v;
            __syncthreads();
        }
        const int wtot = s_pre[RF_THREADS];
        if (tid < 64) {
            const int t = g * 64 + tid - base;
            if (t >= 0 && t < wtot) {
                int lo = 0, hi = RF_THREADS;  // largest c with s_pre[c] <= t
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= t)
                        lo = mid;
                    else
                        hi = mid;
                }
                s_sys[tid] = sys0 + lo;
                s_k[tid] = t - s_pre[lo];
            }
        }
        base += wtot;
    }
    if (tid == 0) s_total = base;
    __syncthreads();
    if (g * 64 >= s_total) return;  // whole block: no image here
    const int sys = s_sys[lane];
    const bool act = sys >= 0;
    size_t slot = 0;
    double x = 0.0, y = 0.0, f = 1.0, bx = 0.0, by = 0.0;
    if (act) {
        slot = ((size_t)s * a.nsys + sys) * a.kmax + s_k[lane];
        x = a.ix[slot];
        y = a.iy[slot];
        f = a.f[sys];
        bx = a.sx[(size_t)s * a.nsys + sys];
        by = a.sy[(size_t)s * a.nsys + sys];
    }
    const double x0 = x, y0 = y, tol2 = a.tol * a.tol;
    int state = act ? 0 : 1;  // 0 iterating, 1 converged (or no image), -1 failed
    const int nfix = a.fixedt.n, nf = a.freet.n;
    const int k0 = min(max(a.free_off[m], 0), nf), k1 = min(max(a.free_off[m + 1], k0), nf);
    for (int it = 0; it < a.max_iter; ++it) {
        double acc[5] = {0, 0, 0, 0, 0};
        for (int pass = 0; pass < 2; ++pass) {
            const Derived T = pass == 0 ? a.fixedt : a.freet;
            const int lo_k = pass == 0 ? 0 : k0, hi_k = pass == 0 ? nfix : k1;
            for (int kc = lo_k; kc < hi_k; kc += RF_CHUNK) {
                const int cnt = min(RF_CHUNK, hi_k - kc);
                __syncthreads();
                for (int e = tid; e < cnt * NDER; e += RF_THREADS) {
                    const int ci = e / cnt, kk = e - ci * cnt;
                    pd[kk * NDER + ci] = T.d[(size_t)ci * T.stride + kc + kk];
                }
                __syncthreads();
                for (int kk = wave; kk < cnt; kk += RF_WAVES)
                    eval_pot_f64<true, true>(ConstD{pd + kk * NDER, 1}, x, y, acc, a.S);
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) red[wave][c][lane] = acc[c];
        __syncthreads();
        double h[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            double v = red[0][c][lane];
            for (int w = 1; w < RF_WAVES; ++w) v += red[w][c][lane];
            h[c] = v;
        }
        hess_of_parts(h[2], h[3], h[4], &h[2]);
        if (state == 0) {
            const double rx = bx - (x - f * h[0]);
            const double ry = by - (y - f * h[1]);
            const double a11 = 1.0 - f * h[2];
            const double a12 = -(f * h[3]);
            const double a22 = 1.0 - f * h[4];
            const double det = a11 * a22 - a12 * a12;
            const double sx = (a22 * rx - a12 * ry) / det;
            const double sy = (a11 * ry - a12 * rx) / det;
            x = x + sx;
            y = y + sy;
            if (!(fabs(x - x0) <= a.max_shift && fabs(y - y0) <= a.max_shift))
                state = -1;
            else if (sx * sx + sy * sy < tol2)
                state = 1;
        }
        if (!__syncthreads_or(state == 0)) break;
    }
    if (wave == 0 && act && state == 1) {
        a.ix[slot] = x;
        a.iy[slot] = y;
    }
}

hipError_t launch_refine_images(const RefineLaunch &L0, hipStream_t st) {
    if (L0.nsamp <= 0 || L0.max_iter <= 0 || L0.nsys <= 0) return hipSuccess;
    RefineLaunch L = L0;
    L.S = make_series();
    const long long groups = ((long long)L.nsys * L.kmax + 63) / 64;
    if (groups > 65535) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(refine_images_kernel, dim3(L.nsamp, (unsigned)groups), dim3(RF_THREADS), 0,
                       st, L);
    return hipGetLastError();
}

}  // namespace lens
