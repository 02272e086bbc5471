// The evolution kernels of libens (plain per-sample search and ENS sweeps):
// device routines, the kernels and their typed launch wrapper.  Each
// storage type's kernels are compiled in a translation unit of their own
// (search_f32.hip, search_f16.hip, search_bf16.hip).
#pragma once

#include "eval.h"

namespace ens {

// ---------------------------------------------------------------------------
// evolution

// Best member of the population occupying lanes [base, base+np): highest
// score, lowest slot on ties (section "Sorting" with P = 1).
__device__ __forceinline__ int32_t group_argmax(float S, int32_t base, int32_t np)
{
    float best = __shfl(S, base, WAVE);
    int32_t bi = 0;
    for (int32_t q = 1; q < np; ++q) {
        const float v = __shfl(S, base + q, WAVE);
        if (v > best) {
            best = v;
            bi = q;
        }
    }
    return bi;
}

// Trial vector of this lane's slot: current-to-best/1 mutant from the slot,
// the best and two other random members, binomial crossover (section
// "Mutation and crossover").  Every lane of the wave must call it.
// With an archive (JADE), lane base + a holds archive entry a in `arch`
// and r2 ranges over the np members and the n_arch entries.
template <int P, bool ARCHIVE = false>
__device__ __forceinline__ void make_trial(const float *x, float S, int32_t base, int32_t np,
                                          int32_t slot, const uint64_t w[4], float F, uint64_t cr_thr,
                                          const float *lo, const float *hi, float *u,
                                          const float *arch = nullptr, int32_t n_arch = 0)
{
    const int32_t b = group_argmax(S, base, np);
    const TrialDraw dr = trial_draw(w, slot, np, P, cr_thr, ARCHIVE ? np + n_arch : np);
    const bool from_arch = ARCHIVE && dr.r2 >= static_cast<uint32_t>(np);
    const int32_t r2_lane = base + static_cast<int32_t>(from_arch ? dr.r2 - np : dr.r2);
#pragma unroll
    for (int d = 0; d < P; ++d) {
        const float xb = __shfl(x[d], base + b, WAVE);
        const float xr1 = __shfl(x[d], base + static_cast<int32_t>(dr.r1), WAVE);
        float xr2 = __shfl(x[d], r2_lane, WAVE);
        if constexpr (ARCHIVE) {
            const float ar2 = __shfl(arch[d], r2_lane, WAVE);
            xr2 = from_arch ? ar2 : xr2;
        }
        const float v = mutant(x[d], xb, xr1, xr2, F, lo[d], hi[d]);
        u[d] = dr.take[d] ? v : x[d];
    }
}

// JADE bookkeeping after a generation's evaluation, in slot order within
// each population: every slot whose trial replaces its parent (ok) puts the
// parent into the archive (appended while it holds fewer than np entries,
// else at that slot's drawn position) and adds its F and CR to the
// population's sums; then the means move toward the successful values.
// Every lane of the wave must call it; populations are lane groups.
template <int P>
__device__ __forceinline__ void jade_update(bool ok, const float *x, int32_t k_cr, int32_t k_f, int32_t a_idx,
                                           int32_t grp, int32_t np, int32_t slot, float *arch, int32_t &n_arch,
                                           double &mu_cr, double &mu_f)
{
    uint64_t pending = __ballot(ok);
    int64_t s_cr = 0, s_f = 0, s_f2 = 0;
    int32_t n_s = 0;
    while (pending) {
        const int32_t L = __builtin_ctzll(pending);
        pending &= pending - 1;
        float xs[3];
#pragma unroll
        for (int d = 0; d < P; ++d) xs[d] = __shfl(x[d], L, WAVE);
        const int32_t kc = __shfl(k_cr, L, WAVE), kf = __shfl(k_f, L, WAVE), ai = __shfl(a_idx, L, WAVE);
        if (L / np == grp) {
            const int32_t pos = n_arch < np ? n_arch : ai;
            if (slot == pos) {
#pragma unroll
                for (int d = 0; d < P; ++d) arch[d] = xs[d];
            }
            n_arch = n_arch < np ? n_arch + 1 : np;
            n_s += 1;
            s_cr += kc;
            s_f += kf;
            s_f2 += static_cast<int64_t>(kf) * kf;
        }
    }
    if (n_s > 0) {
        const double mean_cr = static_cast<double>(s_cr) / (static_cast<double>(n_s) * JADE_GRID);
        const double lehmer_f = static_cast<double>(s_f2) / (static_cast<double>(s_f) * JADE_GRID);
        mu_cr = 0.9 * mu_cr + 0.1 * mean_cr;
        mu_f = 0.9 * mu_f + 0.1 * lehmer_f;
    }
}

template <int P>
__device__ __forceinline__ void load_clamped(const float *__restrict__ src, const float *lo,
                                             const float *hi, float *x)
{
#pragma unroll
    for (int d = 0; d < P; ++d) {
        float v = src[d];
        v = v < lo[d] ? lo[d] : v;
        v = v > hi[d] ? hi[d] : v;
        x[d] = v;
    }
}

// Semblance of each lane's candidate, the trace loop split over the
// workgroup's nsl waves (in every CMP, wave w takes the CMP's traces w,
// w + nsl, w + 2 nsl, ...);
// partial sums meet in LDS and every wave adds them in the same order.
// The LDS-staged windows of a workgroup (search_body with TILES).
struct TileCtx {
    const int2 *tab;      // the step's table of staged column ranges
    int32_t i0;           // first trace of the table
    float *stage;         // this wave's two staging buffers
    const float *zero8;
};

template <int DT, int W, bool TILES = false>
__device__ __forceinline__ float eval_slices(const StoreView &sv, const Cand<float> &cand, int32_t c_lo,
                                             int32_t c_hi, int32_t wave, int32_t nsl, int32_t lane,
                                             float *lds, int &buf, int32_t &M, const TileCtx &tc)
{
    Acc<W, float> acc;
    acc.reset();
    if constexpr (TILES)
        accumulate_cmps_tiles<W>(sv, cand, c_lo, c_hi, wave, nsl, acc, tc.tab, tc.i0, tc.stage, tc.zero8, lane);
    else
        accumulate_range<DT, W, float>(sv, cand, c_lo, c_hi, wave, nsl, acc);
    if (nsl > 1) {
        float *mine = lds + ((buf * nsl + wave) * (W + 2)) * WAVE + lane;
#pragma unroll
        for (int k = 0; k < W; ++k) mine[k * WAVE] = acc.s[k];
        mine[W * WAVE] = acc.E;
        mine[(W + 1) * WAVE] = __int_as_float(acc.M);
        __syncthreads();
        acc.reset();
        for (int32_t v = 0; v < nsl; ++v) {
            const float *r = lds + ((buf * nsl + v) * (W + 2)) * WAVE + lane;
#pragma unroll
            for (int k = 0; k < W; ++k) acc.s[k] += r[k * WAVE];
            acc.E += r[W * WAVE];
            acc.M += __float_as_int(r[(W + 1) * WAVE]);
        }
        buf ^= 1;
    }
    M = acc.M;
    return finish_semblance(acc);
}

// Evolution of a group of samples: lane = (sample, slot), floor(64/NP)
// samples of one output CMP per wave, the trace loop split over nsl waves.
// Sweep pacing.  Every workgroup of an ENS launch sweeps the same number of
// trace steps and all of them are resident together, so the launch lasts as
// long as its slowest sweep.  The wave arbiter favours older waves, which lets
// the first-dispatched sweeps race ahead and leaves the last ones to finish
// alone on a half-empty chip.  Before each step a wave compares its progress
// with the launch's mean (steps counts every finished step of every
// workgroup) and takes a high issue priority when behind, a low one when
// ahead; the results do not depend on it.
__device__ __forceinline__ void pace_by_progress(const unsigned long long *steps, int32_t done_here)
{
    const unsigned long long all = __hip_atomic_load(steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(all)));
    const int64_t mine = static_cast<int64_t>(done_here) * gridDim.x;
    const int64_t half = gridDim.x / 2;
    if (mine + half < total)
        __builtin_amdgcn_s_setprio(3);
    else if (mine > total + half)
        __builtin_amdgcn_s_setprio(0);
    else
        __builtin_amdgcn_s_setprio(1);
}

// Column range of every trace of CMPs c_lo..c_hi that a window may read for
// any candidate in the boxes of the samples t_start + m stride (m < ns) at
// output CMP j: tau^2 = (n0 + As dm)^2 + B n0 dm^2 / dt + C n0 h^2 / dt (CRS;
// CMP: n0^2 + C h^2 / dt^2) is monotone in B and C and convex in As, so the
// box's ends bound it; two columns of margin cover the kernel's binary32
// rounding.  Ranges longer than TILE_STAGE_MAX are marked for direct reads.
template <int OP, int W>
__device__ void build_tile_table(const SearchArgs &a, int2 *tab, int32_t j, int32_t c_lo, int32_t c_hi,
                                 int32_t t_start, int32_t ns, int32_t stride)
{
    const StoreView &sv = a.sv;
    const int64_t i0 = sv.cmp_ptr[c_lo], i1 = sv.cmp_ptr[c_hi + 1];
    const double inv_dt = 1.0 / static_cast<double>(sv.dt);
    for (int64_t idx = threadIdx.x; idx < i1 - i0; idx += blockDim.x) {
        const TraceMeta m = sv.meta[i0 + idx];
        const double dm = static_cast<double>(static_cast<float>(m.cmp - j) * sv.dx);
        const double h2 = static_cast<double>(m.h2);
        double qlo = 1e300, qhi = -1e300;
        for (int32_t q = 0; q < ns; ++q) {
            const int32_t n0 = t_start + q * stride;
            const double nd = static_cast<double>(n0);
            const float *lo = a.lo_tab + n0 * 3, *hi = a.hi_tab + n0 * 3;
            double mn, mx;
            if constexpr (OP == 1) {
                const double cc = inv_dt * inv_dt * h2;
                mn = nd * nd + fmin(lo[0] * cc, hi[0] * cc);
                mx = nd * nd + fmax(lo[0] * cc, hi[0] * cc);
            } else {
                const double e1 = nd + lo[0] * inv_dt * dm, e2 = nd + hi[0] * inv_dt * dm;
                const double amin = e1 * e2 <= 0.0 ? 0.0 : fmin(e1 * e1, e2 * e2), amax = fmax(e1 * e1, e2 * e2);
                const double bc = nd * inv_dt * dm * dm, cc = nd * inv_dt * h2;
                mn = amin + fmin(lo[1] * bc, hi[1] * bc) + fmin(lo[2] * cc, hi[2] * cc);
                mx = amax + fmax(lo[1] * bc, hi[1] * bc) + fmax(lo[2] * cc, hi[2] * cc);
            }
            qlo = fmin(qlo, mn);
            qhi = fmax(qhi, mx);
        }
        int2 e = make_int2(0, 0);
        if (qhi >= 0.0) {
            const double tlo = sqrt(fmax(qlo, 0.0)), thi = fmin(sqrt(qhi), static_cast<double>(sv.nt - 1));
            const int32_t clo = max(0, static_cast<int32_t>(floor(tlo)) + PAD - W / 2 - 2);
            const int32_t chi = static_cast<int32_t>(floor(thi)) + PAD - W / 2 + 2;
            const int32_t len = chi + W + 1 - clo;
            if (len > TILE_STAGE_MAX)
                e = make_int2(0, -1);
            else if (len > 0)
                e = make_int2(clo, len);
        }
        tab[idx] = e;
    }
}

// Plain search: each workgroup runs the whole evolution (initial population
// and NG generations) of its samples.  ENS: each workgroup sweeps its time
// samples through the traces of its bucket, one trace after another: within
// a stage, sample (t, trace) depends only on (t, previous trace) of the same
// stage and on the complete previous stage, so the sweeps of different t
// never wait for each other and one launch covers many steps.
// KIND 0: exploration (plain evolution or ENS stage 0); KIND 1: ENS
// exploitation stages.  KIND selects the counters and names the kernel.
// k_search_dense is the same code held to 64 VGPRs (8 waves per SIMD), for
// launches whose wave count fits the chip in one round at that occupancy.
template <int OP, int DT, int W, int KIND, bool ADAPT, bool TILES = false>
__device__ __forceinline__ void search_body(const SearchArgs &a)
{
    extern __shared__ float lds[];
    const int32_t nsl = a.nsl;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(threadIdx.x) >> 6);
    const int32_t lane = threadIdx.x & (WAVE - 1);
    const int4 it = a.items[a.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int32_t>(blockIdx.x)];
    // the traces this workgroup sweeps: one for the plain search, else the
    // steps [k_begin, k_end) of its bucket's sweep (fewer for a short bucket)
    int32_t b0 = 0, nb = 1, k_end = 1, k_begin = 0;
    if (!a.plain) {
        b0 = it.x * a.n_bucket;
        nb = min(a.n_bucket, a.n_out - b0);
        k_begin = a.k_begin;
        k_end = min(a.k_end, nb);
    }
    // item: t_start, ns samples t_start + m stride (stride in bits 8..15), NP
    const int32_t t_start = it.y, ns = it.z & 0xff, stride = it.z >> 8, np = it.w;
    const int32_t grp = lane / np;
    const bool live = grp < ns;
    const int32_t slot = lane - grp * np;
    const int32_t base = grp * np;
    const int32_t n0 = t_start + (live ? grp : ns - 1) * stride;
    const int32_t tt = n0 - a.t_begin;
    const int32_t ap = a.sv.ap_tab[n0];
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < OP; ++d) {
        lo[d] = a.lo_tab[n0 * 3 + d];
        hi[d] = a.hi_tab[n0 * 3 + d];
    }
    // apertures grow or shrink linearly in t: the item's extreme samples bound them
    const int32_t amax = max(a.sv.ap_tab[t_start], a.sv.ap_tab[t_start + (ns - 1) * stride]);
    const uint64_t stage = static_cast<uint64_t>(a.stage);
    int buf = 0;
    int32_t M = 0;
    uint32_t n_ev = 0;
    uint64_t sum_m = 0;
    float pbest[3] = {0.f, 0.f, 0.f};  // this sample's best on the previous trace of the sweep
    // TILES: the step's table, 16 zeros and two staging buffers per wave after
    // the slices' merge area
    TileCtx tc{nullptr, 0, nullptr, nullptr};
    if constexpr (TILES) {
        float *base = lds + (nsl > 1 ? 2 * nsl * (W + 2) * WAVE : 0);
        float *zero = base + 2 * a.tile_cap;
        if (threadIdx.x < 16) zero[threadIdx.x] = 0.0f;
        tc.tab = reinterpret_cast<const int2 *>(base);
        tc.zero8 = zero;
        tc.stage = zero + 16 + wave * 2 * (TILE_STAGE_MAX + 8);
    }

    for (int32_t k = k_begin; k < k_end; ++k) {
        if (a.progress) pace_by_progress(a.progress, k - k_begin);
        const int32_t o = a.plain ? it.x : b0 + (a.forward ? k : nb - 1 - k);
        const int32_t prev = k > 0 ? (a.forward ? o - 1 : o + 1) : -1;
        const int32_t j = __builtin_amdgcn_readfirstlane(a.cmp_out[o]);
        const int32_t c_lo = max(0, j - amax), c_hi = min(a.sv.n_cmp - 1, j + amax);
        const uint64_t sid =
            static_cast<uint64_t>(n0) + static_cast<uint64_t>(a.sv.nt) * static_cast<uint64_t>(j);
        const int64_t here = static_cast<int64_t>(o) * a.n_t + tt;
        if constexpr (TILES) {
            __syncthreads();   // every wave is done with the previous step's table
            build_tile_table<OP, W>(a, const_cast<int2 *>(tc.tab), j, c_lo, c_hi, t_start, ns, stride);
            tc.i0 = static_cast<int32_t>(a.sv.cmp_ptr[c_lo]);
            __syncthreads();
        }

        // initial population (section "Initializing") and ENS seeds
        float x[3] = {0.f, 0.f, 0.f};
        uint64_t w[4];
        philox4x64_10(sid, stage, 0, static_cast<uint64_t>(slot), a.seed, 0, w);
#pragma unroll
        for (int d = 0; d < OP; ++d) x[d] = init_coord(w[d], lo[d], hi[d]);
        float S = 0.0f;
        bool scored = false;
        if (!a.plain) {
            // the previous trace of this sweep: kept in registers within the
            // launch, read back from the stage state at a launch's first step
            const int prev_slot = a.stage == 0 ? 0 : 2;
            if (a.inject && slot == prev_slot && prev >= 0) {
                if (k > k_begin) {
#pragma unroll
                    for (int d = 0; d < OP; ++d) x[d] = fminf(fmaxf(pbest[d], lo[d]), hi[d]);
                } else {
                    load_clamped<OP>(a.Yp + (static_cast<int64_t>(prev) * a.n_t + tt) * OP, lo, hi, x);
                }
            }
            if (a.stage > 0) {
                if (a.inject && slot == 0 && tt > 0) load_clamped<OP>(a.Xp + (here - 1) * OP, lo, hi, x);
                if (a.inject && slot == 1 && tt < a.n_t - 1)
                    load_clamped<OP>(a.Xp + (here + 1) * OP, lo, hi, x);
                if (slot == 3) {
#pragma unroll
                    for (int d = 0; d < OP; ++d) x[d] = a.Xp[here * OP + d];
                    S = a.XS[here];
                    scored = true;
                }
            }
        }
        {
            const Cand<float> cand = make_cand<OP, float>(x, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            const float Sev = eval_slices<DT, W, TILES>(a.sv, cand, c_lo, c_hi, wave, nsl, lane, lds, buf, M, tc);
            if (!scored) {
                S = Sev;
                if (live) {
                    n_ev += 1;
                    sum_m += static_cast<uint64_t>(M);
                }
            }
        }
        // generations (sections "Mutation and crossover", "Selection"); with
        // ADAPT, JADE's control parameters and archive, reset per domain
        double mu_cr = static_cast<double>(a.CR), mu_f = static_cast<double>(a.F);
        int32_t n_arch = 0;
        float arch[3] = {0.f, 0.f, 0.f};
        for (int32_t g = 1; g <= a.ng; ++g) {
            philox4x64_10(sid, stage, static_cast<uint64_t>(g), static_cast<uint64_t>(slot), a.seed, 0,
                          w);
            float u[3] = {0.f, 0.f, 0.f};
            int32_t k_cr = 0, k_f = 0, a_idx = 0;
            if constexpr (ADAPT) {
                uint64_t jw[4];
                philox4x64_10(sid, stage + (1ULL << 32), static_cast<uint64_t>(g), static_cast<uint64_t>(slot),
                              a.seed, 0, jw);
                jade_draws(jw, mu_cr, mu_f, np, k_cr, k_f, a_idx);
                const float F = static_cast<float>(k_f) * 0x1p-24f;
                make_trial<OP, true>(x, S, base, np, slot, w, F, static_cast<uint64_t>(k_cr) << 8, lo, hi, u,
                                     arch, n_arch);
            } else {
                make_trial<OP>(x, S, base, np, slot, w, a.F, a.cr_thr, lo, hi, u);
            }
            const Cand<float> cand = make_cand<OP, float>(u, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            const float St = eval_slices<DT, W, TILES>(a.sv, cand, c_lo, c_hi, wave, nsl, lane, lds, buf, M, tc);
            if (live) {
                n_ev += 1;
                sum_m += static_cast<uint64_t>(M);
            }
            if constexpr (ADAPT)
                jade_update<OP>(St >= S, x, k_cr, k_f, a_idx, grp, np, slot, arch, n_arch, mu_cr, mu_f);
            if (St >= S) {
#pragma unroll
                for (int d = 0; d < OP; ++d) x[d] = u[d];
                S = St;
            }
        }
        const int32_t b = group_argmax(S, base, np);
#pragma unroll
        for (int d = 0; d < OP; ++d) pbest[d] = __shfl(x[d], base + b, WAVE);
        if (wave == 0 && live && slot == b) {
#pragma unroll
            for (int d = 0; d < OP; ++d) a.Yp[here * OP + d] = x[d];
            a.YS[here] = S;
        }
        if (a.progress && threadIdx.x == 0) atomicAdd(a.progress, 1ull);
    }
    if (wave == 0) {
        const uint64_t tot_ev = wave_sum(static_cast<uint64_t>(n_ev));
        const uint64_t tot_m = wave_sum(sum_m);
        if (lane == 0) {
            atomicAdd(a.counters + 2 * KIND, static_cast<unsigned long long>(tot_ev));
            atomicAdd(a.counters + 2 * KIND + 1, static_cast<unsigned long long>(tot_m));
        }
    }
}

// Exploration (plain search, or ENS stage 0) with fixed F and CR, the
// populations of consecutive time samples laid end to end over all lanes of
// the workgroup's nsl waves, so that a population may straddle two waves and
// no lane idles for want of a whole population (NP_f between 33 and 63 leaves
// most of a wave empty in the layout above).  Each wave evaluates its own
// lanes' candidates over every trace of the union aperture, in the order of
// one slice (the same sums as nsl = 1 there); the members and scores meet in
// LDS, where each lane finds its population's best (lowest slot among equal
// scores) and reads the best and its two random members.  The draws, the
// trial arithmetic and the selection are those of search_body, so the result
// equals search_body's with one slice bit for bit.
template <int OP, int DT, int W>
__device__ __forceinline__ void search_packed_body(const SearchArgs &a)
{
    extern __shared__ float lds[];
    const int32_t nl = WAVE * a.nsl;              // lane slots of the workgroup
    const int32_t pmax = PACK_MAX_SAMPLES_PER_WAVE * a.nsl;
    float *lx = lds;                              // [3][nl] members
    float *ls = lds + 3 * nl;                     // [nl] scores
    float *lp = lds + 4 * nl;                     // [3][pmax] each sample's best on the previous trace
    const int32_t L = threadIdx.x;
    const int32_t lane = L & (WAVE - 1);
    const int4 it = a.items[a.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int32_t>(blockIdx.x)];
    int32_t b0 = 0, nb = 1, k_end = 1, k_begin = 0;
    if (!a.plain) {
        b0 = it.x * a.n_bucket;
        nb = min(a.n_bucket, a.n_out - b0);
        k_begin = a.k_begin;
        k_end = min(a.k_end, nb);
    }
    const int32_t t_start = it.y, ns = it.z & 0xff, stride = it.z >> 8;
    // this lane's sample m and slot; lanes past the last population are idle
    // and stand in as slot 0 of the last one (reads stay inside it, nothing is
    // written but their own LDS entries)
    int32_t m = 0, base = 0, np = a.np_tab[t_start];
    while (m + 1 < ns && L >= base + np) {
        base += np;
        m += 1;
        np = a.np_tab[t_start + m * stride];
    }
    const bool live = L < base + np;
    const int32_t slot = live ? L - base : 0;
    const int32_t n0 = t_start + m * stride;
    const int32_t tt = n0 - a.t_begin;
    const int32_t ap = a.sv.ap_tab[n0];
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < OP; ++d) {
        lo[d] = a.lo_tab[n0 * 3 + d];
        hi[d] = a.hi_tab[n0 * 3 + d];
    }
    const int32_t amax = max(a.sv.ap_tab[t_start], a.sv.ap_tab[t_start + (ns - 1) * stride]);
    const uint64_t stage = static_cast<uint64_t>(a.stage);
    uint32_t n_ev = 0;
    uint64_t sum_m = 0;

    for (int32_t k = k_begin; k < k_end; ++k) {
        if (a.progress) pace_by_progress(a.progress, k - k_begin);
        const int32_t o = a.plain ? it.x : b0 + (a.forward ? k : nb - 1 - k);
        const int32_t prev = k > 0 ? (a.forward ? o - 1 : o + 1) : -1;
        const int32_t j = __builtin_amdgcn_readfirstlane(a.cmp_out[o]);
        const int32_t c_lo = max(0, j - amax), c_hi = min(a.sv.n_cmp - 1, j + amax);
        const uint64_t sid =
            static_cast<uint64_t>(n0) + static_cast<uint64_t>(a.sv.nt) * static_cast<uint64_t>(j);
        const int64_t here = static_cast<int64_t>(o) * a.n_t + tt;

        float x[3] = {0.f, 0.f, 0.f};
        uint64_t w[4];
        philox4x64_10(sid, stage, 0, static_cast<uint64_t>(slot), a.seed, 0, w);
#pragma unroll
        for (int d = 0; d < OP; ++d) x[d] = init_coord(w[d], lo[d], hi[d]);
        if (!a.plain && a.inject && slot == 0 && prev >= 0) {
            if (k > k_begin) {
#pragma unroll
                for (int d = 0; d < OP; ++d) x[d] = fminf(fmaxf(lp[d * pmax + m], lo[d]), hi[d]);
            } else {
                load_clamped<OP>(a.Yp + (static_cast<int64_t>(prev) * a.n_t + tt) * OP, lo, hi, x);
            }
        }
        float S;
        {
            const Cand<float> cand = make_cand<OP, float>(x, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            Acc<W, float> acc;
            acc.reset();
            accumulate_range<DT, W, float>(a.sv, cand, c_lo, c_hi, 0, 1, acc);
            S = finish_semblance(acc);
            if (live) {
                n_ev += 1;
                sum_m += static_cast<uint64_t>(acc.M);
            }
        }
        for (int32_t g = 1; g <= a.ng; ++g) {
            __syncthreads();   // the previous generation's readers are done
#pragma unroll
            for (int d = 0; d < OP; ++d) lx[d * nl + L] = x[d];
            ls[L] = S;
            __syncthreads();
            float best = ls[base];
            int32_t bi = 0;
            for (int32_t q = 1; q < np; ++q) {
                const float v = ls[base + q];
                if (v > best) {
                    best = v;
                    bi = q;
                }
            }
            philox4x64_10(sid, stage, static_cast<uint64_t>(g), static_cast<uint64_t>(slot), a.seed, 0, w);
            const TrialDraw dr = trial_draw(w, slot, np, OP, a.cr_thr, np);
            float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < OP; ++d) {
                const float xb = lx[d * nl + base + bi];
                const float xr1 = lx[d * nl + base + static_cast<int32_t>(dr.r1)];
                const float xr2 = lx[d * nl + base + static_cast<int32_t>(dr.r2)];
                const float v = mutant(x[d], xb, xr1, xr2, a.F, lo[d], hi[d]);
                u[d] = dr.take[d] ? v : x[d];
            }
            const Cand<float> cand = make_cand<OP, float>(u, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            Acc<W, float> acc;
            acc.reset();
            accumulate_range<DT, W, float>(a.sv, cand, c_lo, c_hi, 0, 1, acc);
            const float St = finish_semblance(acc);
            if (live) {
                n_ev += 1;
                sum_m += static_cast<uint64_t>(acc.M);
            }
            if (St >= S) {
#pragma unroll
                for (int d = 0; d < OP; ++d) x[d] = u[d];
                S = St;
            }
        }
        // the sample's best: the state of the sample and the seed of its next trace
        __syncthreads();
#pragma unroll
        for (int d = 0; d < OP; ++d) lx[d * nl + L] = x[d];
        ls[L] = S;
        __syncthreads();
        float best = ls[base];
        int32_t bi = 0;
        for (int32_t q = 1; q < np; ++q) {
            const float v = ls[base + q];
            if (v > best) {
                best = v;
                bi = q;
            }
        }
        if (live && slot == bi) {
#pragma unroll
            for (int d = 0; d < OP; ++d) {
                a.Yp[here * OP + d] = x[d];
                lp[d * pmax + m] = x[d];
            }
            a.YS[here] = S;
        }
        __syncthreads();   // the seeds are in place before the next trace step reads them
        if (a.progress && threadIdx.x == 0) atomicAdd(a.progress, 1ull);
    }
    const uint64_t tot_ev = wave_sum(static_cast<uint64_t>(n_ev));
    const uint64_t tot_m = wave_sum(sum_m);
    if (lane == 0) {
        atomicAdd(a.counters, static_cast<unsigned long long>(tot_ev));
        atomicAdd(a.counters + 1, static_cast<unsigned long long>(tot_m));
    }
}

template <int OP, int DT, int W>
__global__ __launch_bounds__(512) void k_search_packed(SearchArgs a)
{
    search_packed_body<OP, DT, W>(a);
}

template <int OP, int DT, int W>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_search_packed_dense(SearchArgs a)
{
    search_packed_body<OP, DT, W>(a);
}

template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) void k_search(SearchArgs a)
{
    search_body<OP, DT, W, KIND, false>(a);
}

template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_search_dense(SearchArgs a)
{
    search_body<OP, DT, W, KIND, false>(a);
}

// the same search with the windows of binary32 rows staged per trace in LDS
// (ens_tuning.gather = 1): bit for bit the results of k_search
template <int OP, int W, int KIND>
__global__ __launch_bounds__(512) void k_search_tiles(SearchArgs a)
{
    search_body<OP, DT_F32, W, KIND, false, true>(a);
}

// the same search with JADE's control-parameter adaptation and archive
template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) void k_search_jade(SearchArgs a)
{
    search_body<OP, DT, W, KIND, true>(a);
}

template <int DT>
hipError_t launch_search_dt(int op, int window, int kind, int dense, const SearchArgs &a, int32_t n_blocks,
                           hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(n_blocks)), block(WAVE * a.nsl);
    if (a.packed) {
        if (a.adapt || kind != 0 || a.stage != 0) return hipErrorInvalidValue;
        const size_t lds = sizeof(float) * (4 * WAVE + 3 * PACK_MAX_SAMPLES_PER_WAVE) * a.nsl;
        if (!dense) {
            ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
                hipLaunchKernelGGL((k_search_packed<OP, DT, W>), grid, block, lds, s, a)));
        } else {
            ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
                hipLaunchKernelGGL((k_search_packed_dense<OP, DT, W>), grid, block, lds, s, a)));
        }
        return hipGetLastError();
    }
    size_t lds = a.nsl > 1 ? sizeof(float) * 2 * a.nsl * (window + 2) * WAVE : 0;
    if (a.tiles) {
        if constexpr (DT != DT_F32) {
            return hipErrorInvalidValue;
        } else {
            if (a.adapt) return hipErrorInvalidValue;
            lds += sizeof(float) * (2 * static_cast<size_t>(a.tile_cap) + 16 + 2 * a.nsl * (TILE_STAGE_MAX + 8));
            if (kind == 0) {
                ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
                    hipLaunchKernelGGL((k_search_tiles<OP, W, 0>), grid, block, lds, s, a)));
            } else {
                ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
                    hipLaunchKernelGGL((k_search_tiles<OP, W, 1>), grid, block, lds, s, a)));
            }
            return hipGetLastError();
        }
    }
    if (a.adapt && kind == 0) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_jade<OP, DT, W, 0>), grid, block, lds, s, a)));
    } else if (a.adapt) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_jade<OP, DT, W, 1>), grid, block, lds, s, a)));
    } else if (kind == 0 && !dense) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search<OP, DT, W, 0>), grid, block, lds, s, a)));
    } else if (kind == 0) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_dense<OP, DT, W, 0>), grid, block, lds, s, a)));
    } else if (!dense) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search<OP, DT, W, 1>), grid, block, lds, s, a)));
    } else {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_dense<OP, DT, W, 1>), grid, block, lds, s, a)));
    }
    return hipGetLastError();
}


}  // namespace ens
