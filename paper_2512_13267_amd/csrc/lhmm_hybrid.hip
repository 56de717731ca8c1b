// lhmm_hybrid.hip -- the LHMM macro step with the stress surrogate in the
// loop and plain micro-DPD as its fallback (include/lhmm.h, lhmm_hybrid_*).
//
// Per macro step t (the exchange interval of the coupling protocol, one SPH
// step per interval):
//   1. SPH step with the stresses of the last interval; micro gradients L_I;
//   2. L_I enters each particle's history ring (sample t);
//   3. surrogate mode: features -> ensemble forward -> gate; a flagged
//      particle is held on DPD for `hold` macro steps after its last flag.
//      A particle that enters DPD gets its micro-domain back from the
//      equilibrated snapshot and replays its last `replay` gradient samples
//      (k_micro steps each), so its polymer memory matches its history;
//   4. the micro-domains on DPD (all of them in DPD mode) advance k_micro
//      steps under L_I; their mean stresses replace the surrogate's mean on
//      those particles;
//   5. boxes whose cell became thin (LHMM_FLAG_THIN) are restored and
//      replayed the same way, after their stress has been used.
// Host work per step: one readback of the gate flags and one of the micro
// flags; the particle lists are built on the host and uploaded once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lhmm.h"
#include "lhmm_internal.h"

struct lhmm_hybrid {
    lhmm_hybrid_params p{};
    lhmm_sph* sph = nullptr;
    lhmm_micro* micro = nullptr;
    lhmm_sur* sur = nullptr;
    hipStream_t stream = nullptr;
    int n = 0, nm = 0, E = 0;
    long long t = 0;
    lhmm_hybrid_stats last{};
    long long box_steps = 0;
    // device
    float *ring = nullptr, *phi = nullptr, *X = nullptr, *Y = nullptr, *mean = nullptr;
    unsigned *gflag = nullptr, *on_d = nullptr;
    double *sigma = nullptr, *sigma_dpd = nullptr, *gradL = nullptr, *gradL_r = nullptr, *scratch = nullptr;
    double* sigma_sum = nullptr;  // running sum of the stresses handed to SPH
    long long n_sum = 0;
    std::vector<void*> bufs;
    // host (pinned)
    unsigned *gflag_h = nullptr, *on_h = nullptr;
    std::vector<int> hold_left;
    std::vector<unsigned char> was_on;   // DPD stress used in the last step
    std::vector<unsigned char> was_run;  // box advanced in the last step (used or warming)
    std::vector<uint32_t> mflags;
};

namespace {

// Input-range gate: bit 1 of flag[b] is set when the micro gradient of
// particle b (row-major 3 x 3, FP64) has squared Frobenius norm above max2,
// bit 2 when above warm2 (the warm band below it); the sum of squares is
// formed in this fixed order without fused products, so a host computation
// in FP64 takes the same decisions.
__global__ void k_input_gate(const double* __restrict__ L, int n, double max2, double warm2,
                             unsigned* __restrict__ flag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double* l = L + 9 * (long)b;
    double q = 0.0;
    for (int k = 0; k < 9; ++k) q = __dadd_rn(q, __dmul_rn(l[k], l[k]));
    if (q > max2) flag[b] |= 2u;
    if (q > warm2) flag[b] |= 4u;
}

__global__ void k_accumulate(const double* __restrict__ x, long n, double* __restrict__ sum) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sum[i] += x[i];
}

__global__ void k_zero(double* __restrict__ x, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

template <typename T>
int hy_alloc(lhmm_hybrid* h, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess)
        return lhmm_fail(LHMM_ERR_OOM, "hipMalloc(%zu) failed", count * sizeof(T));
    h->bufs.push_back(q);
    *p = (T*)q;
    return LHMM_OK;
}

void hy_release(lhmm_hybrid* h) {
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void* b : h->bufs) (void)hipFree(b);
    h->bufs.clear();
    if (h->gflag_h) (void)hipHostFree(h->gflag_h);
    if (h->on_h) (void)hipHostFree(h->on_h);
}

// Restore the listed boxes from the snapshot and replay history samples
// s_first .. s_last (inclusive, those >= 0) on them.
int restore_and_replay(lhmm_hybrid* h, const std::vector<int>& boxes, long long s_first, long long s_last) {
    if (boxes.empty()) return LHMM_OK;
    int rc = lhmm_micro_restore(h->micro, boxes.data(), (int32_t)boxes.size());
    if (rc != LHMM_OK) return rc;
    for (long long s = std::max(0LL, s_first); s <= s_last; ++s) {
        rc = lhmm_sur_history_gradient(h->ring, h->nm, s, 1.0f / h->p.grad_scale, h->gradL_r, h->stream);
        if (rc == LHMM_OK)
            rc = lhmm_micro_step_subset(h->micro, h->gradL_r, h->p.k_micro, h->scratch, boxes.data(),
                                        (int32_t)boxes.size());
        if (rc != LHMM_OK) return rc;
        h->box_steps += (long long)h->p.k_micro * (long long)boxes.size();
    }
    return LHMM_OK;
}

}  // namespace

extern "C" {

int lhmm_hybrid_create(const lhmm_hybrid_params* p, lhmm_sph* sph, lhmm_micro* micro, lhmm_sur* sur,
                       const float* phi, lhmm_hybrid** out) {
    lhmm_clear_error();
    if (!p || !sph || !micro || !phi || !out) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->mode != LHMM_HYBRID_SURROGATE && p->mode != LHMM_HYBRID_DPD)
        return lhmm_fail(LHMM_ERR_ARG, "unknown mode %d", p->mode);
    if (p->mode == LHMM_HYBRID_SURROGATE && !sur) return lhmm_fail(LHMM_ERR_ARG, "surrogate mode needs a surrogate");
    if (p->k_micro < 1 || p->hold < 1 || p->replay < 0 || p->replay > LHMM_SUR_HIST - 1)
        return lhmm_fail(LHMM_ERR_ARG, "need k_micro >= 1, hold >= 1, 0 <= replay < %d", LHMM_SUR_HIST);
    if (!(p->grad_scale > 0.0f) || !(p->stress_scale > 0.0f) || !(p->threshold >= 0.0f) || !(p->floor >= 0.0f) ||
        !(p->max_grad >= 0.0f))
        return lhmm_fail(LHMM_ERR_ARG, "scales must be positive, threshold, floor and max_grad non-negative");
    if (!(p->warm_frac >= 0.0f && p->warm_frac <= 1.0f))
        return lhmm_fail(LHMM_ERR_ARG, "warm_frac must lie in [0, 1]");
    int n = 0, nm = 0;
    lhmm_sph_counts(sph, &n, &nm);
    int32_t nb = 0;
    int rc = lhmm_micro_sizes(micro, nullptr, &nb);
    if (rc != LHMM_OK) return rc;
    if (nb != nm) return lhmm_fail(LHMM_ERR_ARG, "micro engine holds %d boxes for %d mobile SPH particles", nb, nm);
    hipStream_t st = lhmm_sph_caller_stream(sph);
    if (lhmm_micro_caller_stream(micro) != st) return lhmm_fail(LHMM_ERR_ARG, "engines must share one stream");
    int E = 0;
    if (sur) {
        int nin = 0, nout = 0, bmax = 0;
        lhmm_sur_dims(sur, &E, &nin, &nout, &bmax);
        if (nin != LHMM_SUR_FEATURES || nout != 3 || bmax < nm)
            return lhmm_fail(LHMM_ERR_ARG, "surrogate must map %d features to 3 outputs for batches of %d",
                             LHMM_SUR_FEATURES, nm);
        if (lhmm_sur_caller_stream(sur) != st) return lhmm_fail(LHMM_ERR_ARG, "engines must share one stream");
    }
    lhmm_hybrid* h = new (std::nothrow) lhmm_hybrid();
    if (!h) return lhmm_fail(LHMM_ERR_OOM, "host allocation failed");
    h->p = *p;
    h->sph = sph;
    h->micro = micro;
    h->sur = sur;
    h->stream = st;
    h->n = n;
    h->nm = nm;
    h->E = E;
    const size_t m = (size_t)nm;
    rc = hy_alloc(h, &h->ring, m * LHMM_SUR_HIST * 4);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->phi, m);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->X, m * LHMM_SUR_FEATURES);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->Y, (size_t)std::max(E, 1) * m * 3);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->mean, m * 3);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->gflag, m);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->on_d, m);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->sigma, (size_t)n * 6);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->sigma_dpd, m * 6);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->gradL, (size_t)n * 9);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->gradL_r, m * 9);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->scratch, m * 6);
    if (rc == LHMM_OK) rc = hy_alloc(h, &h->sigma_sum, (size_t)n * 6);
    if (rc == LHMM_OK && hipHostMalloc((void**)&h->gflag_h, m * sizeof(unsigned)) != hipSuccess)
        rc = lhmm_fail(LHMM_ERR_OOM, "pinned allocation failed");
    if (rc == LHMM_OK && hipHostMalloc((void**)&h->on_h, m * sizeof(unsigned)) != hipSuccess)
        rc = lhmm_fail(LHMM_ERR_OOM, "pinned allocation failed");
    auto init = [&]() -> int {
        LHMM_HIPCHK(hipStreamSynchronize(st));
        LHMM_HIPCHK(hipMemset(h->ring, 0, m * LHMM_SUR_HIST * 4 * sizeof(float)));
        LHMM_HIPCHK(hipMemset(h->sigma, 0, (size_t)n * 6 * sizeof(double)));
        LHMM_HIPCHK(hipMemset(h->sigma_sum, 0, (size_t)n * 6 * sizeof(double)));
        LHMM_HIPCHK(hipMemset(h->sigma_dpd, 0, m * 6 * sizeof(double)));
        LHMM_HIPCHK(hipMemset(h->gradL, 0, (size_t)n * 9 * sizeof(double)));
        LHMM_HIPCHK(hipMemset(h->mean, 0, m * 3 * sizeof(float)));
        LHMM_HIPCHK(hipMemcpy(h->phi, phi, m * sizeof(float), hipMemcpyHostToDevice));
        return LHMM_OK;
    };
    if (rc == LHMM_OK) rc = init();
    // the equilibrated state every restored box starts from
    if (rc == LHMM_OK) rc = lhmm_micro_snapshot(micro);
    if (rc == LHMM_OK) {
        h->mflags.assign(m, 0u);
        rc = lhmm_micro_flags(micro, h->mflags.data(), 1);
    }
    if (rc != LHMM_OK) {
        hy_release(h);
        delete h;
        return rc;
    }
    h->hold_left.assign(m, 0);
    h->was_on.assign(m, 0);
    h->was_run.assign(m, 0);
    *out = h;
    return LHMM_OK;
}

int lhmm_hybrid_step(lhmm_hybrid* h, lhmm_hybrid_stats* stats) {
    lhmm_clear_error();
    if (!h) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    const int nm = h->nm;
    const long long t = h->t;
    lhmm_hybrid_stats S{};
    // 1-2: SPH step and history
    int rc = lhmm_sph_step(h->sph, h->sigma, h->gradL);
    if (rc == LHMM_OK) rc = lhmm_sur_push_history(h->ring, nm, h->gradL, t, h->p.grad_scale, h->stream);
    if (rc != LHMM_OK) return rc;
    std::vector<int> on, entering;
    if (h->p.mode == LHMM_HYBRID_DPD) {
        rc = lhmm_micro_step(h->micro, h->gradL, h->p.k_micro, h->sigma);
        if (rc != LHMM_OK) return rc;
        h->box_steps += (long long)h->p.k_micro * nm;
        S.n_dpd = nm;
        on.resize(nm);
        for (int b = 0; b < nm; ++b) on[b] = b;
    } else {
        // 3: surrogate and gate
        rc = lhmm_sur_features(h->ring, nm, t, h->phi, h->X, h->stream);
        if (rc == LHMM_OK) rc = lhmm_sur_forward(h->sur, h->X, nm, h->Y);
        if (rc == LHMM_OK)
            rc = lhmm_sur_gate(h->Y, h->E, nm, 3, h->p.threshold, h->p.floor, h->mean, h->gflag, h->stream);
        if (rc != LHMM_OK) return rc;
        if (h->p.max_grad > 0.0f) {
            const double mg = (double)h->p.max_grad, wg = mg * (h->p.warm_frac > 0.0f ? (double)h->p.warm_frac : 1.0);
            k_input_gate<<<(nm + 255) / 256, 256, 0, h->stream>>>(h->gradL, nm, mg * mg, wg * wg, h->gflag);
            LHMM_HIPCHK(hipGetLastError());
        }
        LHMM_HIPCHK(hipMemcpyAsync(h->gflag_h, h->gflag, nm * sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
        LHMM_HIPCHK(hipStreamSynchronize(h->stream));
        // run: boxes advanced this step, the flagged ones (their DPD stress
        // is used) and, with a warm band, those whose gradient lies in it
        // (kept live so that a later flag finds their memory built);
        // entering: flagged boxes that were not live, restored and replayed;
        // warming: band boxes that were not live, restored only
        std::vector<int> run, warming;
        const bool band = h->p.max_grad > 0.0f && h->p.warm_frac > 0.0f;
        for (int b = 0; b < nm; ++b) {
            const unsigned fl = h->gflag_h[b];
            if (fl & 3u) {
                h->hold_left[b] = h->p.hold;
                S.n_flagged += 1;
                if (fl & 2u) S.n_out_of_range += 1;
            }
            const bool is_on = h->hold_left[b] > 0;
            const bool is_warm = !is_on && band && (fl & 4u);
            if (is_on) {
                on.push_back(b);
                if (!h->was_run[b]) entering.push_back(b);
                h->hold_left[b] -= 1;
            }
            if (is_warm) {
                S.n_warm += 1;
                if (!h->was_run[b]) warming.push_back(b);
            }
            if (is_on || is_warm) run.push_back(b);
            h->was_on[b] = is_on;
            h->was_run[b] = is_on || is_warm;
            h->on_h[b] = is_on ? 1u : 0u;
        }
        S.n_dpd = (int)on.size();
        S.n_entered = (int)entering.size();
        // entering boxes relive the intervals before this one; warming boxes
        // start from the snapshot
        rc = restore_and_replay(h, entering, t - h->p.replay, t - 1);
        if (rc == LHMM_OK) rc = restore_and_replay(h, warming, 0, -1);
        if (rc != LHMM_OK) return rc;
        // 4: DPD where the gate asked for it, and in the warm band
        if (!run.empty()) {
            rc = lhmm_micro_step_subset(h->micro, h->gradL, h->p.k_micro, h->sigma_dpd, run.data(),
                                        (int32_t)run.size());
            if (rc != LHMM_OK) return rc;
            h->box_steps += (long long)h->p.k_micro * (long long)run.size();
        }
        on.swap(run);  // the thin-cell check below covers every box that moved
        LHMM_HIPCHK(hipMemcpyAsync(h->on_d, h->on_h, nm * sizeof(unsigned), hipMemcpyHostToDevice, h->stream));
        rc = lhmm_sur_blend(h->mean, h->on_d, h->sigma_dpd, nm, h->p.stress_scale, h->sigma, h->stream);
        if (rc != LHMM_OK) return rc;
    }
    // 5: thin cells among the boxes that moved
    if (!on.empty()) {
        rc = lhmm_micro_flags(h->micro, h->mflags.data(), 1);
        if (rc != LHMM_OK) return rc;
        // a box whose stress is used relives its history; a warming box
        // starts again from the snapshot
        std::vector<int> reset, reset_warm;
        for (int b : on)
            if (h->mflags[b] & (LHMM_FLAG_THIN | LHMM_FLAG_CELL))
                (h->p.mode == LHMM_HYBRID_DPD || h->was_on[b] ? reset : reset_warm).push_back(b);
        S.n_reset = (int)(reset.size() + reset_warm.size());
        rc = restore_and_replay(h, reset, t + 1 - h->p.replay, t);
        if (rc == LHMM_OK) rc = restore_and_replay(h, reset_warm, 0, -1);
        if (rc != LHMM_OK) return rc;
    }
    const long n6 = 6L * h->n;
    k_accumulate<<<(n6 + 255) / 256, 256, 0, h->stream>>>(h->sigma, n6, h->sigma_sum);
    LHMM_HIPCHK(hipGetLastError());
    h->n_sum += 1;
    h->t += 1;
    S.macro_step = h->t;
    S.micro_box_steps = h->box_steps;
    h->last = S;
    if (stats) *stats = S;
    return LHMM_OK;
}

int lhmm_hybrid_state(lhmm_hybrid* h, double* sigma, uint32_t* on_dpd) {
    lhmm_clear_error();
    if (!h) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    LHMM_HIPCHK(hipStreamSynchronize(h->stream));
    if (sigma) LHMM_HIPCHK(hipMemcpy(sigma, h->sigma, (size_t)h->n * 6 * sizeof(double), hipMemcpyDeviceToHost));
    if (on_dpd) {
        if (h->p.mode == LHMM_HYBRID_DPD) {
            for (int b = 0; b < h->nm; ++b) on_dpd[b] = 1u;
        } else {
            for (int b = 0; b < h->nm; ++b) on_dpd[b] = h->was_on[b] ? 1u : 0u;
        }
    }
    return LHMM_OK;
}

int lhmm_hybrid_mean_stress(lhmm_hybrid* h, double* sigma_mean, int32_t reset) {
    lhmm_clear_error();
    if (!h) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    LHMM_HIPCHK(hipStreamSynchronize(h->stream));
    const size_t n6 = 6 * (size_t)h->n;
    if (sigma_mean) {
        std::vector<double> buf(n6);
        LHMM_HIPCHK(hipMemcpy(buf.data(), h->sigma_sum, n6 * sizeof(double), hipMemcpyDeviceToHost));
        const double w = h->n_sum > 0 ? 1.0 / (double)h->n_sum : 0.0;
        for (size_t i = 0; i < n6; ++i) sigma_mean[i] = buf[i] * w;
    }
    if (reset) {
        k_zero<<<(n6 + 255) / 256, 256, 0, h->stream>>>(h->sigma_sum, (long)n6);
        LHMM_HIPCHK(hipGetLastError());
        LHMM_HIPCHK(hipStreamSynchronize(h->stream));
        h->n_sum = 0;
    }
    return LHMM_OK;
}

int lhmm_hybrid_destroy(lhmm_hybrid* h) {
    lhmm_clear_error();
    if (!h) return LHMM_OK;
    hy_release(h);
    delete h;
    return LHMM_OK;
}

}  // extern "C"
