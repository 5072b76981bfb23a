// Autotuner of the engine's tile and fusion widths.
//
// The fused passes (a4) and the batched trajectory passes (a7) have shape
// knobs whose best values depend on the register size, the element type and
// the circuit: how many index bits a tile holds, how many of them are the
// contiguous low bits, how many amplitudes each thread keeps in registers,
// whether complex64 dense ops run on the matrix cores, and how many
// trajectory registers one launch covers.  The tuner times the caller's own
// workload on the device under candidate settings (kernel time from HIP
// events on the state's stream, median of several runs after an untimed run
// that compiles the candidate's pass kernels) and leaves the fastest set.
// The search is coordinate descent from the current values: one knob at a
// time over its candidate values, keeping a change only when it is at least
// 1% faster.
#include <algorithm>
#include <cstring>
#include <vector>

#include "sv_internal.h"

namespace {

struct Knob {
    const char *key;
    std::vector<int> values;
};

int get(const char *key) {
    int v = 0;
    (void)sv_config_get(key, &v);
    return v;
}

void fill_names(sv_tune_result *res, const std::vector<Knob> &knobs) {
    res->nkeys = int32_t(knobs.size());
    for (size_t i = 0; i < knobs.size(); ++i) {
        std::memset(res->key[i], 0, sizeof res->key[i]);
        std::strncpy(res->key[i], knobs[i].key, sizeof res->key[i] - 1);
    }
}

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

// Kernel time of one fused run of the gate list on s: sum of the profiled
// steps' durations.  The first run compiles and is not timed.
int time_fused(sv_state *s, const sv_gate *gates, int64_t ng, int reps, double *ms) {
    int rc = sv_run(s, gates, ng, SV_RUN_FUSED, nullptr);
    if (rc != SV_OK) return rc;
    std::vector<double> t;
    std::vector<double> step;
    for (int r = 0; r < reps; ++r) {
        rc = sv_run(s, gates, ng, SV_RUN_FUSED | SV_RUN_PROFILE, nullptr);
        if (rc != SV_OK) return rc;
        int64_t cnt = 0;
        rc = sv_run_profile(s, nullptr, nullptr, 0, &cnt);
        if (rc != SV_OK) return rc;
        step.assign(size_t(cnt), 0.0);
        rc = sv_run_profile(s, step.data(), nullptr, cnt, &cnt);
        if (rc != SV_OK) return rc;
        double sum = 0.0;
        for (double x : step) sum += x;
        t.push_back(sum);
    }
    *ms = median(t);
    return SV_OK;
}

}  // namespace

extern "C" int sv_tune_fused(sv_state *s, const sv_gate *gates, int64_t ng, int reps, sv_tune_result *res) {
    if (!s || !res || ng < 1 || !gates || reps < 1 || reps > 100) return SV_EINVAL;
    std::memset(res, 0, sizeof *res);
    std::vector<Knob> knobs;
    if (s->dtype == SV_C128) {
        knobs = {{"fused_tile_bits_c128", {10, 11, 12}}, {"fused_low_bits", {3, 4, 5}}, {"fused_reg_bits", {3, 4}}};
    } else {
        knobs = {{"fused_tile_bits_c64", {11, 12, 13}},
                 {"fused_low_bits", {3, 4, 5}},
                 {"fused_reg_bits", {3, 4}},
                 {"fused_mfma", {0, 1}}};
    }
    fill_names(res, knobs);
    std::vector<int> cur(knobs.size());
    for (size_t i = 0; i < knobs.size(); ++i) cur[i] = res->start[i] = get(knobs[i].key);
    auto set_all = [&](const std::vector<int> &v) {
        for (size_t i = 0; i < knobs.size(); ++i) (void)sv_config_set(knobs[i].key, v[i]);
    };
    double best_ms = 0.0;
    int rc = time_fused(s, gates, ng, reps, &best_ms);
    if (rc != SV_OK) return rc;
    res->start_ms = best_ms;
    res->tried = 1;
    for (size_t k = 0; k < knobs.size(); ++k) {
        for (int v : knobs[k].values) {
            if (v == cur[k]) continue;
            std::vector<int> cand = cur;
            cand[k] = v;
            set_all(cand);
            double ms = 0.0;
            const int rk = time_fused(s, gates, ng, reps, &ms);
            ++res->tried;
            if (rk == SV_EDEVICE) {
                set_all(cur);
                return rk;
            }
            if (rk == SV_OK && ms < 0.99 * best_ms) {
                best_ms = ms;
                cur = cand;
            }
        }
        set_all(cur);
    }
    for (size_t i = 0; i < knobs.size(); ++i) res->best[i] = cur[i];
    res->best_ms = best_ms;
    return SV_OK;
}

extern "C" int svb_tune_group(svb_batch *b, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter,
                              int iters, int reps, sv_tune_result *res) {
    int B = 0;
    if (!b || !res || reps < 1 || reps > 100 || svb_info(b, nullptr, &B, nullptr) != SV_OK) return SV_EINVAL;
    std::memset(res, 0, sizeof *res);
    // candidates: the whole batch per launch, then halvings down to 32
    // registers (a group's registers stay cache-resident between passes)
    std::vector<int> vals = {0};
    for (int g = B / 2; g >= 32 && B % g == 0; g /= 2) vals.push_back(g);
    // then the register budget of the batch pass kernels (waves per SIMD;
    // 0: the compiler's choice)
    std::vector<Knob> knobs = {{"svb_group", vals}, {"batch_waves", {0, 3, 4}}};
    fill_names(res, knobs);
    int cur = 0;
    (void)svb_get_group(b, &cur);
    res->start[0] = cur;
    const int waves0 = get("batch_waves");
    res->start[1] = waves0;
    auto time_group = [&](int g, double *ms) -> int {
        int rc = svb_set_group(b, g);
        if (rc != SV_OK) return rc;
        rc = svb_run_noisy(b, init, n_init, iter, n_iter, iters, 1e-2, 1e-4, 1, 0, 0, nullptr, nullptr);
        if (rc != SV_OK) return rc;
        std::vector<double> t;
        for (int r = 0; r < reps; ++r) {
            rc = svb_run_noisy(b, init, n_init, iter, n_iter, iters, 1e-2, 1e-4, 1, 0, 0, nullptr, nullptr);
            if (rc != SV_OK) return rc;
            double x = 0.0;
            (void)svb_last_run_ms(b, &x);
            t.push_back(x);
        }
        *ms = median(t);
        return SV_OK;
    };
    double best_ms = 0.0;
    int rc = time_group(cur, &best_ms);
    if (rc != SV_OK) return rc;
    res->start_ms = best_ms;
    res->tried = 1;
    int best = cur;
    for (int g : vals) {
        if (g == cur) continue;
        double ms = 0.0;
        rc = time_group(g, &ms);
        ++res->tried;
        if (rc == SV_EDEVICE) {
            (void)svb_set_group(b, best);
            return rc;
        }
        if (rc == SV_OK && ms < 0.99 * best_ms) {
            best_ms = ms;
            best = g;
        }
    }
    rc = svb_set_group(b, best);
    if (rc != SV_OK) return rc;
    res->best[0] = best;
    int best_w = waves0;
    for (int w : knobs[1].values) {
        if (w == waves0) continue;
        (void)sv_config_set("batch_waves", w);
        double ms = 0.0;
        rc = time_group(best, &ms);
        ++res->tried;
        if (rc == SV_EDEVICE) {
            (void)sv_config_set("batch_waves", best_w);
            return rc;
        }
        if (rc == SV_OK && ms < 0.99 * best_ms) {
            best_ms = ms;
            best_w = w;
        }
    }
    (void)sv_config_set("batch_waves", best_w);
    res->best[1] = best_w;
    res->best_ms = best_ms;
    return SV_OK;
}
