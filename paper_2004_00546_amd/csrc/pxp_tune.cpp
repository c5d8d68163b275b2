// Autotuner for the Paraexp gradient: slice count, Krylov flavour, schedule
// of the direct pieces and Krylov workgroup size, chosen by measurement.
//
// The paper sizes the partition from measured solve times per unit of
// simulated time (section 3.5, the tau ratios of the hybrid model); here the
// whole gradient is timed on the device for each candidate, and a candidate
// only counts if its gradient agrees with the serial method's gradient (the
// exact discrete adjoint of the same RK4 march) to the caller's tolerance.
// Host code over the public C ABI; it synchronises the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/paraexp.h"

namespace {

constexpr size_t TUNE_ALIGN = 256;

size_t align_up(size_t v) { return (v + TUNE_ALIGN - 1) / TUNE_ALIGN * TUNE_ALIGN; }

int64_t npts(const pxp_problem& p) { return (int64_t)p.nx * p.ny; }

bool same_group(const pxp_problem& a, const pxp_problem& b) {
    return a.op == b.op && a.nx == b.nx && a.ny == b.ny && a.prec == b.prec &&
           a.ctrl == b.ctrl;
}

// Divisors of n_steps in [lo, hi] (and at most four steps per slice for the
// 2D band marches), thinned to at most six spread geometrically.
std::vector<int> p_candidates(const pxp_problem& p, int lo, int hi) {
    std::vector<int> all;
    for (int64_t d = std::max(1, lo); d <= hi && d <= p.n_steps; ++d) {
        if (p.n_steps % d) continue;
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND && p.n_steps / d > 4) continue;
        all.push_back((int)d);
    }
    if (all.size() <= 6) return all;
    std::vector<int> out;
    const double a = std::log((double)all.front()), b = std::log((double)all.back());
    for (int k = 0; k < 6; ++k) {
        const double target = a + (b - a) * k / 5.0;
        int best = all.front();
        for (int d : all)
            if (std::fabs(std::log((double)d) - target) < std::fabs(std::log((double)best) - target))
                best = d;
        if (std::find(out.begin(), out.end(), best) == out.end()) out.push_back(best);
    }
    return out;
}

std::vector<pxp_problem> candidates(const pxp_problem& base, int lo, int hi) {
    std::vector<pxp_problem> out;
    // the problem as given comes first, so tuning never picks settings
    // slower than the untuned ones (e.g. AUTO, which chooses the flavour
    // per instance)
    {
        size_t bytes = 0;
        if (pxp_workspace_size(&base, 1, &bytes) == PXP_OK) out.push_back(base);
    }
    const bool linear = base.op != PXP_OP_BURGERS1D;
    const bool twod = base.op == PXP_OP_ADVDIFF2D_UPWIND;
    for (int P : p_candidates(base, lo, hi))
        for (int kr : {PXP_KRYLOV_POLY, PXP_KRYLOV_SHIFT_INVERT, PXP_KRYLOV_TAYLOR,
                       PXP_KRYLOV_CHEBYSHEV})
            for (int sc : {PXP_SCHED_CLASSIC, PXP_SCHED_CHAIN}) {
                if (!linear && sc == PXP_SCHED_CHAIN) continue;
                // 2D shift-and-invert pays two 2D Fourier transforms per
                // Krylov dimension: a named choice, not a tuning candidate
                if (twod && kr == PXP_KRYLOV_SHIFT_INVERT) continue;
                for (int kb : {256, 512}) {
                    if (twod && kb == 512) continue;
                    pxp_problem c = base;
                    c.P = P;
                    c.krylov = kr;
                    c.sched = sc;
                    c.kblock = twod ? 0 : kb;
                    size_t bytes = 0;
                    if (pxp_workspace_size(&c, 1, &bytes) == PXP_OK) out.push_back(c);
                }
            }
    return out;
}

// Offsets of instance i in the packed arrays.
struct Off {
    size_t n, k, kn;
};
Off offsets(const pxp_problem* pb, int i) {
    Off o{0, 0, 0};
    for (int j = 0; j < i; ++j) {
        o.n += (size_t)npts(pb[j]);
        o.k += (size_t)pb[j].K;
        o.kn += (size_t)pb[j].K * (size_t)npts(pb[j]);
    }
    return o;
}

// Divisors of n_steps usable as slice counts, ascending (the 2D band
// marches take at most four steps per slice).
std::vector<int> slice_counts(const pxp_problem& p) {
    std::vector<int> v;
    for (int64_t d = 1; d <= p.n_steps && d <= (1 << 20); ++d) {
        if (p.n_steps % d) continue;
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND && p.n_steps / d > 4) continue;
        v.push_back((int)d);
    }
    return v;
}

// Slice count of an instance whose slices last about `dur` time units,
// kept within [lo, hi] when that range has a divisor.
int map_P(const pxp_problem& p, double dur, int lo, int hi) {
    int best = -1;
    double bd = 1e300;
    for (int d : slice_counts(p)) {
        const bool inside = d >= lo && d <= hi;
        const double dist = std::fabs(std::log(p.T / d / dur)) + (inside ? 0.0 : 1e6);
        if (dist < bd) {
            bd = dist;
            best = d;
        }
    }
    return best > 0 ? best : p.P;
}

struct Trial {
    pxp_status st;
    double ms, warm_ms;
    std::vector<double> grad;
};

}  // namespace

extern "C" {

pxp_status pxp_tune_workspace_size(const pxp_problem* pb, int32_t batch, int32_t p_min,
                                   int32_t p_max, size_t* bytes) {
    if (!bytes || batch < 0 || (batch > 0 && !pb)) return PXP_EINVAL;
    size_t need = 0;
    for (int i = 0; i < batch; ++i) {
        size_t b = 0;
        pxp_status st = pxp_workspace_size(&pb[i], 1, &b);
        if (st != PXP_OK) return st;
        need = std::max(need, b);
        for (const pxp_problem& c : candidates(pb[i], p_min, p_max)) {
            pxp_workspace_size(&c, 1, &b);
            need = std::max(need, b);
        }
        need = std::max(need, b);
    }
    size_t kmax = 0;
    for (int i = 0; i < batch; ++i) kmax = std::max(kmax, (size_t)pb[i].K);
    *bytes = align_up((1 + kmax) * sizeof(double)) + need;
    return PXP_OK;
}

pxp_status pxp_autotune(pxp_problem* pb, int32_t batch, const double* ctrl,
                        const double* basis, const double* q0, const double* u_tgt,
                        int32_t p_min, int32_t p_max, double rtol, int32_t reps, void* ws,
                        size_t ws_bytes, pxp_tune_report* report, void* stream) {
    if (batch < 0 || (batch > 0 && !pb) || !u_tgt || !(rtol > 0.0)) return PXP_EINVAL;
    if (batch == 0) return PXP_OK;
    if (p_min <= 0) p_min = 8;
    if (p_max <= 0) p_max = 256;
    if (reps <= 0) reps = 2;
    size_t need = 0;
    pxp_status st = pxp_tune_workspace_size(pb, batch, p_min, p_max, &need);
    if (st != PXP_OK) return st;
    if (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % TUNE_ALIGN)
        return PXP_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t kmax = 0;
    for (int i = 0; i < batch; ++i) kmax = std::max(kmax, (size_t)pb[i].K);
    double* dJ = static_cast<double*>(ws);
    double* dgrad = dJ + 1;
    char* wsl = static_cast<char*>(ws) + align_up((1 + kmax) * sizeof(double));
    const size_t wsl_bytes = ws_bytes - align_up((1 + kmax) * sizeof(double));

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PXP_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PXP_EHIP;
    }
    // one gradient of instance i with settings c: status, time, gradient
    auto trial = [&](const pxp_problem& c, int i, int method, int nrep) -> Trial {
        Trial r{PXP_OK, 0.0, 0.0, {}};
        const auto t0 = std::chrono::steady_clock::now();
        const Off o = offsets(pb, i);
        const double* a = ctrl ? ctrl + o.k : nullptr;
        const double* G = basis ? basis + o.kn : nullptr;
        const double* z = q0 ? q0 + o.n : nullptr;
        r.st = pxp_workspace_init(wsl, wsl_bytes, stream);
        if (r.st != PXP_OK) return r;
        for (int rep = 0; rep <= nrep; ++rep) {
            if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) r.st = PXP_EHIP;
            if (r.st != PXP_OK) return r;
            r.st = pxp_gradient(&c, 1, method, a, G, z, u_tgt + o.n, dJ, dgrad, nullptr,
                                nullptr, wsl, wsl_bytes, stream);
            if (r.st != PXP_OK) return r;
            if (rep == 0) {
                // the first run is the warm-up and the accuracy sample
                r.st = pxp_device_status(wsl, wsl_bytes, stream, nullptr);
                r.warm_ms = std::chrono::duration<double, std::milli>(
                                std::chrono::steady_clock::now() - t0)
                                .count();
                if (r.st != PXP_OK) return r;
                r.grad.resize((size_t)c.K);
                if (c.K > 0 &&
                    hipMemcpy(r.grad.data(), dgrad, (size_t)c.K * sizeof(double),
                              hipMemcpyDeviceToHost) != hipSuccess) {
                    r.st = PXP_EHIP;
                    return r;
                }
            }
        }
        if (nrep > 0) {
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                r.st = PXP_EHIP;
                return r;
            }
            r.ms = ms / nrep;
        }
        return r;
    };
    auto rel = [](const std::vector<double>& x, const std::vector<double>& y) {
        double num = 0.0, den = 0.0;
        for (size_t k = 0; k < x.size(); ++k) {
            num += (x[k] - y[k]) * (x[k] - y[k]);
            den += y[k] * y[k];
        }
        return den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
    };

    std::vector<int> done(batch, 0);
    st = PXP_OK;
    for (int g = 0; g < batch && st == PXP_OK; ++g) {
        if (done[g]) continue;
        // the group's representative: its longest march
        int rep_i = g;
        for (int i = g; i < batch; ++i)
            if (!done[i] && same_group(pb[i], pb[g]) &&
                pb[i].n_steps * npts(pb[i]) > pb[rep_i].n_steps * npts(pb[rep_i]))
                rep_i = i;
        const pxp_problem base = pb[rep_i];
        Trial ref = trial(base, rep_i, PXP_METHOD_SERIAL, reps);
        if (ref.st != PXP_OK) {
            st = ref.st;
            break;
        }
        pxp_problem best = base;
        double best_ms = 1e300, best_err = 0.0;
        bool best_is_base = false;
        int tried = 0;
        for (const pxp_problem& c : candidates(base, p_min, p_max)) {
            // the warm-up alone decides for candidates far slower than the
            // best so far
            Trial w = trial(c, rep_i, PXP_METHOD_PARAEXP, 0);
            ++tried;
            if (w.st == PXP_EHIP) {
                st = w.st;
                break;
            }
            if (w.st != PXP_OK) continue;  // not converged or non-finite
            const double err = rel(w.grad, ref.grad);
            if (!(err <= rtol)) continue;
            if (w.warm_ms > 4.0 * best_ms) continue;
            Trial t = trial(c, rep_i, PXP_METHOD_PARAEXP, reps);
            if (t.st != PXP_OK) continue;
            if (t.ms < best_ms) {
                best_ms = t.ms;
                best = c;
                best_err = err;
                best_is_base = (tried == 1);
            }
        }
        if (st != PXP_OK) break;
        // The other instances of the group take the tuned settings with
        // slices of the tuned duration; each is checked against its own
        // serial gradient, and its slice count doubled (up to the next
        // divisor) until it passes, at most four times.
        const double dur = base.T / best.P;
        for (int i = g; i < batch; ++i) {
            if (done[i] || !same_group(pb[i], pb[g])) continue;
            done[i] = 1;
            double err_i = best_err;
            if (best_ms < 1e300) {
                pxp_problem c = pb[i];
                if (!best_is_base) {
                    c.krylov = best.krylov;
                    c.sched = best.sched;
                    c.kblock = best.kblock;
                    c.P = (i == rep_i) ? best.P : map_P(pb[i], dur, p_min, p_max);
                }
                // when the untuned settings won, every instance keeps its own
                bool ok = (i == rep_i) || best_is_base;
                if (!ok) {
                    Trial r = trial(pb[i], i, PXP_METHOD_SERIAL, 0);
                    if (r.st == PXP_EHIP) {
                        st = r.st;
                        break;
                    }
                    const std::vector<int> counts = slice_counts(pb[i]);
                    for (int attempt = 0; attempt < 5 && r.st == PXP_OK; ++attempt) {
                        size_t b = 0;
                        if (pxp_workspace_size(&c, 1, &b) == PXP_OK && b <= wsl_bytes) {
                            Trial w = trial(c, i, PXP_METHOD_PARAEXP, 0);
                            if (w.st == PXP_EHIP) {
                                st = w.st;
                                break;
                            }
                            err_i = (w.st == PXP_OK) ? rel(w.grad, r.grad) : 1e300;
                            if (err_i <= rtol) {
                                ok = true;
                                break;
                            }
                        }
                        auto nxt = std::lower_bound(counts.begin(), counts.end(), 2 * c.P);
                        if (nxt == counts.end()) break;
                        c.P = *nxt;
                    }
                    if (st != PXP_OK) break;
                }
                if (ok) {
                    pb[i].krylov = c.krylov;
                    pb[i].sched = c.sched;
                    pb[i].kblock = c.kblock;
                    pb[i].P = c.P;
                } else {
                    err_i = -1.0;
                }
            }
            if (report) {
                pxp_tune_report& r = report[i];
                r.P = pb[i].P;
                r.krylov = pb[i].krylov;
                r.sched = pb[i].sched;
                r.kblock = pb[i].kblock;
                r.candidates = tried;
                r.group = rep_i;
                r.ms = best_ms < 1e300 ? best_ms : -1.0;
                r.serial_ms = ref.ms;
                r.rel_err = best_ms < 1e300 ? err_i : -1.0;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // extern "C"
