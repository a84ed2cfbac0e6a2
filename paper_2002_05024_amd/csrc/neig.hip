// neig.hip -- host driver and C ABI of libneig (one translation unit with the
// kernels it launches).
//
// Control flow of neig_schur (Section 3.2): split the active block at
// negligible subdiagonals; blocks of at most nmin rows are finished by the
// in-LDS double-shift QR; larger ones alternate an aggressive early deflation
// step on the trailing window with a multishift sweep that uses the window's
// undeflated Ritz values as shifts.  Each AED and each small solve ends with one
// small device-to-host read of its status; sweeps are launched without
// synchronisation.  All launches go to the caller's stream.
#include "neig.h"

#include "small.hip"
#include "chase.hip"
#include "gemm.hip"
#include "util.hip"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <vector>

namespace {

struct HipFail {
    hipError_t e;
};

inline void ck(hipError_t e) {
    if (e != hipSuccess) throw HipFail{e};
}

neig_params g_params = {};
neig_stats g_stats = {};
std::mutex g_mutex;

constexpr int kMaxDevices = 64;
constexpr int kStatusInts = 64;

template <class T>
void grow(T **p, size_t *cap, size_t need) {
    if (need <= *cap) return;
    if (*p) ck(hipFree(*p));
    *p = nullptr;
    ck(hipMalloc((void **)p, need * sizeof(T)));
    *cap = need;
}

template <class T>
void grow_host(T **p, size_t *cap, size_t need) {
    if (need <= *cap) return;
    if (*p) ck(hipHostFree(*p));
    *p = nullptr;
    ck(hipHostMalloc((void **)p, need * sizeof(T), hipHostMallocDefault));
    *cap = need;
}

// Per-device workspace, allocated on first use and grown on demand.
struct DeviceWs {
    bool ready = false;
    size_t lds_max = 0;
    int small_max = 0;  // largest order the LDS QR / AED kernels take
    int chase_max = 0;  // largest chase window (U order)
    double *ut = nullptr; size_t ut_cap = 0;      // chase U^T slots
    double *vt = nullptr; size_t vt_cap = 0;      // AED / small-solve U^T
    double *poly = nullptr; size_t poly_cap = 0;  // bulge polynomials (tr, det)
    double *dbuf = nullptr; size_t dbuf_cap = 0;  // shifts, gathers, norm partials
    double *rot = nullptr; size_t rot_cap = 0;
    int *ist = nullptr;                           // device status ints
    int *flag = nullptr; size_t flag_cap = 0;
    int *h_ist = nullptr; size_t h_ist_cap = 0;   // pinned mirrors
    double *h_dbuf = nullptr; size_t h_dbuf_cap = 0;
    double *h_poly = nullptr; size_t h_poly_cap = 0;
    int *h_flag = nullptr; size_t h_flag_cap = 0;
    std::vector<hipEvent_t> events;               // pool for timing mode
};

DeviceWs g_ws[kMaxDevices];

DeviceWs &workspace() {
    int dev = 0;
    ck(hipGetDevice(&dev));
    DeviceWs &w = g_ws[dev];
    if (w.ready) return w;
    int lds = 0;
    ck(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    w.lds_max = (size_t)lds;
    int m = NEIG_SMALL_MAX;
    while (m > 4 && (size_t)(2 * m * (m + 1) + m) * 8 > w.lds_max) --m;
    w.small_max = m;
    int c = NEIG_CHASE_MAX;
    while (c > 8 && (size_t)(2 * (c + 1) * (c + 2)) * 8 + 2048 > w.lds_max) --c;
    w.chase_max = c;
    (void)hipFuncSetAttribute((const void *)k_small_qr, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_aed, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_chase, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_update, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();
    ck(hipMalloc((void **)&w.ist, kStatusInts * sizeof(int)));
    grow_host(&w.h_ist, &w.h_ist_cap, (size_t)kStatusInts);
    w.ready = true;
    return w;
}

void free_workspace(DeviceWs &w) {
    if (!w.ready) return;
    for (void *p : {(void *)w.ut, (void *)w.vt, (void *)w.poly, (void *)w.dbuf, (void *)w.rot, (void *)w.ist,
                    (void *)w.flag})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)w.h_ist, (void *)w.h_dbuf, (void *)w.h_poly, (void *)w.h_flag})
        if (p) (void)hipHostFree(p);
    for (hipEvent_t e : w.events) (void)hipEventDestroy(e);
    w = DeviceWs();
}

struct Eig {
    double re, im;
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ----------------------------------------------------------------------------
class Solver {
  public:
    Solver(int n, double *H, int ldh, double *Z, int ldz, hipStream_t st)
        : n_(n), H_(H), ldh_(ldh), Z_(Z), ldz_(ldz), st_(st), ws_(workspace()) {
        p_ = g_params;
        nsmall_ = ws_.small_max;
        nmin_ = p_.nmin > 0 ? std::min(p_.nmin, nsmall_) : nsmall_;
        wchase_ = p_.chase_w > 0 ? std::min(p_.chase_w, ws_.chase_max) : ws_.chase_max;
        nbc_ = p_.chain > 0 ? p_.chain : 16;
        nbc_ = std::max(1, std::min(nbc_, std::min(CHASE_MAX_BULGES, (wchase_ - 2) / 3)));
        maxit_ = p_.maxit > 0 ? p_.maxit : 30 * std::max(10, n);
        nibble_ = p_.nibble > 0 ? p_.nibble : 14;
        exc_ = p_.exc > 0 ? p_.exc : 6;
        smlnum_ = NEIG_DBL_MIN * ((double)std::max(n, 1) / NEIG_EPS);
        stats_ = neig_stats();
    }

    neig_stats stats_;

    // ---- timing mode: HIP events around launches, per kernel class ---------
    enum Kind { kUpdate = 0, kChase = 1, kAed = 2, kSmall = 3, kOther = 4 };
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks_;
    size_t ev_next_ = 0;

    hipEvent_t next_event() {
        if (ev_next_ == ws_.events.size()) {
            hipEvent_t e;
            ck(hipEventCreate(&e));
            ws_.events.push_back(e);
        }
        return ws_.events[ev_next_++];
    }

    template <class F>
    void timed(int kind, F &&launch) {
        if (!p_.timing) {
            launch();
            return;
        }
        hipEvent_t a = next_event(), b = next_event();
        ck(hipEventRecord(a, st_));
        launch();
        ck(hipEventRecord(b, st_));
        marks_.push_back({kind, a, b});
    }

    void sync_collect() {
        ck(hipStreamSynchronize(st_));
        collect();
    }

    // after the stream is synchronised: fold the event intervals into stats_
    void collect() {
        for (const Mark &m : marks_) {
            float ms = 0.0f;
            ck(hipEventElapsedTime(&ms, m.a, m.b));
            switch (m.kind) {
                case kUpdate: stats_.gpu_update_ms += ms; stats_.n_update += 1; break;
                case kChase: stats_.gpu_chase_ms += ms; stats_.n_chase += 1; break;
                case kAed: stats_.gpu_aed_ms += ms; break;
                case kSmall: stats_.gpu_small_ms += ms; break;
                default: stats_.gpu_other_ms += ms; break;
            }
        }
        marks_.clear();
        ev_next_ = 0;
    }

    // ||H||_F, zeros below the subdiagonal; returns false on non-finite input.
    bool prep() {
        const int nb = 512;
        grow(&ws_.dbuf, &ws_.dbuf_cap, (size_t)std::max(2 * nb, 4 * n_ + 64));
        grow_host(&ws_.h_dbuf, &ws_.h_dbuf_cap, (size_t)std::max(2 * nb, 4 * n_ + 64));
        ck(hipMemsetAsync(ws_.ist, 0, kStatusInts * sizeof(int), st_));
        hipLaunchKernelGGL(k_prep, dim3(nb), dim3(256), 0, st_, H_, ldh_, n_, ws_.ist, ws_.dbuf);
        ck(hipGetLastError());
        ck(hipMemcpyAsync(ws_.h_dbuf, ws_.dbuf, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, st_));
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, sizeof(int), hipMemcpyDeviceToHost, st_));
        sync_collect();
        if (ws_.h_ist[0]) return false;
        double scale = 0.0, ssq = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double sb = ws_.h_dbuf[2 * b], qb = ws_.h_dbuf[2 * b + 1];
            if (sb <= 0.0) continue;
            if (sb > scale) {
                ssq = ssq * (scale / sb) * (scale / sb) + qb;
                scale = sb;
            } else {
                ssq += qb * (sb / scale) * (sb / scale);
            }
        }
        hnorm_ = (scale > 0.0) ? scale * std::sqrt(ssq) : 0.0;
        return true;
    }

    double hnorm() const { return hnorm_; }

    // Largest k in [1, kbot] with a negligible (now zeroed) subdiagonal, else 0.
    int scan(int kbot) {
        if (kbot <= 0) return 0;
        ck(hipMemsetAsync(ws_.ist, 0, sizeof(int), st_));
        const int blocks = (kbot + 255) / 256;
        hipLaunchKernelGGL(k_scan, dim3(blocks), dim3(256), 0, st_, H_, ldh_, kbot, hnorm_, smlnum_, ws_.ist);
        ck(hipGetLastError());
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, sizeof(int), hipMemcpyDeviceToHost, st_));
        sync_collect();
        return ws_.h_ist[0];
    }

    // ---- off-diagonal update launches ------------------------------------
    struct Task {
        double *C;
        const double *Ut;
        int ldc, ldu, w, len, side;
    };

    void run_updates(const std::vector<Task> &tasks) {
        size_t i = 0;
        while (i < tasks.size()) {
            UpdArgs a;
            std::memset(&a, 0, sizeof(a));
            int tiles = 0, nt = 0, wmaxp = 16;
            bool any_left = false;
            for (; i < tasks.size() && nt < UPD_MAX_TASKS; ++i) {
                const Task &t = tasks[i];
                if (t.len <= 0 || t.w <= 0) continue;
                UpdTask &u = a.t[nt++];
                u.C = t.C; u.Ut = t.Ut; u.ldc = t.ldc; u.ldu = t.ldu; u.w = t.w; u.len = t.len; u.side = t.side;
                u.tile0 = tiles;
                tiles += (t.len + UPD_SLICE - 1) / UPD_SLICE;
                wmaxp = std::max(wmaxp, (t.w + 15) & ~15);
                if (t.side == 0) any_left = true;
                stats_.gemm_flops += 2.0 * t.w * (double)t.w * t.len;
            }
            a.ntask = nt;
            if (nt == 0 || tiles == 0) continue;
            size_t lds = any_left ? (size_t)(wmaxp + 1) * UPD_SLICE * sizeof(double) : 0;
            timed(kUpdate, [&] {
                hipLaunchKernelGGL(k_update, dim3(tiles), dim3(UPD_THREADS), lds, st_, a);
                ck(hipGetLastError());
            });
        }
    }

    // updates of everything outside the diagonal block [lo, hi] by its factor
    void add_block_updates(std::vector<Task> &tasks, int lo, int hi, const double *ut, int ldut) {
        const int w = hi - lo + 1;
        if (hi + 1 < n_) tasks.push_back({H_ + lo + (size_t)(hi + 1) * ldh_, ut, ldh_, ldut, w, n_ - hi - 1, 0});
        if (lo > 0) tasks.push_back({H_ + (size_t)lo * ldh_, ut, ldh_, ldut, w, lo, 1});
        tasks.push_back({Z_ + (size_t)lo * ldz_, ut, ldz_, ldut, w, n_, 1});
    }

    // ---- small block ------------------------------------------------------
    // Solve the diagonal block [ktop, kbot] in LDS and update the rest.  Returns the
    // number of leading rows of the block that did not converge (0 on success).
    int small_block(int ktop, int kbot) {
        const int m = kbot - ktop + 1;
        if (m <= 1) return 0;
        double t0 = now_ms();
        grow(&ws_.vt, &ws_.vt_cap, (size_t)m * m);
        const size_t lds = (size_t)2 * m * (m + 1) * sizeof(double);
        const int maxit = 30 * std::max(10, m);
        timed(kSmall, [&] {
            hipLaunchKernelGGL(k_small_qr, dim3(1), dim3(NT), lds, st_, H_, ldh_, ktop, m, hnorm_, smlnum_, maxit,
                               ws_.vt, m, ws_.ist);
            ck(hipGetLastError());
        });
        std::vector<Task> tasks;
        add_block_updates(tasks, ktop, kbot, ws_.vt, m);
        run_updates(tasks);
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
        sync_collect();
        stats_.small_solves++;
        stats_.small_flops += 10.0 * m * (double)m * m;
        stats_.alg_flops += 10.0 * m * (double)m * m + 2.0 * m * (double)m * (ktop + (n_ - kbot - 1) + n_);
        stats_.t_small_ms += now_ms() - t0;
        return ws_.h_ist[0];
    }

    // ---- aggressive early deflation -------------------------------------
    // Returns the number of deflated eigenvalues; fills the undeflated Ritz values.
    int aed(int ktop, int kbot, int nw, std::vector<Eig> &ritz, int *infqr = nullptr) {
        double t0 = now_ms();
        nw = std::min(nw, kbot - ktop + 1);
        nw = std::min(nw, nsmall_);
        const int kwtop = kbot - nw + 1;
        grow(&ws_.vt, &ws_.vt_cap, (size_t)nw * nw);
        grow(&ws_.dbuf, &ws_.dbuf_cap, (size_t)4 * nw + 64);
        grow_host(&ws_.h_dbuf, &ws_.h_dbuf_cap, (size_t)4 * nw + 64);
        const size_t lds = (size_t)(2 * nw * (nw + 1) + nw) * sizeof(double);
        const int maxit = 30 * std::max(10, nw);
        timed(kAed, [&] {
            hipLaunchKernelGGL(k_aed, dim3(1), dim3(NT), lds, st_, H_, ldh_, ktop, kbot, nw, hnorm_, smlnum_,
                               p_.deflation, maxit, ws_.vt, nw, ws_.ist, ws_.dbuf, ws_.dbuf + nw);
            ck(hipGetLastError());
        });
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, 12 * sizeof(int), hipMemcpyDeviceToHost, st_));
        ck(hipMemcpyAsync(ws_.h_dbuf, ws_.dbuf, 2 * nw * sizeof(double), hipMemcpyDeviceToHost, st_));
        sync_collect();
        const int nd = ws_.h_ist[0], nr = ws_.h_ist[1], applied = ws_.h_ist[2];
        if (infqr) *infqr = ws_.h_ist[3];
        if (ws_.h_ist[4]) stats_.swap_failures++;
        stats_.aed_qr_iters += ws_.h_ist[5];
        stats_.aed_swaps += ws_.h_ist[6];
        stats_.aed_cyc_qr += ws_.h_ist[7];
        stats_.aed_cyc_defl += ws_.h_ist[8];
        if (applied) stats_.aed_cyc_hess += ws_.h_ist[9];
        stats_.aed_late += ws_.h_ist[10];
        ritz.clear();
        for (int t = 0; t < nr; ++t) ritz.push_back({ws_.h_dbuf[t], ws_.h_dbuf[nw + t]});
        if (applied) {
            std::vector<Task> tasks;
            add_block_updates(tasks, kwtop, kbot, ws_.vt, nw);
            run_updates(tasks);
        }
        stats_.aeds++;
        stats_.aed_deflated += nd;
        stats_.small_flops += 10.0 * nw * (double)nw * nw;
        stats_.alg_flops += 10.0 * nw * (double)nw * nw;
        if (applied) stats_.alg_flops += 2.0 * nw * (double)nw * (kwtop + (n_ - kbot - 1) + n_);
        stats_.t_aed_ms += now_ms() - t0;
        return nd;
    }

    // ---- multishift sweep ------------------------------------------------
    struct Win {
        int r0, r1, t0, t1;
    };

    void sweep(int ktop, int kbot, const std::vector<Eig> &sh) {
        double t0ms = now_ms();
        const int nbulge = (int)sh.size() / 2;
        if (nbulge < 1 || kbot - ktop < 2) return;
        grow(&ws_.poly, &ws_.poly_cap, (size_t)2 * nbulge);
        grow_host(&ws_.h_poly, &ws_.h_poly_cap, (size_t)2 * nbulge);
        for (int g = 0; g < nbulge; ++g) {
            const Eig a = sh[2 * g], b = sh[2 * g + 1];
            ws_.h_poly[2 * g] = a.re + b.re;
            ws_.h_poly[2 * g + 1] = a.re * b.re - a.im * b.im;
        }
        ck(hipMemcpyAsync(ws_.poly, ws_.h_poly, 2 * nbulge * sizeof(double), hipMemcpyHostToDevice, st_));
        const int nbc = std::min(nbc_, nbulge);
        const int nchain = (nbulge + nbc - 1) / nbc;
        const int wmax = wchase_;
        const int ldut = wmax;
        grow(&ws_.ut, &ws_.ut_cap, (size_t)std::min(nchain, NEIG_MAX_CHAINS) * ldut * ldut);
        std::vector<std::vector<Win>> wins(nchain);
        std::vector<int> nbs(nchain);
        for (int c = 0; c < nchain; ++c) {
            const int nb = std::min(nbc, nbulge - c * nbc);
            nbs[c] = nb;
            const int tend = kbot - 1 - ktop + 3 * (nb - 1);
            int t = 0;
            while (t <= tend) {
                const int r0 = std::max(ktop, ktop + t - 3 * (nb - 1));
                const int r1 = std::min(kbot, r0 + wmax - 1);
                const int t1 = (r1 < kbot) ? r1 - 3 - ktop + 1 : tend + 1;
                wins[c].push_back({r0, r1, t, t1});
                t = t1;
            }
        }
        std::vector<size_t> idx(nchain, 0);
        for (;;) {
            ChaseArgs ca;
            std::memset(&ca, 0, sizeof(ca));
            ca.ktop = ktop; ca.kbot = kbot; ca.nbc = nbc; ca.ldut = ldut;
            int prev_r0 = 0;
            bool prev_done = true, prev_ran = false;
            int nact = 0;
            size_t lds = 0;
            bool any_left = false;
            for (int c = 0; c < nchain && nact < NEIG_MAX_CHAINS; ++c) {
                if (idx[c] >= wins[c].size()) {
                    prev_done = true; prev_ran = false;
                    continue;
                }
                any_left = true;
                const Win &wn = wins[c][idx[c]];
                bool ok = (c == 0) || prev_done || (prev_ran && wn.r1 < prev_r0 - 1);
                if (!ok) break;
                ChaseWin &cw = ca.win[nact++];
                cw.r0 = wn.r0; cw.r1 = wn.r1; cw.t0 = wn.t0; cw.t1 = wn.t1; cw.chain = c; cw.nb = nbs[c];
                const int b0 = wn.r0 > 0 ? wn.r0 - 1 : 0;
                const int mb = wn.r1 - b0 + 1, w = wn.r1 - wn.r0 + 1;
                lds = std::max(lds, (size_t)(mb * (mb + 1) + w * (w + 1)) * sizeof(double));
                stats_.chase_flops += 2.0 * 3 * nbs[c] * (double)(wn.t1 - wn.t0) * (2.0 * w + mb) * 2.0;
                prev_r0 = wn.r0; prev_done = false; prev_ran = true;
                ++idx[c];
            }
            if (!any_left) break;
            if (nact == 0) throw HipFail{hipErrorUnknown};  // schedule cannot stall
            ca.nwin = nact;
            timed(kChase, [&] {
                hipLaunchKernelGGL(k_chase, dim3(nact), dim3(CHASE_THREADS), lds, st_, H_, ldh_, ws_.poly, ws_.ut,
                                   ca);
                ck(hipGetLastError());
            });
            std::vector<Task> left, right;
            for (int k = 0; k < nact; ++k) {
                const ChaseWin &cw = ca.win[k];
                const double *ut = ws_.ut + (size_t)k * ldut * ldut;
                const int w = cw.r1 - cw.r0 + 1;
                const int b0 = cw.r0 > 0 ? cw.r0 - 1 : 0;
                if (cw.r1 + 1 < n_)
                    left.push_back({H_ + cw.r0 + (size_t)(cw.r1 + 1) * ldh_, ut, ldh_, ldut, w, n_ - cw.r1 - 1, 0});
                if (b0 > 0) right.push_back({H_ + (size_t)cw.r0 * ldh_, ut, ldh_, ldut, w, b0, 1});
                right.push_back({Z_ + (size_t)cw.r0 * ldz_, ut, ldz_, ldut, w, n_, 1});
            }
            if (nact == 1) {
                left.insert(left.end(), right.begin(), right.end());
                run_updates(left);
            } else {
                run_updates(left);
                run_updates(right);
            }
        }
        stats_.sweeps++;
        stats_.shifts_used += 2 * nbulge;
        stats_.alg_flops += 20.0 * n_ * (double)nbulge * (kbot - ktop);
        stats_.t_sweep_ms += now_ms() - t0ms;
    }

    // ---- shifts ------------------------------------------------------------
    std::vector<double> gather(int lo, int hi) {
        const int m = hi - lo + 1;
        grow(&ws_.dbuf, &ws_.dbuf_cap, (size_t)3 * m + 64);
        grow_host(&ws_.h_dbuf, &ws_.h_dbuf_cap, (size_t)3 * m + 64);
        hipLaunchKernelGGL(k_gather, dim3(1), dim3(256), 0, st_, H_, ldh_, lo, hi, ws_.dbuf);
        ck(hipGetLastError());
        ck(hipMemcpyAsync(ws_.h_dbuf, ws_.dbuf, 3 * m * sizeof(double), hipMemcpyDeviceToHost, st_));
        sync_collect();
        return std::vector<double>(ws_.h_dbuf, ws_.h_dbuf + 3 * m);
    }

    static void eig2(double a, double b, double c, double d, Eig *e1, Eig *e2) {
        double p = 0.5 * (a - d), disc = p * p + b * c, m = 0.5 * (a + d);
        if (disc >= 0.0) {
            double r = std::sqrt(disc);
            *e1 = {m + r, 0.0};
            *e2 = {m - r, 0.0};
        } else {
            double r = std::sqrt(-disc);
            *e1 = {m, r};
            *e2 = {m, -r};
        }
    }

    // Choose up to ns shifts from the Ritz values: complex pairs stay together,
    // real values are paired; smallest magnitudes first (bottom of the list on ties).
    static std::vector<Eig> pick_shifts(const std::vector<Eig> &ritz, int ns) {
        struct Item {
            Eig a, b;
            double mag;
            bool pair;
        };
        std::vector<Item> cpx;
        std::vector<Eig> real;
        for (size_t t = 0; t < ritz.size();) {
            if (ritz[t].im != 0.0 && t + 1 < ritz.size()) {
                cpx.push_back({ritz[t], ritz[t + 1], std::hypot(ritz[t].re, ritz[t].im), true});
                t += 2;
            } else {
                real.push_back(ritz[t]);
                ++t;
            }
        }
        std::sort(real.begin(), real.end(), [](const Eig &x, const Eig &y) { return std::fabs(x.re) < std::fabs(y.re); });
        std::vector<Item> items = cpx;
        for (size_t t = 0; t + 1 < real.size(); t += 2)
            items.push_back({real[t], real[t + 1], std::max(std::fabs(real[t].re), std::fabs(real[t + 1].re)), false});
        std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.mag < y.mag; });
        std::vector<Eig> out;
        for (const Item &it : items) {
            if ((int)out.size() + 2 > ns) break;
            out.push_back(it.a);
            out.push_back(it.b);
        }
        return out;
    }

    // Defaults measured on MI355X for random Hessenberg input: the AED window QR is a
    // latency-bound chain on one CU, so moderate windows deflate the most per unit time.
    int default_ns(int m) const {
        int ns = p_.ns > 0 ? p_.ns : (m < 300 ? 16 : 32);
        ns = std::min(ns, std::max(2, m / 3));
        ns -= ns % 2;
        return std::max(ns, 2);
    }

    int default_nw(int m) const {
        int nw = p_.nw > 0 ? p_.nw : (m < 300 ? 48 : 64);
        nw = std::min(nw, nsmall_);
        return std::min(nw, m);
    }

    // ---- whole solve -----------------------------------------------------
    int run() {
        double t0 = now_ms();
        if (!prep()) return -2;
        int kbot = n_ - 1;
        int total = 0, ndefl = 0;
        std::vector<Eig> ritz;
        int info = 0;
        while (kbot >= 0) {
            const int ktop = scan(kbot);
            const int m = kbot - ktop + 1;
            if (m <= nmin_) {
                int bad = small_block(ktop, kbot);
                if (bad > 0) {
                    info = ktop + bad;
                    break;
                }
                kbot = ktop - 1;
                ndefl = 0;
                continue;
            }
            if (++total > maxit_) {
                info = kbot + 1;
                break;
            }
            stats_.iterations++;
            const int nw = default_nw(m);
            const int nd = aed(ktop, kbot, nw, ritz);
            kbot -= nd;
            ndefl = (nd > 0) ? 0 : ndefl + 1;
            const int m2 = kbot - ktop + 1;
            if (m2 <= nmin_) continue;
            if (nd > 0 && 100 * nd > nibble_ * nw) continue;
            const int ns = default_ns(m2);
            std::vector<Eig> sh;
            if (ndefl > 0 && ndefl % exc_ == 0) {
                const int lo = std::max(ktop, kbot - ns - 1);
                std::vector<double> g = gather(lo, kbot);
                const int gm = kbot - lo + 1;
                for (int i = kbot; i >= lo + 2 && (int)sh.size() + 2 <= ns; i -= 2) {
                    const double s = std::fabs(g[gm + (i - lo)]) + std::fabs(g[gm + (i - 1 - lo)]);
                    const double x = g[i - lo];
                    sh.push_back({x + 0.75 * s, std::sqrt(0.4375) * s});
                    sh.push_back({x + 0.75 * s, -std::sqrt(0.4375) * s});
                }
                stats_.exceptional++;
            } else {
                sh = pick_shifts(ritz, ns);
            }
            if (sh.size() < 2) {
                std::vector<double> g = gather(kbot - 1, kbot);
                Eig e1, e2;
                eig2(g[0], g[4], g[3], g[1], &e1, &e2);
                if (e1.im == 0.0) {
                    const double hb = g[1];
                    const Eig pick = std::fabs(e1.re - hb) < std::fabs(e2.re - hb) ? e1 : e2;
                    e1 = pick;
                    e2 = pick;
                }
                sh = {e1, e2};
            }
            sweep(ktop, kbot, sh);
        }
        finish();
        stats_.t_total_ms = now_ms() - t0;
        return info;
    }

    // Standardise any 2x2 block not yet in standard form, then read off (wr, wi).
    void finish_std() {
        if (n_ < 2) return;
        grow(&ws_.flag, &ws_.flag_cap, (size_t)n_);
        grow(&ws_.rot, &ws_.rot_cap, (size_t)6 * n_);
        ck(hipMemsetAsync(ws_.ist, 0, sizeof(int), st_));
        hipLaunchKernelGGL(k_std_check, dim3((n_ + 255) / 256), dim3(256), 0, st_, H_, ldh_, n_, ws_.flag, ws_.rot,
                           ws_.ist);
        ck(hipGetLastError());
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, sizeof(int), hipMemcpyDeviceToHost, st_));
        sync_collect();
        if (ws_.h_ist[0] == 0) return;
        grow_host(&ws_.h_flag, &ws_.h_flag_cap, (size_t)n_);
        ck(hipMemcpyAsync(ws_.h_flag, ws_.flag, (n_ - 1) * sizeof(int), hipMemcpyDeviceToHost, st_));
        sync_collect();
        for (int j = 0; j + 1 < n_; ++j) {
            if (!ws_.h_flag[j]) continue;
            hipLaunchKernelGGL(k_std_apply, dim3((n_ + 255) / 256), dim3(256), 0, st_, H_, ldh_, Z_, ldz_, n_, j,
                               ws_.rot);
            ck(hipGetLastError());
        }
    }

    void finish() { finish_std(); }

    void eigenvalues(double *wr, double *wi) {
        if (n_ == 0) return;
        hipLaunchKernelGGL(k_eigs, dim3((n_ + 255) / 256), dim3(256), 0, st_, H_, ldh_, n_, wr, wi);
        ck(hipGetLastError());
    }

    void sync() { sync_collect(); }
    int nsmall() const { return nsmall_; }

  private:
    int n_;
    double *H_;
    int ldh_;
    double *Z_;
    int ldz_;
    hipStream_t st_;
    DeviceWs &ws_;
    neig_params p_;
    int nsmall_, nmin_, wchase_, nbc_, maxit_, nibble_, exc_;
    double hnorm_ = 0.0, smlnum_ = 0.0;
};

int check_args(int n, const void *H, int ldh, const void *Z, int ldz) {
    if (n < 0) return -1;
    if (n > 0 && !H) return -2;
    if (ldh < std::max(1, n)) return -3;
    if (n > 0 && !Z) return -4;
    if (ldz < std::max(1, n)) return -5;
    return 0;
}

}  // namespace

// ============================================================================ C ABI

extern "C" int neig_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi, hipStream_t stream) {
    int a = check_args(n, H, ldh, Z, ldz);
    if (a) return a;
    if (n > 0 && !wr) return -6;
    if (n > 0 && !wi) return -7;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        Solver s(n, H, ldh, Z, ldz, stream);
        int info = s.run();
        if (info == -2) return -2;
        s.eigenvalues(wr, wi);
        s.sync();
        g_stats = s.stats_;
        return info;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_small_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi,
                                hipStream_t stream) {
    int a = check_args(n, H, ldh, Z, ldz);
    if (a) return a;
    if (n > 0 && !wr) return -6;
    if (n > 0 && !wi) return -7;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        Solver s(n, H, ldh, Z, ldz, stream);
        if (n > s.nsmall()) return -1;
        if (!s.prep()) return -2;
        int info = s.small_block(0, n - 1);
        s.finish();
        s.eigenvalues(wr, wi);
        s.sync();
        g_stats = s.stats_;
        return info;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_sweep(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nshifts,
                          const double *sr, const double *si, hipStream_t stream) {
    int a = check_args(n, H, ldh, Z, ldz);
    if (a) return a;
    if (ktop < 0 || ktop >= n) return -6;
    if (kbot < ktop + 2 || kbot >= n) return -7;
    if (nshifts < 2 || nshifts % 2) return -8;
    if (!sr) return -9;
    if (!si) return -10;
    for (int i = 0; i < nshifts; i += 2) {
        const bool pair = si[i] != 0.0 || si[i + 1] != 0.0;
        if (pair && !(sr[i] == sr[i + 1] && si[i] == -si[i + 1])) return -10;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        Solver s(n, H, ldh, Z, ldz, stream);
        std::vector<Eig> sh;
        for (int i = 0; i < nshifts; ++i) sh.push_back({sr[i], si[i]});
        s.sweep(ktop, kbot, sh);
        s.sync();
        g_stats = s.stats_;
        return 0;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_aed(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nw, int *nd,
                        int *nshift, double *sr, double *si, hipStream_t stream) {
    int a = check_args(n, H, ldh, Z, ldz);
    if (a) return a;
    if (ktop < 0 || ktop >= n) return -6;
    if (kbot < ktop || kbot >= n) return -7;
    if (nw < 1 || nw > kbot - ktop + 1) return -8;
    if (!nd) return -9;
    if (!nshift) return -10;
    if (!sr) return -11;
    if (!si) return -12;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        Solver s(n, H, ldh, Z, ldz, stream);
        if (nw > s.nsmall()) return -8;
        if (!s.prep()) return -2;
        std::vector<Eig> ritz;
        *nd = s.aed(ktop, kbot, nw, ritz);
        *nshift = (int)ritz.size();
        for (size_t i = 0; i < ritz.size(); ++i) {
            sr[i] = ritz[i].re;
            si[i] = ritz[i].im;
        }
        s.sync();
        g_stats = s.stats_;
        return 0;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_schur_batched(int batch, const int *n, double *const *H, const int *ldh, double *const *Z,
                                  const int *ldz, double *const *wr, double *const *wi, int *info,
                                  hipStream_t stream) {
    if (batch < 0) return -1;
    if (batch == 0) return 0;
    if (!n) return -2;
    if (!H) return -3;
    if (!ldh) return -4;
    if (!Z) return -5;
    if (!ldz) return -6;
    if (!wr) return -7;
    if (!wi) return -8;
    if (!info) return -9;
    // device pointer tables -> host copies
    std::vector<double *> hH(batch), hZ(batch), hwr(batch), hwi(batch);
    try {
        ck(hipMemcpyAsync(hH.data(), H, batch * sizeof(double *), hipMemcpyDeviceToHost, stream));
        ck(hipMemcpyAsync(hZ.data(), Z, batch * sizeof(double *), hipMemcpyDeviceToHost, stream));
        ck(hipMemcpyAsync(hwr.data(), wr, batch * sizeof(double *), hipMemcpyDeviceToHost, stream));
        ck(hipMemcpyAsync(hwi.data(), wi, batch * sizeof(double *), hipMemcpyDeviceToHost, stream));
        ck(hipStreamSynchronize(stream));
        std::vector<int> inf(batch, 0);
        for (int b = 0; b < batch; ++b) inf[b] = neig_schur(n[b], hH[b], ldh[b], hZ[b], ldz[b], hwr[b], hwi[b], stream);
        ck(hipMemcpyAsync(info, inf.data(), batch * sizeof(int), hipMemcpyHostToDevice, stream));
        ck(hipStreamSynchronize(stream));
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

extern "C" int neig_set_params(const neig_params *p) {
    if (!p) return -1;
    if (p->ns < 0 || p->ns % 2) return -1;
    if (p->nw < 0) return -2;
    if (p->nmin < 0) return -3;
    if (p->chain < 0 || p->chain > CHASE_MAX_BULGES) return -4;
    if (p->chase_w < 0 || (p->chase_w > 0 && p->chase_w < 8)) return -5;
    if (p->deflation < 0 || p->deflation > 1) return -6;
    if (p->maxit < 0) return -7;
    if (p->nibble < 0 || p->nibble > 100) return -8;
    if (p->exc < 0) return -9;
    std::lock_guard<std::mutex> lock(g_mutex);
    g_params = *p;
    return 0;
}

extern "C" int neig_get_params(neig_params *p) {
    if (!p) return -1;
    std::lock_guard<std::mutex> lock(g_mutex);
    *p = g_params;
    return 0;
}

extern "C" int neig_get_stats(neig_stats *s) {
    if (!s) return -1;
    std::lock_guard<std::mutex> lock(g_mutex);
    *s = g_stats;
    return 0;
}

extern "C" void neig_finalize(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    for (int d = 0; d < kMaxDevices; ++d) free_workspace(g_ws[d]);
}

extern "C" const char *neig_version(void) { return "libneig 0.1 (gfx950, FP64 multishift QR + AED)"; }
