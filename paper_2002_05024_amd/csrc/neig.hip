// neig.hip -- host driver and C ABI of libneig (one translation unit with the
// kernels it launches).
//
// Control flow of neig_schur (Section 3.2): split the active block at
// negligible subdiagonals; blocks of at most nmin rows are finished by the
// in-LDS double-shift QR; larger ones alternate an aggressive early deflation
// step on the trailing window with a multishift sweep that uses the window's
// undeflated Ritz values as shifts.  Each AED and each small solve ends with one
// small device-to-host read of its status; sweeps are launched without
// synchronisation.  Launches go to the caller's stream, except the far part of
// a sweep step's updates, which runs on the library's second stream beside the
// next chase launch; the caller's stream waits for it before the sweep ends.
//
// Also here: the batched entry points (descriptor packing and the persistent
// solver of batched.hip), eigenvalue reordering (rounds of concurrent windows,
// k_reorder_window in small.hip), the Hessenberg reduction (hessenberg.hip),
// the proposal network's hooks and kernels (mlp.hip), and the per-device
// workspace.
#include "neig.h"

#include "small.hip"
#include "aedwide.hip"
#include "chase.hip"
#include "gemm.hip"
#include "util.hip"
#include "batched.hip"
#include "mlp.hip"
#include "hessenberg.hip"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
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

// Per-size-bucket settings of the batched solver (problems with n <= hi use the
// bucket); the autotuner replaces these through neig_set_batched_tune.
struct BatchTable {
    int hi[B_NBUCKET];
    BTune t[B_NBUCKET];
};
BatchTable g_btab = {{96, 256, 512, 768, 1024, 1 << 30},
                     {{48, 16, 96, 96}, {48, 16, 96, 96}, {64, 32, 96, 96}, {64, 32, 96, 96}, {64, 32, 96, 96},
                      {64, 32, 96, 96}}};
neig_stats g_stats = {};
std::mutex g_mutex;

// Parameter-proposal network: bins of the two proposals, the weights (host copy,
// uploaded to each device on first use after a change), the confidence below
// which the default heuristics are used, and the log of the last run.
const int kNsBins[MLP_NBIN] = {8, 16, 24, 32, 48, 64, 96, 128};
const int kNwBins[MLP_NBIN] = {32, 40, 48, 56, 64, 72, 80, 96};
struct PolicyState {
    std::vector<float> theta;  // empty: no network installed
    long long version = 0;
    float min_conf = 0.0f;
};
PolicyState g_policy;
struct PolicySample {
    float feat[MLP_NIN];
    int bins[2];
    float nd, ms, m;
    int used_net;
};
std::vector<PolicySample> g_policy_log;

constexpr int kMaxDevices = 64;
constexpr int kStatusInts = 64;
constexpr int kOverlapMinN = 8192;  // automatic overlap of sweep updates from this order on

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
    double *aw = nullptr; size_t aw_cap = 0;      // wide AED window: T, V, V^T, vectors
    int *ist = nullptr;                           // device status ints
    int *flag = nullptr; size_t flag_cap = 0;
    int *h_ist = nullptr; size_t h_ist_cap = 0;   // pinned mirrors
    double *h_dbuf = nullptr; size_t h_dbuf_cap = 0;
    double *h_poly = nullptr; size_t h_poly_cap = 0;
    int *h_flag = nullptr; size_t h_flag_cap = 0;
    std::vector<hipEvent_t> events;               // pool for timing mode
    int cus = 0;                                  // compute units (persistent grid size)
    // batched path: problem descriptors, processing order, work counter; fixed
    // capacity, allocated once, so a captured batched launch never refers to
    // memory that a later call frees
    BProb *bprob = nullptr;
    int *border = nullptr;
    int *bnext = nullptr;
    // network: weights, per-decision output (24 features, 2 bins, 2 probabilities),
    // training partials
    float *theta = nullptr;
    long long theta_version = -1;
    float *pol_out = nullptr;
    float *h_pol_out = nullptr;
    float *mlp_part = nullptr; size_t mlp_part_cap = 0;
    // Hessenberg reduction: V, Y, T, partials (one block, carved per call) and
    // the column state with its two workgroup counters (zero between launches)
    double *hrd = nullptr; size_t hrd_cap = 0;
    // reordering: window descriptors and statuses of one round
    ReorderWin *rwin = nullptr; size_t rwin_cap = 0;
    ReorderWin *h_rwin = nullptr; size_t h_rwin_cap = 0;
    int *rstat = nullptr; size_t rstat_cap = 0;
    int *h_rstat = nullptr; size_t h_rstat_cap = 0;
    HrdState *hrd_st = nullptr;
    // a second stream for a sweep's off-diagonal updates, which run beside the
    // next chase launch, and the events that order it with the caller's stream
    hipStream_t ust = nullptr;
    hipEvent_t ev_near = nullptr, ev_far = nullptr, ev_join = nullptr;
};

DeviceWs g_ws[kMaxDevices];

// Let a kernel take all the LDS its static arrays leave free as dynamic LDS.
void allow_dynamic_lds(const void *fn, size_t lds_max) {
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) == hipSuccess && at.sharedSizeBytes < lds_max)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(lds_max - at.sharedSizeBytes));
    (void)hipGetLastError();
}

// LDS per workgroup, the largest orders the LDS kernels take with it, and the
// compute-unit count of device dev.
struct DevLimits {
    size_t lds_max;
    int small_max, chase_max, cus;
};

DevLimits device_limits(int dev) {
    DevLimits d;
    int lds = 0;
    ck(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    d.lds_max = (size_t)lds;
    int m = NEIG_SMALL_MAX;
    while (m > 4 && (size_t)(2 * m * (m + 1) + m) * 8 > d.lds_max) --m;
    d.small_max = m;
    int c = NEIG_CHASE_MAX;
    while (c > 8 && (size_t)(2 * (c + 1) * (c + 2)) * 8 + 2048 > d.lds_max) --c;
    d.chase_max = c;
    ck(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    return d;
}

DeviceWs &workspace() {
    int dev = 0;
    ck(hipGetDevice(&dev));
    DeviceWs &w = g_ws[dev];
    if (w.ready) return w;
    const DevLimits lim = device_limits(dev);
    w.lds_max = lim.lds_max;
    w.small_max = lim.small_max;
    w.chase_max = lim.chase_max;
    for (const void *fn : {(const void *)k_small_qr, (const void *)k_aed, (const void *)k_chase,
                           (const void *)k_update, (const void *)k_update_wide, (const void *)k_batched,
                           (const void *)k_reorder_window})
        allow_dynamic_lds(fn, w.lds_max);
    w.cus = lim.cus;
    ck(hipMalloc((void **)&w.ist, kStatusInts * sizeof(int)));
    ck(hipMalloc((void **)&w.bprob, (size_t)NEIG_BATCH_MAX * sizeof(BProb)));
    ck(hipMalloc((void **)&w.border, (size_t)NEIG_BATCH_MAX * sizeof(int)));
    ck(hipMalloc((void **)&w.bnext, 4 * sizeof(int)));  // work counter, pad, flop count (a double)
    ck(hipMalloc((void **)&w.theta, (size_t)MLP_NPARAM * sizeof(float)));
    ck(hipMalloc((void **)&w.pol_out, 32 * sizeof(float)));
    ck(hipHostMalloc((void **)&w.h_pol_out, 32 * sizeof(float), hipHostMallocDefault));
    grow_host(&w.h_ist, &w.h_ist_cap, (size_t)kStatusInts);
    ck(hipStreamCreateWithFlags(&w.ust, hipStreamNonBlocking));
    for (hipEvent_t *e : {&w.ev_near, &w.ev_far, &w.ev_join}) ck(hipEventCreateWithFlags(e, hipEventDisableTiming));
    w.ready = true;
    return w;
}

void free_workspace(DeviceWs &w) {
    if (!w.ready) return;
    for (void *p : {(void *)w.ut, (void *)w.vt, (void *)w.poly, (void *)w.dbuf, (void *)w.rot, (void *)w.aw,
                    (void *)w.ist,
                    (void *)w.flag, (void *)w.bprob, (void *)w.border, (void *)w.bnext,
                    (void *)w.theta, (void *)w.pol_out, (void *)w.mlp_part, (void *)w.hrd, (void *)w.hrd_st,
                    (void *)w.rwin, (void *)w.rstat})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)w.h_ist, (void *)w.h_dbuf, (void *)w.h_poly, (void *)w.h_flag, (void *)w.h_pol_out,
                    (void *)w.h_rwin, (void *)w.h_rstat})
        if (p) (void)hipHostFree(p);
    for (hipEvent_t e : w.events) (void)hipEventDestroy(e);
    for (hipEvent_t e : {w.ev_near, w.ev_far, w.ev_join})
        if (e) (void)hipEventDestroy(e);
    if (w.ust) (void)hipStreamDestroy(w.ust);
    w = DeviceWs();
}

struct Eig {
    double re, im;
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Dynamic LDS of k_update_p<nrt>: one slice buffer.
size_t update_p_lds(int nrt) {
    const size_t wp = 16 * (size_t)nrt;
    return std::max((wp + 1) * UPD_SLICE, (size_t)(UPD_SLICE + 1) * wp) * sizeof(double);
}

// Resident workgroups of k_update_p<NRT> per compute unit (queried once per device).
template <int NRT>
int update_p_occupancy(DeviceWs &ws) {
    static int occ[kMaxDevices] = {0};
    int dev = 0;
    ck(hipGetDevice(&dev));
    if (occ[dev] == 0) {
        allow_dynamic_lds((const void *)k_update_p<NRT>, ws.lds_max);
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_p<NRT>, 64 * NRT, update_p_lds(NRT)) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        (void)hipGetLastError();
        occ[dev] = nb;
    }
    return occ[dev];
}

// ----------------------------------------------------------------------------
class Solver {
  public:
    Solver(int n, double *H, int ldh, double *Z, int ldz, hipStream_t st)
        : Solver(n, H, ldh, Z, ldz, st, g_params) {}

    Solver(int n, double *H, int ldh, double *Z, int ldz, hipStream_t st, const neig_params &prm)
        : n_(n), H_(H), ldh_(ldh), Z_(Z), ldz_(ldz), st_(st), ws_(workspace()) {
        p_ = prm;
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
    enum Kind { kUpdate = 0, kChase = 1, kAed = 2, kSmall = 3, kOther = 4, kRecDefl = 5, kUpdateFar = 6 };
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
        timed_on(st_, kind, launch);
    }

    template <class F>
    void timed_on(hipStream_t s, int kind, F &&launch) {
        if (!p_.timing) {
            launch();
            return;
        }
        hipEvent_t a = next_event(), b = next_event();
        ck(hipEventRecord(a, s));
        launch();
        ck(hipEventRecord(b, s));
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
                case kUpdateFar:
                    stats_.gpu_update_ms += ms; stats_.n_update += 1;
                    stats_.gpu_update_far_ms += ms; stats_.n_update_far += 1;
                    break;
                case kChase: stats_.gpu_chase_ms += ms; stats_.n_chase += 1; break;
                case kAed: stats_.gpu_aed_ms += ms; break;
                case kSmall: stats_.gpu_small_ms += ms; break;
                case kRecDefl: stats_.gpu_rec_defl_ms += ms; break;
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

    void run_updates(const std::vector<Task> &all) { run_updates(all, st_, kUpdate); }

    // kind: kUpdate, or kUpdateFar for the far part of an overlapped sweep step
    void run_updates(const std::vector<Task> &all, hipStream_t s, int kind) {
        std::vector<Task> tasks, wide;
        for (const Task &t : all) (t.w > UPD_WMAX ? wide : tasks).push_back(t);
        run_updates_wide(wide, s, kind);
        size_t i = 0;
        while (i < tasks.size()) {
            UpdArgs a;
            std::memset(&a, 0, sizeof(a));
            int tiles = 0, nt = 0, wmaxp = 16;
            for (; i < tasks.size() && nt < UPD_MAX_TASKS; ++i) {
                const Task &t = tasks[i];
                if (t.len <= 0 || t.w <= 0) continue;
                UpdTask &u = a.t[nt++];
                u.C = t.C; u.Ut = t.Ut; u.ldc = t.ldc; u.ldu = t.ldu; u.w = t.w; u.len = t.len; u.side = t.side;
                u.tile0 = tiles;
                tiles += (t.len + UPD_SLICE - 1) / UPD_SLICE;
                wmaxp = std::max(wmaxp, (t.w + 15) & ~15);
                count_update_flops(2.0 * t.w * (double)t.w * t.len, kind);
            }
            a.ntask = nt;
            if (nt == 0 || tiles == 0) continue;
            launch_update_p(a, tiles, (wmaxp + 15) / 16, s, kind);
        }
    }

    void count_update_flops(double f, int kind) {
        stats_.gemm_flops += f;
        if (kind == kUpdateFar) stats_.gemm_flops_far += f;
    }

    void launch_update_p(const UpdArgs &a, int nslice, int nrt, hipStream_t s, int kind) {
        switch (nrt) {
            case 1: launch_update_nrt<1>(a, nslice, s, kind); break;
            case 2: launch_update_nrt<2>(a, nslice, s, kind); break;
            case 3: launch_update_nrt<3>(a, nslice, s, kind); break;
            case 4: launch_update_nrt<4>(a, nslice, s, kind); break;
            case 5: launch_update_nrt<5>(a, nslice, s, kind); break;
            default: launch_update_nrt<6>(a, nslice, s, kind); break;
        }
    }

    template <int NRT>
    void launch_update_nrt(const UpdArgs &a, int nslice, hipStream_t s, int kind) {
        const int grid = std::min(nslice, ws_.cus * update_p_occupancy<NRT>(ws_));
        timed_on(s, kind, [&] {
            hipLaunchKernelGGL(k_update_p<NRT>, dim3(grid), dim3(64 * NRT), update_p_lds(NRT), s, a, nslice);
            ck(hipGetLastError());
        });
    }

    // tasks with factors of order UPD_WMAX+1 .. UPW_WMAX: U^T streamed from L2,
    // only the strip's slice staged in LDS
    void run_updates_wide(const std::vector<Task> &tasks, hipStream_t s, int kind) {
        size_t i = 0;
        while (i < tasks.size()) {
            UpdArgs a;
            std::memset(&a, 0, sizeof(a));
            int tiles = 0, nt = 0, wmaxp = 64;
            for (; i < tasks.size() && nt < UPD_MAX_TASKS; ++i) {
                const Task &t = tasks[i];
                if (t.len <= 0 || t.w <= 0) continue;
                if (t.w > UPW_WMAX) throw HipFail{hipErrorInvalidValue};
                UpdTask &u = a.t[nt++];
                u.C = t.C; u.Ut = t.Ut; u.ldc = t.ldc; u.ldu = t.ldu; u.w = t.w; u.len = t.len; u.side = t.side;
                u.tile0 = tiles;
                tiles += (t.len + UPW_SLICE - 1) / UPW_SLICE;
                wmaxp = std::max(wmaxp, (t.w + 63) & ~63);
                count_update_flops(2.0 * t.w * (double)t.w * t.len, kind);
            }
            a.ntask = nt;
            if (nt == 0 || tiles == 0) continue;
            // side 0 stages wp x UPW_SLICE with leading dimension wp + 1, side 1
            // UPW_SLICE x wp with leading dimension UPW_SLICE + 1
            const size_t lds = (size_t)(wmaxp + 1) * (UPW_SLICE + 1) * sizeof(double);
            timed_on(s, kind, [&] {
                hipLaunchKernelGGL(k_update_wide, dim3(tiles), dim3(UPW_THREADS), lds, s, a);
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
        nw = std::min(nw, kbot - ktop + 1);
        nw = std::min(nw, NEIG_AED_MAX);
        if (nw > nsmall_) return aed_wide(ktop, kbot, nw, ritz, infqr);
        std::vector<Eig> unused;
        AedEnd r = aed_ends(ktop, kbot, nw, 0, ritz, unused);
        if (infqr) *infqr = r.infqr;
        return r.nd;
    }

    // AED at the two ends of the active block [ktop, kbot] in one k_aed launch
    // (one workgroup per window): the trailing window of nw_bot rows (Section
    // 3.2) and, when nw_top > 0, the leading window of nw_top rows, handled as
    // the trailing window of the flipped block.  Either size may be 0 (that end
    // is skipped); both at most nsmall_, and the two windows must not overlap.
    // The windows' factors are applied to the rest of H and to Z; the leading
    // window's row strip overlaps the trailing window's column strip, so those
    // go in separate update launches.  Returns the trailing window's result;
    // the leading window's deflation count goes to *nd_top.
    struct AedEnd {
        int nd, infqr;
    };

    AedEnd aed_ends(int ktop, int kbot, int nw_bot, int nw_top, std::vector<Eig> &ritz_bot,
                    std::vector<Eig> &ritz_top, int *nd_top = nullptr) {
        double t0 = now_ms();
        const int nwm = std::max(nw_bot, nw_top);
        grow(&ws_.vt, &ws_.vt_cap, (size_t)2 * nwm * nwm);
        grow(&ws_.dbuf, &ws_.dbuf_cap, (size_t)4 * nwm + 64);
        grow_host(&ws_.h_dbuf, &ws_.h_dbuf_cap, (size_t)4 * nwm + 64);
        AedJobs jobs;
        std::memset(&jobs, 0, sizeof(jobs));
        // job j: factor at vt + j nwm^2, status at ist + 16 j, Ritz values at dbuf + 2 nwm j
        int nj = 0, jb = -1;
        auto add_job = [&](int nw, int flip) {
            const int j = nj++;
            jobs.j[j] = {ktop, kbot, nw, flip, ws_.vt + (size_t)j * nwm * nwm, ws_.ist + 16 * j,
                         ws_.dbuf + (size_t)2 * nwm * j, ws_.dbuf + (size_t)2 * nwm * j + nwm};
            return j;
        };
        if (nw_bot > 0) jb = add_job(nw_bot, 0);
        if (nw_top > 0) add_job(nw_top, 1);
        AedEnd res{0, 0};
        if (nd_top) *nd_top = 0;
        if (nj == 0) return res;
        const size_t lds = (size_t)(2 * nwm * (nwm + 1) + nwm) * sizeof(double);
        const int maxit = 30 * std::max(10, nwm);
        stats_.aed_launches += 1;
        timed(kAed, [&] {
            hipLaunchKernelGGL(k_aed, dim3(nj), dim3(NT), lds, st_, H_, ldh_, jobs, hnorm_, smlnum_, p_.deflation,
                               maxit, nwm);
            ck(hipGetLastError());
        });
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, 28 * sizeof(int), hipMemcpyDeviceToHost, st_));
        ck(hipMemcpyAsync(ws_.h_dbuf, ws_.dbuf, 4 * (size_t)nwm * sizeof(double), hipMemcpyDeviceToHost, st_));
        sync_collect();
        for (int j = 0; j < nj; ++j) {
            const int *st = ws_.h_ist + 16 * j;
            const AedJob &J = jobs.j[j];
            const int nw = J.nw, nd = st[0], nr = st[1], applied = st[2];
            if (st[4]) stats_.swap_failures++;
            stats_.aed_qr_iters += st[5];
            stats_.aed_swaps += st[6];
            stats_.aed_cyc_qr += st[7];
            stats_.aed_cyc_defl += st[8];
            if (applied) stats_.aed_cyc_hess += st[9];
            stats_.aed_late += st[10];
            std::vector<Eig> &ritz = (j == jb) ? ritz_bot : ritz_top;
            const double *hsr = ws_.h_dbuf + (size_t)2 * nwm * j;
            ritz.clear();
            for (int t = 0; t < nr; ++t) ritz.push_back({hsr[t], hsr[nwm + t]});
            if (j == jb) {
                res.nd = nd;
                res.infqr = st[3];
            } else {
                if (nd_top) *nd_top = nd;
                stats_.aeds_top += 1;
                stats_.aed_top_deflated += nd;
            }
            stats_.aeds++;
            stats_.aed_deflated += nd;
            stats_.small_flops += 10.0 * nw * (double)nw * nw;
            stats_.aed_flops += 10.0 * nw * (double)nw * nw;
            stats_.alg_flops += 10.0 * nw * (double)nw * nw;
            if (applied) {
                const int lo = J.flip ? ktop : kbot - nw + 1, hi = lo + nw - 1;
                std::vector<Task> tasks;
                add_block_updates(tasks, lo, hi, J.Vt, nwm);
                run_updates(tasks);  // one launch per window (see above)
                stats_.alg_flops += 2.0 * nw * (double)nw * (lo + (n_ - hi - 1) + n_);
            }
        }
        stats_.t_aed_ms += now_ms() - t0;
        return res;
    }

    // AED on a window of more than nsmall_ rows (Section 3.2: the window's Schur
    // form by a recursive application of the QR algorithm): the window is copied
    // to the workspace and reduced by the whole method run on it (its own AED
    // windows of at most nsmall_ rows, sweeps, small blocks), then k_aed_wide
    // does the spike test, swaps and re-Hessenberg reduction there.
    int aed_wide(int ktop, int kbot, int nw, std::vector<Eig> &ritz, int *infqr_out) {
        double t0 = now_ms();
        const int kwtop = kbot - nw + 1;
        const int ld = nw;
        const size_t nn = (size_t)nw * nw;
        grow(&ws_.aw, &ws_.aw_cap, 3 * nn + 4 * (size_t)nw + 64);
        grow_host(&ws_.h_dbuf, &ws_.h_dbuf_cap, (size_t)4 * nw + 64);
        double *T = ws_.aw, *V = T + nn, *Vt = V + nn, *x = Vt + nn, *sr = x + nw, *si = sr + nw, *sp0 = si + nw;
        const int gb = (int)std::min<size_t>((nn + 255) / 256, 1024);
        timed(kOther, [&] {
            hipLaunchKernelGGL(k_win_load, dim3(gb), dim3(256), 0, st_, H_, ldh_, kwtop, nw, T, ld, V, ld);
            ck(hipGetLastError());
        });
        neig_params ip = p_;
        ip.nw = p_.rec_nw > 0 ? std::min(p_.rec_nw, nsmall_) : 0;
        ip.ns = p_.rec_ns;
        ip.policy = 0;
        ip.maxit = 0;
        int inner_info = 0;
        if (p_.timing) sync_collect();  // the inner solve reuses the event pool from its start
        {
            Solver in(nw, T, ld, V, ld, st_, ip);
            inner_info = in.run();
            if (inner_info < 0) throw HipFail{hipErrorInvalidValue};  // non-finite window
            const neig_stats &q = in.stats_;
            stats_.rec_inner_aeds += (double)q.aeds;
            stats_.rec_inner_sweeps += (double)q.sweeps;
            stats_.gemm_flops += q.gemm_flops;
            stats_.chase_flops += q.chase_flops;
            stats_.small_flops += q.small_flops;
            stats_.aed_flops += q.aed_flops;  // the inner k_aed launches
            stats_.aed_launches += q.aed_launches;
            stats_.gpu_update_ms += q.gpu_update_ms;
            stats_.gpu_update_far_ms += q.gpu_update_far_ms;
            stats_.n_update_far += q.n_update_far;
            stats_.gemm_flops_far += q.gemm_flops_far;
            stats_.gpu_chase_ms += q.gpu_chase_ms;
            stats_.gpu_aed_ms += q.gpu_aed_ms;
            stats_.gpu_small_ms += q.gpu_small_ms;
            stats_.gpu_other_ms += q.gpu_other_ms;
            stats_.n_update += q.n_update;
            stats_.n_chase += q.n_chase;
            stats_.chase_bytes += q.chase_bytes;
            stats_.aed_qr_iters += q.aed_qr_iters;
            stats_.aed_swaps += q.aed_swaps;
            stats_.aed_cyc_qr += q.aed_cyc_qr;
            stats_.aed_cyc_defl += q.aed_cyc_defl;
            stats_.aed_cyc_hess += q.aed_cyc_hess;
            stats_.aed_late += q.aed_late;
            stats_.swap_failures += q.swap_failures;
        }
        timed(kRecDefl, [&] {
            hipLaunchKernelGGL(k_aed_wide, dim3(1), dim3(NT), 0, st_, H_, ldh_, ktop, kbot, T, V, ld, nw,
                               inner_info, hnorm_, smlnum_, p_.deflation, x, ws_.ist, sr, si, sp0);
            ck(hipGetLastError());
        });
        ck(hipMemcpyAsync(ws_.h_ist, ws_.ist, 12 * sizeof(int), hipMemcpyDeviceToHost, st_));
        ck(hipMemcpyAsync(ws_.h_dbuf, sr, 2 * (size_t)nw * sizeof(double), hipMemcpyDeviceToHost, st_));
        sync_collect();
        const int nd = ws_.h_ist[0], nr = ws_.h_ist[1], applied = ws_.h_ist[2];
        if (infqr_out) *infqr_out = ws_.h_ist[3];
        if (ws_.h_ist[4]) stats_.swap_failures++;
        stats_.aed_swaps += ws_.h_ist[6];
        stats_.aed_cyc_defl += ws_.h_ist[8];
        if (applied) stats_.aed_cyc_hess += ws_.h_ist[9];
        stats_.aed_late += ws_.h_ist[10];
        ritz.clear();
        for (int t = 0; t < nr; ++t) ritz.push_back({ws_.h_dbuf[t], ws_.h_dbuf[nw + t]});
        if (applied) {
            timed(kOther, [&] {
                hipLaunchKernelGGL(k_win_store, dim3(gb), dim3(256), 0, st_, H_, ldh_, ktop, kwtop, nw, T, V, ld,
                                   Vt, ld, sp0);
                ck(hipGetLastError());
            });
            std::vector<Task> tasks;
            add_block_updates(tasks, kwtop, kbot, Vt, ld);
            run_updates(tasks);
        }
        stats_.aeds++;
        stats_.rec_aeds++;
        stats_.aed_deflated += nd;
        stats_.alg_flops += 10.0 * nw * (double)nw * nw;
        if (applied) stats_.alg_flops += 2.0 * nw * (double)nw * (kwtop + (n_ - kbot - 1) + n_);
        stats_.t_aed_ms += now_ms() - t0;
        return nd;
    }

    // ---- multishift sweep ------------------------------------------------
    struct Win {
        int r0, r1, t0, t1;
    };

    // Update tasks of one part of a sweep step: left strips (rows of a window,
    // columns right of it), right strips of H (rows above a window, its
    // columns) and the Z tasks, with the H rectangles they cover.
    struct Rect {
        int r0, r1, c0, c1;
    };
    struct Parts {
        std::vector<Task> l, r, z;
        std::vector<Rect> lr, rr;
        void left(double *H, int ldh, const double *ut, int ldut, int r0, int r1, int c0, int c1) {
            l.push_back({H + r0 + (size_t)c0 * ldh, ut, ldh, ldut, r1 - r0 + 1, c1 - c0 + 1, 0});
            lr.push_back({r0, r1, c0, c1});
        }
        void right(double *H, int ldh, const double *ut, int ldut, int a, int b, int c0, int c1) {
            r.push_back({H + a + (size_t)c0 * ldh, ut, ldh, ldut, c1 - c0 + 1, b - a + 1, 1});
            rr.push_back({a, b, c0, c1});
        }
        bool cross() const {  // does a left strip meet a right strip?
            for (const Rect &x : lr)
                for (const Rect &y : rr)
                    if (x.r0 <= y.r1 && y.r0 <= x.r1 && x.c0 <= y.c1 && y.c0 <= x.c1) return true;
            return false;
        }
    };

    // One launch when no left strip meets a right strip, else every left strip
    // first (each pair commutes, but not within one launch).
    void run_parts(Parts &p, hipStream_t s, int kind) {
        if (!p.cross()) {
            p.l.insert(p.l.end(), p.r.begin(), p.r.end());
            p.l.insert(p.l.end(), p.z.begin(), p.z.end());
            run_updates(p.l, s, kind);
        } else {
            run_updates(p.l, s, kind);
            p.r.insert(p.r.end(), p.z.begin(), p.z.end());
            run_updates(p.r, s, kind);
        }
    }

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
        // two sets of U^T slots, used by alternate steps
        const size_t slot = (size_t)std::min(nchain, NEIG_MAX_CHAINS) * ldut * ldut;
        grow(&ws_.ut, &ws_.ut_cap, 2 * slot);
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
        // With overlap on, the updates of each step are split in two parts: the
        // near part (the entries of H that the next step's windows may cover,
        // rows and columns lo..hi) runs on the caller's stream right after the
        // step's chase launch, and the far part (the rest of H, all of Z) on
        // the update stream, beside the next step's chase launch; the next
        // step's near part waits for it (their left strips share rows).  The
        // windows of the next step are each chain's next window or a subset of
        // them.  Where one window's left strip crosses another's right strip
        // (rows of a window behind, columns of one ahead), the two updates
        // commute only as wholes, so that block is never split between the
        // parts: a left strip that reaches the next windows' rows keeps every
        // window's columns that start at or before hi in its near part, and a
        // right strip is split only if its window's columns start at or before
        // hi.
        const bool ovl = p_.overlap == 1 || (p_.overlap == 0 && n_ >= kOverlapMinN);
        if (ovl) {
            ck(hipEventRecord(ws_.ev_join, st_));
            ck(hipStreamWaitEvent(ws_.ust, ws_.ev_join, 0));
        }
        std::vector<size_t> idx(nchain, 0);
        int step = 0;
        for (;; ++step) {
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
                stats_.chase_bytes += 8.0 * (2.0 * mb * (double)mb + (double)w * w);
                prev_r0 = wn.r0; prev_done = false; prev_ran = true;
                ++idx[c];
            }
            if (!any_left) break;
            if (nact == 0) throw HipFail{hipErrorUnknown};  // schedule cannot stall
            ca.nwin = nact;
            double *uts = ws_.ut + (size_t)(step & 1) * slot;
            timed(kChase, [&] {
                hipLaunchKernelGGL(k_chase, dim3(nact), dim3(CHASE_THREADS), lds, st_, H_, ldh_, ws_.poly, uts, ca);
                ck(hipGetLastError());
            });
            // rows and columns lo..hi hold every window of the next step
            int lo = n_, hi = -1;
            if (ovl)
                for (int c = 0; c < nchain; ++c)
                    if (idx[c] < wins[c].size()) {
                        const Win &wn = wins[c][idx[c]];
                        lo = std::min(lo, wn.r0 > 0 ? wn.r0 - 1 : 0);
                        hi = std::max(hi, wn.r1);
                    }
            int hi_left = hi;  // near columns of the left strips
            for (int k = 0; k < nact; ++k)
                if (ca.win[k].r0 <= hi) hi_left = std::max(hi_left, ca.win[k].r1);
            Parts near, far;
            for (int k = 0; k < nact; ++k) {
                const ChaseWin &cw = ca.win[k];
                const double *ut = uts + (size_t)k * ldut * ldut;
                const int w = cw.r1 - cw.r0 + 1;
                const int b0 = cw.r0 > 0 ? cw.r0 - 1 : 0;
                if (cw.r1 + 1 < n_) {  // rows r0..r1, columns r1+1..n-1: near up to column cm
                    const int c0 = cw.r1 + 1;
                    const int cm = (cw.r1 >= lo) ? std::min(std::max(hi_left, cw.r1), n_ - 1) : cw.r1;
                    if (cm >= c0) near.left(H_, ldh_, ut, ldut, cw.r0, cw.r1, c0, cm);
                    if (cm + 1 < n_) far.left(H_, ldh_, ut, ldut, cw.r0, cw.r1, cm + 1, n_ - 1);
                }
                if (b0 > 0) {  // rows 0..b0-1, columns r0..r1: near from row rm
                    const int rm = (cw.r0 <= hi) ? std::min(lo, b0) : b0;
                    if (rm < b0) near.right(H_, ldh_, ut, ldut, rm, b0 - 1, cw.r0, cw.r1);
                    if (rm > 0) far.right(H_, ldh_, ut, ldut, 0, rm - 1, cw.r0, cw.r1);
                }
                far.z.push_back({Z_ + (size_t)cw.r0 * ldz_, ut, ldz_, ldut, w, n_, 1});
            }
            if (ovl) {
                if (step > 0) ck(hipStreamWaitEvent(st_, ws_.ev_far, 0));
                run_parts(near, st_, kUpdate);
                ck(hipEventRecord(ws_.ev_near, st_));
                ck(hipStreamWaitEvent(ws_.ust, ws_.ev_near, 0));
                run_parts(far, ws_.ust, kUpdateFar);
                ck(hipEventRecord(ws_.ev_far, ws_.ust));
            } else {
                run_parts(far, st_, kUpdate);  // lo > hi: everything is in the far part
            }
        }
        if (ovl && step > 0) ck(hipStreamWaitEvent(st_, ws_.ev_far, 0));
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
        nw = std::min(nw, NEIG_AED_MAX);
        return std::min(nw, m);
    }

    // ---- whole solve -----------------------------------------------------
    // ---- parameter proposals ----------------------------------------------
    // The features of the active block [ktop, kbot] and the network's bins, by
    // one k_policy launch and one read-back.  The last four features come from
    // the host: Ritz-value statistics of the previous deflation window and the
    // share of it that deflated.
    struct Decision {
        float feat[MLP_NIN];
        int bins[2];
        float conf[2];
    };

    void upload_policy() {
        if (ws_.theta_version == g_policy.version) return;
        std::vector<float> th = g_policy.theta;
        if (th.empty()) {  // neutral weights: features are still computed
            th.assign(MLP_NPARAM, 0.0f);
            for (int k = 0; k < MLP_NIN; ++k) th[MLP_O_SD + k] = 1.0f;
        }
        ck(hipMemcpy(ws_.theta, th.data(), (size_t)MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
        ws_.theta_version = g_policy.version;
    }

    Decision propose(int ktop, int kbot, const std::vector<Eig> &ritz, int nd_prev, int nw_prev) {
        upload_policy();
        const double scale = hnorm_ > 0.0 ? hnorm_ / std::sqrt((double)n_) : 1.0;
        float f20 = 0.0f, f21 = 0.0f, f22 = 0.0f;
        if (!ritz.empty()) {
            double sum = 0.0, sq = 0.0, cplx = 0.0;
            for (const Eig &e : ritz) {
                const double r = std::hypot(e.re, e.im);
                sum += r;
                sq += r * r;
                cplx += (e.im != 0.0) ? 1.0 : 0.0;
            }
            const double k = (double)ritz.size(), mean = sum / k;
            const double var = std::max(0.0, sq / k - mean * mean);
            f20 = (float)std::log(1e-30 + mean / scale);
            f21 = (float)(std::sqrt(var) / (mean + 1e-300));
            f22 = (float)(cplx / k);
        }
        const float f23 = nw_prev > 0 ? (float)nd_prev / (float)nw_prev : 0.0f;
        float *out = ws_.pol_out;
        timed(kOther, [&] {
            hipLaunchKernelGGL(k_policy, dim3(1), dim3(256), 0, st_, H_, ldh_, n_, ktop, kbot, hnorm_, f20, f21, f22,
                               f23, ws_.theta, out, (int *)(out + MLP_NIN), out + MLP_NIN + 2);
            ck(hipGetLastError());
        });
        ck(hipMemcpyAsync(ws_.h_pol_out, out, (MLP_NIN + 4) * sizeof(float), hipMemcpyDeviceToHost, st_));
        sync_collect();
        Decision d;
        std::memcpy(d.feat, ws_.h_pol_out, MLP_NIN * sizeof(float));
        std::memcpy(d.bins, ws_.h_pol_out + MLP_NIN, 2 * sizeof(int));
        std::memcpy(d.conf, ws_.h_pol_out + MLP_NIN + 2, 2 * sizeof(float));
        return d;
    }

    // counter-based generator for exploration (splitmix64 of seed and counter)
    uint64_t rng_state_ = 0;
    int explore_bin() {
        uint64_t z = (rng_state_ += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return (int)(z % MLP_NBIN);
    }

    int run() {
        double t0 = now_ms();
        if (!prep()) return -2;
        int kbot = n_ - 1;
        int total = 0, ndefl = 0;
        std::vector<Eig> ritz;
        int info = 0;
        const int mode = p_.policy;
        rng_state_ = 0x243f6a8885a308d3ull ^ (uint64_t)(unsigned)p_.seed;
        policy_log_.clear();
        int nw_next = 0, ns_next = 0;
        bool held_set = false;
        int held_used = 0, held_bins[2] = {0, 0};
        PolicySample pending;
        bool have_pending = false;
        double t_decide = 0.0;
        std::map<int, int> done;  // rows [first, last] deflated at the top of an active block, by last
        int top_fail = 0;         // leading-window AEDs in a row that deflated nothing
        while (kbot >= 0) {
            const auto dn = done.find(kbot);
            if (dn != done.end()) {  // already in Schur form: skip to the rows above
                kbot = dn->second - 1;
                continue;
            }
            int ktop = scan(kbot);
            const int m = kbot - ktop + 1;
            if (m <= nmin_) {
                int bad = small_block(ktop, kbot);
                if (bad > 0) {
                    info = ktop + bad;
                    break;
                }
                kbot = ktop - 1;
                top_fail = 0;
                ndefl = 0;
                have_pending = false;
                nw_next = ns_next = 0;
                continue;
            }
            if (++total > maxit_) {
                info = kbot + 1;
                break;
            }
            stats_.iterations++;
            const int nw = nw_next > 0 ? std::min(nw_next, m) : default_nw(m);
            int nd = 0;
            if (nw <= nsmall_) {
                // the leading window too while the block is large enough for two
                // disjoint windows and that end keeps deflating
                const int nw_top = (p_.aed_ends == 0 && top_fail < 3 && m >= 2 * nw + 32) ? nw : 0;
                int nd_top = 0;
                std::vector<Eig> ritz_top;
                nd = aed_ends(ktop, kbot, nw, nw_top, ritz, ritz_top, &nd_top).nd;
                if (nd_top > 0) {
                    const int last = ktop + nd_top - 1;
                    int first = ktop;
                    const auto prev = done.find(ktop - 1);  // extend the range deflated just above
                    if (prev != done.end()) {
                        first = prev->second;
                        done.erase(prev);
                    }
                    done[last] = first;
                    ktop += nd_top;
                    top_fail = 0;
                } else if (nw_top > 0) {
                    ++top_fail;
                }
            } else {
                nd = aed(ktop, kbot, nw, ritz);
            }
            if (have_pending) {  // reward of the last proposal: this window's deflations per ms
                pending.nd = (float)nd;
                pending.ms = (float)(now_ms() - t_decide);
                policy_log_.push_back(pending);
                have_pending = false;
            }
            nw_next = ns_next = 0;
            kbot -= nd;
            ndefl = (nd > 0) ? 0 : ndefl + 1;
            const int m2 = kbot - ktop + 1;
            if (m2 <= nmin_) continue;
            if (mode == 4 && held_set) {
                // per-matrix proposal: the bins of the first decision hold
                if (held_used) {
                    ns_next = kNsBins[held_bins[0]];
                    nw_next = kNwBins[held_bins[1]];
                    stats_.policy_used++;
                } else {
                    stats_.policy_fallback++;
                }
            } else if (mode != 0) {
                t_decide = now_ms();
                Decision d = propose(ktop, kbot, ritz, nd, nw);
                int bns = d.bins[0], bnw = d.bins[1];
                int used = 0;
                if (mode == 2) {
                    bns = explore_bin();
                    bnw = explore_bin();
                    used = 1;
                } else if (mode == 3) {
                    const unsigned sd = (unsigned)p_.seed;
                    bns = (int)(sd % MLP_NBIN);
                    bnw = (int)((sd / MLP_NBIN) % MLP_NBIN);
                    used = 1;
                } else if (!g_policy.theta.empty() && d.conf[0] >= g_policy.min_conf &&
                           d.conf[1] >= g_policy.min_conf) {
                    used = 1;
                }
                if (used) {
                    ns_next = kNsBins[bns];
                    nw_next = kNwBins[bnw];
                    stats_.policy_used++;
                } else {
                    stats_.policy_fallback++;
                }
                std::memcpy(pending.feat, d.feat, sizeof(pending.feat));
                pending.bins[0] = bns;
                pending.bins[1] = bnw;
                pending.m = (float)m2;
                pending.used_net = used;
                have_pending = true;
                if (mode == 4) {
                    held_set = true;
                    held_used = used;
                    held_bins[0] = bns;
                    held_bins[1] = bnw;
                }
            }
            if (nd > 0 && 100 * nd > nibble_ * nw) continue;
            int ns = default_ns(m2);
            if (ns_next > 0) {
                ns = std::min(ns_next, std::max(2, m2 / 3));
                ns = std::max(2, ns - ns % 2);
            }
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

    std::vector<PolicySample> policy_log_;

    // ---- eigenvalue reordering -----------------------------------------------
    // Move the eigenvalues flagged in sel (per diagonal position; a 2x2 block is
    // selected as a whole) to the leading diagonal block, keeping their order.
    // Windows of at most REORDER_WMAX rows: in each, the selected blocks go to
    // the window's top (k_reorder_window) and the window's factor is applied to
    // the rest of S and to Z by the update kernel.  Each window ends at the last
    // block of a group of selected blocks (the first one not yet in place and
    // those following it within a window, at most a third of a window of
    // rows) and reaches at most REORDER_WMAX rows up, so each window moves the
    // whole group up by most of a window.
    // Returns 0, or 1 when a swap was rejected (S, Z remain a valid Schur
    // decomposition, partly reordered).  *m = selected eigenvalues in place.
    int reorder(std::vector<int> sel, int *m_out) {
        const int n = n_;
        const int W = std::min(REORDER_WMAX, nsmall_);
        std::vector<char> nz(n + 1, 0);  // nz[i]: rows i-1, i form a 2x2 block
        {
            std::vector<double> g = gather(0, n - 1);
            for (int i = 1; i < n; ++i) nz[i] = g[n + i] != 0.0;
        }
        auto bsize = [&](int j) { return (j + 1 < n && nz[j + 1]) ? 2 : 1; };
        for (int j = 0; j < n;) {  // a pair is selected as a whole
            const int bs = bsize(j);
            const int v = (sel[j] || (bs == 2 && sel[j + 1])) ? 1 : 0;
            for (int t = 0; t < bs; ++t) sel[j + t] = v;
            j += bs;
        }
        int total = 0;
        for (int j = 0; j < n; ++j) total += sel[j];
        grow(&ws_.vt, &ws_.vt_cap, (size_t)W * W);
        // per-round window descriptors (device, with a pinned host mirror),
        // factors and statuses for up to kMaxWins concurrent windows
        const int kMaxWins = std::max(1, std::min(ws_.cus, 64));
        grow(&ws_.vt, &ws_.vt_cap, (size_t)kMaxWins * W * W);
        grow(&ws_.rwin, &ws_.rwin_cap, (size_t)kMaxWins);
        grow_host(&ws_.h_rwin, &ws_.h_rwin_cap, (size_t)kMaxWins);
        grow(&ws_.rstat, &ws_.rstat_cap, (size_t)2 * kMaxWins);
        grow_host(&ws_.h_rstat, &ws_.h_rstat_cap, (size_t)2 * kMaxWins);
        int placed = 0, info = 0;
        while (placed < total) {
            // one round: windows for successive groups of selected blocks, each
            // window ending at its group's last block and starting at most W rows
            // up but not above the previous window's end (windows never overlap)
            const int placed_before = placed;
            int nwin = 0, floor_row = placed, p = placed;
            while (nwin < kMaxWins) {
                while (p < n && !sel[p]) p += bsize(p);
                if (p >= n) break;
                const int bs = bsize(p);
                if (p == floor_row) {  // already in place behind the previous group
                    if (nwin == 0) placed += bs;
                    floor_row = p + bs;
                    p += bs;
                    continue;
                }
                int gend = p + bs, grows = bs, j = gend;
                while (j < n && grows < W / 3) {
                    const int bj = bsize(j);
                    if (j + bj - p > W) break;
                    if (sel[j]) {
                        gend = j + bj;
                        grows += bj;
                    }
                    j += bj;
                }
                int hi = gend;
                int lo = std::max(floor_row, hi - W);
                if (lo > floor_row && nz[lo]) ++lo;  // do not split the 2x2 block at lo-1, lo
                if (hi < n && nz[hi]) --hi;           // nor the one at hi-1, hi
                ReorderWin &rw = ws_.h_rwin[nwin++];
                rw.off = lo;
                rw.w = hi - lo;
                for (int t = 0; t < rw.w; ++t) rw.sel[t] = sel[lo + t];
                floor_row = hi;
                p = hi;
            }
            if (nwin == 0) {  // only blocks already in place were passed
                if (placed == placed_before) break;
                continue;
            }
            ck(hipMemcpyAsync(ws_.rwin, ws_.h_rwin, (size_t)nwin * sizeof(ReorderWin), hipMemcpyHostToDevice, st_));
            const size_t lds = (size_t)(2 * W * (W + 1)) * sizeof(double);
            timed(kSmall, [&] {
                hipLaunchKernelGGL(k_reorder_window, dim3(nwin), dim3(NT), lds, st_, H_, ldh_, ws_.rwin, ws_.vt, W,
                                   ws_.rstat);
                ck(hipGetLastError());
            });
            // left updates (rows of a window, columns right of it) touch rows the
            // right updates of later windows also touch in other columns: two launches
            std::vector<Task> left, right;
            for (int b = 0; b < nwin; ++b) {
                const ReorderWin &rw = ws_.h_rwin[b];
                const double *ut = ws_.vt + (size_t)b * W * W;
                const int lo = rw.off, hi = rw.off + rw.w - 1;
                if (hi + 1 < n) left.push_back({H_ + lo + (size_t)(hi + 1) * ldh_, ut, ldh_, W, rw.w, n - hi - 1, 0});
                if (lo > 0) right.push_back({H_ + (size_t)lo * ldh_, ut, ldh_, W, rw.w, lo, 1});
                right.push_back({Z_ + (size_t)lo * ldz_, ut, ldz_, W, rw.w, n, 1});
            }
            run_updates(left);
            run_updates(right);
            ck(hipMemcpyAsync(ws_.h_rstat, ws_.rstat, (size_t)2 * nwin * sizeof(int), hipMemcpyDeviceToHost, st_));
            const int glo = ws_.h_rwin[0].off, ghi = ws_.h_rwin[nwin - 1].off + ws_.h_rwin[nwin - 1].w - 1;
            std::vector<double> g = gather(glo, ghi);  // also waits for the status copy
            const int gm = ghi - glo + 1;
            for (int b = 0; b < nwin; ++b) {
                const ReorderWin &rw = ws_.h_rwin[b];
                const int k = ws_.h_rstat[2 * b];
                for (int t = 0; t < rw.w; ++t) {
                    sel[rw.off + t] = t < k ? 1 : 0;
                    if (t > 0) nz[rw.off + t] = g[gm + (rw.off + t - glo)] != 0.0;
                }
                if (ws_.h_rstat[2 * b + 1]) info = 1;
                stats_.small_solves++;
            }
            if (info) break;
            if (ws_.h_rwin[0].off == placed) placed += ws_.h_rstat[0];
        }
        *m_out = placed;
        return info;
    }

    // Standardise any 2x2 block not yet in standard form, then (wr, wi).
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

// ---------------------------------------------------------------- Hessenberg reduction

// Thin product out = (sum over splits of op(C) V - X B) T (X, T optional) with
// op(C) M x K, V K x nbc; the long dimension K is split so that the launch has
// about two workgroups per compute unit, but into at most 64 parts (the
// partials are summed by one workgroup per 64 rows).
void hrd_thin(DeviceWs &ws, double *sk, const double *C, int ldc, int trans, int M, int K, const double *V,
              int ldv, int nbc, const double *X, int ldx, const double *B, const double *T, double *out, int ldo,
              hipStream_t s) {
    if (M <= 0) return;
    const int rb = (M + 63) / 64;
    int nsplit = std::max(1, std::min({(2 * ws.cus + rb - 1) / rb, (K + 31) / 32, 64}));
    const int kper = ((K + nsplit - 1) / nsplit + 31) / 32 * 32;
    nsplit = (K + kper - 1) / kper;
    const size_t sp = (size_t)M * nbc;
    SkArgs a{C, V, sk, sp, ldc, ldv, M, K, nbc, kper, trans};
    if (trans)
        hipLaunchKernelGGL(k_hrd_skinny_t, dim3(rb, nsplit), dim3(HRD_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_hrd_skinny_n, dim3(rb, nsplit), dim3(HRD_THREADS), 0, s, a);
    RdArgs r{sk, sp, nsplit, X, ldx, B, T, out, ldo, M, nbc};
    hipLaunchKernelGGL(k_hrd_reduce, dim3(rb), dim3(HRD_THREADS), 0, s, r);
}

// C (M x N) -= L1 R1^T + L2 R2^T
void hrd_rank(double *C, int ldc, int M, int N, const double *L1, int ldl1, const double *R1, int ldr1, int r1,
              const double *L2, int ldl2, const double *R2, int ldr2, int r2, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    RkArgs a{C, L1, R1, L2, R2, ldc, ldl1, ldr1, ldl2, ldr2, M, N, r1, r2};
    hipLaunchKernelGGL(k_hrd_rank, dim3((M + 63) / 64, (N + 63) / 64), dim3(HRD_THREADS), 0, s, a);
}

// A (n x n) <- H = Q1^T A Q1 upper Hessenberg; Q <- Q Q1 when Q is given.
void hessenberg_run(int n, double *A, int lda, double *Q, int ldq, hipStream_t s) {
    DeviceWs &ws = workspace();
    if (n <= 2) return;
    const int NB = HRD_NB;
    const int ldw = (n + 7) & ~7;
    const size_t nrb_max = (size_t)(n + HRD_RB - 1) / HRD_RB;
    const size_t nch_max = (size_t)(n + HRD_GC - 1) / HRD_GC;
    const size_t sk_cap = ((size_t)128 * ws.cus + (size_t)n + 64) * NB;
    const size_t need = 4 * (size_t)ldw * NB + 2 * (size_t)NB * NB + nrb_max * (NB + 2) + nch_max * ldw + sk_cap;
    grow(&ws.hrd, &ws.hrd_cap, need);
    if (!ws.hrd_st) {
        ck(hipMalloc((void **)&ws.hrd_st, sizeof(HrdState)));
        ck(hipMemset(ws.hrd_st, 0, sizeof(HrdState)));
    }
    double *V = ws.hrd, *Y = V + (size_t)ldw * NB, *P = Y + (size_t)ldw * NB, *Mt = P + (size_t)ldw * NB;
    double *T = Mt + (size_t)ldw * NB, *Gt = T + (size_t)NB * NB;
    double *part = Gt + (size_t)NB * NB, *zpart = part + nrb_max * (NB + 2), *sk = zpart + nch_max * ldw;
    // the two workgroup counters start at zero (the last workgroup of every
    // column kernel resets its counter; this also clears them after an
    // interrupted call)
    ck(hipMemsetAsync(ws.hrd_st, 0, sizeof(HrdState), s));
    HrdArgs ha{A, V, Y, T, part, zpart, ws.hrd_st, lda, ldw, n, 0, 0, 0, 0, 0, HRD_GC};
    for (int k0 = 0; k0 < n - 2; k0 += NB) {
        const int jb = std::min(NB, n - 2 - k0);
        const int m = n - k0 - 1;
        const int nrb = (m + HRD_RB - 1) / HRD_RB;
        ha.k0 = k0;
        ha.m = m;
        ha.jb = jb;
        // wider GEMV chunks on large trailing blocks: fewer partial sums per row
        // while the grid still has thousands of workgroups
        ha.cw = m > 8192 ? HRD_GC_MAX : HRD_GC;
        int nch = 0;
        for (int i = 0; i <= jb; ++i) {
            ha.i = i;
            ha.nch = nch;
            if (i > 0) hipLaunchKernelGGL(k_hrd_a, dim3(nrb), dim3(HRD_THREADS), 0, s, ha);
            if (i == jb) break;
            hipLaunchKernelGGL(k_hrd_b, dim3(nrb), dim3(HRD_THREADS), 0, s, ha);
            nch = (m - i - 1 + ha.cw - 1) / ha.cw;
            hipLaunchKernelGGL(k_hrd_gemv, dim3((m + HRD_GR - 1) / HRD_GR, nch), dim3(HRD_THREADS), 0, s, ha);
        }
        const int nt = n - k0 - jb;  // trailing columns k0 + jb .. n-1
        double *Atop = A + (size_t)(k0 + 1) * lda;
        double *At = Atop + (size_t)(jb - 1) * lda + (k0 + 1);
        // Y(0:k0, :) = A(0:k0, k0+1:n) V T
        hrd_thin(ws, sk, Atop, lda, 0, k0 + 1, m, V, ldw, jb, nullptr, 0, nullptr, T, Y, ldw, s);
        // G^T = Y_low^T V;  Mt = (A_t^T V - V_t G^T) T
        hrd_thin(ws, sk, Y + k0 + 1, ldw, 1, jb, m, V, ldw, jb, nullptr, 0, nullptr, nullptr, Gt, NB, s);
        hrd_thin(ws, sk, At, lda, 1, nt, m, V, ldw, jb, V + (jb - 1), ldw, Gt, T, Mt, ldw, s);
        // A_t <- (I - V T V^T)^T (A_t - Y_low V_t^T) = A_t - Y_low V_t^T - V Mt^T
        hrd_rank(At, lda, m, nt, Y + k0 + 1, ldw, V + (jb - 1), ldw, jb, V, ldw, Mt, ldw, jb, s);
        // A(0:k0, k0+1:n) -= Y_top V^T
        hrd_rank(Atop, lda, k0 + 1, m, Y, ldw, V, ldw, jb, nullptr, 0, nullptr, 0, 0, s);
        if (Q) {
            // Q(:, k0+1:n) -= (Q(:, k0+1:n) V T) V^T
            double *Qc = Q + (size_t)(k0 + 1) * ldq;
            hrd_thin(ws, sk, Qc, ldq, 0, n, m, V, ldw, jb, nullptr, 0, nullptr, T, P, ldw, s);
            hrd_rank(Qc, ldq, n, m, P, ldw, V, ldw, jb, nullptr, 0, nullptr, 0, 0, s);
        }
    }
    ck(hipGetLastError());
}

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
        g_policy_log.swap(s.policy_log_);
        if (info == -2) return -2;
        s.eigenvalues(wr, wi);
        s.sync();
        g_stats = s.stats_;
        return info;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_reorder(int n, double *S, int lds, double *Z, int ldz, const int *select, double *wr, double *wi,
                            int *m, hipStream_t stream) {
    int a = check_args(n, S, lds, Z, ldz);
    if (a) return a;
    if (n > 0 && !select) return -6;
    if (n > 0 && !wr) return -7;
    if (n > 0 && !wi) return -8;
    if (!m) return -9;
    *m = 0;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        Solver s(n, S, lds, Z, ldz, stream);
        std::vector<int> sel(select, select + n);
        const int info = s.reorder(sel, m);
        s.eigenvalues(wr, wi);
        s.sync();
        g_stats = s.stats_;
        return info;
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
}

extern "C" int neig_hessenberg(int n, double *A, int lda, double *Q, int ldq, hipStream_t stream) {
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max(1, n)) return -3;
    if (Q && ldq < std::max(1, n)) return -5;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        hessenberg_run(n, A, lda, Q, ldq, stream);
        ck(hipStreamSynchronize(stream));
        return 0;
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
        if (nw > NEIG_AED_MAX) return -8;
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

namespace {

int check_batched_args(int batch, int cap, const int *n, double *const *H, const int *ldh, double *const *Z,
                       const int *ldz, double *const *wr, double *const *wi, int *info) {
    if (batch < 0 || batch > cap) return -1;
    if (batch == 0) return 0;
    if (!n) return -2;
    if (!H) return -3;
    if (!ldh) return -4;
    if (!Z) return -5;
    if (!ldz) return -6;
    if (!wr) return -7;
    if (!wi) return -8;
    if (!info) return -9;
    return 0;
}

// The launch pair of the batched solver: descriptors, order and counter live in
// the buffers the caller of this function provides (library workspace, or the
// fixed array of the no-allocation entry point).
void launch_batched_pair(int batch, const int *n, double *const *H, const int *ldh, double *const *Z,
                         const int *ldz, double *const *wr, double *const *wi, int *info, BProb *probs, int *order,
                         int *next, int small_max, int chase_max, int cus, hipStream_t stream) {
    hipLaunchKernelGGL(k_batched_pack, dim3((batch + 255) / 256), dim3(256), 0, stream, probs, order, next, info, n,
                       ldh, ldz, H, Z, wr, wi, batch);
    ck(hipGetLastError());
    BArgs A;
    std::memset(&A, 0, sizeof(A));
    A.probs = probs;
    A.order = order;
    A.nprob = batch;
    A.next = next;
    A.info = info;
    for (int k = 0; k < B_NBUCKET; ++k) {
        A.bucket_hi[k] = g_btab.hi[k];
        A.tune[k] = g_btab.t[k];
        A.tune[k].nw = std::min(A.tune[k].nw, small_max);
        A.tune[k].nmin = std::min(A.tune[k].nmin, small_max);
        A.tune[k].wchase = std::min(A.tune[k].wchase, chase_max);
        A.tune[k].ns = std::min(A.tune[k].ns, 2 * B_MAX_BULGES);
    }
    A.criterion = g_params.deflation;
    A.nibble = g_params.nibble > 0 ? g_params.nibble : 14;
    A.exc = g_params.exc > 0 ? g_params.exc : 6;
    A.maxit_factor = 30;
    const int grid = std::max(1, std::min(batch, cus > 0 ? cus : 256));
    const size_t lds = (size_t)(NEIG_CHASE_MAX + 1) * (NEIG_CHASE_MAX + 2) * sizeof(double) +
                       (size_t)NEIG_CHASE_MAX * (NEIG_CHASE_MAX + 1) * sizeof(double);
    hipLaunchKernelGGL(k_batched, dim3(grid), dim3(NT), lds, stream, A);
    ck(hipGetLastError());
}

}  // namespace

extern "C" int neig_aed_top(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nw, int *nd,
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
        std::vector<Eig> unused, ritz;
        int ndt = 0;
        s.aed_ends(ktop, kbot, 0, nw, unused, ritz, &ndt);
        *nd = ndt;
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
    const int a = check_batched_args(batch, NEIG_BATCH_MAX, n, H, ldh, Z, ldz, wr, wi, info);
    if (a || batch == 0) return a;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        DeviceWs &ws = workspace();
        launch_batched_pair(batch, n, H, ldh, Z, ldz, wr, wi, info, ws.bprob, ws.border, ws.bnext, ws.small_max,
                            ws.chase_max, ws.cus, stream);
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

extern "C" int neig_batched_flops(double *flops) {
    if (!flops) return -1;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        DeviceWs &ws = workspace();
        ck(hipDeviceSynchronize());
        ck(hipMemcpy(flops, ws.bnext + 2, sizeof(double), hipMemcpyDeviceToHost));
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

// ---------------------------------------------------------------- no-allocation batched entry
//
// The descriptor table, order and work counter of neig_schur_batched_noalloc
// live in this fixed device array.  In host code its name is only a stand-in for
// the symbol: the device address of each GPU's copy comes from
// hipGetSymbolAddress, once per device, and only that address is passed on.
namespace {
constexpr size_t kNaOrderOff = ((size_t)NEIG_BATCH_NOALLOC_MAX * sizeof(BProb) + 255) & ~(size_t)255;
constexpr size_t kNaNextOff = kNaOrderOff + (((size_t)NEIG_BATCH_NOALLOC_MAX * sizeof(int) + 255) & ~(size_t)255);
constexpr size_t kNaBytes = kNaNextOff + 256;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

struct NoAllocDev {
    bool ready = false;
    unsigned char *ptr = nullptr;  // device address of this GPU's scratch
    int small_max = 0, chase_max = 0, cus = 0;
};
NoAllocDev g_na[kMaxDevices];

// Set-up on the current device (no allocation): the scratch address, the LDS
// limits and the compute-unit count.
NoAllocDev &noalloc_device() {
    int dev = 0;
    ck(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw HipFail{hipErrorInvalidDevice};
    NoAllocDev &d = g_na[dev];
    if (d.ready) return d;
    void *ptr = nullptr;
    ck(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    const DevLimits lim = device_limits(dev);
    allow_dynamic_lds((const void *)k_batched, lim.lds_max);
    d.ptr = (unsigned char *)ptr;
    d.small_max = lim.small_max;
    d.chase_max = lim.chase_max;
    d.cus = lim.cus;
    d.ready = true;
    return d;
}

}  // namespace

extern "C" int neig_schur_batched_noalloc(int batch, const int *n, double *const *H, const int *ldh,
                                          double *const *Z, const int *ldz, double *const *wr, double *const *wi,
                                          int *info, hipStream_t stream) {
    const int a = check_batched_args(batch, NEIG_BATCH_NOALLOC_MAX, n, H, ldh, Z, ldz, wr, wi, info);
    if (a || batch == 0) return a;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        NoAllocDev &d = noalloc_device();
        launch_batched_pair(batch, n, H, ldh, Z, ldz, wr, wi, info, (BProb *)d.ptr, (int *)(d.ptr + kNaOrderOff),
                            (int *)(d.ptr + kNaNextOff), d.small_max, d.chase_max, d.cus, stream);
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

static_assert(B_NBUCKET == NEIG_BATCH_CLASSES, "size classes of the batched solver");

extern "C" int neig_set_batched_tune(int nclass, const int *n_hi, const int *nw, const int *ns, const int *nmin,
                                     const int *chase_w) {
    if (nclass < 1 || nclass > B_NBUCKET) return -1;
    if (!n_hi) return -2;
    if (!nw) return -3;
    if (!ns) return -4;
    if (!nmin) return -5;
    if (!chase_w) return -6;
    for (int k = 0; k < nclass; ++k) {
        if (k > 0 && k < nclass - 1 && n_hi[k] <= n_hi[k - 1]) return -2;
        if (nw[k] < 2 || nw[k] > NEIG_SMALL_MAX) return -3;
        if (ns[k] < 2 || ns[k] % 2 || ns[k] > 2 * B_MAX_BULGES) return -4;
        if (nmin[k] < 2 || nmin[k] > NEIG_SMALL_MAX) return -5;
        if (chase_w[k] < 3 * (ns[k] / 2) + 2 || chase_w[k] > NEIG_CHASE_MAX) return -6;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    BatchTable t;
    for (int k = 0; k < B_NBUCKET; ++k) {
        const int src = std::min(k, nclass - 1);
        t.hi[k] = k < nclass - 1 ? n_hi[k] : (1 << 30);
        t.t[k] = {nw[src], ns[src], nmin[src], chase_w[src]};
    }
    g_btab = t;
    return 0;
}

extern "C" int neig_get_batched_tune(int *nclass, int *n_hi, int *nw, int *ns, int *nmin, int *chase_w) {
    if (!nclass) return -1;
    if (!n_hi) return -2;
    if (!nw) return -3;
    if (!ns) return -4;
    if (!nmin) return -5;
    if (!chase_w) return -6;
    std::lock_guard<std::mutex> lock(g_mutex);
    *nclass = B_NBUCKET;
    for (int k = 0; k < B_NBUCKET; ++k) {
        n_hi[k] = g_btab.hi[k];
        nw[k] = g_btab.t[k].nw;
        ns[k] = g_btab.t[k].ns;
        nmin[k] = g_btab.t[k].nmin;
        chase_w[k] = g_btab.t[k].wchase;
    }
    return 0;
}

static_assert(MLP_NPARAM == NEIG_MLP_NPARAM, "network parameter count");

extern "C" int neig_policy_bins(int *ns_bins, int *nw_bins) {
    if (!ns_bins) return -1;
    if (!nw_bins) return -2;
    for (int k = 0; k < MLP_NBIN; ++k) {
        ns_bins[k] = kNsBins[k];
        nw_bins[k] = kNwBins[k];
    }
    return 0;
}

extern "C" int neig_policy_set(const float *theta, int nparam, float min_conf) {
    if (theta && nparam != MLP_NPARAM) return -1;
    if (!(min_conf >= 0.0f && min_conf <= 1.0f)) return -3;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (theta) g_policy.theta.assign(theta, theta + MLP_NPARAM);
    else g_policy.theta.clear();
    g_policy.min_conf = min_conf;
    g_policy.version++;
    return 0;
}

extern "C" int neig_policy_log(int cap, float *feat, int *bins, float *stats) {
    std::lock_guard<std::mutex> lock(g_mutex);
    const int count = (int)g_policy_log.size();
    const int k = std::min(std::max(cap, 0), count);
    for (int i = 0; i < k; ++i) {
        const PolicySample &q = g_policy_log[i];
        if (feat) std::memcpy(feat + (size_t)MLP_NIN * i, q.feat, sizeof(q.feat));
        if (bins) {
            bins[2 * i] = q.bins[0];
            bins[2 * i + 1] = q.bins[1];
        }
        if (stats) {
            stats[4 * i] = q.nd;
            stats[4 * i + 1] = q.ms;
            stats[4 * i + 2] = q.m;
            stats[4 * i + 3] = (float)q.used_net;
        }
    }
    return count;
}

extern "C" int neig_policy_features(int n, const double *H, int ldh, int ktop, int kbot, double hnorm,
                                    const float *extra, float *feat, int *bins, float *conf, hipStream_t stream) {
    if (n < 1) return -1;
    if (!H) return -2;
    if (ldh < n) return -3;
    if (ktop < 0 || ktop >= n) return -4;
    if (kbot < ktop || kbot >= n) return -5;
    if (!(hnorm >= 0.0)) return -6;
    if (!extra) return -7;
    if (!feat) return -8;
    if (!bins) return -9;
    if (!conf) return -10;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        DeviceWs &ws = workspace();
        Solver s(n, const_cast<double *>(H), ldh, nullptr, n, stream);
        s.upload_policy();
        float *out = ws.pol_out;
        hipLaunchKernelGGL(k_policy, dim3(1), dim3(256), 0, stream, H, ldh, n, ktop, kbot, hnorm, extra[0], extra[1],
                           extra[2], extra[3], ws.theta, out, (int *)(out + MLP_NIN), out + MLP_NIN + 2);
        ck(hipGetLastError());
        ck(hipMemcpyAsync(ws.h_pol_out, out, (MLP_NIN + 4) * sizeof(float), hipMemcpyDeviceToHost, stream));
        ck(hipStreamSynchronize(stream));
        std::memcpy(feat, ws.h_pol_out, MLP_NIN * sizeof(float));
        std::memcpy(bins, ws.h_pol_out + MLP_NIN, 2 * sizeof(int));
        std::memcpy(conf, ws.h_pol_out + MLP_NIN + 2, 2 * sizeof(float));
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

extern "C" int neig_mlp_grad(int batch, const float *X, const int *a, const int *c, const float *w,
                             const float *theta, float *grad, float *loss, hipStream_t stream) {
    if (batch < 1) return -1;
    if (!X) return -2;
    if (!a) return -3;
    if (!c) return -4;
    if (!w) return -5;
    if (!theta) return -6;
    if (!grad) return -7;
    if (!loss) return -8;
    std::lock_guard<std::mutex> lock(g_mutex);
    try {
        DeviceWs &ws = workspace();
        const int nblk = (batch + MLP_TILE - 1) / MLP_TILE;
        grow(&ws.mlp_part, &ws.mlp_part_cap, (size_t)nblk * (MLP_NPARAM + 1));
        float *lossp = ws.mlp_part + (size_t)nblk * MLP_NPARAM;
        hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, stream, theta, X, a, c, w, batch,
                           1.0f / (float)batch, ws.mlp_part, lossp);
        ck(hipGetLastError());
        hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, stream, ws.mlp_part,
                           lossp, nblk, grad, loss);
        ck(hipGetLastError());
    } catch (const HipFail &f) {
        return -100 - (int)f.e;
    }
    return 0;
}

extern "C" int neig_mlp_adam(float *theta, const float *grad, float *m, float *v, int step, float lr,
                             hipStream_t stream) {
    if (!theta) return -1;
    if (!grad) return -2;
    if (!m) return -3;
    if (!v) return -4;
    if (step < 1) return -5;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, step)), bc2 = (float)(1.0 - std::pow(b2, step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, stream, theta, grad, m, v, lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, bc1, bc2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : -100 - (int)e;
}

extern "C" int neig_mlp_infer(int batch, const float *X, const float *theta, float *logits, int *bins, float *conf,
                              hipStream_t stream) {
    if (batch < 1) return -1;
    if (!X) return -2;
    if (!theta) return -3;
    if (!logits) return -4;
    if (!bins) return -5;
    if (!conf) return -6;
    const int grid = std::min((batch + 3) / 4, 1024);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, stream, theta, X, batch, logits, bins, conf);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : -100 - (int)e;
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
    if (p->timing < 0 || p->timing > 1) return -10;
    if (p->policy < 0 || p->policy > 4) return -11;
    if (p->nw > NEIG_AED_MAX) return -2;
    if (p->rec_nw < 0 || p->rec_nw > NEIG_SMALL_MAX) return -13;
    if (p->rec_ns < 0 || p->rec_ns % 2) return -14;
    if (p->aed_ends < 0 || p->aed_ends > 1) return -15;
    if (p->overlap < 0 || p->overlap > 2) return -16;
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
