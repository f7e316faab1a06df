// C ABI of the IPT library: handles, argument checks, workspace, and the host loop
// that launches the sweeps of Alg. 1 / Alg. 2 on one stream.  Every step of a
// sweep runs in the device kernels; the host only launches and, every
// sync_every sweeps, reads the device stop flag.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ipt_internal.h"

using namespace ipt;

// Workspace of ipt_solve_dense_noalloc: one copy per device, held until the process
// ends.  Host code never passes this name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address that hipGetSymbolAddress
// returned for the device, kept in g_scratch_ptr by ipt_create.
__device__ __align__(256) unsigned char scratch[IPT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Called by ipt_create with the handle's device current.
hipError_t init_scratch(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return hipSuccess;  // the no-allocation solve then refuses
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

struct ipt_context {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *pws = nullptr;  // near-degenerate pair rotation: rotated copies of the inputs
    size_t pws_bytes = 0;
    Ctrl *host_ctrl = nullptr;  // pinned copy of the control block
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    std::vector<hipEvent_t> tev;  // kernel-timing events (IPT_FLAG_TIME_KERNELS), reused across solves
    // batched solves: tile size per size bucket (bucket q holds 64q < n <= 64(q + 1))
    int32_t batch_tile[IPT_TILE_BUCKETS];
    hipStream_t cap_stream = nullptr;          // capture-only stream for the batched sweep graph
    hipGraphExec_t bgraph = nullptr;           // instantiated chunk of batched sweeps
    std::vector<unsigned char> bgraph_key;     // the launch arguments it was captured with
    int32_t *poll_host = nullptr;              // pinned [2][2]: error/done words of two polls in flight
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    // debug mode (IPT_GUARD at ipt_create): guard bands of the running solve's workspace
    bool guard = false, guard_poke = false, guard_armed = false;
    std::vector<size_t> bands;                 // byte offsets of the bands from guard_base
    char *guard_base = nullptr;
    void *band_mem = nullptr;                  // device copy of the offsets, then the damage word
    size_t band_bytes = 0;
    ipt_context() {
        for (int q = 0; q < IPT_TILE_BUCKETS; ++q) batch_tile[q] = q < 3 ? 64 : 128;
    }
    std::string last_error;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

ipt_status fail(ipt_handle h, ipt_status st, const std::string &msg) {
    if (h) h->last_error = msg;
    return st;
}

#define IPT_HIP(h, expr)                                                                              \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return fail((h), IPT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Bump allocator over the handle's workspace (256-byte aligned slices).  In the debug
// mode every slice is followed by a guard band (and one precedes the first); the pass
// with a base records where the bands are.
constexpr size_t GUARD_BYTES = 4096;
struct Carve {
    size_t off = 0;
    char *base = nullptr;
    size_t gbytes = 0;
    std::vector<size_t> *bands = nullptr;
    void band() {
        if (!gbytes) return;
        off = (off + 255) & ~size_t(255);
        if (bands) bands->push_back(off);
        off += gbytes;
    }
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        band();
        return p;
    }
};

ipt_status ensure_buf(ipt_handle h, void *&buf, size_t &have, size_t bytes) {
    if (bytes <= have) return IPT_OK;
    IPT_HIP(h, hipStreamSynchronize(h->stream));
    if (buf) IPT_HIP(h, hipFree(buf));
    buf = nullptr;
    have = 0;
    size_t want = bytes + bytes / 8;  // head-room for slightly larger follow-up solves
    hipError_t e = hipMalloc(&buf, want);
    if (e != hipSuccess) {
        want = bytes;
        e = hipMalloc(&buf, want);
    }
    if (e != hipSuccess) {
        buf = nullptr;
        (void)hipGetLastError();
        return fail(h, IPT_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    have = want;
    return IPT_OK;
}

ipt_status ensure_ws(ipt_handle h, size_t bytes) { return ensure_buf(h, h->ws, h->ws_bytes, bytes); }

// A workspace carve for handle h: base NULL for the sizing pass.  Guard bands only in
// the debug mode and where the solve may allocate (the no-allocation solve has none).
Carve carve(ipt_handle h, char *base, bool guarded = true) {
    Carve c;
    c.base = base;
    if (h->guard && guarded) {
        c.gbytes = GUARD_BYTES;
        if (base) {
            h->bands.clear();
            c.bands = &h->bands;
        }
        c.band();
    }
    return c;
}

// Debug mode: fill the bands of the carve just laid out with the guard pattern (and,
// in the self-test mode, overwrite 8 bytes of the second band from the host, as a
// kernel writing past the first slice would).  Stream-ordered before the solve.
ipt_status guard_arm(ipt_handle h, const Carve &cv) {
    h->guard_armed = false;
    if (!cv.bands || h->bands.empty()) return IPT_OK;
    const size_t nb = h->bands.size(), list_bytes = round_up(nb * sizeof(uint64_t), 256);
    if (ipt_status st = ensure_buf(h, h->band_mem, h->band_bytes, list_bytes + 256)) return st;
    uint64_t *list = (uint64_t *)h->band_mem;
    int32_t *damage = (int32_t *)((char *)h->band_mem + list_bytes);
    IPT_HIP(h, hipMemcpyAsync(list, h->bands.data(), nb * sizeof(uint64_t), hipMemcpyHostToDevice, h->stream));
    IPT_HIP(h, launch_guard_fill(h->stream, cv.base, list, (int64_t)nb, (int64_t)(GUARD_BYTES / 8), damage));
    if (h->guard_poke && nb > 1) IPT_HIP(h, hipMemsetAsync(cv.base + h->bands[1] + 64, 0, 8, h->stream));
    IPT_HIP(h, hipStreamSynchronize(h->stream));  // the host list may change with the next solve
    h->guard_base = cv.base;
    h->guard_armed = true;
    return IPT_OK;
}

// Debug mode, after the solve's last kernel: IPT_EGUARD names the first damaged band.
ipt_status guard_check(ipt_handle h) {
    if (!h->guard_armed) return IPT_OK;
    h->guard_armed = false;
    const size_t nb = h->bands.size(), list_bytes = round_up(nb * sizeof(uint64_t), 256);
    const uint64_t *list = (const uint64_t *)h->band_mem;
    int32_t *damage = (int32_t *)((char *)h->band_mem + list_bytes);
    IPT_HIP(h, launch_guard_check(h->stream, h->guard_base, list, (int64_t)nb, (int64_t)(GUARD_BYTES / 8), damage));
    int32_t bad = 0;
    IPT_HIP(h, hipMemcpyAsync(&bad, damage, sizeof(bad), hipMemcpyDeviceToHost, h->stream));
    IPT_HIP(h, hipStreamSynchronize(h->stream));
    if (bad == INT32_MAX) return IPT_OK;
    return fail(h, IPT_EGUARD,
                "workspace guard band " + std::to_string(bad) + " (byte offset " + std::to_string(h->bands[bad]) +
                    ") was overwritten: a kernel wrote past the end of slice " + std::to_string(bad - 1));
}

ipt_status check_opts(ipt_handle h, const ipt_opts *in, ipt_opts &o) {
    ipt_opts_default(&o);
    if (in) o = *in;
    if (!(o.tol >= 0.0) || !isfinite(o.tol)) return fail(h, IPT_EINVAL, "opts.tol must be finite and >= 0");
    if (o.max_iter < 1 || o.max_iter > 100000) return fail(h, IPT_EINVAL, "opts.max_iter must be in [1, 100000]");
    if (o.precision != IPT_PREC_FP64 && o.precision != IPT_PREC_LADDER)
        return fail(h, IPT_EINVAL, "opts.precision must be IPT_PREC_FP64 or IPT_PREC_LADDER");
    if (o.low_type < IPT_LOW_BF16 || o.low_type > IPT_LOW_NONE) return fail(h, IPT_EINVAL, "opts.low_type invalid");
    if (o.sync_every < 0) return fail(h, IPT_EINVAL, "opts.sync_every must be >= 0");
    if (!(o.div_norm > 0.0)) return fail(h, IPT_EINVAL, "opts.div_norm must be > 0");
    if (o.div_growth < 1) return fail(h, IPT_EINVAL, "opts.div_growth must be >= 1");
    if (!(o.tau_low >= 0.0) || !(o.tau_32 >= 0.0)) return fail(h, IPT_EINVAL, "opts.tau_low/tau_32 must be >= 0");
    if ((o.flags & IPT_FLAG_ACX) && o.precision != IPT_PREC_FP64)
        return fail(h, IPT_EINVAL, "IPT_FLAG_ACX runs FP64 sweeps: set precision = IPT_PREC_FP64");
    if (!(o.cont_alpha >= 0.0 && o.cont_alpha < 1.0))
        return fail(h, IPT_EINVAL, "opts.cont_alpha must be in [0, 1)");
    if (o.cont_alpha > 0.0 && (o.precision != IPT_PREC_FP64 || (o.flags & IPT_FLAG_ACX)))
        return fail(h, IPT_EINVAL, "opts.cont_alpha needs precision = IPT_PREC_FP64 and no IPT_FLAG_ACX");
    if (o.homotopy_q < 0 || o.homotopy_q > 1000) return fail(h, IPT_EINVAL, "opts.homotopy_q must be in [0, 1000]");
    if (o.homotopy_q > 1 && o.cont_alpha > 0.0)
        return fail(h, IPT_EINVAL, "opts.homotopy_q and opts.cont_alpha do not combine");
    return IPT_OK;
}

DevOpts dev_opts(const ipt_opts &o) {
    DevOpts d;
    memset(&d, 0, sizeof(d));  // padding too: batched graphs are keyed on the argument bytes
    d.tol = o.tol;
    d.tau_low = o.tau_low;
    d.tau_32 = o.tau_32;
    d.div_norm = o.div_norm;
    d.cont_alpha = o.cont_alpha;
    d.max_iter = o.max_iter;
    d.div_growth = o.div_growth;
    d.ladder = o.precision == IPT_PREC_LADDER;
    d.low_type = o.low_type;
    d.first_product = 0;
    d.acx = (o.flags & IPT_FLAG_ACX) ? 1 : 0;
    d.mid_x3 = (d.ladder && !(o.flags & IPT_FLAG_MID_FP32)) ? 1 : 0;  // the dense GEMM's FP32-class rung
    return d;
}

void fill_info(const Ctrl &c, ipt_info *info, float ms) {
    if (!info) return;
    memset(info, 0, sizeof(*info));
    info->sweeps = c.sweeps;
    info->converged = c.n_conv;
    info->not_converged = c.n_notconv;
    info->diverged = c.n_div;
    info->matvecs = c.matvecs;
    uint64_t b;
    double v;
    b = c.dec_maxstep;
    memcpy(&v, &b, 8);
    info->max_step = v;
    b = c.norm1_bits;
    memcpy(&v, &b, 8);
    info->norm1 = v;
    b = c.acc_maxres;
    memcpy(&v, &b, 8);
    info->max_resid = v;
    info->time_ms = ms;
    info->hist_len = c.sweeps < IPT_HIST ? c.sweeps : IPT_HIST;
    for (int q = 0; q < info->hist_len; ++q) {
        info->sweep_prec[q] = c.hist_prec[q];
        info->sweep_active[q] = c.hist_active[q];
        info->sweep_max_step[q] = c.hist_step[q];
    }
}

// Kernel timing: one pair of events brackets the product launch of each sweep;
// the time is attributed to the sweep's precision through hist_prec.
struct Timer {
    ipt_handle h;
    bool on;
    int max_iter;
    hipError_t ensure() {
        if (!on) return hipSuccess;
        const size_t want = (size_t)(max_iter < IPT_HIST ? max_iter : IPT_HIST) * 2;
        while (h->tev.size() < want) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            h->tev.push_back(e);
        }
        return hipSuccess;
    }
    hipError_t mark(int32_t t, int end, hipStream_t s) {
        if (!on || t - 1 >= IPT_HIST) return hipSuccess;
        return hipEventRecord(h->tev[(size_t)(t - 1) * 2 + end], s);
    }
    void collect(const Ctrl &c, ipt_info *info) {
        if (!on || !info) return;
        const int hl = c.sweeps < IPT_HIST ? c.sweeps : IPT_HIST;
        for (int t = 1; t <= hl; ++t) {
            const int q = c.hist_prec[t - 1];
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h->tev[(size_t)(t - 1) * 2], h->tev[(size_t)(t - 1) * 2 + 1]) == hipSuccess) {
                info->prec_ms[q] += ms;
                info->prec_sweeps[q] += 1;
                info->sweep_ms[t - 1] = ms;
            }
        }
    }
};

// Host polling of the device stop flag: after the first `first` sweeps, then every
// `every` sweeps, and always at max_iter.  Sweeps launched after the device has
// set its done flag return at once.
struct PollPlan {
    int first, every;
    bool at(int t, int max_iter) const { return t == max_iter || t == first || (t > first && (t - first) % every == 0); }
};

PollPlan poll_plan(const ipt_opts &o, bool cold) {
    if (o.sync_every > 0) return PollPlan{o.sync_every, o.sync_every};
    // A cold start certifies after about four sweeps on well-separated spectra.
    return PollPlan{cold ? 4 : 3, 1};
}

// IPT_LOG set (and not "0") in the environment: every solve prints a summary line and
// one line per sweep to stderr, from the history the device keeps (nothing is added
// to the solve itself; the lines are written after its final synchronisation).
bool log_enabled() {
    const char *e = getenv("IPT_LOG");  // read at every solve, so it can be switched at run time
    return e && *e && strcmp(e, "0") != 0;
}

void log_solve(const char *kind, int64_t k, const ipt_info &inf, ipt_status st, bool timed) {
    static const char *prec_name[4] = {"exact-first", "low", "fp32", "fp64"};
    fprintf(stderr,
            "[ipt] %s: columns=%lld status=%s sweeps=%d converged=%d not_converged=%d diverged=%d matvecs=%lld "
            "max_step=%.3e max_resid=%.3e norm1=%.6e time_ms=%.3f\n",
            kind, (long long)k, st == IPT_OK ? "IPT_OK" : "IPT_ENOTCONV", inf.sweeps, inf.converged, inf.not_converged, inf.diverged,
            (long long)inf.matvecs, inf.max_step, inf.max_resid, inf.norm1, inf.time_ms);
    for (int q = 0; q < inf.hist_len; ++q) {
        const int p = inf.sweep_prec[q];
        fprintf(stderr, "[ipt] %s sweep %d: %s active=%d max_step=%.3e", kind, q + 1,
                (p >= 0 && p < 4) ? prec_name[p] : "?", inf.sweep_active[q], inf.sweep_max_step[q]);
        if (timed) fprintf(stderr, " product_ms=%.4f", inf.sweep_ms[q]);
        fputc('\n', stderr);
    }
    fflush(stderr);
}

// End of a solve: wait for it, turn device errors into status codes, fill *info.
// maxres_dev (batched solves): the max residual the copy-out reduced on the device.
ipt_status finish(ipt_handle h, Ctrl *dev, int64_t k, ipt_info *info, Timer *timer, const char *kind,
                  const double *maxres_dev, const uint64_t *norm_bits_dev = nullptr) {
    IPT_HIP(h, hipEventRecord(h->ev_stop, h->stream));
    IPT_HIP(h, hipMemcpyAsync(h->host_ctrl, dev, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    IPT_HIP(h, hipStreamSynchronize(h->stream));
    float ms = 0.f;
    IPT_HIP(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
    if (ipt_status st = guard_check(h)) return st;
    const Ctrl &c = *h->host_ctrl;
    if (c.error == IPT_EDEGENERATE)
        return fail(h, IPT_EDEGENERATE, "theta_j == theta_idx[c] for some j != idx[c]: inverse gap undefined");
    if (c.error) return fail(h, IPT_EINVAL, "idx out of range or repeated, or theta not finite");
    const bool logging = log_enabled();
    ipt_info local;
    ipt_info *out = info ? info : (logging ? &local : nullptr);
    fill_info(c, out, ms);
    if (timer) timer->collect(c, out);
    if (out && maxres_dev) {
        double mr = 0.0, nm = 0.0;
        IPT_HIP(h, hipMemcpy(&mr, maxres_dev, sizeof(double), hipMemcpyDeviceToHost));
        if (norm_bits_dev) IPT_HIP(h, hipMemcpy(&nm, norm_bits_dev, sizeof(double), hipMemcpyDeviceToHost));
        out->max_resid = mr;
        out->norm1 = nm;  // a batch of one problem reports its |M|_1
    }
    const ipt_status st = (c.n_conv == k) ? IPT_OK : IPT_ENOTCONV;
    if (logging) log_solve(kind, k, *out, st, timer && timer->on);
    if (st == IPT_OK) return IPT_OK;
    h->last_error = "some columns did not converge";
    return IPT_ENOTCONV;
}

// ------------------------------------------------------------- batched
ipt_status ensure_poll(ipt_handle h) {
    if (h->poll_host) return IPT_OK;
    IPT_HIP(h, hipEventCreateWithFlags(&h->poll_ev[0], hipEventDisableTiming));
    IPT_HIP(h, hipEventCreateWithFlags(&h->poll_ev[1], hipEventDisableTiming));
    IPT_HIP(h, hipHostMalloc((void **)&h->poll_host, 4 * sizeof(int32_t), hipHostMallocDefault));
    return IPT_OK;
}

// Look-ahead polling of the device stop words: each poll enqueues a copy of them
// and then waits for the previous poll's copy, so the sweeps launched in between
// keep the device busy (sweeps launched after the device stopped return at once).
// The first poll, placed where the solve is expected to stop, waits for itself.
struct LookaheadPoll {
    ipt_handle h;
    const Ctrl *ctrl;
    int pend = -1, slot = 0;
    bool first = true;
    ipt_status push(bool &stop) {
        stop = false;
        IPT_HIP(h, hipMemcpyAsync(h->poll_host + 2 * slot, ctrl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        IPT_HIP(h, hipEventRecord(h->poll_ev[slot], h->stream));
        const int wait = first ? slot : pend;
        first = false;
        if (wait >= 0) {
            IPT_HIP(h, hipEventSynchronize(h->poll_ev[wait]));
            stop = h->poll_host[2 * wait] != 0 || h->poll_host[2 * wait + 1] != 0;
        }
        pend = (wait == slot) ? -1 : slot;
        slot ^= 1;
        return IPT_OK;
    }
};

// Everything a captured chunk of batched sweeps depends on; the graph is reused
// while these bytes are unchanged.
struct BatchGraphKey {
    BatchLaunch L;
    BatchLists lists;
    DevOpts dopt;
    Ctrl *ctrl;
    int64_t total_cols;
    int32_t grid[NCLS], has[NCLS], chunk;
};

template <typename F>
ipt_status ensure_batch_graph(ipt_handle h, const BatchGraphKey &key, F capture) {
    const unsigned char *kb = (const unsigned char *)&key;
    std::vector<unsigned char> want(kb, kb + sizeof(key));
    if (h->bgraph && h->bgraph_key == want) return IPT_OK;
    if (h->bgraph) {
        IPT_HIP(h, hipGraphExecDestroy(h->bgraph));
        h->bgraph = nullptr;
    }
    if (!h->cap_stream) IPT_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    IPT_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    const hipError_t e1 = capture(h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(h, IPT_EHIP, std::string("capture of the batched sweep graph failed: ") +
                                     hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&h->bgraph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        h->bgraph = nullptr;
        return fail(h, IPT_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    h->bgraph_key = want;
    return IPT_OK;
}

// The batched solve; force_T != 0 gives every problem that tile size (autotuner).
ipt_status batched_run(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                       const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                       const double *delta_pool, const ipt_opts &o, double *z_pool, double *lambda_pool,
                       int32_t *status_pool, ipt_info *info, int force_T, const ipt_colinfo *ci = nullptr) {
    if (count < 1) return fail(h, IPT_EINVAL, "count must be >= 1");
    if (!ns || !theta_off || !delta_off || !z_off || !theta_pool || !delta_pool || !z_pool || !lambda_pool ||
        !status_pool)
        return fail(h, IPT_EINVAL, "NULL argument");
    DevOpts dopt = dev_opts(o);
    dopt.low_type = IPT_LOW_NONE;  // batched ladder: FP32 split-form sweeps, then FP64
    dopt.mid_x3 = 0;
    const bool ladder = dopt.ladder, acx = dopt.acx != 0;
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;

    // Host plan: problems laid out largest first (so the work lists the finalize
    // appends run roughly largest first), tile size per size bucket.
    std::vector<int32_t> order(count);
    for (int32_t b = 0; b < count; ++b) {
        if (ns[b] < 1 || ns[b] > 4096) return fail(h, IPT_EINVAL, "every problem size must be in [1, 4096]");
        if (theta_off[b] < 0 || delta_off[b] < 0 || z_off[b] < 0) return fail(h, IPT_EINVAL, "negative offset");
        order[b] = b;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return ns[x] > ns[y]; });
    std::vector<BatchMeta> meta(count);
    std::vector<int4> it_s1;
    int64_t offz = 0, offc = 0, offp = 0, offq = 0, offf = 0, cap[NCLS] = {0, 0, 0, 0}, capx[NCLS][NXCD] = {};
    double load[3][NXCD] = {};
    for (int32_t b : order) {
        const int64_t n = ns[b];
        const int T = force_T ? force_T : h->batch_tile[(n - 1) / 64];
        const int64_t np = round_up(n, T), nt = np / T, ncb = (np + 63) / 64;
        const int cl = T == 32 ? 0 : (T == 64 ? 1 : 2);
        // deal the problem to the least loaded die of its class (work ~ np^3)
        int x = 0;
        for (int y = 1; y < NXCD; ++y)
            if (load[cl][y] < load[cl][x]) x = y;
        load[cl][x] += (double)np * np * np;
        BatchMeta &m = meta[b];
        m.n = (int32_t)n;
        m.T = T;
        m.np = (int32_t)np;
        m.xcd = x;
        capx[cl][x] += nt * nt;
        m.offd = delta_off[b];
        m.offt = theta_off[b];
        m.offo = z_off[b];
        m.offz = offz;
        m.offc = offc;
        m.offp = offp;
        m.offq = offq;
        m.offf = offf;
        offz += np * np;
        offc += n;
        offp += nt * n * NPART;
        offq += nt * n;
        offf += nt;
        cap[cl] += nt * nt;
        if (np % 64 == 0) {  // at most one narrow column tile per problem: its nt row tiles
            cap[CLS_NARROW] += nt;
            capx[CLS_NARROW][x] += nt;
        }
        for (int tm = 0; tm < nt; ++tm)
            for (int cb = 0; cb < ncb; ++cb) it_s1.push_back(make_int4(b, tm, cb, 0));
    }
    const int64_t total_cols = offc, total_tiles = offf, total_q = offq;
    if (total_cols > INT32_MAX / 2 || cap[0] > INT32_MAX / 2 || cap[1] > INT32_MAX / 2 || cap[2] > INT32_MAX / 2 ||
        cap[3] > INT32_MAX / 2)
        return fail(h, IPT_EINVAL, "batch too large");

    BatchLaunch L;
    memset(&L, 0, sizeof(L));
    BatchLists lists;
    memset(&lists, 0, sizeof(lists));
    int64_t segcap[NCLS] = {0, 0, 0, 0};
    for (int c = 0; c < NCLS; ++c) {
        for (int x = 0; x < NXCD; ++x) segcap[c] = std::max(segcap[c], capx[c][x]);
        if (NXCD * segcap[c] > INT32_MAX / 2) return fail(h, IPT_EINVAL, "batch too large");
        lists.segcap[c] = (int32_t)segcap[c];
    }
    BatchMeta *dmeta;
    int4 *ds1;
    double *maxres;
    int32_t *cnt;
    Ctrl *ctrl;
    auto layout = [&](Carve &cv) {
        dmeta = cv.take<BatchMeta>(count);
        ds1 = cv.take<int4>(it_s1.size());
        L.dpad = cv.take<double>(offz);
        for (int q = 0; q < 4; ++q) L.zs[q] = (q < 2 || acx) ? cv.take<double>(offz) : nullptr;
        L.col.dslot = cv.take<double>(acx ? 4 * total_cols : 1);
        L.col.alist = cv.take<int32_t>(total_cols);
        L.col.cprec = cv.take<int32_t>(total_cols);
        L.col.want = cv.take<int32_t>(total_cols);
        L.col.kact = cv.take<int32_t>(count);
        L.col.asym = cv.take<int32_t>(count);
        L.d32 = cv.take<float>(ladder ? offz : 1);
        L.zlo0 = cv.take<float>(ladder ? offz : 1);
        L.zlo1 = cv.take<float>(ladder ? offz : 1);
        L.bpart = cv.take<uint64_t>((size_t)bfinalize_blocks(total_cols) * 8);
        L.col.state = cv.take<int32_t>(total_cols);
        L.col.sweeps = cv.take<int32_t>(total_cols);
        L.col.grow = cv.take<int32_t>(total_cols);
        L.col.par = cv.take<int32_t>(total_cols);
        L.col.prob = cv.take<int32_t>(total_cols);
        L.col.prev = cv.take<double>(total_cols);
        L.col.step = cv.take<double>(total_cols);
        L.col.lam = cv.take<double>(total_cols);
        L.col.resid = cv.take<double>(total_cols);
        L.col.d = cv.take<double>(total_cols);
        L.col.norm_bits = cv.take<uint64_t>(count);
        L.part = cv.take<double>(offp);
        L.dpart = cv.take<double>(total_q);
        L.normpart = cv.take<double>(total_q);
        L.tflag = cv.take<uint32_t>(2 * total_tiles);
        L.ncols = cv.take<int32_t>((size_t)count * 16);
        for (int c = 0; c < NCLS; ++c)
            for (int p = 0; p < 2; ++p) lists.l[c][p] = cv.take<int4>(NXCD * segcap[c] + 1);
        cnt = cv.take<int32_t>(BLIST_WORDS);
        maxres = cv.take<double>(1);
        ctrl = cv.take<Ctrl>(1);
    };
    Carve sizing = carve(h, nullptr);
    layout(sizing);
    if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
    if (ipt_status st = ensure_poll(h)) return st;
    Carve cv = carve(h, (char *)h->ws);
    layout(cv);
    if (ipt_status st = guard_arm(h, cv)) return st;
    lists.counts = cnt;
    lists.tickets = cnt + BLIST_COUNTS;
    L.meta = dmeta;
    L.theta = theta_pool;
    L.delta = delta_pool;
    L.total_tiles = total_tiles;
    L.total_q = total_q;

    // Upload the plan (ordered on the stream; the host vectors live until the
    // synchronisation below).
    IPT_HIP(h, hipMemcpyAsync(dmeta, meta.data(), sizeof(BatchMeta) * count, hipMemcpyHostToDevice, s));
    IPT_HIP(h, hipMemcpyAsync(ds1, it_s1.data(), sizeof(int4) * it_s1.size(), hipMemcpyHostToDevice, s));
    IPT_HIP(h, hipStreamSynchronize(s));

    const int tsize[3] = {32, 64, 128};
    BatchGraphKey key;
    memset(&key, 0, sizeof(key));
    key.L = L;
    key.lists = lists;
    key.dopt = dopt;
    key.ctrl = ctrl;
    key.total_cols = total_cols;
    key.chunk = o.sync_every > 0 ? o.sync_every : 4;
    for (int c = 0; c < NCLS; ++c) {
        key.has[c] = cap[c] > 0;
        // a multiple of NXCD blocks, so that every die has blocks starting on its own segment
        const int64_t full = c == CLS_NARROW ? bnarrow_grid() : bgemm_grid(tsize[c]);
        key.grid[c] = cap[c] > 0 ? (int32_t)round_up(std::min<int64_t>(full, cap[c]), NXCD) : 0;
    }
    // One sweep after the first: the GEMM per tile class (largest tiles first), the
    // finalize, the control kernel.
    Timer timer{h, (o.flags & IPT_FLAG_TIME_KERNELS) != 0, o.max_iter};
    auto sweep = [&](hipStream_t st, int32_t t_host) -> hipError_t {
        hipError_t e = timer.mark(t_host, 0, st);
        for (int c = 2; c >= 0 && e == hipSuccess; --c)
            if (key.has[c]) e = launch_bgemm(st, ctrl, L, lists, tsize[c], key.grid[c], dopt.acx);
        if (e == hipSuccess && key.has[CLS_NARROW])
            e = launch_bnarrow(st, ctrl, L, lists, key.grid[CLS_NARROW], dopt.acx);
        if (e == hipSuccess) e = timer.mark(t_host, 1, st);
        if (e == hipSuccess) e = launch_bfinalize(st, ctrl, dopt, L, total_cols, lists);
        if (e == hipSuccess) e = launch_bplan(st, ctrl, L, lists, count);
        if (e == hipSuccess) e = launch_bcontrol(st, ctrl, dopt, L, total_cols, lists);
        if (e == hipSuccess && acx) e = launch_bacx(st, ctrl, L, lists, total_cols);
        return e;
    };
    const bool use_graph = !(o.flags & (IPT_FLAG_NO_GRAPH | IPT_FLAG_TIME_KERNELS));
    if (use_graph) {
        if (ipt_status st = ensure_batch_graph(h, key, [&](hipStream_t cs) -> hipError_t {
                for (int q = 0; q < key.chunk; ++q)
                    if (hipError_t e = sweep(cs, 0)) return e;
                return hipSuccess;
            }))
            return st;
    }

    IPT_HIP(h, timer.ensure());
    IPT_HIP(h, hipEventRecord(h->ev_start, s));
    IPT_HIP(h, launch_ctrl_init(s, ctrl, PREC_EXACT_FIRST, total_cols));
    IPT_HIP(h, launch_fill_f32(s, (float *)cnt, BLIST_WORDS));
    IPT_HIP(h, launch_fill_f32(s, (float *)maxres, 2));
    IPT_HIP(h, launch_binit(s, ctrl, L, count, ladder ? PREC_F32 : PREC_F64));
    // sweep 1: product-free
    IPT_HIP(h, timer.mark(1, 0, s));
    IPT_HIP(h, launch_bsweep1(s, ctrl, L, ds1, (int64_t)it_s1.size(), ladder ? 1 : 0, dopt.acx));
    IPT_HIP(h, timer.mark(1, 1, s));
    IPT_HIP(h, launch_bfinalize(s, ctrl, dopt, L, total_cols, lists));
    IPT_HIP(h, launch_bplan(s, ctrl, L, lists, count));
    IPT_HIP(h, launch_bcontrol(s, ctrl, dopt, L, total_cols, lists));
    if (acx) IPT_HIP(h, launch_bacx(s, ctrl, L, lists, total_cols));
    // Later sweeps in chunks; the host reads the stop words of chunk i while chunk
    // i + 1 runs (sweeps launched after the device stopped return at once).
    int32_t launched = 1;
    LookaheadPoll poll{h, ctrl};
    while (launched < o.max_iter) {
        if (use_graph) {
            IPT_HIP(h, hipGraphLaunch(h->bgraph, s));
            launched += key.chunk;
        } else {
            const int32_t m = std::min<int32_t>(key.chunk, o.max_iter - launched);
            for (int32_t q = 0; q < m; ++q) IPT_HIP(h, sweep(s, launched + q + 1));
            launched += m;
        }
        bool stop;
        if (ipt_status st = poll.push(stop)) return st;
        if (stop) break;
    }
    IPT_HIP(h, launch_bcopyout(s, ctrl, L, ds1, (int64_t)it_s1.size(), z_pool, lambda_pool, status_pool, maxres,
                               ci ? ci->sweeps : nullptr, ci ? ci->step : nullptr, ci ? ci->resid : nullptr));
    return finish(h, ctrl, total_cols, info, &timer, "batched", maxres,
                  count == 1 ? L.col.norm_bits : nullptr);
}

}  // namespace

extern "C" {

void ipt_opts_default(ipt_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_iter = 100;
    o->precision = IPT_PREC_FP64;
    o->low_type = IPT_LOW_BF16;
    o->sync_every = 0;
    o->tau_low = 1e-5;
    o->tau_32 = 1e-9;
    o->div_norm = 1e3;
    o->div_growth = 8;
    o->flags = 0;
}

ipt_status ipt_create(ipt_handle *out, void *stream) {
    if (!out) return IPT_EINVAL;
    *out = nullptr;
    ipt_context *h = new (std::nothrow) ipt_context();
    if (!h) return IPT_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess || hipEventCreate(&h->ev_start) != hipSuccess ||
        hipEventCreate(&h->ev_stop) != hipSuccess) {
        delete h;
        return IPT_EHIP;
    }
    if (hipHostMalloc((void **)&h->host_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
        (void)hipEventDestroy(h->ev_start);
        (void)hipEventDestroy(h->ev_stop);
        delete h;
        return IPT_ENOMEM;
    }
    h->stream = (hipStream_t)stream;
    if (const char *g = getenv("IPT_GUARD")) {
        h->guard = *g && strcmp(g, "0") != 0;
        h->guard_poke = strcmp(g, "selftest") == 0;
    }
    // set-up that no solve may do later: the poll buffers (pinned host memory) and the
    // device address of the no-allocation workspace on this device
    const hipError_t es = init_scratch(h->device);
    if (es != hipSuccess || ensure_poll(h) != IPT_OK) {
        (void)hipGetLastError();
        ipt_destroy(h);
        return es != hipSuccess ? IPT_EHIP : IPT_ENOMEM;
    }
    *out = h;
    return IPT_OK;
}

ipt_status ipt_destroy(ipt_handle h) {
    if (!h) return IPT_EINVAL;
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->ws) (void)hipFree(h->ws);
    if (h->pws) (void)hipFree(h->pws);
    if (h->band_mem) (void)hipFree(h->band_mem);
    if (h->host_ctrl) (void)hipHostFree(h->host_ctrl);
    (void)hipEventDestroy(h->ev_start);
    (void)hipEventDestroy(h->ev_stop);
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->poll_host) (void)hipHostFree(h->poll_host);
    for (hipEvent_t e : h->poll_ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return IPT_OK;
}

ipt_status ipt_set_stream(ipt_handle h, void *stream) {
    if (!h) return IPT_EINVAL;
    h->stream = (hipStream_t)stream;
    return IPT_OK;
}

const char *ipt_status_string(ipt_status s) {
    switch (s) {
        case IPT_OK: return "IPT_OK";
        case IPT_EINVAL: return "IPT_EINVAL: invalid argument";
        case IPT_EDEGENERATE: return "IPT_EDEGENERATE: repeated unperturbed eigenvalue, inverse gap undefined";
        case IPT_ENOTCONV: return "IPT_ENOTCONV: some columns did not converge";
        case IPT_EHIP: return "IPT_EHIP: HIP runtime error";
        case IPT_ENOMEM: return "IPT_ENOMEM: out of device memory";
        case IPT_EGUARD: return "IPT_EGUARD: a workspace guard band was overwritten (debug mode)";
    }
    return "unknown ipt_status";
}

const char *ipt_last_error(ipt_handle h) { return h ? h->last_error.c_str() : "invalid handle"; }

// The homotopy restart (concluding section): stages q = 1..Q on a scaled copy of
// Delta (the handle's second workspace), each a full dense solve started from the
// previous stage's vectors; the last stage runs on Delta itself into the caller's
// outputs.
static ipt_status homotopy_dense(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                          const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts &o, double *z_out,
                          int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info,
                          const ipt_colinfo *ci) {
    const int32_t Q = o.homotopy_q;
    Carve sizing;
    (void)sizing.take<double>(n * n);
    (void)sizing.take<double>(n * k);
    (void)sizing.take<double>(n * k);
    if (ipt_status st = ensure_buf(h, h->pws, h->pws_bytes, sizing.off + 256)) return st;
    Carve cv;
    cv.base = (char *)h->pws;
    double *dq = cv.take<double>(n * n);
    double *zs[2] = {cv.take<double>(n * k), cv.take<double>(n * k)};
    ipt_opts os = o;
    os.homotopy_q = 0;
    const double *zin = z0;
    int64_t ldin = ldz0, sweeps = 0, matvecs = 0;
    float ms = 0.f;
    for (int32_t q = 1; q <= Q; ++q) {
        const bool last = q == Q;
        if (!last) {
            DeviceGuard guard(h->device);
            IPT_HIP(h, launch_scale_copy(h->stream, dq, delta, lda, n, (double)q / (double)Q));
        }
        double *zo = last ? z_out : zs[q & 1];
        ipt_info inf;
        const ipt_status st = ipt_solve_dense(h, n, theta, last ? delta : dq, last ? lda : n, k, idx, zin, ldin, &os,
                                              zo, last ? ldz : k, lambda_out, col_status, &inf, last ? ci : nullptr);
        if (st != IPT_OK && st != IPT_ENOTCONV) return st;
        sweeps += inf.sweeps;
        matvecs += inf.matvecs;
        ms += inf.time_ms;
        if (last) {
            if (info) {
                *info = inf;
                info->sweeps = (int32_t)sweeps;
                info->matvecs = matvecs;
                info->time_ms = ms;
            }
            return st;
        }
        zin = zo;
        ldin = k;
    }
    return IPT_OK;
}

namespace {

// The dense solve.  noalloc: the workspace is the device's no-allocation array
// (scratch_ptr) instead of the handle's, and nothing is allocated.
ipt_status batched_pairs(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                         const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                         const double *delta_pool, const ipt_opts &o, double *z_pool, double *lambda_pool,
                         int32_t *status_pool, ipt_info *info, const ipt_colinfo *ci);

ipt_status solve_dense(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                       const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts *opts, double *z_out,
                       int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info, const ipt_colinfo *ci,
                       bool noalloc) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (n < 1 || n > (int64_t(1) << 20)) return fail(h, IPT_EINVAL, "n must be in [1, 2^20]");
    if (k < 1 || k > n) return fail(h, IPT_EINVAL, "k must be in [1, n]");
    if (lda < n) return fail(h, IPT_EINVAL, "lda must be >= n");
    if (ldz < k) return fail(h, IPT_EINVAL, "ldz must be >= k");
    if (z0 && ldz0 < k) return fail(h, IPT_EINVAL, "ldz0 must be >= k");
    if (!theta || !delta || !z_out || !lambda_out || !col_status)
        return fail(h, IPT_EINVAL, "theta, delta, z_out, lambda_out and col_status must be non-NULL");
    ipt_opts o;
    if (ipt_status st = check_opts(h, opts, o)) return st;
    if (noalloc && (o.homotopy_q > 1 || (o.flags & IPT_FLAG_TIME_KERNELS)))
        return fail(h, IPT_EINVAL, "the no-allocation solve takes neither opts.homotopy_q > 1 nor IPT_FLAG_TIME_KERNELS");
    if (o.flags & IPT_FLAG_CHOOSE_D) {
        // the choice of D re-partitions the whole problem: a full-spectrum cold solve, run
        // as a batch of one problem (ns = n, every offset 0)
        if (noalloc || idx || z0 || k != n || lda != n || ldz != n || n > 4096 || o.cont_alpha > 0.0 ||
            o.homotopy_q > 1)
            return fail(h, IPT_EINVAL,
                        "IPT_FLAG_CHOOSE_D on a dense solve: full spectrum (k = n, idx NULL), cold start, lda = ldz = n, "
                        "n <= 4096, no continuation, homotopy or no-allocation entry");
        DeviceGuard guard(h->device);
        const int32_t nn = (int32_t)n;
        const int64_t zero = 0;
        return batched_pairs(h, 1, &nn, &zero, &zero, &zero, theta, delta, o, z_out, lambda_out, col_status, info, ci);
    }
    if (o.homotopy_q > 1) return homotopy_dense(h, n, theta, delta, lda, k, idx, z0, ldz0, o, z_out, ldz, lambda_out,
                                                col_status, info, ci);
    const DevOpts dopt = dev_opts(o);
    const bool ladder = dopt.ladder;
    const bool cold = (z0 == nullptr);
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;

    const int64_t np = round_up(n, TILE_M), kp = round_up(k, TILE_N);
    const int64_t nrt = np / TILE_M, ntn = kp / TILE_N;
    const bool direct = (n % TILE_M == 0) && (lda % 2 == 0) && (((uintptr_t)delta & 15) == 0);
    const bool norm = !(o.flags & IPT_FLAG_NO_NORM);
    const int32_t lt = (o.low_type == IPT_LOW_FP16) ? LT_F16 : LT_BF16;
    const bool use_low = ladder && o.low_type != IPT_LOW_NONE;
    // FP16 shadows of Delta (the FP16 low rung, the three-product rung) need max |Delta|
    const bool mid_x3 = dopt.mid_x3 != 0;
    const bool low16 = use_low && lt == LT_F16;
    const bool want_max = low16 || mid_x3;

    // Workspace layout (sizes first, then carve).
    const bool acx = dopt.acx != 0;
    // The caller's z_out serves as iterate buffer 0 when it has that buffer's shape (no
    // padding rows or columns, ldz = kp) and is not the warm start: a column certified by
    // a sweep that read buffer 0 (odd sweeps) is then already in place, and the copy-out
    // skips it.  Not with ACX, whose slots have other roles.
    const bool alias_out = !acx && np == n && kp == k && ldz == kp && (const double *)z_out != z0;
    double *acx_part = nullptr, *acx_sigma = nullptr, *ypart = nullptr;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
        cus = 256;
    const int nblk = 2 * cus;  // the sweep GEMM keeps two 256-thread blocks per CU
    const SplitBounds sb = split_bounds(np, kp, nblk);
    auto layout = [&](Carve &cv, double **zb, ColState &cs, double **dnp, double **dvec, double **part, uint32_t **bitmap,
                      double **scratch, double **dpad, void **dlo, float **d32, void **zt, Ctrl **ctrl) {
        zb[0] = alias_out ? z_out : cv.take<double>(np * kp);
        zb[1] = cv.take<double>(np * kp);
        zb[2] = acx ? cv.take<double>(np * kp) : nullptr;
        zb[3] = acx ? cv.take<double>(np * kp) : nullptr;
        acx_part = acx ? cv.take<double>((size_t)acx_splits(n, kp) * kp * 2) : nullptr;
        acx_sigma = acx ? cv.take<double>(kp) : nullptr;
        ypart = sb.ypart_tiles ? cv.take<double>((size_t)sb.ypart_tiles * TILE_M * TILE_N) : nullptr;
        *dvec = cv.take<double>(kp);
        *part = cv.take<double>(nrt * kp * NPART);
        *dnp = cv.take<double>(nrt * kp);
        cs.state = cv.take<int32_t>(kp);
        cs.sweeps = cv.take<int32_t>(kp);
        cs.grow = cv.take<int32_t>(kp);
        cs.par = cv.take<int32_t>(kp);
        cs.idx = cv.take<int32_t>(kp);
        cs.tile_stamp = cv.take<int32_t>(ntn < kp ? kp : ntn);
        cs.alist = cv.take<int32_t>(kp);
        cs.prev = cv.take<double>(kp);
        cs.step = cv.take<double>(kp);
        cs.lam = cv.take<double>(kp);
        cs.resid = cv.take<double>(kp);
        *bitmap = cv.take<uint32_t>((n + 31) / 32);
        // column partials of |M|_1, then the per-block maxima of |Delta|
        *scratch = (norm || want_max) ? cv.take<double>(prep_delta_chunks(np) * n + prep_delta_blocks(np)) : nullptr;
        *dpad = direct ? nullptr : cv.take<double>(np * np);
        *dlo = use_low ? (void *)cv.take<uint16_t>(np * np) : nullptr;
        *d32 = ladder ? cv.take<float>(np * np) : nullptr;
        *zt = ladder ? (void *)cv.take<float>(kp * np) : nullptr;
        *ctrl = cv.take<Ctrl>(1);
    };
    double *zb[4];
    ColState cs;
    double *dnp, *dvec, *part, *scratch, *dpad;
    uint32_t *bitmap;
    void *dlo, *zt;
    float *d32;
    Ctrl *ctrl;
    Carve sizing = carve(h, nullptr, !noalloc);
    layout(sizing, zb, cs, &dnp, &dvec, &part, &bitmap, &scratch, &dpad, &dlo, &d32, &zt, &ctrl);
    Carve cv;
    if (noalloc) {
        cv = carve(h, (char *)scratch_ptr(h->device), false);
        if (!cv.base) return fail(h, IPT_EINVAL, "no no-allocation workspace on this device");
        if (sizing.off > IPT_NOALLOC_SCRATCH_BYTES)
            return fail(h, IPT_EINVAL, "this solve needs " + std::to_string(sizing.off) +
                                           " bytes of workspace, more than the no-allocation limit of " +
                                           std::to_string((size_t)IPT_NOALLOC_SCRATCH_BYTES));
    } else {
        if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
        cv = carve(h, (char *)h->ws);
    }
    layout(cv, zb, cs, &dnp, &dvec, &part, &bitmap, &scratch, &dpad, &dlo, &d32, &zt, &ctrl);
    if (ipt_status st = guard_arm(h, cv)) return st;

    Timer timer{h, (o.flags & IPT_FLAG_TIME_KERNELS) != 0, o.max_iter};
    IPT_HIP(h, timer.ensure());
    IPT_HIP(h, hipEventRecord(h->ev_start, s));
    const int32_t start_prec = cold ? PREC_EXACT_FIRST : (ladder ? PREC_F32 : PREC_F64);
    // The pass over Delta goes first (it needs only the control block), so that the
    // small column-setup kernels queue behind it instead of idling the device.
    // Plain sweeps take d of the next sweep from the product epilogue; for an exactly
    // symmetric Delta (checked once here) it reads Delta_ji, coalesced, for Delta_ij.
    // continuation sweeps rescale W after the product, so d comes from the pass over Delta
    const bool cont = o.cont_alpha > 0.0;
    const bool fuse_d = !acx && !cont;
    IPT_HIP(h, launch_ctrl_init(s, ctrl, start_prec, k, fuse_d ? 1 : 0, o.cont_alpha, bitmap, n));
    // Row-major pass over Delta (copy, BF16/FP32 shadows, |M|_1, max |Delta|), then the
    // tile-pair pass (symmetry, FP16 shadows at the power-of-two scale from that max)
    const double *dA = direct ? delta : dpad;
    const int64_t ldA = direct ? lda : np;
    if (!direct || ladder || norm)
        IPT_HIP(h, launch_prep_delta(s, ctrl, theta, delta, lda, n, np, direct ? nullptr : dpad,
                                     (use_low && !low16) ? (__bf16 *)dlo : nullptr, (ladder && !mid_x3) ? d32 : nullptr,
                                     norm ? scratch : nullptr,
                                     want_max ? (uint64_t *)(scratch + prep_delta_chunks(np) * n) : nullptr));
    if (fuse_d || want_max)
        IPT_HIP(h, launch_scan_delta(s, ctrl, delta, lda, n, np, fuse_d, low16 ? (_Float16 *)dlo : nullptr,
                                     mid_x3 ? (_Float16 *)d32 : nullptr));
    // column state, the packed list of the first sweep and theta's order in one launch
    IPT_HIP(h, launch_init_cols(s, ctrl, cs, idx, n, k, kp, bitmap, (int32_t)ntn, 0, true, theta));
    IPT_HIP(h, launch_check_theta(s, ctrl, theta, cs.idx, n, k, true));
    const bool padded = (np != n) || (kp != k);
    if (cold && !acx) {
        if (padded) IPT_HIP(h, launch_zero_pad(s, zb[0], kp, n, np, k, kp));
    } else {
        // warm start, or the base iterate E of the first ACX cycle
        IPT_HIP(h, launch_load_z0(s, ctrl, z0, ldz0, zb[0], kp, cs.idx, n, np, k, kp, mid_x3 ? 1 : 0));
        if (padded)
            for (int q = 1; q < (acx ? 4 : 2); ++q) IPT_HIP(h, launch_zero_pad(s, zb[q], kp, n, np, k, kp));
    }

    const PollPlan plan = poll_plan(o, cold);
    if (ipt_status st = ensure_poll(h)) return st;
    LookaheadPoll poll{h, ctrl};
    // d of a sweep comes from the previous sweep's product epilogue (plain sweeps: the
    // input is the previous output W), else from a pass over Delta and Z.
    bool d_ready = false, copied = false;
    for (int32_t t = 1; t <= o.max_iter; ++t) {
        const bool first_exact = cold && t == 1;
        // Plain sweeps ping-pong between two buffers; an ACX cycle runs slot q -> q + 1
        // from its base iterate in slot 0 and extrapolates back into slot 0.
        int32_t q, pc;
        acx_phase(dopt.acx, t, q, pc);
        const int32_t in_par = first_exact ? PAR_UNIT : (acx ? PAR_BUF0 : ((t - 1) & 1));
        const int32_t out_par = acx ? PAR_BUF1 : (t & 1);
        double *zin = acx ? zb[q] : zb[(t - 1) & 1], *zout = acx ? zb[q + 1] : zb[t & 1];
        if (first_exact) {
            IPT_HIP(h, timer.mark(t, 0, s));
            IPT_HIP(h, launch_sweep1_dense(s, ctrl, theta, dA, ldA, cs, dvec, zout, kp, part, n, np, kp,
                                           fuse_d ? dnp : nullptr));
            IPT_HIP(h, timer.mark(t, 1, s));
        } else {
            if (ladder) IPT_HIP(h, launch_cast_z(s, ctrl, zin, kp, cs, zt, np, np, kp, lt, dopt.mid_x3));
            if (!d_ready) IPT_HIP(h, launch_diag_dense(s, ctrl, dA, ldA, zin, kp, cs, dnp, dvec, n, kp));
            IPT_HIP(h, timer.mark(t, 0, s));
            IPT_HIP(h, launch_sweep_gemm(s, ctrl, dA, ldA, dlo, d32, zt, zin, zout, theta, cs, dvec, part, n, np, kp, t,
                                         lt, ypart, nblk, fuse_d ? dnp : nullptr, dopt.mid_x3));
            IPT_HIP(h, timer.mark(t, 1, s));
        }
        if (cont) IPT_HIP(h, launch_cont_blend(s, ctrl, zout, kp, cs, n, kp));
        const bool fused_d = fuse_d;  // every plain sweep (the product-free first one too) forms the next d
        IPT_HIP(h, launch_finalize(s, ctrl, dopt, cs, dvec, theta, part, nrt, kp, t, in_par, out_par,
                                   fused_d ? dnp : nullptr));
        d_ready = fused_d;
        IPT_HIP(h, launch_control_plan(s, ctrl, dopt, t, cs, kp));
        if (acx && q == pc - 1)
            IPT_HIP(h, launch_acx(s, ctrl, cs.state, zb[0], zb[1], zb[2], zb[3], kp, n, kp, pc, acx_part, acx_sigma));
        if (plan.at(t, o.max_iter)) {
            // The first poll sits where the solve is expected to stop and waits for
            // itself: a copy-out that runs only if the device is done goes before it,
            // so the outputs are written while the host reads the stop words.
            const bool spec = poll.first;
            if (spec)
                IPT_HIP(h, launch_copyout(s, ctrl, cs, zb[0], zb[1], kp, z_out, ldz, lambda_out, col_status, n, k, ci,
                                          true));
            bool stop;
            if (ipt_status st = poll.push(stop)) return st;
            if (stop) {
                copied = spec;
                break;
            }
        }
    }
    if (!copied)
        IPT_HIP(h, launch_copyout(s, ctrl, cs, zb[0], zb[1], kp, z_out, ldz, lambda_out, col_status, n, k, ci));
    return finish(h, ctrl, k, info, &timer, "dense", nullptr);
}

}  // namespace

ipt_status ipt_solve_dense(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                           const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts *opts, double *z_out,
                           int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info,
                           const ipt_colinfo *ci) {
    return solve_dense(h, n, theta, delta, lda, k, idx, z0, ldz0, opts, z_out, ldz, lambda_out, col_status, info, ci,
                       false);
}

ipt_status ipt_solve_dense_noalloc(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda,
                                   int64_t k, const int32_t *idx, const double *z0, int64_t ldz0,
                                   const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out,
                                   int32_t *col_status, ipt_info *info, const ipt_colinfo *ci) {
    return solve_dense(h, n, theta, delta, lda, k, idx, z0, ldz0, opts, z_out, ldz, lambda_out, col_status, info, ci,
                       true);
}

ipt_status ipt_solve_dense_z(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda,
                             int64_t k, const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts *opts,
                             double *z_out, int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info,
                             const ipt_colinfo *ci) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (n < 1 || n > (int64_t(1) << 20)) return fail(h, IPT_EINVAL, "n must be in [1, 2^20]");
    if (k < 1 || k > n) return fail(h, IPT_EINVAL, "k must be in [1, n]");
    if (lda < n) return fail(h, IPT_EINVAL, "lda must be >= n");
    if (ldz < k) return fail(h, IPT_EINVAL, "ldz must be >= k");
    if (z0 && ldz0 < k) return fail(h, IPT_EINVAL, "ldz0 must be >= k");
    if (!theta || !delta || !z_out || !lambda_out || !col_status)
        return fail(h, IPT_EINVAL, "theta, delta, z_out, lambda_out and col_status must be non-NULL");
    if ((((uintptr_t)theta | (uintptr_t)delta | (uintptr_t)z_out | (uintptr_t)lambda_out | (uintptr_t)z0) & 15) != 0)
        return fail(h, IPT_EINVAL, "complex arrays must be 16-byte aligned");
    ipt_opts o;
    if (ipt_status st = check_opts(h, opts, o)) return st;
    if (o.precision != IPT_PREC_FP64 || (o.flags & (IPT_FLAG_ACX | IPT_FLAG_CHOOSE_D)) || o.cont_alpha > 0.0 ||
        o.homotopy_q > 1)
        return fail(h, IPT_EINVAL,
                    "complex solves run plain FP64 sweeps (no ladder, ACX, choice of D, continuation or homotopy)");
    const DevOpts dopt = dev_opts(o);
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;

    const int64_t zt = zsweep_tile();
    const int64_t np = round_up(n, zt), kp = round_up(k, TILE_N);
    const int64_t nrt = np / zt, ntn = kp / TILE_N;
    const bool norm = !(o.flags & IPT_FLAG_NO_NORM);
    auto layout = [&](Carve &cv, double **zb, ColState &cs, double **d_re, double **d_im, double **dpart,
                      double **lam_im, double **th_re, double **th_im, double **part, double **part2,
                      uint32_t **bitmap, Ctrl **ctrl) {
        zb[0] = cv.take<double>(2 * np * kp);
        zb[1] = cv.take<double>(2 * np * kp);
        *d_re = cv.take<double>(kp);
        *d_im = cv.take<double>(kp);
        *dpart = cv.take<double>(zdiag_part_doubles(kp));
        *lam_im = cv.take<double>(kp);
        *th_re = cv.take<double>(n);
        *th_im = cv.take<double>(n);
        *part = cv.take<double>(nrt * kp * NPART);
        *part2 = norm ? cv.take<double>(zsetup_part2_doubles(n)) : nullptr;
        cs.state = cv.take<int32_t>(kp);
        cs.sweeps = cv.take<int32_t>(kp);
        cs.grow = cv.take<int32_t>(kp);
        cs.par = cv.take<int32_t>(kp);
        cs.idx = cv.take<int32_t>(kp);
        cs.tile_stamp = cv.take<int32_t>(ntn < kp ? kp : ntn);
        cs.alist = cv.take<int32_t>(kp);
        cs.prev = cv.take<double>(kp);
        cs.step = cv.take<double>(kp);
        cs.lam = cv.take<double>(kp);
        cs.resid = cv.take<double>(kp);
        *bitmap = cv.take<uint32_t>((n + 31) / 32);
        *ctrl = cv.take<Ctrl>(1);
    };
    double *zb[2], *d_re, *d_im, *dpart, *lam_im, *th_re, *th_im, *part, *part2;
    ColState cs;
    uint32_t *bitmap;
    Ctrl *ctrl;
    Carve sizing = carve(h, nullptr);
    layout(sizing, zb, cs, &d_re, &d_im, &dpart, &lam_im, &th_re, &th_im, &part, &part2, &bitmap, &ctrl);
    if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
    Carve cv = carve(h, (char *)h->ws);
    layout(cv, zb, cs, &d_re, &d_im, &dpart, &lam_im, &th_re, &th_im, &part, &part2, &bitmap, &ctrl);
    if (ipt_status st = guard_arm(h, cv)) return st;

    Timer timer{h, (o.flags & IPT_FLAG_TIME_KERNELS) != 0, o.max_iter};
    IPT_HIP(h, timer.ensure());
    IPT_HIP(h, hipEventRecord(h->ev_start, s));
    // the first sweep of a cold start needs no product (Delta E is a gather)
    const bool cold = (z0 == nullptr);
    IPT_HIP(h, launch_ctrl_init(s, ctrl, cold ? PREC_EXACT_FIRST : PREC_F64, k, 0, 0.0, bitmap, n));
    IPT_HIP(h, launch_zsetup(s, ctrl, theta, delta, lda, th_re, th_im, part2, n));
    IPT_HIP(h, launch_init_cols(s, ctrl, cs, idx, n, k, kp, bitmap, (int32_t)ntn, 0, true));
    IPT_HIP(h, launch_zcheck_gaps(s, ctrl, th_re, th_im, cs.idx, n, k));
    IPT_HIP(h, launch_zload(s, ctrl, z0, ldz0, zb[0], kp, cs.idx, n, np, k));
    IPT_HIP(h, launch_zload(s, ctrl, nullptr, 0, zb[1], kp, cs.idx, n, np, k));

    const PollPlan plan = poll_plan(o, false);
    if (ipt_status st = ensure_poll(h)) return st;
    LookaheadPoll poll{h, ctrl};
    for (int32_t t = 1; t <= o.max_iter; ++t) {
        const int32_t in_par = (t - 1) & 1, out_par = t & 1;
        const double *zin = zb[(t - 1) & 1];
        double *zout = zb[t & 1];
        if (cold && t == 1) {
            IPT_HIP(h, timer.mark(t, 0, s));
            IPT_HIP(h, launch_zsweep1(s, ctrl, delta, lda, th_re, th_im, cs, d_re, d_im, zout, kp, part, n, np));
            IPT_HIP(h, timer.mark(t, 1, s));
        } else {
            IPT_HIP(h, launch_zdiag(s, ctrl, delta, lda, zin, kp, cs, dpart, d_re, d_im, n));
            IPT_HIP(h, timer.mark(t, 0, s));
            IPT_HIP(h, launch_zsweep(s, ctrl, delta, lda, th_re, th_im, zin, zout, cs, d_re, d_im, part, n, np, kp));
            IPT_HIP(h, timer.mark(t, 1, s));
        }
        IPT_HIP(h, launch_finalize(s, ctrl, dopt, cs, d_re, th_re, part, nrt, kp, t, in_par, out_par, nullptr, th_im,
                                   d_im, lam_im));
        IPT_HIP(h, launch_control_plan(s, ctrl, dopt, t, cs, kp));
        if (plan.at(t, o.max_iter)) {
            bool stop;
            if (ipt_status st = poll.push(stop)) return st;
            if (stop) break;
        }
    }
    IPT_HIP(h, launch_zcopyout(s, ctrl, cs, zb[0], zb[1], kp, z_out, ldz, lam_im, lambda_out, col_status, n, k, ci));
    return finish(h, ctrl, k, info, &timer, "complex", nullptr);
}

ipt_status ipt_solve_csr_z(ipt_handle h, int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                           const double *val, int64_t nnz, int64_t k, const int32_t *idx, const double *z0,
                           int64_t ldz0, const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out,
                           int32_t *col_status, ipt_info *info, const ipt_colinfo *ci) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (n < 1 || n > (int64_t(1) << 30)) return fail(h, IPT_EINVAL, "n must be in [1, 2^30]");
    if (k < 1 || k > n) return fail(h, IPT_EINVAL, "k must be in [1, n]");
    if (nnz < 0 || nnz > INT32_MAX) return fail(h, IPT_EINVAL, "nnz must be in [0, 2^31)");
    if (ldz < k) return fail(h, IPT_EINVAL, "ldz must be >= k");
    if (z0 && ldz0 < k) return fail(h, IPT_EINVAL, "ldz0 must be >= k");
    if (!theta || !row_ptr || (nnz > 0 && (!col || !val)) || !z_out || !lambda_out || !col_status)
        return fail(h, IPT_EINVAL, "theta, row_ptr, col, val, z_out, lambda_out and col_status must be non-NULL");
    if ((((uintptr_t)theta | (uintptr_t)val | (uintptr_t)z_out | (uintptr_t)lambda_out | (uintptr_t)z0) & 15) != 0)
        return fail(h, IPT_EINVAL, "complex arrays must be 16-byte aligned");
    ipt_opts o;
    if (ipt_status st = check_opts(h, opts, o)) return st;
    if (o.precision != IPT_PREC_FP64 || (o.flags & (IPT_FLAG_ACX | IPT_FLAG_CHOOSE_D)) || o.cont_alpha > 0.0 ||
        o.homotopy_q > 1)
        return fail(h, IPT_EINVAL,
                    "complex solves run plain FP64 sweeps (no ladder, ACX, choice of D, continuation or homotopy)");
    const DevOpts dopt = dev_opts(o);
    const bool cold = (z0 == nullptr);
    const bool norm = !(o.flags & IPT_FLAG_NO_NORM);
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;

    const int64_t kpc = round_up(k, 64);  // column-state and partial-sum layout
    const int64_t ldzb = k;               // Z buffers: n x k complex
    const int64_t nrb = zspmm_row_blocks(n);
    auto layout = [&](Carve &cv, double **zb, ColState &cs, double **d_re, double **d_im, double **lam_im,
                      double **th_re, double **th_im, double **part, uint32_t **bitmap, double **scratch,
                      Ctrl **ctrl) {
        zb[0] = cv.take<double>(2 * n * ldzb);
        zb[1] = cv.take<double>(2 * n * ldzb);
        *d_re = cv.take<double>(kpc);
        *d_im = cv.take<double>(kpc);
        *lam_im = cv.take<double>(kpc);
        *th_re = cv.take<double>(n);
        *th_im = cv.take<double>(n);
        *part = cv.take<double>(nrb * kpc * NPART);
        cs.state = cv.take<int32_t>(kpc);
        cs.sweeps = cv.take<int32_t>(kpc);
        cs.grow = cv.take<int32_t>(kpc);
        cs.par = cv.take<int32_t>(kpc);
        cs.idx = cv.take<int32_t>(kpc);
        cs.tile_stamp = cv.take<int32_t>(kpc / TILE_N + 1);
        cs.alist = nullptr;
        cs.prev = cv.take<double>(kpc);
        cs.step = cv.take<double>(kpc);
        cs.lam = cv.take<double>(kpc);
        cs.resid = cv.take<double>(kpc);
        *bitmap = cv.take<uint32_t>((n + 31) / 32);
        *scratch = norm ? cv.take<double>(norm1_csr_scratch_doubles(n)) : nullptr;
        *ctrl = cv.take<Ctrl>(1);
    };
    double *zb[2], *d_re, *d_im, *lam_im, *th_re, *th_im, *part, *scratch;
    ColState cs;
    uint32_t *bitmap;
    Ctrl *ctrl;
    Carve sizing = carve(h, nullptr);
    layout(sizing, zb, cs, &d_re, &d_im, &lam_im, &th_re, &th_im, &part, &bitmap, &scratch, &ctrl);
    if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
    Carve cv = carve(h, (char *)h->ws);
    layout(cv, zb, cs, &d_re, &d_im, &lam_im, &th_re, &th_im, &part, &bitmap, &scratch, &ctrl);
    if (ipt_status st = guard_arm(h, cv)) return st;

    Timer timer{h, (o.flags & IPT_FLAG_TIME_KERNELS) != 0, o.max_iter};
    IPT_HIP(h, timer.ensure());
    IPT_HIP(h, hipEventRecord(h->ev_start, s));
    // A cold start's first sweep multiplies Delta by E, which is exact, so it may certify.
    IPT_HIP(h, launch_init(s, ctrl, cs, idx, n, k, kpc, bitmap, cold ? PREC_EXACT_FIRST : PREC_F64,
                           (int32_t)(kpc / TILE_N + 1), 0));
    IPT_HIP(h, launch_zsetup(s, ctrl, theta, nullptr, 0, th_re, th_im, nullptr, n));  // theta's parts, finiteness
    IPT_HIP(h, launch_zcheck_gaps(s, ctrl, th_re, th_im, cs.idx, n, k));
    IPT_HIP(h, launch_check_csr(s, ctrl, row_ptr, col, n, nnz));
    if (norm) IPT_HIP(h, launch_norm1_csr(s, ctrl, th_re, row_ptr, col, val, n, nnz, scratch, th_im));
    // a cold start's first sweep reads no iterate (Z = E: the product-free sweep)
    if (!cold) IPT_HIP(h, launch_zload(s, ctrl, z0, ldz0, zb[0], ldzb, cs.idx, n, n, k));

    PollPlan plan = poll_plan(o, cold);
    if (o.sync_every <= 0) plan.first = cold ? 3 : 2;  // sparse near-diagonal solves take few sweeps
    if (ipt_status st = ensure_poll(h)) return st;
    LookaheadPoll poll{h, ctrl};
    for (int32_t t = 1; t <= o.max_iter; ++t) {
        const bool unit = cold && t == 1;
        const int32_t in_par = unit ? PAR_UNIT : ((t - 1) & 1), out_par = t & 1;
        const double *zin = zb[(t - 1) & 1];
        double *zout = zb[t & 1];
        if (!unit) IPT_HIP(h, launch_zdiag_csr(s, ctrl, row_ptr, col, val, zin, ldzb, cs, d_re, d_im, k));
        IPT_HIP(h, timer.mark(t, 0, s));
        IPT_HIP(h, launch_zspmm_sweep(s, ctrl, row_ptr, col, val, th_re, th_im, zin, zout, cs, d_re, d_im, part, n,
                                      k, ldzb, unit ? 1 : 0));
        IPT_HIP(h, timer.mark(t, 1, s));
        IPT_HIP(h, launch_reduce_parts(s, ctrl, cs, part, nrb, k, kpc));
        IPT_HIP(h, launch_finalize(s, ctrl, dopt, cs, d_re, th_re, part, 1, kpc, t, in_par, out_par, nullptr, th_im,
                                   d_im, lam_im));
        IPT_HIP(h, launch_control(s, ctrl, dopt, t));
        if (plan.at(t, o.max_iter)) {
            bool stop;
            if (ipt_status st = poll.push(stop)) return st;
            if (stop) break;
        }
    }
    IPT_HIP(h, launch_zcopyout(s, ctrl, cs, zb[0], zb[1], ldzb, z_out, ldz, lam_im, lambda_out, col_status, n, k, ci));
    return finish(h, ctrl, k, info, &timer, "csr_z", nullptr);
}

ipt_status ipt_solve_csr(ipt_handle h, int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                         const double *val, int64_t nnz, int64_t k, const int32_t *idx, const double *z0, int64_t ldz0,
                         const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out, int32_t *col_status,
                         ipt_info *info, const ipt_colinfo *ci) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (n < 1 || n > (int64_t(1) << 30)) return fail(h, IPT_EINVAL, "n must be in [1, 2^30]");
    if (k < 1 || k > n) return fail(h, IPT_EINVAL, "k must be in [1, n]");
    if (nnz < 0 || nnz > INT32_MAX) return fail(h, IPT_EINVAL, "nnz must be in [0, 2^31)");
    if (ldz < k) return fail(h, IPT_EINVAL, "ldz must be >= k");
    if (z0 && ldz0 < k) return fail(h, IPT_EINVAL, "ldz0 must be >= k");
    if (!theta || !row_ptr || (nnz > 0 && (!col || !val)) || !z_out || !lambda_out || !col_status)
        return fail(h, IPT_EINVAL, "theta, row_ptr, col, val, z_out, lambda_out and col_status must be non-NULL");
    ipt_opts o;
    if (ipt_status st = check_opts(h, opts, o)) return st;
    if (o.homotopy_q > 1) return fail(h, IPT_EINVAL, "opts.homotopy_q: the homotopy restart is for dense solves");
    DevOpts dopt = dev_opts(o);
    dopt.low_type = IPT_LOW_NONE;  // the sparse ladder runs FP32 then FP64 sweeps
    dopt.mid_x3 = 0;
    const bool ladder = dopt.ladder;
    const bool cold = (z0 == nullptr);
    const bool norm = !(o.flags & IPT_FLAG_NO_NORM);
    const bool cont = o.cont_alpha > 0.0;  // FP64 sweeps, no ACX (check_opts)
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;

    const int64_t kpc = round_up(k, 64);   // column-state and partial-sum layout
    const int64_t ldzb = round_up(k, 2);   // Z buffers: n x ldzb
    const int64_t nrt = spmm_row_tiles(n);
    const bool acx = dopt.acx != 0;
    double *acx_part = nullptr, *acx_sigma = nullptr;
    // z_out as iterate buffer 0 when it has its shape (ldz = ldzb = k), as in the dense solve
    const bool alias_out = !acx && ldz == ldzb && k == ldzb && (const double *)z_out != z0;
    auto layout = [&](Carve &cv, double **zb, float **zlo, ColState &cs, double **dvec, double **part,
                      uint32_t **bitmap, double **scratch, float **val32, Ctrl **ctrl) {
        zb[0] = alias_out ? z_out : cv.take<double>(n * ldzb);
        zb[1] = cv.take<double>(n * ldzb);
        zb[2] = acx ? cv.take<double>(n * ldzb) : nullptr;
        zb[3] = acx ? cv.take<double>(n * ldzb) : nullptr;
        acx_part = acx ? cv.take<double>((size_t)acx_splits(n, k) * kpc * 2) : nullptr;
        acx_sigma = acx ? cv.take<double>(kpc) : nullptr;
        zlo[0] = ladder ? cv.take<float>(n * ldzb) : nullptr;
        zlo[1] = ladder ? cv.take<float>(n * ldzb) : nullptr;
        *dvec = cv.take<double>(kpc);
        *part = cv.take<double>(nrt * kpc * NPART);
        cs.state = cv.take<int32_t>(kpc);
        cs.sweeps = cv.take<int32_t>(kpc);
        cs.grow = cv.take<int32_t>(kpc);
        cs.par = cv.take<int32_t>(kpc);
        cs.idx = cv.take<int32_t>(kpc);
        cs.tile_stamp = cv.take<int32_t>(kpc / TILE_N + 1);
        cs.alist = nullptr;
        cs.prev = cv.take<double>(kpc);
        cs.step = cv.take<double>(kpc);
        cs.lam = cv.take<double>(kpc);
        cs.resid = cv.take<double>(kpc);
        *bitmap = cv.take<uint32_t>((n + 31) / 32);
        *scratch = norm ? cv.take<double>(norm1_csr_scratch_doubles(n)) : nullptr;
        *val32 = (ladder && nnz > 0) ? cv.take<float>(nnz) : nullptr;
        *ctrl = cv.take<Ctrl>(1);
    };
    double *zb[4], *dvec, *part, *scratch;
    float *zlo[2], *val32;
    ColState cs;
    uint32_t *bitmap;
    Ctrl *ctrl;
    Carve sizing = carve(h, nullptr);
    layout(sizing, zb, zlo, cs, &dvec, &part, &bitmap, &scratch, &val32, &ctrl);
    if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
    Carve cv = carve(h, (char *)h->ws);
    layout(cv, zb, zlo, cs, &dvec, &part, &bitmap, &scratch, &val32, &ctrl);
    if (ipt_status st = guard_arm(h, cv)) return st;

    Timer timer{h, (o.flags & IPT_FLAG_TIME_KERNELS) != 0, o.max_iter};
    IPT_HIP(h, timer.ensure());
    IPT_HIP(h, hipEventRecord(h->ev_start, s));
    // A cold start's first sweep multiplies Delta by E, which is exact in every
    // precision (the low-precision part Z - E is zero), so it may certify.
    const int32_t start_prec = cold ? PREC_EXACT_FIRST : (ladder ? PREC_F32 : PREC_F64);
    IPT_HIP(h, launch_init(s, ctrl, cs, idx, n, k, kpc, bitmap, start_prec, (int32_t)(kpc / TILE_N + 1), 0, theta,
                           o.cont_alpha));
    IPT_HIP(h, launch_check_theta(s, ctrl, theta, cs.idx, n, k, true));
    IPT_HIP(h, launch_check_csr(s, ctrl, row_ptr, col, n, nnz, val, val32));
    if (norm) IPT_HIP(h, launch_norm1_csr(s, ctrl, theta, row_ptr, col, val, n, nnz, scratch));
    // A cold start's first sweep reads no iterate (Z = E: the product-free sweep); only
    // ACX keeps E in slot 0 as the base of its first cycle.
    if (!cold || acx) IPT_HIP(h, launch_load_z0(s, ctrl, z0, ldz0, zb[0], ldzb, cs.idx, n, n, k, ldzb));
    if (ladder && !cold) IPT_HIP(h, launch_zlo_init(s, zb[0], zlo[0], ldzb, cs.idx, n, k));
    if (ldzb != k) {  // padding column of the other buffers
        for (int q = 1; q < (acx ? 4 : 2); ++q)
            IPT_HIP(h, launch_load_z0(s, ctrl, nullptr, 0, zb[q], ldzb, cs.idx, n, n, k, ldzb));
        if (ladder) IPT_HIP(h, launch_fill_f32(s, zlo[1], n * ldzb));
    }

    PollPlan plan = poll_plan(o, cold);
    if (o.sync_every <= 0) plan.first = cold ? 3 : 2;  // sparse near-diagonal solves take few sweeps
    if (ipt_status st = ensure_poll(h)) return st;
    LookaheadPoll poll{h, ctrl};
    bool copied = false;
    for (int32_t t = 1; t <= o.max_iter; ++t) {
        int32_t q, pc;
        acx_phase(dopt.acx, t, q, pc);
        const bool unit = cold && t == 1;  // the product-free first sweep (d from row i inside it)
        const int32_t in_par = acx ? PAR_BUF0 : (unit ? PAR_UNIT : ((t - 1) & 1)), out_par = acx ? PAR_BUF1 : (t & 1);
        double *zin = acx ? zb[q] : zb[(t - 1) & 1], *zout = acx ? zb[q + 1] : zb[t & 1];
        // d of a plain sweep after the first comes from the previous sweep's tail
        const bool tail = !acx && !cont;
        if (!unit && (!tail || t == 1)) IPT_HIP(h, launch_diag_csr(s, ctrl, row_ptr, col, val, zin, ldzb, cs, dvec, k));
        IPT_HIP(h, timer.mark(t, 0, s));
        IPT_HIP(h, launch_spmm_sweep(s, ctrl, row_ptr, col, val, val32, theta, zin, zout,
                                     ladder ? zlo[(t - 1) & 1] : nullptr, ladder ? zlo[t & 1] : nullptr, cs, dvec,
                                     part, n, k, ldzb, kpc, unit ? 1 : 0));
        IPT_HIP(h, timer.mark(t, 1, s));
        // continuation: W <- E + s (W - E) on this sweep's active columns (scale s < 1)
        if (cont) IPT_HIP(h, launch_cont_blend_cols(s, ctrl, zout, ldzb, cs, n, k));
        if (!tail) {
            IPT_HIP(h, launch_reduce_parts(s, ctrl, cs, part, nrt, k, kpc));
            IPT_HIP(h, launch_finalize(s, ctrl, dopt, cs, dvec, theta, part, 1, kpc, t, in_par, out_par));
            IPT_HIP(h, launch_control(s, ctrl, dopt, t));
        } else {
            IPT_HIP(h, launch_csr_tail(s, ctrl, dopt, cs, dvec, theta, part, nrt, k, kpc, t, in_par, out_par, row_ptr,
                                       col, val, zout, ldzb));
        }
        if (acx && q == pc - 1)
            IPT_HIP(h, launch_acx(s, ctrl, cs.state, zb[0], zb[1], zb[2], zb[3], ldzb, n, k, pc, acx_part, acx_sigma));
        if (plan.at(t, o.max_iter)) {
            const bool spec = poll.first;  // as in the dense solve: copy-out before the first poll
            if (spec)
                IPT_HIP(h, launch_copyout(s, ctrl, cs, zb[0], zb[1], ldzb, z_out, ldz, lambda_out, col_status, n, k,
                                          ci, true));
            bool stop;
            if (ipt_status st = poll.push(stop)) return st;
            if (stop) {
                copied = spec;
                break;
            }
        }
    }
    if (!copied)
        IPT_HIP(h, launch_copyout(s, ctrl, cs, zb[0], zb[1], ldzb, z_out, ldz, lambda_out, col_status, n, k, ci));
    return finish(h, ctrl, k, info, &timer, "csr", nullptr);
}

namespace {

// IPT_FLAG_CHOOSE_D on a batch: copies of the pools (at the caller's offsets) are
// re-partitioned (near-degenerate pairs rotated out, level shifts moved into D), the
// batch is solved on them, and the eigenvectors are rotated back in z_pool.
ipt_status batched_pairs(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                         const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                         const double *delta_pool, const ipt_opts &o, double *z_pool, double *lambda_pool,
                         int32_t *status_pool, ipt_info *info, const ipt_colinfo *ci) {
    if (count < 1 || !ns || !theta_off || !delta_off || !z_off || !theta_pool || !delta_pool || !z_pool)
        return fail(h, IPT_EINVAL, "bad batch description");
    int64_t tlo = INT64_MAX, thi = 0, dhi = 0;
    int32_t max_n = 0;
    for (int32_t b = 0; b < count; ++b) {
        const int64_t n = ns[b];
        if (n < 1 || n > 4096) return fail(h, IPT_EINVAL, "every problem size must be in [1, 4096]");
        if (theta_off[b] < 0 || delta_off[b] < 0 || z_off[b] < 0) return fail(h, IPT_EINVAL, "negative pool offset");
        tlo = std::min(tlo, theta_off[b]);
        thi = std::max(thi, theta_off[b] + n);
        dhi = std::max(dhi, delta_off[b] + n * n);
        max_n = std::max(max_n, (int32_t)n);
    }
    // scratch: theta' [thi], Delta' [dhi], best [thi], partner [thi], rmax [thi], cs [2 thi], th2 [thi],
    // then the per-problem n, ld = n, offsets
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_dp = up(thi * 8), o_best = o_dp + up(dhi * 8), o_part = o_best + up(thi * 4),
                 o_rmax = o_part + up(thi * 4), o_cs = o_rmax + up(thi * 8), o_th2 = o_cs + up(thi * 16),
                 o_meta = o_th2 + up(thi * 8);
    const size_t meta_bytes = (size_t)count * (4 + 4 + 8 * 4);
    if (ipt_status st = ensure_buf(h, h->pws, h->pws_bytes, o_meta + meta_bytes)) return st;
    char *base = (char *)h->pws;
    double *tp = (double *)base, *dp = (double *)(base + o_dp), *rmax = (double *)(base + o_rmax);
    double *cs = (double *)(base + o_cs), *th2 = (double *)(base + o_th2);
    int32_t *best = (int32_t *)(base + o_best), *partner = (int32_t *)(base + o_part);
    std::vector<unsigned char> meta(meta_bytes);
    int32_t *hn = (int32_t *)meta.data(), *hk = hn + count;
    int64_t *hto = (int64_t *)(hk + count), *hdo = hto + count, *hzo = hdo + count, *hld = hzo + count;
    for (int32_t b = 0; b < count; ++b) {
        hn[b] = hk[b] = ns[b];
        hto[b] = theta_off[b];
        hdo[b] = delta_off[b];
        hzo[b] = z_off[b];
        hld[b] = ns[b];
    }
    char *dm = base + o_meta;
    int32_t *dn = (int32_t *)dm, *dk = dn + count;
    int64_t *dto = (int64_t *)(dk + count), *ddo = dto + count, *dzo = ddo + count, *dld = dzo + count;
    hipStream_t s = h->stream;
    IPT_HIP(h, hipMemcpyAsync(dm, meta.data(), meta_bytes, hipMemcpyHostToDevice, s));
    IPT_HIP(h, hipMemcpyAsync(tp + tlo, theta_pool + tlo, (size_t)(thi - tlo) * 8, hipMemcpyDeviceToDevice, s));
    IPT_HIP(h, hipStreamSynchronize(s));  // the host copy of the metadata is released below
    IPT_HIP(h, launch_pair_rotate(s, count, max_n, dn, dto, ddo, theta_pool, delta_pool, tp, dp, best, rmax, partner,
                                  cs, IPT_PAIR_TAU, th2));
    ipt_opts o2 = o;
    o2.flags &= ~IPT_FLAG_CHOOSE_D;
    const ipt_status st = batched_run(h, count, ns, theta_off, delta_off, z_off, tp, dp, o2, z_pool, lambda_pool,
                                      status_pool, info, 0, ci);
    if (st != IPT_OK && st != IPT_ENOTCONV) return st;
    IPT_HIP(h, launch_pair_rows(s, count, dn, dto, dzo, dld, dk, z_pool, partner, cs, 0));
    IPT_HIP(h, hipStreamSynchronize(s));
    return st;
}

}  // namespace

ipt_status ipt_solve_batched(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                             const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                             const double *delta_pool, const ipt_opts *opts, double *z_pool, double *lambda_pool,
                             int32_t *status_pool, ipt_info *info) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    ipt_opts o;
    if (ipt_status st = check_opts(h, opts, o)) return st;
    if (o.cont_alpha > 0.0) return fail(h, IPT_EINVAL, "opts.cont_alpha: continuation is for dense solves");
    if (o.homotopy_q > 1) return fail(h, IPT_EINVAL, "opts.homotopy_q: the homotopy restart is for dense solves");
    if (o.flags & IPT_FLAG_CHOOSE_D) {
        DeviceGuard guard(h->device);
        return batched_pairs(h, count, ns, theta_off, delta_off, z_off, theta_pool, delta_pool, o, z_pool,
                             lambda_pool, status_pool, info, nullptr);
    }
    return batched_run(h, count, ns, theta_off, delta_off, z_off, theta_pool, delta_pool, o, z_pool, lambda_pool,
                       status_pool, info, 0);
}

ipt_status ipt_batched_tune(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                            const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                            const double *delta_pool, double *z_pool, double *lambda_pool, int32_t *status_pool,
                            int32_t *tiles_out) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (count < 1 || !ns || !theta_off || !delta_off || !z_off) return fail(h, IPT_EINVAL, "bad batch description");
    // Per size bucket: time two FP32 and two FP64 GEMM sweeps of (up to 512 of) its
    // problems with each tile size and keep the fastest sum.  tol = 0 keeps every
    // column active, so each sweep multiplies whole problems.
    std::vector<std::vector<int32_t>> members(IPT_TILE_BUCKETS);
    for (int32_t b = 0; b < count; ++b) {
        if (ns[b] < 1 || ns[b] > 4096) return fail(h, IPT_EINVAL, "every problem size must be in [1, 4096]");
        std::vector<int32_t> &v = members[(ns[b] - 1) / 64];
        if (v.size() < 512) v.push_back(b);
    }
    int32_t tiles[IPT_TILE_BUCKETS];
    memcpy(tiles, h->batch_tile, sizeof(tiles));
    for (int q = 0; q < IPT_TILE_BUCKETS; ++q) {
        const std::vector<int32_t> &v = members[q];
        if (v.empty()) continue;
        std::vector<int32_t> sn(v.size());
        std::vector<int64_t> sto(v.size()), sdo(v.size()), szo(v.size());
        for (size_t u = 0; u < v.size(); ++u) {
            sn[u] = ns[v[u]];
            sto[u] = theta_off[v[u]];
            sdo[u] = delta_off[v[u]];
            szo[u] = z_off[v[u]];
        }
        float best = INFINITY;
        int best_t = tiles[q];
        for (int T : {32, 64, 128}) {
            if (q == 0 && T == 128) continue;  // n <= 64: a 128 tile is mostly padding
            float total = 0.f;
            for (int prec : {IPT_PREC_LADDER, IPT_PREC_FP64}) {
                ipt_opts o;
                ipt_opts_default(&o);
                o.tol = 0.0;
                o.max_iter = 3;
                o.precision = prec;
                o.tau_32 = 0.0;
                o.sync_every = 3;
                o.flags = IPT_FLAG_TIME_KERNELS | IPT_FLAG_NO_GRAPH;
                float run_best = INFINITY;
                for (int rep = 0; rep < 2; ++rep) {
                    ipt_info inf;
                    ipt_status st = batched_run(h, (int32_t)v.size(), sn.data(), sto.data(), sdo.data(), szo.data(),
                                                theta_pool, delta_pool, o, z_pool, lambda_pool, status_pool, &inf, T);
                    if (st != IPT_OK && st != IPT_ENOTCONV) return st;
                    const float ms = inf.prec_ms[IPT_SWEEP_FP32] + inf.prec_ms[IPT_SWEEP_FP64];
                    run_best = ms < run_best ? ms : run_best;
                }
                total += run_best;
            }
            if (total < best) {
                best = total;
                best_t = T;
            }
        }
        tiles[q] = best_t;
    }
    h->last_error.clear();
    memcpy(h->batch_tile, tiles, sizeof(tiles));
    if (tiles_out) memcpy(tiles_out, tiles, sizeof(tiles));
    return IPT_OK;
}

ipt_status ipt_batched_get_tiles(ipt_handle h, int32_t *tiles) {
    if (!h || !tiles) return IPT_EINVAL;
    memcpy(tiles, h->batch_tile, sizeof(h->batch_tile));
    return IPT_OK;
}

ipt_status ipt_batched_set_tiles(ipt_handle h, const int32_t *tiles) {
    if (!h || !tiles) return IPT_EINVAL;
    for (int q = 0; q < IPT_TILE_BUCKETS; ++q)
        if (tiles[q] != 32 && tiles[q] != 64 && tiles[q] != 128)
            return fail(h, IPT_EINVAL, "tile sizes must be 32, 64 or 128");
    memcpy(h->batch_tile, tiles, sizeof(h->batch_tile));
    return IPT_OK;
}

}  // extern "C"

// ======================================================================= MLP
struct ipt_mlp_context {
    ipt_handle h = nullptr;
    int in = 0, hid = 0, depth = 0, out = 0;
    int nl = 0;                        // linear layers (depth + 1)
    int ip = 0, hp = 0, op = 0;        // in, hidden, out padded to MLP_TILE
    int64_t nparam = 0;
    std::vector<int64_t> woff, boff;   // per linear layer
    std::vector<int> lin, lout, linp, loutp;
    float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;  // FP32 weights, gradient, Adam moments
    void *wmem = nullptr;              // BF16 copies W_l and W_l^T of every layer
    std::vector<__bf16 *> wb, wbt;
    int32_t *adam_t = nullptr;         // Adam steps taken (device)
    float *loss_dev = nullptr;
    // batch buffers, for batches up to cap_bp (a multiple of MLP_TILE)
    int cap_bp = 0;
    void *bmem = nullptr;
    __bf16 *xb = nullptr, *xt = nullptr;
    std::vector<__bf16 *> hb, ht;      // hidden activations H_1..H_depth and their transposes
    __bf16 *gy = nullptr, *gyt = nullptr;
    __bf16 *gp[2] = {nullptr, nullptr}, *gpt[2] = {nullptr, nullptr};
    float *split = nullptr;
    std::vector<float *> colp;
    double *lossp = nullptr;
    hipStream_t cap = nullptr;         // capture stream of the training step's graph
};

namespace {

ipt_status mlp_fail(ipt_mlp m, ipt_status st, const std::string &msg) { return fail(m ? m->h : nullptr, st, msg); }

#define IPT_MHIP(m, expr)                                                                                      \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) return mlp_fail((m), IPT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline int pad_tile(int v) { return (int)round_up(v, MLP_TILE); }

void mlp_free_batch(ipt_mlp m) {
    if (m->bmem) (void)hipFree(m->bmem);
    m->bmem = nullptr;
    m->cap_bp = 0;
}

// split counts of the three products of layer l at padded batch bp
int split_dh(const ipt_mlp m, int bp, int l) { return mlp_split_count(bp, m->linp[l], m->loutp[l]); }
int split_fwd(const ipt_mlp m, int bp, int l) { return mlp_split_count(bp, m->loutp[l], m->linp[l]); }
int split_dw(const ipt_mlp m, int bp, int l) { return mlp_split_count(m->loutp[l], m->linp[l], bp); }

ipt_status mlp_ensure_batch(ipt_mlp m, int batch) {
    const int bp = pad_tile(batch);
    if (bp <= m->cap_bp) return IPT_OK;
    IPT_MHIP(m, hipStreamSynchronize(m->h->stream));
    mlp_free_batch(m);
    int64_t split_floats = 0;
    for (int l = 0; l < m->nl; ++l) {
        if (l > 0) split_floats = std::max(split_floats, (int64_t)split_dh(m, bp, l) * bp * m->linp[l]);
        if (l < m->depth) split_floats = std::max(split_floats, (int64_t)split_fwd(m, bp, l) * bp * m->loutp[l]);
        split_floats = std::max(split_floats, (int64_t)split_dw(m, bp, l) * m->loutp[l] * m->linp[l]);
    }
    auto layout = [&](Carve &cv) {
        m->xb = cv.take<__bf16>((size_t)bp * m->ip);
        m->xt = cv.take<__bf16>((size_t)bp * m->ip);
        m->hb.assign(m->depth, nullptr);
        m->ht.assign(m->depth, nullptr);
        for (int l = 0; l < m->depth; ++l) {
            m->hb[l] = cv.take<__bf16>((size_t)bp * m->hp);
            m->ht[l] = cv.take<__bf16>((size_t)bp * m->hp);
        }
        m->gy = cv.take<__bf16>((size_t)bp * m->op);
        m->gyt = cv.take<__bf16>((size_t)bp * m->op);
        for (int q = 0; q < 2; ++q) {
            m->gp[q] = cv.take<__bf16>((size_t)bp * m->hp);
            m->gpt[q] = cv.take<__bf16>((size_t)bp * m->hp);
        }
        m->split = cv.take<float>((size_t)std::max<int64_t>(split_floats, 1));
        m->colp.assign(m->nl, nullptr);
        for (int l = 0; l < m->nl; ++l) m->colp[l] = cv.take<float>((size_t)(bp / MLP_SLAB) * m->loutp[l]);
        m->lossp = cv.take<double>((size_t)(bp / MLP_TILE) * (m->op / MLP_TILE));
    };
    Carve sizing;
    layout(sizing);
    if (hipMalloc(&m->bmem, sizing.off + 256) != hipSuccess) {
        (void)hipGetLastError();
        m->bmem = nullptr;
        return mlp_fail(m, IPT_ENOMEM, "MLP activation buffers");
    }
    Carve cv;
    cv.base = (char *)m->bmem;
    layout(cv);
    m->cap_bp = bp;
    return IPT_OK;
}

MlpEpi epi0() {
    MlpEpi e;
    memset(&e, 0, sizeof(e));
    return e;
}

// Input packing and the hidden layers: H_l = tanh(H_{l-1} W_l^T + b_l), stored with H_l^T.
// The arguments of the one-launch hidden layers; false when the network does not fit them.
static bool mlp_fused_args(ipt_mlp m, MlpFused &f) {
    if (!mlp_fused_fits(m->depth, m->linp.data(), m->loutp.data())) return false;
    memset(&f, 0, sizeof(f));
    f.xb = m->xb;
    f.ip = m->ip;
    f.hp = m->hp;
    f.depth = m->depth;
    for (int l = 0; l < m->depth; ++l) {
        f.w[l] = m->wb[l];
        f.bias[l] = m->w + m->boff[l];
        f.hb[l] = m->hb[l];
        f.ht[l] = m->ht[l];
        f.linp[l] = m->linp[l];
        f.loutp[l] = m->loutp[l];
        f.lout[l] = m->lout[l];
    }
    return true;
}

hipError_t mlp_hidden(ipt_mlp m, hipStream_t s, int batch) {
    const int bp = pad_tile(batch);
    MlpFused f;
    if (mlp_fused_args(m, f)) {
        // narrow hidden layers: all of them in one launch, activations kept in LDS
        return mlp_hidden_fused(s, f, batch, bp);
    }
    for (int l = 0; l < m->depth; ++l) {
        MlpEpi e = epi0();
        e.mvalid = batch;
        e.nvalid = m->lout[l];
        e.bias = m->w + m->boff[l];
        e.tanh_act = 1;
        e.c16 = m->hb[l];
        e.ldc16 = m->hp;
        e.ct16 = m->ht[l];
        e.ldct16 = bp;
        const __bf16 *A = l == 0 ? m->xb : m->hb[l - 1];
        const int S = split_fwd(m, bp, l);
        hipError_t err;
        if (S > 1) {  // few tiles: split K, then bias and tanh in the reduction
            MlpEpi es = epi0();
            es.c32 = m->split;
            err = mlp_gemm(s, MLP_EPI_SPLIT, A, m->linp[l], m->wb[l], m->linp[l], bp, m->loutp[l], m->linp[l], S, es);
            if (err == hipSuccess) err = mlp_split_reduce(s, MLP_EPI_ACT, m->split, S, bp, m->loutp[l], e);
        } else {
            err = mlp_gemm(s, MLP_EPI_ACT, A, m->linp[l], m->wb[l], m->linp[l], bp, m->loutp[l], m->linp[l], 1, e);
        }
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// One step of the loss and its gradient after the hidden layers: output layer with the
// loss epilogue, then layer by layer the input gradient (split K, with the tanh
// derivative) before the weight gradient (which, with adam, updates W_l and its BF16
// copies), then the biases and the loss.
hipError_t mlp_backward(ipt_mlp m, hipStream_t s, const float *tg, const float *roww, int batch, bool adam, float lr) {
    const int bp = pad_tile(batch), L = m->nl, last = L - 1;
    hipError_t err;
    {
        MlpEpi e = epi0();
        e.mvalid = batch;
        e.nvalid = m->out;
        e.bias = m->w + m->boff[last];
        e.tgt = tg;
        e.roww = roww;
        e.ldt = m->out;
        e.scale = (float)(2.0 / ((double)batch * (double)m->out));
        e.lossp = m->lossp;
        e.c16 = m->gy;
        e.ldc16 = m->op;
        e.ct16 = m->gyt;
        e.ldct16 = bp;
        e.colp = m->colp[last];
        e.ldcolp = m->op;
        if ((err = mlp_gemm(s, MLP_EPI_MSE, m->hb[m->depth - 1], m->hp, m->wb[last], m->linp[last], bp, m->op,
                            m->linp[last], 1, e)) != hipSuccess)
            return err;
    }
    const __bf16 *cur = m->gy, *curt = m->gyt;
    int64_t ldcur = m->op;
    for (int l = last; l >= 0; --l) {
        if (l > 0) {
            const int S = split_dh(m, bp, l);
            MlpEpi es = epi0();
            es.c32 = m->split;
            if ((err = mlp_gemm(s, MLP_EPI_SPLIT, cur, ldcur, m->wbt[l], m->loutp[l], bp, m->linp[l], m->loutp[l], S,
                                es)) != hipSuccess)
                return err;
            const int q = l & 1;
            MlpEpi e = epi0();
            e.mvalid = batch;
            e.nvalid = m->lin[l];
            e.h = m->hb[l - 1];
            e.ldh = m->hp;
            e.c16 = m->gp[q];
            e.ldc16 = m->hp;
            e.ct16 = m->gpt[q];
            e.ldct16 = bp;
            e.colp = m->colp[l - 1];
            e.ldcolp = m->loutp[l - 1];
            if ((err = mlp_split_reduce(s, MLP_EPI_SPLIT, m->split, S, bp, m->linp[l], e)) != hipSuccess) return err;
        }
        MlpEpi e = epi0();
        e.mvalid = m->lout[l];
        e.nvalid = m->lin[l];
        if (adam) {
            e.w = m->w + m->woff[l];
            e.am = m->am + m->woff[l];
            e.av = m->av + m->woff[l];
            e.adam_t = m->adam_t;
            e.lr = lr;
            e.c16 = m->wb[l];
            e.ldc16 = m->linp[l];
            e.ct16 = m->wbt[l];
            e.ldct16 = m->loutp[l];
        } else {
            e.c32 = m->g + m->woff[l];
            e.ldc32 = m->lin[l];
        }
        const __bf16 *B = l == 0 ? m->xt : m->ht[l - 1];
        const int S = adam ? split_dw(m, bp, l) : 1;
        if (S > 1) {  // few tiles: split K (the batch), then Adam in the reduction
            MlpEpi es = epi0();
            es.c32 = m->split;
            if ((err = mlp_gemm(s, MLP_EPI_SPLIT, curt, bp, B, bp, m->loutp[l], m->linp[l], bp, S, es)) != hipSuccess ||
                (err = mlp_split_reduce(s, MLP_EPI_ADAM, m->split, S, m->loutp[l], m->linp[l], e)) != hipSuccess)
                return err;
        } else if ((err = mlp_gemm(s, adam ? MLP_EPI_ADAM : MLP_EPI_GRAD, curt, bp, B, bp, m->loutp[l], m->linp[l], bp,
                                   1, e)) != hipSuccess) {
            return err;
        }
        if (l > 0) {
            cur = m->gp[l & 1];
            curt = m->gpt[l & 1];
            ldcur = m->hp;
        }
    }
    MlpBiasLayers bl;
    memset(&bl, 0, sizeof(bl));
    bl.count = L;
    for (int l = 0; l < L; ++l) {
        bl.lout[l] = m->lout[l];
        bl.boff[l] = m->boff[l];
        bl.colp[l] = m->colp[l];
        bl.ldcolp[l] = m->loutp[l];
        // the output layer's sums come per GEMM tile, the hidden layers' per reduction slab
        bl.mtiles[l] = l == L - 1 ? bp / MLP_TILE : bp / MLP_SLAB;
    }
    if ((err = mlp_bias_step(s, bl, adam ? 1 : 0, m->w, m->g, m->am, m->av, m->adam_t, lr)) != hipSuccess)
        return err;
    return mlp_loss_step(s, m->lossp, (bp / MLP_TILE) * (m->op / MLP_TILE),
                         1.0 / ((double)batch * (double)m->out), m->loss_dev, m->adam_t, adam ? 1 : 0);
}

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

hipError_t mlp_pack_all_weights(ipt_mlp m, hipStream_t s) {
    for (int l = 0; l < m->nl; ++l) {
        hipError_t e = mlp_pack_weights(s, m->w + m->woff[l], m->lout[l], m->lin[l], m->wb[l], m->wbt[l], m->loutp[l],
                                        m->linp[l]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

ipt_status mlp_check_x(ipt_mlp m, const float *x, int32_t batch) {
    if (!x || batch < 1 || batch > (1 << 20)) return mlp_fail(m, IPT_EINVAL, "bad MLP input (batch in [1, 2^20])");
    return IPT_OK;
}

}  // namespace

extern "C" {

ipt_status ipt_mlp_create(ipt_handle h, int32_t in_dim, int32_t hidden, int32_t depth, int32_t out_dim, uint64_t seed,
                          ipt_mlp *out) {
    if (!h || !out) return IPT_EINVAL;
    *out = nullptr;
    if (in_dim < 1 || hidden < 1 || depth < 1 || depth > 16 || out_dim < 1 || in_dim > (1 << 16) ||
        hidden > (1 << 16) || out_dim > (1 << 26))
        return fail(h, IPT_EINVAL, "MLP sizes must be >= 1 (depth <= 16, in and hidden <= 2^16, out <= 2^26)");
    DeviceGuard guard(h->device);
    ipt_mlp m = new (std::nothrow) ipt_mlp_context();
    if (!m) return IPT_ENOMEM;
    m->h = h;
    m->in = in_dim;
    m->hid = hidden;
    m->depth = depth;
    m->out = out_dim;
    m->nl = depth + 1;
    m->ip = pad_tile(in_dim);
    m->hp = pad_tile(hidden);
    m->op = pad_tile(out_dim);
    int64_t off = 0, wbytes = 0;
    for (int l = 0; l <= depth; ++l) {
        const int li = l == 0 ? in_dim : hidden, lo = l == depth ? out_dim : hidden;
        m->lin.push_back(li);
        m->lout.push_back(lo);
        m->linp.push_back(pad_tile(li));
        m->loutp.push_back(pad_tile(lo));
        m->woff.push_back(off);
        off += (int64_t)li * lo;
        m->boff.push_back(off);
        off += lo;
        wbytes += 2 * (int64_t)m->linp[l] * m->loutp[l];
    }
    m->nparam = off;
    std::vector<float> host(off, 0.f);
    uint64_t st = seed;
    for (int l = 0; l <= depth; ++l) {
        const double a = sqrt(6.0 / (double)(m->lin[l] + m->lout[l]));  // Glorot uniform
        for (int64_t e = 0; e < (int64_t)m->lin[l] * m->lout[l]; ++e) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            host[m->woff[l] + e] = (float)((2.0 * u - 1.0) * a);
        }
    }
    const size_t bytes = sizeof(float) * off;
    if (hipMalloc(&m->w, bytes) != hipSuccess || hipMalloc(&m->g, bytes) != hipSuccess ||
        hipMalloc(&m->am, bytes) != hipSuccess || hipMalloc(&m->av, bytes) != hipSuccess ||
        hipMalloc(&m->wmem, sizeof(__bf16) * wbytes + 256 * 2 * m->nl) != hipSuccess ||
        hipMalloc(&m->adam_t, sizeof(int32_t)) != hipSuccess || hipMalloc(&m->loss_dev, sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        ipt_mlp_destroy(m);
        return fail(h, IPT_ENOMEM, "MLP parameter buffers");
    }
    Carve cv;
    cv.base = (char *)m->wmem;
    for (int l = 0; l <= depth; ++l) {
        m->wb.push_back(cv.take<__bf16>((size_t)m->linp[l] * m->loutp[l]));
        m->wbt.push_back(cv.take<__bf16>((size_t)m->linp[l] * m->loutp[l]));
    }
    hipStream_t s = h->stream;
    if (hipMemcpyAsync(m->w, host.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(m->am, 0, bytes, s) != hipSuccess || hipMemsetAsync(m->av, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(m->adam_t, 0, sizeof(int32_t), s) != hipSuccess || mlp_pack_all_weights(m, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        ipt_mlp_destroy(m);
        return fail(h, IPT_EHIP, "MLP initialisation");
    }
    *out = m;
    return IPT_OK;
}

ipt_status ipt_mlp_destroy(ipt_mlp m) {
    if (!m) return IPT_EINVAL;
    DeviceGuard guard(m->h->device);
    (void)hipStreamSynchronize(m->h->stream);
    mlp_free_batch(m);
    for (void *p : {(void *)m->w, (void *)m->g, (void *)m->am, (void *)m->av, (void *)m->wmem, (void *)m->adam_t,
                    (void *)m->loss_dev})
        if (p) (void)hipFree(p);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    delete m;
    return IPT_OK;
}

int64_t ipt_mlp_num_params(ipt_mlp m) { return m ? m->nparam : -1; }

ipt_status ipt_mlp_get_params(ipt_mlp m, float *dst) {
    if (!m || !dst) return IPT_EINVAL;
    DeviceGuard guard(m->h->device);
    IPT_MHIP(m, hipMemcpyAsync(dst, m->w, sizeof(float) * m->nparam, hipMemcpyDeviceToDevice, m->h->stream));
    IPT_MHIP(m, hipStreamSynchronize(m->h->stream));
    return IPT_OK;
}

ipt_status ipt_mlp_set_params(ipt_mlp m, const float *src) {
    if (!m || !src) return IPT_EINVAL;
    DeviceGuard guard(m->h->device);
    IPT_MHIP(m, hipMemcpyAsync(m->w, src, sizeof(float) * m->nparam, hipMemcpyDeviceToDevice, m->h->stream));
    IPT_MHIP(m, mlp_pack_all_weights(m, m->h->stream));
    IPT_MHIP(m, hipStreamSynchronize(m->h->stream));
    return IPT_OK;
}

ipt_status ipt_mlp_forward(ipt_mlp m, const float *x, int32_t batch, float *y) {
    if (!m) return IPT_EINVAL;
    if (ipt_status st = mlp_check_x(m, x, batch)) return st;
    if (!y) return mlp_fail(m, IPT_EINVAL, "y must be non-NULL");
    DeviceGuard guard(m->h->device);
    if (ipt_status st = mlp_ensure_batch(m, batch)) return st;
    hipStream_t s = m->h->stream;
    const int bp = pad_tile(batch);
    MlpEpi e = epi0();
    e.mvalid = batch;
    e.nvalid = m->out;
    e.bias = m->w + m->boff[m->nl - 1];
    e.c32 = y;
    e.ldc32 = m->out;
    IPT_MHIP(m, mlp_gemm(s, MLP_EPI_F32, m->hb[m->depth - 1], m->hp, m->wb[m->nl - 1], m->hp, bp, m->op, m->hp, 1, e));
    IPT_MHIP(m, hipStreamSynchronize(s));
    return IPT_OK;
}

ipt_status ipt_mlp_loss_grad(ipt_mlp m, const float *x, const float *targets, const float *weights, int32_t batch,
                             float *loss, float *grad) {
    if (!m) return IPT_EINVAL;
    if (ipt_status st = mlp_check_x(m, x, batch)) return st;
    if (!targets) return mlp_fail(m, IPT_EINVAL, "targets must be non-NULL");
    DeviceGuard guard(m->h->device);
    if (ipt_status st = mlp_ensure_batch(m, batch)) return st;
    hipStream_t s = m->h->stream;
    IPT_MHIP(m, mlp_pack_x(s, x, batch, m->in, m->xb, m->xt, pad_tile(batch), m->ip));
    IPT_MHIP(m, mlp_hidden(m, s, batch));
    IPT_MHIP(m, mlp_backward(m, s, targets, weights, batch, false, 0.f));
    if (grad) IPT_MHIP(m, hipMemcpyAsync(grad, m->g, sizeof(float) * m->nparam, hipMemcpyDeviceToDevice, s));
    float l = 0.f;
    IPT_MHIP(m, hipMemcpyAsync(&l, m->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s));
    IPT_MHIP(m, hipStreamSynchronize(s));
    if (loss) *loss = l;
    return IPT_OK;
}

ipt_status ipt_mlp_train(ipt_mlp m, const float *x, const float *targets, const float *weights, int32_t batch,
                         int32_t steps, float lr, float *loss) {
    if (!m) return IPT_EINVAL;
    if (ipt_status st = mlp_check_x(m, x, batch)) return st;
    if (!targets || steps < 0 || !(lr > 0.f)) return mlp_fail(m, IPT_EINVAL, "bad MLP training arguments");
    DeviceGuard guard(m->h->device);
    if (ipt_status st = mlp_ensure_batch(m, batch)) return st;
    hipStream_t s = m->h->stream;
    IPT_MHIP(m, mlp_pack_x(s, x, batch, m->in, m->xb, m->xt, pad_tile(batch), m->ip));
    if (steps > 0) {
        // one Adam step as a graph (its launches depend only on this call's arguments;
        // the step count lives on the device), replayed `steps` times on the stream
        if (!m->cap) IPT_MHIP(m, hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking));
        IPT_MHIP(m, hipStreamBeginCapture(m->cap, hipStreamCaptureModeRelaxed));
        hipError_t e1 = mlp_hidden(m, m->cap, batch);
        if (e1 == hipSuccess) e1 = mlp_backward(m, m->cap, targets, weights, batch, true, lr);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(m->cap, &graph);
        hipGraphExec_t exec = nullptr;
        hipError_t e3 = (e1 == hipSuccess && e2 == hipSuccess) ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)
                                                                : (e1 != hipSuccess ? e1 : e2);
        if (graph) (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            if (exec) (void)hipGraphExecDestroy(exec);
            return mlp_fail(m, IPT_EHIP, std::string("training-step graph: ") + hipGetErrorString(e3));
        }
        hipError_t e4 = hipSuccess;
        for (int32_t it = 0; it < steps && e4 == hipSuccess; ++it) e4 = hipGraphLaunch(exec, s);
        const hipError_t e5 = hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(exec);
        if (e4 != hipSuccess || e5 != hipSuccess)
            return mlp_fail(m, IPT_EHIP, std::string("training steps: ") + hipGetErrorString(e4 != hipSuccess ? e4 : e5));
    }
    float l = 0.f;
    IPT_MHIP(m, hipMemcpyAsync(&l, m->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s));
    IPT_MHIP(m, hipStreamSynchronize(s));
    if (loss) *loss = l;
    return IPT_OK;
}

ipt_status ipt_mlp_predict_z0(ipt_mlp m, const float *x, int32_t batch, const float *mu, const float *sigma,
                              const double *eps, int32_t order, const double *terms, int64_t n, int64_t k,
                              const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride) {
    if (!m) return IPT_EINVAL;
    if (ipt_status st = mlp_check_x(m, x, batch)) return st;
    if (!mu || !sigma || !eps || !idx || !z0 || n < 1 || k < 1 || k > n || ldz0 < k || n * k != m->out ||
        pstride < (n - 1) * ldz0 + k || order < 0 || order > 16 || (order > 0 && !terms))
        return mlp_fail(m, IPT_EINVAL, "bad warm-start arguments (out_dim must be n k, 0 <= order <= 16)");
    DeviceGuard guard(m->h->device);
    if (ipt_status st = mlp_ensure_batch(m, batch)) return st;
    hipStream_t s = m->h->stream;
    const int bp = pad_tile(batch);
    IPT_MHIP(m, mlp_pack_x(s, x, batch, m->in, m->xb, m->xt, bp, m->ip));
    IPT_MHIP(m, mlp_hidden(m, s, batch));
    MlpEpi e = epi0();
    e.mvalid = batch;
    e.nvalid = m->out;
    e.bias = m->w + m->boff[m->nl - 1];
    e.z0 = z0;
    e.ldz0 = ldz0;
    e.pstride = pstride;
    e.kcols = k;
    e.idx = idx;
    e.mu = mu;
    e.sigma = sigma;
    e.eps = eps;
    e.terms = terms;
    e.order = order;
    MlpFused f;
    if (mlp_fused_args(m, f)) {
        // narrow hidden layers: one launch reading x itself (no packed copy, no H^T)
        IPT_MHIP(m, mlp_hidden_fused(s, f, batch, bp, x, m->in));
    } else {
        IPT_MHIP(m, mlp_pack_x(s, x, batch, m->in, m->xb, m->xt, bp, m->ip));
        IPT_MHIP(m, mlp_hidden(m, s, batch));
    }
    IPT_MHIP(m, mlp_gemm(s, MLP_EPI_WARM, m->hb[m->depth - 1], m->hp, m->wb[m->nl - 1], m->hp, bp, m->op, m->hp, 1, e));
    IPT_MHIP(m, hipStreamSynchronize(s));
    return IPT_OK;
}

ipt_status ipt_mlp_targets(ipt_handle h, const double *z, int32_t batch, int64_t n, int64_t k, int64_t ldz,
                           int64_t pstride, const int32_t *idx, const double *eps, int32_t order, const double *terms,
                           const double *weights, float *targets, float *mu, float *sigma) {
    if (!h) return IPT_EINVAL;
    if (!z || !idx || !eps || !targets || !mu || !sigma || batch < 1 || n < 1 || k < 1 || k > n || ldz < k ||
        pstride < (n - 1) * ldz + k || order < 0 || order > 16 || (order > 0 && !terms))
        return fail(h, IPT_EINVAL, "bad target arguments");
    DeviceGuard guard(h->device);
    IPT_HIP(h, mlp_targets(h->stream, z, batch, n, k, ldz, pstride, idx, eps, order, terms, weights, targets, mu,
                           sigma));
    IPT_HIP(h, hipStreamSynchronize(h->stream));
    return IPT_OK;
}

ipt_status ipt_rs_terms(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                        const int32_t *idx, int32_t order, double *terms) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (n < 1 || n > (int64_t(1) << 20) || k < 1 || k > n || lda < n || order < 1 || order > 16)
        return fail(h, IPT_EINVAL, "need 1 <= k <= n <= 2^20, lda >= n, 1 <= order <= 16");
    if (!theta || !delta || !idx || !terms) return fail(h, IPT_EINVAL, "theta, delta, idx and terms must be non-NULL");
    DeviceGuard guard(h->device);
    hipStream_t s = h->stream;
    Carve sizing;
    sizing.take<double>((size_t)n * k);
    sizing.take<double>((size_t)order * k);
    sizing.take<int32_t>(1);
    if (ipt_status st = ensure_ws(h, sizing.off + 256)) return st;
    Carve cv;
    cv.base = (char *)h->ws;
    double *y = cv.take<double>((size_t)n * k);
    double *d = cv.take<double>((size_t)order * k);
    int32_t *err = cv.take<int32_t>(1);
    IPT_HIP(h, rs_clear(s, err));
    IPT_HIP(h, rs_gather(s, delta, lda, idx, n, k, y, err));
    for (int32_t l = 1; l <= order; ++l) {
        if (l > 1) IPT_HIP(h, rs_product(s, delta, lda, terms + (int64_t)(l - 2) * n * k, n, k, y));
        IPT_HIP(h, rs_term(s, theta, idx, y, terms, d, l, n, k, err));
    }
    int32_t herr = 0;
    IPT_HIP(h, hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IPT_HIP(h, hipStreamSynchronize(s));
    if (herr & 1) return fail(h, IPT_EINVAL, "idx out of range");
    if (herr & 2) return fail(h, IPT_EDEGENERATE, "theta_j == theta_idx[c] for some j != idx[c], or theta not finite");
    return IPT_OK;
}

ipt_status ipt_rs_start(ipt_handle h, const double *eps, int32_t count, int32_t order, const double *terms, int64_t n,
                        int64_t k, const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride) {
    if (!h) return IPT_EINVAL;
    h->last_error.clear();
    if (!eps || !idx || !z0 || (order > 0 && !terms) || count < 1 || n < 1 || k < 1 || k > n || ldz0 < k ||
        pstride < (n - 1) * ldz0 + k || order < 0 || order > 16)
        return fail(h, IPT_EINVAL, "bad series-start arguments");
    DeviceGuard guard(h->device);
    IPT_HIP(h, rs_start(h->stream, eps, count, order, terms, n, k, idx, z0, ldz0, pstride));
    IPT_HIP(h, hipStreamSynchronize(h->stream));
    return IPT_OK;
}

}  // extern "C"
