// api.cpp -- the C ABI of include/clgc.h on top of the kernels.
//
// A lattice lives entirely inside the caller's device buffer:
//   [links U][drift K][clover F][partials][cooling partials][Ctrl][RunArgs][BatchHdr][record]
// (K and F are adjacent so that together they can stage the host link
// array in set/get_links).  Parameters reach the device through a one-thread
// kernel that copies a RunArgs struct passed by value, so every call stays
// stream-ordered and nothing is read from host memory after the call
// returns.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/clgc.h"
#include "engine.hpp"
#include "host.hpp"

using namespace clgc;

namespace {
thread_local std::string g_err;
}  // namespace

namespace clgc {

cl_status fail(cl_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

Layout layout_of(const cl_lattice_desc& d)
{
    const size_t V = (size_t)d.dims[0] * d.dims[1] * d.dims[2] * d.dims[3];
    const size_t rs = d.precision == CL_MIXED ? sizeof(float) : sizeof(double);
    int nb[NKIND];
    blocks_per_kind((int)V, d.precision == CL_MIXED ? 1 : 0, nb);
    int maxb = 0;
    for (int k = 0; k < NKIND; ++k) maxb = nb[k] > maxb ? nb[k] : maxb;
    Layout L;
    size_t off = 0;
    L.U = off;
    off = align256(off + 72 * V * rs);
    L.K = off;
    off = align256(off + 72 * V * rs);
    L.F = off;
    off = align256(off + 108 * V * rs);
    L.part = off;
    off = align256(off + sizeof(double) * kNumPartials * (size_t)maxb);
    L.cpart = off;
    off = align256(off + sizeof(double) * kMaxCoolBlocks);
    L.ctrl = off;
    off = align256(off + sizeof(Ctrl));
    L.args = off;
    off = align256(off + sizeof(RunArgs));
    L.hdr = off;
    off = align256(off + sizeof(BatchHdr));
    L.rec = off;
    off = align256(off + sizeof(double) * kRecCap * kRecFields);
    L.total = off;
    return L;
}

cl_status check_desc(const cl_lattice_desc* d)
{
    if (!d) return fail(CL_EINVAL, "desc is NULL");
    double V = 1;
    for (int m = 0; m < 4; ++m) {
        if (d->dims[m] < 2 || (d->dims[m] & 1))
            return fail(CL_EINVAL, "extent L%d = %d must be even and >= 2", m, d->dims[m]);
        V *= d->dims[m];
    }
    // the largest field (clover: 9 x 6V complex) must stay addressable by one
    // 32-bit buffer resource
    const double cbytes = d->precision == CL_MIXED ? 8.0 : 16.0;
    if (9.0 * 6.0 * V * cbytes >= 4294967296.0)
        return fail(CL_EINVAL, "lattice of %.0f sites too large (a field must stay below 4 GiB)", V);
    if (!(d->beta > 0)) return fail(CL_EINVAL, "beta must be > 0");
    if (!std::isfinite(d->theta_re) || !std::isfinite(d->theta_im)) return fail(CL_EINVAL, "theta not finite");
    if (d->precision != CL_FP64 && d->precision != CL_MIXED) return fail(CL_EINVAL, "unknown precision");
    return CL_OK;
}

}  // namespace clgc

namespace {

hipEvent_t take_event(cl_lattice* lat)
{
    if (!lat->pool.empty()) {
        hipEvent_t e = lat->pool.back();
        lat->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void recycle_marks(cl_lattice* lat)
{
    for (auto& m : lat->marks) {
        lat->pool.push_back(m.a);
        lat->pool.push_back(m.b);
    }
    lat->marks.clear();
}

// launch `expr` (a hipError_t-returning launcher using lat->L); when the
// lattice records timings the dispatch records a start and a stop event itself
#define TIMED(lat, KIND, expr)                                                        \
    do {                                                                              \
        if ((lat)->timing) {                                                          \
            hipEvent_t ea_ = take_event(lat), eb_ = take_event(lat);                  \
            if (!ea_ || !eb_) return fail(CL_EHIP, "hipEventCreate failed");         \
            (lat)->L.ev_start = ea_;                                                  \
            (lat)->L.ev_stop = eb_;                                                   \
            const hipError_t te_ = (expr);                                            \
            (lat)->L.ev_start = (lat)->L.ev_stop = nullptr;                           \
            HIP_TRY(te_);                                                             \
            (lat)->marks.push_back({(KIND), ea_, eb_});                               \
        } else {                                                                      \
            HIP_TRY(expr);                                                            \
        }                                                                             \
    } while (0)

// the device RunArgs (read by batched launches and kept for them) and the copy
// that travels in the kernel arguments of this lattice's launches
cl_status push_args(cl_lattice* lat)
{
    HIP_TRY(launch_write_args(lat->d_args, lat->args, lat->stream));
    lat->L.one = lat->args;
    return CL_OK;
}

cl_status read_ctrl(cl_lattice* lat, Ctrl* c)
{
    HIP_TRY(hipMemcpyAsync(c, lat->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return CL_OK;
}

cl_status set_step_params(cl_lattice* lat, const cl_step_desc* s)
{
    if (!s) return fail(CL_EINVAL, "step desc is NULL");
    if (!(s->eps0 > 0) || !std::isfinite(s->eps0)) return fail(CL_EINVAL, "eps0 must be > 0");
    RunArgs& a = lat->args;
    if (a.eps0 != s->eps0 || a.adaptive != (s->adaptive != 0) || a.drift_bound != s->drift_bound) {
        a.eps0 = s->eps0;
        a.adaptive = s->adaptive != 0;
        a.drift_bound = s->drift_bound;
        return push_args(lat);
    }
    return CL_OK;
}

cl_status set_cool_params(cl_lattice* lat, const cl_cool_desc* c)
{
    if (!c) return fail(CL_EINVAL, "cool desc is NULL");
    if (c->n_steps < 0 || c->n_steps > kMaxCoolHist) return fail(CL_EINVAL, "n_steps must be in 0..%d", kMaxCoolHist);
    if (!(c->eps_c >= 0) || !std::isfinite(c->eps_c) || !std::isfinite(c->alpha))
        return fail(CL_EINVAL, "eps_c and alpha must be finite, eps_c >= 0");
    if (c->mode < 0 || c->mode > 2) return fail(CL_EINVAL, "unknown cooling mode %d", c->mode);
    RunArgs& a = lat->args;
    if (a.eps_c != c->eps_c || a.alpha != c->alpha || a.mode != c->mode || a.n_cool != c->n_steps) {
        a.eps_c = c->eps_c;
        a.alpha = c->alpha;
        a.mode = c->mode;
        a.n_cool = c->n_steps;
        return push_args(lat);
    }
    return CL_OK;
}

// device link-layout field (complex-element SoA, checkerboard) -> host layout
void soa_to_host(const cl_lattice* lat, const void* raw, double* host)
{
    const int* L = lat->desc.dims;
    const size_t V = lat->V, Vh = V / 2;
    for (int x3 = 0; x3 < L[3]; ++x3)
        for (int x2 = 0; x2 < L[2]; ++x2)
            for (int x1 = 0; x1 < L[1]; ++x1)
                for (int x0 = 0; x0 < L[0]; ++x0) {
                    const size_t s = x0 + (size_t)L[0] * (x1 + (size_t)L[1] * (x2 + (size_t)L[2] * x3));
                    const size_t p = (x0 + x1 + x2 + x3) & 1;
                    const size_t h = (x0 >> 1) + (size_t)(L[0] / 2) * (x1 + (size_t)L[1] * (x2 + (size_t)L[2] * x3));
                    for (int mu = 0; mu < 4; ++mu)
                        for (int e = 0; e < 9; ++e) {
                            const size_t src = e * 4 * V + (mu * 2 + p) * Vh + h;
                            double* dst = host + (s * 4 + mu) * 18 + 2 * e;
                            if (lat->prec == CL_MIXED) {
                                dst[0] = ((const float*)raw)[2 * src];
                                dst[1] = ((const float*)raw)[2 * src + 1];
                            } else {
                                dst[0] = ((const double*)raw)[2 * src];
                                dst[1] = ((const double*)raw)[2 * src + 1];
                            }
                        }
                }
}

// Measure the current links into the per-step record (the entry of the CL
// step that produced them).  FP64 with a theta term takes the clover field,
// built here unless it is current; otherwise each site forms its clover
// matrices itself in FP64.
cl_status enqueue_record(cl_lattice* lat)
{
    const bool from_f = lat->prec == CL_FP64 && lat->has_theta;
    if (from_f && !lat->F_valid) TIMED(lat, CL_K_CLOVER, launch_clover(lat->L, lat->prec, 0));
    if (from_f) lat->F_valid = true;
    TIMED(lat, CL_K_MEASURE, launch_measure(lat->L, lat->prec, from_f));
    TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_RECORD, 0));
    return CL_OK;
}

// One CL update.  The drift kernel leaves K_max for the update kernel, which
// forms eps itself.  fold: cooling steps follow in the same sequence and the
// first of them finishes the update (norm, step counter); otherwise, or with
// no cooling, a finalize launch does.
cl_status enqueue_step(cl_lattice* lat, bool fold)
{
    const bool theta = lat->has_theta;
    // recording: the links entering this step are the ones the previous step
    // left after its cooling.  FP64 with a theta term measures them with the
    // step's own clover kernel (its first leaf is the plaquette) and a charge
    // pass over the clover field it builds, summed before the update changes
    // the control block; otherwise a measurement kernel runs first.
    const bool rec_in_step = lat->record && theta && lat->prec == CL_FP64;
    if (theta && (!lat->F_valid || rec_in_step)) {
        TIMED(lat, CL_K_CLOVER, launch_clover(lat->L, lat->prec, 0, rec_in_step));
        lat->F_valid = true;
    }
    if (rec_in_step) TIMED(lat, CL_K_MEASURE, launch_record_charge(lat->L));
    if (lat->record && !rec_in_step) {
        cl_status st = enqueue_record(lat);
        if (st) return st;
    }
    TIMED(lat, CL_K_DRIFT, launch_drift(lat->L, lat->prec, theta));
    if (rec_in_step) TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_RECORD_STEP, 0));
    TIMED(lat, CL_K_UPDATE, launch_update(lat->L, lat->prec));
    if (!fold || lat->args.n_cool == 0) TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_UPDATE, 0));
    lat->F_valid = false;
    return CL_OK;
}

// n cooling steps; finalize: sum the last step's norm partials into the
// control block (the norm, its history entry, the status).  Inside
// cl_run_steps only the call's last step is finalized: nothing between two CL
// steps reads that norm (the next update's own partials drive D_1).
cl_status enqueue_cool(cl_lattice* lat, int n, bool finalize)
{
    for (int i = 0; i < n; ++i) {
        if (lat->args.mode == CL_ALPHA_GRAD) {
            TIMED(lat, CL_K_GRADNORM, launch_gradnorm(lat->L, lat->prec, i));
        }
        TIMED(lat, CL_K_COOL_OMEGA, launch_cool(lat->L, lat->prec, 0, i));
        TIMED(lat, CL_K_COOL_APPLY, launch_cool(lat->L, lat->prec, 1, i));
    }
    // the next cooling step reduces the apply partials itself; only the last
    // one is finalized (unitarity norm, history, status)
    if (finalize && n > 0) TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_COOL, -1));
    if (n > 0) lat->F_valid = false;
    return CL_OK;
}

// Capture n_rep full steps (drift, update, n_cool cooling steps and their
// finalize kernels) into a graph.  The kernels take the run's parameters from
// their kernel arguments (a copy of RunArgs) and its evolving state from the
// device Ctrl block, so a graph is keyed by the launch sequence (n_cool, D_2
// mode, theta) and by the RunArgs it was captured with.
cl_status ensure_graph(cl_lattice* lat, int n_cool, int n_rep, hipGraphExec_t& slot, GraphKey& slot_key)
{
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.n_cool = n_cool;
    key.mode = lat->args.mode;
    key.theta = lat->has_theta ? 1 : 0;
    key.record = lat->record ? 1 : 0;
    key.args = lat->args;
    if (slot && std::memcmp(&key, &slot_key, sizeof key) == 0) return CL_OK;
    if (slot) {
        HIP_TRY(hipGraphExecDestroy(slot));
        slot = nullptr;
    }
    if (!lat->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&lat->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = lat->stream;
    lat->stream = lat->cap_stream;
    lat->L.stream = lat->cap_stream;
    lat->F_valid = false;  // every replayed step rebuilds the clover field
    hipGraph_t g = nullptr;
    cl_status st = CL_OK;
    hipError_t e = hipStreamBeginCapture(lat->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int r = 0; r < n_rep && st == CL_OK; ++r) {
            st = enqueue_step(lat, true);
            if (st == CL_OK) st = enqueue_cool(lat, n_cool, false);
        }
        e = hipStreamEndCapture(lat->cap_stream, &g);
    }
    lat->stream = user;
    lat->L.stream = user;
    lat->F_valid = false;
    if (st != CL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CL_EHIP, "stream capture of a CL step: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CL_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    slot = ex;
    std::memcpy(&slot_key, &key, sizeof key);
    // move the graph's launch data to the device now rather than at its first launch
    HIP_TRY(hipGraphUpload(ex, lat->stream));
    return CL_OK;
}

}  // namespace

extern "C" {

const char* cl_last_error(void) { return g_err.c_str(); }

cl_status cl_lattice_bytes(const cl_lattice_desc* desc, size_t* device_bytes)
{
    cl_status st = check_desc(desc);
    if (st) return st;
    if (!device_bytes) return fail(CL_EINVAL, "device_bytes is NULL");
    *device_bytes = layout_of(*desc).total;
    return CL_OK;
}

cl_status cl_lattice_create(const cl_lattice_desc* desc, void* dev_buf, size_t buf_bytes, void* hip_stream,
                            cl_lattice** out)
{
    cl_status st = check_desc(desc);
    if (st) return st;
    if (!dev_buf || !out) return fail(CL_EINVAL, "dev_buf and out must not be NULL");
    if ((uintptr_t)dev_buf & 255) return fail(CL_EINVAL, "dev_buf must be 256-byte aligned");
    const Layout lay = layout_of(*desc);
    if (buf_bytes < lay.total)
        return fail(CL_ENOMEM, "device buffer has %zu bytes, lattice needs %zu", buf_bytes, lay.total);
    cl_lattice* lat = new cl_lattice();
    lat->desc = *desc;
    lat->prec = desc->precision;
    lat->V = desc->dims[0] * desc->dims[1] * desc->dims[2] * desc->dims[3];
    lat->base = (char*)dev_buf;
    lat->bytes = buf_bytes;
    lat->stream = (hipStream_t)hip_stream;
    lat->lay = lay;
    lat->has_theta = desc->theta_re != 0.0 || desc->theta_im != 0.0;
    lat->F_valid = false;
    lat->d_ctrl = (Ctrl*)(lat->base + lay.ctrl);
    lat->d_args = (RunArgs*)(lat->base + lay.args);
    lat->d_hdr = (BatchHdr*)(lat->base + lay.hdr);

    RunArgs& a = lat->args;
    std::memset(&a, 0, sizeof a);
    for (int m = 0; m < 4; ++m) a.L[m] = desc->dims[m];
    a.Lh0 = desc->dims[0] / 2;
    a.V = lat->V;
    a.Vh = lat->V / 2;
    a.has_theta = lat->has_theta;
    a.U = lat->base + lay.U;
    a.K = lat->base + lay.K;
    a.F = lat->base + lay.F;
    a.part = (double*)(lat->base + lay.part);
    a.cpart = (double*)(lat->base + lay.cpart);
    a.ctrl = lat->d_ctrl;
    a.beta = desc->beta;
    a.th_re = desc->theta_re;
    a.th_im = desc->theta_im;
    a.seed = desc->seed;
    a.rec = (double*)(lat->base + lay.rec);
    a.eps0 = 1e-2;
    a.eps_c = 1e-2;
    a.alpha = 1.0;
    blocks_per_kind(lat->V, lat->prec == CL_MIXED ? 1 : 0, a.nblk);

    BatchHdr hdr;
    std::memset(&hdr, 0, sizeof hdr);
    hdr.nrun = 1;
    for (int k = 0; k < NKIND; ++k) {
        hdr.total[k] = a.nblk[k];
        hdr.begin[k][0] = 0;
        hdr.begin[k][1] = a.nblk[k];
    }
    Ctrl c;
    std::memset(&c, 0, sizeof c);
    lat->L.hdr = lat->d_hdr;
    lat->L.runs = lat->d_args;
    for (int k = 0; k < NKIND; ++k) lat->L.blocks[k] = a.nblk[k];
    lat->L.nrun = 1;
    lat->L.fast = 1;
    lat->L.one = a;
    lat->L.stream = lat->stream;

    hipError_t e = hipMemcpyAsync(lat->d_hdr, &hdr, sizeof hdr, hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(lat->d_ctrl, &c, sizeof c, hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(lat->stream);
    if (e != hipSuccess) {
        delete lat;
        return fail(CL_EHIP, "cl_lattice_create: %s", hipGetErrorString(e));
    }
    if ((st = push_args(lat)) != CL_OK) {
        delete lat;
        return st;
    }
    if ((st = cl_lattice_init(lat, 0, 0.0, 0.0)) != CL_OK) {
        delete lat;
        return st;
    }
    *out = lat;
    return CL_OK;
}

cl_status cl_lattice_destroy(cl_lattice* lat)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    hipError_t e = hipStreamSynchronize(lat->stream);
    recycle_marks(lat);
    for (hipEvent_t ev : lat->pool) (void)hipEventDestroy(ev);
    if (lat->step_graph) (void)hipGraphExecDestroy(lat->step_graph);
    if (lat->multi_graph) (void)hipGraphExecDestroy(lat->multi_graph);
    if (lat->cap_stream) (void)hipStreamDestroy(lat->cap_stream);
    delete lat;
    if (e != hipSuccess) return fail(CL_EHIP, "cl_lattice_destroy: %s", hipGetErrorString(e));
    return CL_OK;
}

cl_status cl_lattice_init(cl_lattice* lat, int perturbed, double sigma_x, double sigma_y)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    if (perturbed && (!std::isfinite(sigma_x) || !std::isfinite(sigma_y)))
        return fail(CL_EINVAL, "sigma must be finite");
    HIP_TRY(launch_init(lat->L, lat->prec, perturbed ? 1 : 0, sigma_x, sigma_y));
    HIP_TRY(launch_finalize(lat->L, FIN_INIT, 0));
    // the step counter restarts: no entry of an earlier trajectory may remain
    HIP_TRY(launch_zero(lat->args.rec, kRecCap * kRecFields, lat->stream));
    lat->F_valid = false;
    return CL_OK;
}

cl_status cl_lattice_set_links(cl_lattice* lat, const double* host, size_t n_doubles)
{
    if (!lat || !host) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)lat->V * 72;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    double* stage = (double*)(lat->base + lat->lay.K);  // K and F are free between steps
    HIP_TRY(hipMemcpyAsync(stage, host, n * sizeof(double), hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(launch_unpack(lat->L, lat->prec, stage));
    HIP_TRY(launch_unorm(lat->L, lat->prec));
    HIP_TRY(launch_finalize(lat->L, FIN_UNORM, 0));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->F_valid = false;
    return CL_OK;
}

cl_status cl_lattice_get_links(cl_lattice* lat, double* host, size_t n_doubles)
{
    if (!lat || !host) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)lat->V * 72;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    double* stage = (double*)(lat->base + lat->lay.K);
    HIP_TRY(launch_pack(lat->L, lat->prec, lat->args.U, stage));
    HIP_TRY(hipMemcpyAsync(host, stage, n * sizeof(double), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->F_valid = false;  // the staging area overwrote F
    return CL_OK;
}

cl_status cl_lattice_get_state(cl_lattice* lat, int64_t* step, double* bound)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    Ctrl c;
    cl_status st = read_ctrl(lat, &c);
    if (st) return st;
    if (step) *step = c.step;
    if (bound) *bound = c.bound;
    return CL_OK;
}

cl_status cl_lattice_set_state(cl_lattice* lat, int64_t step, double bound)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    if (step < 0 || step > 0xFFFFFFFFll) return fail(CL_EINVAL, "step out of range");
    HIP_TRY(launch_write_state(lat->d_ctrl, step, bound, lat->stream));
    HIP_TRY(launch_zero(lat->args.rec, kRecCap * kRecFields, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return CL_OK;
}

cl_status cl_langevin_step(cl_lattice* lat, const cl_step_desc* step, double* eps_used)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    cl_status st = set_step_params(lat, step);
    if (st) return st;
    if ((st = enqueue_step(lat, false)) != CL_OK) return st;
    if (eps_used) {
        Ctrl c;
        if ((st = read_ctrl(lat, &c)) != CL_OK) return st;
        *eps_used = c.eps;
        if (c.status != ST_OK) return fail(CL_ENONFINITE, "non-finite drift or unitarity norm (kmax=%g)", c.kmax);
    }
    return CL_OK;
}

cl_status cl_gauge_cool(cl_lattice* lat, const cl_cool_desc* cool, double* unorm_after)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    cl_status st = set_cool_params(lat, cool);
    if (st) return st;
    if ((st = enqueue_cool(lat, cool->n_steps, true)) != CL_OK) return st;
    if (unorm_after) {
        Ctrl c;
        if ((st = read_ctrl(lat, &c)) != CL_OK) return st;
        *unorm_after = c.unorm / (12.0 * lat->V) - 1.0;
        if (c.status != ST_OK) return fail(CL_ENONFINITE, "non-finite unitarity norm");
    }
    return CL_OK;
}

cl_status cl_run_steps(cl_lattice* lat, const cl_step_desc* step, const cl_cool_desc* cool, int n_steps)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    if (n_steps < 0) return fail(CL_EINVAL, "n_steps < 0");
    cl_status st = set_step_params(lat, step);
    if (st) return st;
    if ((st = set_cool_params(lat, cool)) != CL_OK) return st;
    if (n_steps == 0) return CL_OK;
    if (lat->timing) {
        // instrumented path: individual launches bracketed by events
        for (int i = 0; i < n_steps; ++i) {
            if ((st = enqueue_step(lat, true)) != CL_OK) return st;
            if ((st = enqueue_cool(lat, cool->n_steps, false)) != CL_OK) return st;
        }
        if (cool->n_steps > 0) TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_COOL, -1));
        return lat->record ? enqueue_record(lat) : CL_OK;
    }
    // whole blocks of kGraphSteps steps from one graph (the gap between two graph
    // launches is paid once per block), the remainder from the one-step graph
    const int blocks = n_steps / kGraphSteps, rest = n_steps % kGraphSteps;
    if (blocks > 0) {
        if ((st = ensure_graph(lat, cool->n_steps, kGraphSteps, lat->multi_graph, lat->multi_key)) != CL_OK) return st;
        for (int i = 0; i < blocks; ++i) HIP_TRY(hipGraphLaunch(lat->multi_graph, lat->stream));
    }
    if (rest > 0) {
        if ((st = ensure_graph(lat, cool->n_steps, 1, lat->step_graph, lat->graph_key)) != CL_OK) return st;
        for (int i = 0; i < rest; ++i) HIP_TRY(hipGraphLaunch(lat->step_graph, lat->stream));
    }
    lat->F_valid = false;
    // the last cooling step's norm into the control block
    if (cool->n_steps > 0) HIP_TRY(launch_finalize(lat->L, FIN_COOL, -1));
    // the last step's entry (the graph steps recorded the ones before it)
    return lat->record ? enqueue_record(lat) : CL_OK;
}

cl_status cl_run_prepare(cl_lattice* lat, const cl_step_desc* step, const cl_cool_desc* cool)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    cl_status st = set_step_params(lat, step);
    if (st) return st;
    if ((st = set_cool_params(lat, cool)) != CL_OK) return st;
    if ((st = ensure_graph(lat, cool->n_steps, kGraphSteps, lat->multi_graph, lat->multi_key)) != CL_OK) return st;
    return ensure_graph(lat, cool->n_steps, 1, lat->step_graph, lat->graph_key);
}

cl_status cl_record_enable(cl_lattice* lat, int enable)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    lat->record = enable != 0;
    return CL_OK;
}

cl_status cl_record_read(cl_lattice* lat, int64_t first_step, int n, double* host)
{
    if (!lat || (n > 0 && !host)) return fail(CL_EINVAL, "NULL argument");
    if (n < 0 || first_step < 1) return fail(CL_EINVAL, "first_step must be >= 1 and n >= 0");
    Ctrl c;
    cl_status st = read_ctrl(lat, &c);
    if (st) return st;
    const int64_t last = first_step + n - 1;
    if (n > 0 && (last > c.step || first_step <= c.step - kRecCap))
        return fail(CL_EINVAL, "steps %lld..%lld not in the record (it holds the last %d of %lld steps)",
                    (long long)first_step, (long long)last, kRecCap, (long long)c.step);
    const double* rec = lat->args.rec;
    int done = 0;
    while (done < n) {
        const int64_t i = (first_step - 1 + done) % kRecCap;
        const int k = (int)std::min<int64_t>(n - done, kRecCap - i);
        HIP_TRY(hipMemcpyAsync(host + (size_t)done * kRecFields, rec + (size_t)i * kRecFields,
                               sizeof(double) * kRecFields * k, hipMemcpyDeviceToHost, lat->stream));
        done += k;
    }
    HIP_TRY(hipStreamSynchronize(lat->stream));
    // an entry holds its own step number; a step run while the record was off
    // left its slot without one
    for (int k = 0; k < n; ++k)
        if (host[(size_t)k * kRecFields] != (double)(first_step + k))
            return fail(CL_EINVAL, "step %lld was not recorded", (long long)(first_step + k));
    return CL_OK;
}

cl_status cl_unitarity_norm(cl_lattice* lat, double* d)
{
    if (!lat || !d) return fail(CL_EINVAL, "NULL argument");
    Ctrl c;
    cl_status st = read_ctrl(lat, &c);
    if (st) return st;
    *d = c.unorm / (12.0 * lat->V) - 1.0;
    if (c.status != ST_OK) return fail(CL_ENONFINITE, "non-finite state");
    return CL_OK;
}

cl_status cl_measure(cl_lattice* lat, cl_obs* out)
{
    if (!lat || !out) return fail(CL_EINVAL, "NULL argument");
    // FP64 reads the clover field; mixed precision forms it in FP64 per site
    const bool from_f = lat->prec == CL_FP64;
    if (from_f && !lat->F_valid) TIMED(lat, CL_K_CLOVER, launch_clover(lat->L, lat->prec, 0));
    if (from_f) lat->F_valid = true;
    TIMED(lat, CL_K_MEASURE, launch_measure(lat->L, lat->prec, from_f));
    TIMED(lat, CL_K_FINALIZE, launch_finalize(lat->L, FIN_MEASURE, 0));
    Ctrl c;
    cl_status st = read_ctrl(lat, &c);
    if (st) return st;
    const double V = lat->V;
    const double pi = 3.14159265358979323846;
    std::memset(out, 0, sizeof *out);
    out->plaq[0] = c.obs[0] / (18.0 * V);
    out->plaq[1] = c.obs[1] / (18.0 * V);
    const double qs = -1.0 / (256.0 * pi * pi);
    out->q[0] = qs * c.obs[4];
    out->q[1] = qs * c.obs[5];
    // S_W = beta sum_x sum_{mu<nu} [1 - (Tr P + Tr P^{-1}) / 6];  S = S_W - i theta Q
    const double sw_re = lat->desc.beta * (6.0 * V - (c.obs[0] + c.obs[2]) / 6.0);
    const double sw_im = -lat->desc.beta * (c.obs[1] + c.obs[3]) / 6.0;
    const double tr = lat->desc.theta_re, ti = lat->desc.theta_im;
    // -i theta Q = -i (tr + i ti)(qr + i qi) = (ti qr + tr qi) - i (tr qr - ti qi)
    out->action[0] = sw_re + (ti * out->q[0] + tr * out->q[1]);
    out->action[1] = sw_im - (tr * out->q[0] - ti * out->q[1]);
    // d of the links measured here (their norms summed in FP64)
    out->unorm_d = c.obs[6] / (12.0 * V) - 1.0;
    out->d_pre = c.d_pre;
    out->eps = c.eps;
    out->kmax = c.kmax;
    out->alpha = c.alpha_cur;
    out->bound = c.bound;
    out->step = c.step;
    if (c.status != ST_OK) return fail(CL_ENONFINITE, "non-finite state");
    return CL_OK;
}

cl_status cl_compute_drift(cl_lattice* lat, double* host_K, size_t n_doubles)
{
    if (!lat || !host_K) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)lat->V * 72;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    Ctrl saved;
    cl_status st = read_ctrl(lat, &saved);
    if (st) return st;
    if (lat->has_theta && !lat->F_valid) HIP_TRY(launch_clover(lat->L, lat->prec, 0));
    lat->F_valid = lat->has_theta;
    HIP_TRY(launch_drift(lat->L, lat->prec, lat->has_theta));
    HIP_TRY(launch_finalize(lat->L, FIN_DRIFT, 0));
    // raw SoA copy of the drift, reordered on the host
    const size_t rs = lat->prec == CL_MIXED ? sizeof(float) : sizeof(double);
    std::vector<char> raw((size_t)lat->V * 72 * rs);
    HIP_TRY(hipMemcpyAsync(raw.data(), lat->args.K, raw.size(), hipMemcpyDeviceToHost, lat->stream));
    // the drift kernel updated the step-size control; restore it
    HIP_TRY(hipMemcpyAsync(lat->d_ctrl, &saved, sizeof saved, hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    soa_to_host(lat, raw.data(), host_K);
    return CL_OK;
}

cl_status cl_timing_enable(cl_lattice* lat, int enable)
{
    if (!lat) return fail(CL_EINVAL, "lattice is NULL");
    HIP_TRY(hipStreamSynchronize(lat->stream));
    recycle_marks(lat);
    lat->timing = enable != 0;
    return CL_OK;
}

cl_status cl_timing_read(cl_lattice* lat, double* total_ms, int64_t* launches, int cap)
{
    if (!lat || !total_ms || !launches) return fail(CL_EINVAL, "NULL argument");
    if (cap < CL_K_COUNT) return fail(CL_EINVAL, "cap must be >= %d", (int)CL_K_COUNT);
    HIP_TRY(hipStreamSynchronize(lat->stream));
    for (int k = 0; k < cap; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    for (const auto& m : lat->marks) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b));
        total_ms[m.kind] += ms;
        launches[m.kind] += 1;
    }
    return CL_OK;
}

cl_status cl_cool_history(cl_lattice* lat, double* unorm, double* alpha, int cap, int* n)
{
    if (!lat || !n) return fail(CL_EINVAL, "NULL argument");
    Ctrl c;
    cl_status st = read_ctrl(lat, &c);
    if (st) return st;
    *n = c.hist_n;
    for (int i = 0; i <= c.hist_n && i < cap; ++i) {
        if (unorm) unorm[i] = c.hist_un[i];
        if (alpha && i < c.hist_n) alpha[i] = c.hist_alpha[i];
    }
    return CL_OK;
}

}  // extern "C"
