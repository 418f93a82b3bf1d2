// chain_api.cpp -- C ABI of the SU(2) Polyakov chain workload (cl_chain_*).
// A chain set lives in the caller's device buffer:
//   [links: n_chains x n_links x 8 doubles][ChainCtrl x n_chains][record]
// the record holding obs_cap steps x n_chains x 6 doubles, or the drift of
// every link for cl_chain_drift, whichever is larger.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/clgc.h"
#include "chain.hpp"
#include "host.hpp"

namespace clgc {
hipError_t chain_launch_init(const ChainArgs& a, double sx, double sy, hipStream_t st);
hipError_t chain_launch_run(const ChainArgs& a, int n_steps, hipStream_t st);
hipError_t chain_launch_drift(const ChainArgs& a, hipStream_t st);
hipError_t chain_launch_cool(const ChainArgs& a, hipStream_t st);
hipError_t chain_launch_measure(const ChainArgs& a, hipStream_t st);
}  // namespace clgc

using namespace clgc;

struct cl_chain {
    cl_chain_desc desc;
    char* base;
    size_t bytes;
    hipStream_t stream;
    ChainArgs a;
    int recorded;      // steps in the device record from the last recording run
};

namespace {

struct ChainLayout {
    size_t links, ctrl, rec, total;
};

ChainLayout chain_layout(const cl_chain_desc& d)
{
    ChainLayout L;
    const size_t nl = (size_t)d.n_chains * d.n_links * 8;
    const size_t rec = std::max((size_t)d.obs_cap * d.n_chains * kChainObs, nl);
    size_t off = 0;
    L.links = off;
    off = align256(off + sizeof(double) * nl);
    L.ctrl = off;
    off = align256(off + sizeof(ChainCtrl) * (size_t)d.n_chains);
    L.rec = off;
    off = align256(off + sizeof(double) * rec);
    L.total = off;
    return L;
}

cl_status check_chain_desc(const cl_chain_desc* d)
{
    if (!d) return fail(CL_EINVAL, "desc is NULL");
    if (d->n_links < 1 || d->n_links > kChainMaxLinks)
        return fail(CL_EINVAL, "n_links = %d must be in 1..%d", d->n_links, kChainMaxLinks);
    if (d->n_chains < 1 || d->n_chains > (1 << 24)) return fail(CL_EINVAL, "n_chains = %d out of range", d->n_chains);
    if (d->obs_cap < 0) return fail(CL_EINVAL, "obs_cap < 0");
    if (!std::isfinite(d->beta_re) || !std::isfinite(d->beta_im)) return fail(CL_EINVAL, "beta not finite");
    return CL_OK;
}

cl_status set_params(cl_chain* ch, const cl_step_desc* step, const cl_cool_desc* cool)
{
    ChainArgs& a = ch->a;
    if (step) {
        if (!(step->eps0 > 0) || !std::isfinite(step->eps0)) return fail(CL_EINVAL, "eps0 must be > 0");
        a.eps0 = step->eps0;
        a.adaptive = step->adaptive != 0;
        a.drift_bound = step->drift_bound;
    }
    a.n_cool = 0;
    if (cool) {
        if (cool->n_steps < 0 || cool->n_steps > (1 << 20)) return fail(CL_EINVAL, "cooling n_steps out of range");
        if (!(cool->eps_c >= 0) || !std::isfinite(cool->eps_c) || !std::isfinite(cool->alpha))
            return fail(CL_EINVAL, "eps_c and alpha must be finite, eps_c >= 0");
        if (cool->mode < 0 || cool->mode > 2) return fail(CL_EINVAL, "unknown cooling mode %d", cool->mode);
        a.n_cool = cool->n_steps;
        a.eps_c = cool->eps_c;
        a.alpha = cool->alpha;
        a.mode = cool->mode;
    }
    return CL_OK;
}

cl_status reset_ctrl(cl_chain* ch)
{
    std::vector<ChainCtrl> c((size_t)ch->desc.n_chains);
    std::memset(c.data(), 0, c.size() * sizeof(ChainCtrl));
    HIP_TRY(hipMemcpyAsync(ch->a.ctrl, c.data(), c.size() * sizeof(ChainCtrl), hipMemcpyHostToDevice, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    return CL_OK;
}

}  // namespace

extern "C" {

cl_status cl_chain_bytes(const cl_chain_desc* desc, size_t* device_bytes)
{
    cl_status st = check_chain_desc(desc);
    if (st) return st;
    if (!device_bytes) return fail(CL_EINVAL, "device_bytes is NULL");
    *device_bytes = chain_layout(*desc).total;
    return CL_OK;
}

cl_status cl_chain_create(const cl_chain_desc* desc, void* dev_buf, size_t buf_bytes, void* hip_stream,
                          cl_chain** out)
{
    cl_status st = check_chain_desc(desc);
    if (st) return st;
    if (!dev_buf || !out) return fail(CL_EINVAL, "NULL argument");
    if ((uintptr_t)dev_buf & 255) return fail(CL_EINVAL, "dev_buf must be 256-byte aligned");
    const ChainLayout L = chain_layout(*desc);
    if (buf_bytes < L.total) return fail(CL_EINVAL, "buffer of %zu bytes, need %zu", buf_bytes, L.total);
    cl_chain* ch = new cl_chain();
    ch->desc = *desc;
    ch->base = (char*)dev_buf;
    ch->bytes = buf_bytes;
    ch->stream = (hipStream_t)hip_stream;
    ChainArgs& a = ch->a;
    std::memset(&a, 0, sizeof a);
    a.n = desc->n_links;
    a.n_chains = desc->n_chains;
    a.beta_re = desc->beta_re;
    a.beta_im = desc->beta_im;
    a.seed = desc->seed;
    a.links = (double*)(ch->base + L.links);
    a.ctrl = (ChainCtrl*)(ch->base + L.ctrl);
    a.obs = (double*)(ch->base + L.rec);
    a.K = a.obs;
    a.obs_cap = desc->obs_cap;
    a.eps0 = 1e-2;
    a.alpha = 1.0;
    // cold start: every link the identity
    std::vector<double> id((size_t)desc->n_chains * desc->n_links * 8, 0.0);
    for (size_t l = 0; l < id.size() / 8; ++l) id[l * 8] = id[l * 8 + 6] = 1.0;
    hipError_t e = hipMemcpyAsync(a.links, id.data(), id.size() * sizeof(double), hipMemcpyHostToDevice, ch->stream);
    if (e != hipSuccess) {
        delete ch;
        return fail(CL_EHIP, "cl_chain_create: %s", hipGetErrorString(e));
    }
    if ((st = reset_ctrl(ch)) != CL_OK) {
        delete ch;
        return st;
    }
    *out = ch;
    return CL_OK;
}

cl_status cl_chain_destroy(cl_chain* ch)
{
    if (!ch) return fail(CL_EINVAL, "chain is NULL");
    delete ch;
    return CL_OK;
}

cl_status cl_chain_init(cl_chain* ch, double sigma_x, double sigma_y)
{
    if (!ch) return fail(CL_EINVAL, "chain is NULL");
    if (!std::isfinite(sigma_x) || !std::isfinite(sigma_y)) return fail(CL_EINVAL, "sigma not finite");
    HIP_TRY(chain_launch_init(ch->a, sigma_x, sigma_y, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    ch->recorded = 0;
    return CL_OK;
}

cl_status cl_chain_set_links(cl_chain* ch, const double* host, size_t n_doubles)
{
    if (!ch || !host) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)ch->desc.n_chains * ch->desc.n_links * 8;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    HIP_TRY(hipMemcpyAsync(ch->a.links, host, n * sizeof(double), hipMemcpyHostToDevice, ch->stream));
    ch->recorded = 0;
    return reset_ctrl(ch);
}

cl_status cl_chain_get_links(cl_chain* ch, double* host, size_t n_doubles)
{
    if (!ch || !host) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)ch->desc.n_chains * ch->desc.n_links * 8;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    HIP_TRY(hipMemcpyAsync(host, ch->a.links, n * sizeof(double), hipMemcpyDeviceToHost, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    return CL_OK;
}

cl_status cl_chain_run(cl_chain* ch, const cl_step_desc* step, const cl_cool_desc* cool, int n_steps, int record)
{
    if (!ch || !step) return fail(CL_EINVAL, "NULL argument");
    if (n_steps < 0) return fail(CL_EINVAL, "n_steps < 0");
    if (record && n_steps > ch->desc.obs_cap)
        return fail(CL_EINVAL, "record of %d steps exceeds obs_cap = %d", n_steps, ch->desc.obs_cap);
    cl_status st = set_params(ch, step, cool);
    if (st) return st;
    ch->a.record = record != 0;
    HIP_TRY(chain_launch_run(ch->a, n_steps, ch->stream));
    if (record) ch->recorded = n_steps;
    return CL_OK;
}

cl_status cl_chain_cool(cl_chain* ch, const cl_cool_desc* cool)
{
    if (!ch || !cool) return fail(CL_EINVAL, "NULL argument");
    cl_status st = set_params(ch, nullptr, cool);
    if (st) return st;
    HIP_TRY(chain_launch_cool(ch->a, ch->stream));
    return CL_OK;
}

cl_status cl_chain_drift(cl_chain* ch, double* host_K, size_t n_doubles, double* kmax)
{
    if (!ch || !host_K) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)ch->desc.n_chains * ch->desc.n_links * 8;
    if (n_doubles != n) return fail(CL_EINVAL, "expected %zu doubles, got %zu", n, n_doubles);
    HIP_TRY(chain_launch_drift(ch->a, ch->stream));
    HIP_TRY(hipMemcpyAsync(host_K, ch->a.K, n * sizeof(double), hipMemcpyDeviceToHost, ch->stream));
    std::vector<ChainCtrl> c((size_t)ch->desc.n_chains);
    HIP_TRY(hipMemcpyAsync(c.data(), ch->a.ctrl, c.size() * sizeof(ChainCtrl), hipMemcpyDeviceToHost, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    if (kmax)
        for (size_t i = 0; i < c.size(); ++i) kmax[i] = c[i].kmax;
    ch->recorded = 0;
    return CL_OK;
}

cl_status cl_chain_measure(cl_chain* ch, cl_chain_obs* out, int cap)
{
    if (!ch || !out) return fail(CL_EINVAL, "NULL argument");
    if (cap < ch->desc.n_chains) return fail(CL_EINVAL, "cap %d < n_chains %d", cap, ch->desc.n_chains);
    HIP_TRY(chain_launch_measure(ch->a, ch->stream));
    std::vector<ChainCtrl> c((size_t)ch->desc.n_chains);
    HIP_TRY(hipMemcpyAsync(c.data(), ch->a.ctrl, c.size() * sizeof(ChainCtrl), hipMemcpyDeviceToHost, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    for (size_t i = 0; i < c.size(); ++i) {
        cl_chain_obs& o = out[i];
        std::memset(&o, 0, sizeof o);
        o.step = c[i].step;
        o.status = c[i].status;
        o.L[0] = c[i].L_re;
        o.L[1] = c[i].L_im;
        o.d = c[i].d;
        o.d_pre = c[i].d_pre;
        o.eps = c[i].eps;
        o.kmax = c[i].kmax;
        o.sum_L[0] = c[i].sum_L_re;
        o.sum_L[1] = c[i].sum_L_im;
        o.sum_d = c[i].sum_d;
        o.n_sum = c[i].sum_n;
        o.t_sum = c[i].sum_t;
    }
    return CL_OK;
}

cl_status cl_chain_record(cl_chain* ch, double* host, size_t n_doubles)
{
    if (!ch || !host) return fail(CL_EINVAL, "NULL argument");
    const size_t n = (size_t)ch->recorded * ch->desc.n_chains * kChainObs;
    if (n_doubles != n) return fail(CL_EINVAL, "the record holds %zu doubles, asked for %zu", n, n_doubles);
    if (n == 0) return CL_OK;
    HIP_TRY(hipMemcpyAsync(host, ch->a.obs, n * sizeof(double), hipMemcpyDeviceToHost, ch->stream));
    HIP_TRY(hipStreamSynchronize(ch->stream));
    return CL_OK;
}

}  // extern "C"
