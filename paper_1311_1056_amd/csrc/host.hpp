// host.hpp -- host-side internals shared by the C ABI (api.cpp) and the
// run server (server.cpp): error reporting, the device-buffer layout of a
// lattice and the lattice handle itself.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <vector>

#include "../../include/clgc.h"
#include "engine.hpp"
#include "sched.hpp"

namespace clgc {

// sets the thread-local message returned by cl_last_error and returns st
cl_status fail(cl_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return ::clgc::fail(CL_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)


// byte offsets of a lattice's pieces inside its device buffer
struct Layout {
    size_t U, K, F, part, cpart, ctrl, args, hdr, rec, total;
};

Layout layout_of(const cl_lattice_desc& d);
cl_status check_desc(const cl_lattice_desc* d);

}  // namespace clgc

// what a captured step graph depends on: the launch sequence and the RunArgs
// copy its kernel arguments carry (compared bytewise; zero-filled first)
struct GraphKey {
    int n_cool, mode, theta, record;
    clgc::RunArgs args;
};

// steps captured into the block graph that cl_run_steps replays (the idle
// gap between two graph launches is then paid once per block)
constexpr int kGraphSteps = 8;

struct cl_lattice {
    cl_lattice_desc desc;
    int prec;
    int V;
    char* base;
    size_t bytes;
    hipStream_t stream;
    clgc::Layout lay;
    clgc::RunArgs args;      // host mirror of the device RunArgs
    clgc::RunArgs* d_args;
    clgc::BatchHdr* d_hdr;
    clgc::Ctrl* d_ctrl;
    clgc::Launch L;
    bool F_valid;      // clover field matches the current links
    bool has_theta;
    bool record;       // cl_run_steps measures every step into the device record
    // benchmark instrumentation (cl_timing_enable)
    bool timing;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    // one captured CL step (update + cooling) and a block of kGraphSteps of
    // them, replayed by cl_run_steps (captured on a private stream)
    hipStream_t cap_stream;
    hipGraphExec_t step_graph;
    GraphKey graph_key;
    hipGraphExec_t multi_graph;
    GraphKey multi_key;
};
