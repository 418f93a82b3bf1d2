// engine.hpp -- internal interface between the C ABI (api.cpp) and the
// kernels (kernels.hip).  Not installed; the public interface is clgc.h.
#pragma once
#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "philox.hpp"
#include "su3.hpp"

namespace clgc {

// compact per-run state copied to the host after a batched step
struct GatherRec {
    int64_t step;
    int32_t status;
    int32_t pad;
    double eps, kmax, unorm, d_pre;
};

// one launch of a batch: device header and run table, logical blocks per kind
struct Launch {
    const BatchHdr* hdr;
    const RunArgs* runs;
    int blocks[NKIND];
    int nrun;
    int fast = 0;       // a single run whose RunArgs travel in the kernel arguments
    RunArgs one{};      // that copy (kept equal to the device RunArgs by the host)
    hipStream_t stream;
    hipEvent_t ev_start = nullptr;  // if set, the next launch records these two events
    hipEvent_t ev_stop = nullptr;   // at its own start and end (kernel timing)
};

hipError_t launch_init(const Launch& L, int prec, int perturbed, double sx, double sy);
hipError_t launch_unorm(const Launch& L, int prec);
hipError_t launch_unpack(const Launch& L, int prec, const double* aos);
hipError_t launch_pack(const Launch& L, int prec, const void* field, double* aos);
// record (single lattice, FP64 with a theta term): the clover kernel also
// leaves the plaquette traces and link norms and launch_record_charge the
// charge density, as partials for FIN_RECORD_STEP (layout at record_partial)
hipError_t launch_clover(const Launch& L, int prec, int only_theta, bool record = false);
hipError_t launch_drift(const Launch& L, int prec, bool theta);
hipError_t launch_record_charge(const Launch& L);
hipError_t launch_update(const Launch& L, int prec);
// phase 0: even-site Omega (k_cool_omega); phase 1: apply both half-sweeps (k_cool_apply)
hipError_t launch_cool(const Launch& L, int prec, int phase, int iter);
hipError_t launch_gradnorm(const Launch& L, int prec, int iter);
// from_f (FP64 only): the clover field of the current links is in F; otherwise
// each site forms its clover matrices itself in FP64 (always for mixed precision)
hipError_t launch_measure(const Launch& L, int prec, bool from_f);
hipError_t launch_finalize(const Launch& L, int what, int iter);
hipError_t launch_gather(const Launch& L, GatherRec* out);
hipError_t launch_write_args(RunArgs* dst, const RunArgs& src, hipStream_t st);
hipError_t launch_write_state(Ctrl* c, int64_t step, double bound, hipStream_t st);
hipError_t launch_zero(double* p, int n, hipStream_t st);

// The applying cooling kernel, the update and the gradient-norm pass use at
// most kMaxCoolBlocks logical blocks per run; a block loops over contiguous
// chunks of 256 lanes.  The partial sums of one cooling step then stay few
// enough that the next step's blocks reduce them themselves, with no
// finalize launch in between.  cool_blocks picks the
// count: FP64 up to 512 (512 blocks of 256 threads at two waves per SIMD
// already fill the 256 CUs); mixed precision, whose prefetching kernels run
// best at about four chunks per block on large lattices, a quarter of the
// chunks between 512 and 2048.
constexpr int kMaxCoolBlocks = 2048;
__host__ __device__ inline int cool_chunks_total(int V) { return (2 * V + kBlock - 1) / kBlock; }

// the chunks [c0, c1) of logical block lb when nch chunks of kBlock lanes are
// spread over nblk blocks in contiguous runs (empty for blocks past the end)
__host__ __device__ inline void chunk_range(int nch, int nblk, int lb, int& c0, int& c1)
{
    const int per = (nch + nblk - 1) / nblk;
    c0 = lb * per;
    c1 = (lb + 1) * per < nch ? (lb + 1) * per : nch;
}

__host__ __device__ inline int cool_blocks(int V, int prec)
{
    const int nch = cool_chunks_total(V);
    int cap = 512;
    if (prec) {
        cap = nch / 4;
        cap = cap < 512 ? 512 : (cap > kMaxCoolBlocks ? kMaxCoolBlocks : cap);
    }
    return nch < cap ? nch : cap;
}

// Logical blocks of the omega kernel.  It writes no partial sums (it reads
// the applying kernel's and the update's, nblk[KIND_COOL] of them), so its
// count is its own: FP64 one chunk per block, where the plain kernel (about
// 100 registers, four waves per SIMD) beats the prefetching one on large
// lattices; mixed precision the cooling count (its prefetching kernel, four
// chunks per block on large lattices).
__host__ __device__ inline int omega_blocks(int V, int prec)
{
    return prec ? cool_blocks(V, prec) : cool_chunks_total(V);
}

// logical blocks a run of V sites in precision prec (0 FP64, 1 mixed) needs per kind
inline void blocks_per_kind(int V, int prec, int out[NKIND])
{
    out[KIND_LINK] = (4 * V + kBlock - 1) / kBlock;
    out[KIND_SITE] = (V + kBlock - 1) / kBlock;
    out[KIND_COOL] = cool_blocks(V, prec);
    const int Vh = V / 2;
    out[KIND_PLANE] = 12 * ((Vh + kBlock - 1) / kBlock);            // (region, plane, parity)
    out[KIND_DRIFT] = 8 * ((Vh + kBlock - 1) / kBlock);             // (region, mu, parity)
    out[KIND_OMEGA] = omega_blocks(V, prec);
}

constexpr int kNumPartials = 8;  // partial values per logical block of the widest kind

}  // namespace clgc
