// lattice.hpp -- device data layout, run descriptors and index arithmetic.
//
// Link field in HBM ("complex-element SoA", checkerboard order):
//   element e (0..8, row-major) of link (mu, parity p, half-index h) is the
//   complex<T> at  U[e * 4V + (mu * 2 + p) * Vh + h],
//   h = (x0 >> 1) + (L0/2) * (x1 + L1 * (x2 + L2 * x3)),  p = (x0+x1+x2+x3) & 1.
// Consecutive lanes own consecutive h, so every load and store of one
// matrix element by a wavefront is one contiguous 1 KB (FP64) or 512 B
// (FP32) segment.  The drift field K uses the same layout; the clover field F
// stores six planes per site: element e of plane P at site (p, h) is
// F[e * 6V + P * V + p * Vh + h].
//
// Several independent runs (lattices of any even extents, each with its own
// buffers and parameters) can share one launch: the logical blocks of all
// runs are concatenated and a block finds its run by binary search in
// BatchHdr::begin.  A single lattice is a batch of one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "su3.hpp"

namespace clgc {

constexpr int kBlock = 256;        // threads per logical block, all kernels
constexpr int kXcds = 8;           // accelerator complex dies of an MI355X (one L2 each)
constexpr int kMaxRuns = 256;      // runs in one batched launch
constexpr int kMaxCoolHist = 64;   // cooling steps per call kept in the history
constexpr int kRecCap = 4096;      // CL steps kept in a lattice's per-step record (a ring)
// one record entry: step, d_pre, d, P re/im, Q re/im, S re/im, eps, Kmax, alpha_ad
constexpr int kRecFields = 12;

// logical-block kinds: what one thread owns
enum Kind : int {
    KIND_LINK = 0,   // one link: init, drift, update          (4V threads)
    KIND_SITE = 1,   // one site: measurement                  (V threads)
    KIND_COOL = 2,   // one (site of one parity, mu): cooling  (2V threads)
    KIND_PLANE = 3,  // one (site, plane): clover field        (6V threads)
    KIND_DRIFT = 4,  // one (link, 256-site region): drift    (4V threads)
    KIND_OMEGA = 5,  // one (site of one parity, mu): the omega kernel of a cooling step (2V threads)
    NKIND = 6
};

// what a finalize launch reduces
enum Finalize : int { FIN_INIT = 0, FIN_UNORM = 1, FIN_DRIFT = 2, FIN_UPDATE = 3, FIN_COOL = 4,
                      FIN_MEASURE = 6, FIN_RECORD = 7, FIN_RECORD_STEP = 8 };

enum Status : int { ST_OK = 0, ST_NONFINITE = 1 };

// Per-run control block in device memory: everything the step-size and
// cooling-strength control needs stays on the GPU between kernels.
struct Ctrl {
    double eps;         // step size of the last CL update
    double bound;       // adaptive bound B (<= 0: not set)
    double kmax;        // max ||Khat|| of the last drift
    double unorm;       // sum Tr U U^dagger of the current links
    double alpha_cur;   // alpha_ad of the cooling step in progress
    double d_pre;       // distance after the last CL update
    double obs[8];      // sums: Tr P re/im, Tr P^-1 re/im, clover Q bracket re/im, UN
    double hist_un[kMaxCoolHist + 1];
    double hist_alpha[kMaxCoolHist];
    int64_t step;       // CL step counter n (Philox counter word 1)
    int32_t status;     // Status
    int32_t hist_n;     // cooling steps recorded
    int32_t upd_pending;  // 1: the unitarity-norm partials of an applied CL update wait in
                          // cpart, for the next cooling step (or FIN_UPDATE) to finish the step
    int32_t pad;
    // max ||Khat||^2 of the drift of step n, as IEEE bit patterns (their order is the
    // order of non-negative doubles, so an integer atomic max is exact and order-free):
    // slot [n & 1][x] collects the blocks dispatched to XCD x, 128 bytes apart
    unsigned long long kslot[2][kXcds][16];
};

// Per-run descriptor (device copy written by the host when it changes).
struct RunArgs {
    int L[4];
    int Lh0;           // L0 / 2
    int Vh;            // V / 2
    int V;
    int has_theta;
    void* U;           // links, T = double or float
    void* F;           // clover field
    void* K;           // drift
    double* part;      // per-logical-block partials: part[j * nblk + b]
    double* cpart;     // the cooling step's unitarity-norm partials (<= kMaxCoolBlocks), kept
                       // apart so a D_2 gradient pass between two steps cannot overwrite them
    Ctrl* ctrl;
    double beta, th_re, th_im;
    uint64_t seed;
    double eps0, drift_bound;
    int adaptive;
    int mode;          // cl_alpha_mode
    double eps_c, alpha;
    int n_cool;        // cooling steps of the current call (batched: this run's own count)
    int nblk[NKIND];   // logical blocks of this run per kind
    double* rec;       // per-step record, kRecCap entries of kRecFields doubles (NULL: none)
};

struct BatchHdr {
    int nrun;
    int total[NKIND];
    int begin[NKIND][kMaxRuns + 1];
};

// What every kernel of the path receives: the batch tables in device memory
// and, when a single lattice is launched through the lattice API (the FAST
// instance of each kernel), a copy of its RunArgs in the kernel arguments, so
// that a block reaches its field pointers without first reading the tables
// (two dependent memory round trips fewer at every kernel start).
struct KArgs {
    const BatchHdr* hdr;
    const RunArgs* runs;
    RunArgs one;
};

// ---------------------------------------------------------------------------
// index arithmetic

// lattice coordinates; four scalars (not an array) so that runtime direction
// indices compile to selects and the struct stays in registers
struct Site {
    int x0, x1, x2, x3;
};

__host__ __device__ __forceinline__ int site_get(const Site& s, int mu)
{
    return mu == 0 ? s.x0 : (mu == 1 ? s.x1 : (mu == 2 ? s.x2 : s.x3));
}

__host__ __device__ __forceinline__ Site site_coords(const RunArgs& ra, int p, int h)
{
    Site s;
    int r = h / ra.Lh0;
    const int x0h = h - r * ra.Lh0;
    int q = r / ra.L[1];
    s.x1 = r - q * ra.L[1];
    r = q;
    q = r / ra.L[2];
    s.x2 = r - q * ra.L[2];
    s.x3 = q;
    s.x0 = 2 * x0h + ((p + s.x1 + s.x2 + s.x3) & 1);
    return s;
}

__host__ __device__ __forceinline__ int site_half(const RunArgs& ra, const Site& s)
{
    return (s.x0 >> 1) + ra.Lh0 * (s.x1 + ra.L[1] * (s.x2 + ra.L[2] * s.x3));
}

__host__ __device__ __forceinline__ int site_parity(const Site& s) { return (s.x0 + s.x1 + s.x2 + s.x3) & 1; }

__host__ __device__ __forceinline__ int site_lex(const RunArgs& ra, const Site& s)
{
    return s.x0 + ra.L[0] * (s.x1 + ra.L[1] * (s.x2 + ra.L[2] * s.x3));
}

__host__ __device__ __forceinline__ int wrap(int v, int L) { return v >= L ? v - L : (v < 0 ? v + L : v); }

// s + d * mu_hat with periodic wrap, d = +-1
__host__ __device__ __forceinline__ Site site_move(const RunArgs& ra, const Site& s, int mu, int d)
{
    Site r;
    r.x0 = mu == 0 ? wrap(s.x0 + d, ra.L[0]) : s.x0;
    r.x1 = mu == 1 ? wrap(s.x1 + d, ra.L[1]) : s.x1;
    r.x2 = mu == 2 ? wrap(s.x2 + d, ra.L[2]) : s.x2;
    r.x3 = mu == 3 ? wrap(s.x3 + d, ra.L[3]) : s.x3;
    return r;
}

// offset (in complex elements, without the e * 4V term) of link (mu, site)
__host__ __device__ __forceinline__ int link_off(const RunArgs& ra, int mu, const Site& s)
{
    return (mu * 2 + site_parity(s)) * ra.Vh + site_half(ra, s);
}

// Logical block of a launch slot.  Workgroups are dispatched to the eight
// XCDs round-robin (slot w runs on XCD w mod 8) and each XCD has its own L2:
// slot w takes logical block (w mod 8) q + w / 8, q = ceil(total / 8), so XCD
// x works through the contiguous range [x q, (x + 1) q) of the logical-block
// space, where neighbouring sites re-read each other's links.  Slots whose
// block is >= total have no work.  A bijection of [0, 8q) onto itself.
__host__ __device__ __forceinline__ int logical_block(int slot, int total)
{
    const int q = (total + kXcds - 1) / kXcds;
    return (slot % kXcds) * q + slot / kXcds;
}

// decompose a link index l in [0, 4V): l = (mu * 2 + p) * Vh + h
__host__ __device__ __forceinline__ void link_decompose(const RunArgs& ra, int l, int& mu, int& p, int& h)
{
    mu = l / ra.V;
    const int rem = l - mu * ra.V;
    p = rem >= ra.Vh;
    h = rem - p * ra.Vh;
}

// Order of the regions (256 consecutive half-indices) inside one XCD's share
// of a kernel that deals whole regions to XCDs: x3 fastest.  In half-index
// order a region's x3 neighbours come a whole x3 slice of regions later, long
// after its data left the XCD's L2; with the share transposed they run next
// to it.  A bijection on the share; the identity when the share is not a
// whole number of x3 slices.
__host__ __device__ __forceinline__ int xcd_region_order(const RunArgs& ra, int region, int nreg)
{
    const int per = nreg / kXcds;
    const int slice_h = ra.Vh / ra.L[3];
    if (nreg % kXcds || slice_h % kBlock) return region;
    const int slice = slice_h / kBlock;
    if (slice == 0 || per % slice || per / slice < 2) return region;
    const int c3 = per / slice, k = region % per;
    return region - k + (k % c3) * slice + k / c3;
}

// Cooling lanes.  A cooling step runs 4 lanes per site of one parity, in
// chunks of kBlock lanes that cover kCoolSites consecutive half-indices: lane
// t of chunk c takes the site h = kCoolSites c + (t mod kCoolSites) and the
// direction mu = t / kCoolSites, so each wavefront handles one direction for
// 64 consecutive sites and its load of a link element covers 64 neighbouring
// entries of that direction's array (with one site per four lanes, a
// wavefront's load is split over four arrays in pieces of 16 entries, which
// streams measurably slower in FP32).
constexpr int kCoolSites = kBlock / 4;
static_assert(kCoolSites == 64, "one wavefront per direction");
__host__ __device__ __forceinline__ void cool_lane(int c, int t, int& h, int& mu)
{
    h = c * kCoolSites + (t & (kCoolSites - 1));
    mu = t / kCoolSites;
}

// The lane at the site of parity p and half-index h with direction mu owns
// the links U_mu(x) and U_mu(x - mu): each link has exactly one end of each
// parity, so over all h and mu these are every link exactly once.  of / ob:
// their offsets (complex elements, without the element stride).
__host__ __device__ __forceinline__ void cool_lane_links(const RunArgs& ra, int p, int h, int mu, int& of, int& ob)
{
    const Site x = site_coords(ra, p, h);
    of = (mu * 2 + p) * ra.Vh + h;
    ob = link_off(ra, mu, site_move(ra, x, mu, -1));
}

// Field access through raw buffer instructions.  The field pointers come
// from the device-side run table, so plain pointer code compiles to flat
// loads with a 64-bit address per element; a buffer resource instead keeps
// the base in scalar registers, the element's offset (e * stride, uniform) in
// the scalar offset and only the lane's 32-bit byte offset in a vector
// register.  The resource's record count is the whole field (9 element
// slabs of stride complex numbers; the hardware range check includes the
// scalar offset): an offset beyond the field reads zero and drops the store
// instead of touching memory outside it.  Fields are limited to 4 GiB.
constexpr int kBufferWord3 = 0x00020000;  // gfx9-family raw buffer: 32-bit data format, no swizzle

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const cx<T>* base, int stride)
{
    const uint32_t bytes = 9u * (uint32_t)stride * (uint32_t)sizeof(cx<T>);
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, kBufferWord3);
}

template <typename T>
__device__ __forceinline__ cx<T> buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes, int elem_bytes)
{
    if constexpr (sizeof(T) == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 v = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane_bytes, elem_bytes, 0));
        return {v.x, v.y};
    } else {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)lane_bytes, elem_bytes, 0));
        return {v.x, v.y};
    }
}

template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes, int elem_bytes, cx<T> c)
{
    if constexpr (sizeof(T) == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        d2 v;
        v.x = c.re;
        v.y = c.im;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rs, (int)lane_bytes, elem_bytes, 0);
    } else {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        f2 v;
        v.x = c.re;
        v.y = c.im;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, (int)lane_bytes, elem_bytes, 0);
    }
}

// the matrix at lane offset off (complex units) of a field whose elements lie
// stride complex numbers apart
template <typename T>
__device__ __forceinline__ mat3<T> load_mat(const cx<T>* base, int off, int stride)
{
    const __amdgpu_buffer_rsrc_t rs = field_rsrc(base, stride);
    const uint32_t lane = (uint32_t)off * (uint32_t)sizeof(cx<T>);
    const int es = stride * (int)sizeof(cx<T>);
    mat3<T> m;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e / 3][e % 3] = buf_load<T>(rs, lane, e * es);
    return m;
}

template <typename T>
__device__ __forceinline__ void store_mat(cx<T>* base, int off, int stride, const mat3<T>& m)
{
    const __amdgpu_buffer_rsrc_t rs = field_rsrc((const cx<T>*)base, stride);
    const uint32_t lane = (uint32_t)off * (uint32_t)sizeof(cx<T>);
    const int es = stride * (int)sizeof(cx<T>);
#pragma unroll
    for (int e = 0; e < 9; ++e) buf_store<T>(rs, lane, e * es, m.e[e / 3][e % 3]);
}

// dual clover partner of plane P (0..5 = 01,02,03,12,13,23) and its sign:
// Ft01 = F23, Ft02 = -F13, Ft03 = F12, Ft12 = F03, Ft13 = -F02, Ft23 = F01.
__host__ __device__ constexpr int plane_of(int mu, int nu)
{
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}
__host__ __device__ constexpr int dual_plane(int P) { return 5 - P; }
__host__ __device__ constexpr int dual_sign(int P) { return (P == 1 || P == 4) ? -1 : 1; }

// find the run that owns logical block b of a kind (uniform per block)
__device__ __forceinline__ int find_run(const __attribute__((address_space(4))) BatchHdr* hdr, int kind, int b)
{
    int lo = 0, hi = hdr->nrun - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hdr->begin[kind][mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace clgc
