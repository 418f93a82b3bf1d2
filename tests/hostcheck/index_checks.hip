// index_checks.hip -- host-side checks of the library's device index
// arithmetic, compiled for the host only (hipcc --offload-host-only) from the
// same headers the kernels include, so the functions checked are the ones the
// kernels run.  Prints one line per check; exit status 0 iff all pass.
//
//   cooling   the lanes of a cooling kernel (chunks dealt over its logical
//             blocks, four lanes per site of one parity) own every link
//             exactly once, for either parity, lane (x, mu) holding U_mu(x)
//             and U_mu(x - mu); the update's chunks cover every link once; the
//             Omega sites an applying lane reads have the other parity
//   regions   xcd_region_order permutes the regions of the drift and clover
//             launches and keeps each XCD's share on that XCD
//   slots     logical_block is a bijection of the launch slots that deals
//             each XCD a contiguous range
//   butterfly the reduction stages pair lanes by involutions inside their
//             groups; every lane of a group adds every input once and ends
//             with the same bits
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "engine.hpp"
#include "lattice.hpp"
#include "reduce.hpp"

using namespace clgc;

static int g_fail = 0;

static void report(bool ok, const char* what, const int* d)
{
    if (d) std::printf("%s %s %dx%dx%dx%d\n", ok ? "ok" : "FAIL", what, d[0], d[1], d[2], d[3]);
    else std::printf("%s %s\n", ok ? "ok" : "FAIL", what);
    if (!ok) ++g_fail;
}

static RunArgs args_of(const int* d, int prec = 0)
{
    RunArgs a;
    std::memset(&a, 0, sizeof a);
    for (int m = 0; m < 4; ++m) a.L[m] = d[m];
    a.Lh0 = d[0] / 2;
    a.V = d[0] * d[1] * d[2] * d[3];
    a.Vh = a.V / 2;
    blocks_per_kind(a.V, prec, a.nblk);
    return a;
}

static void check_cooling(const int* d, int prec)
{
    const RunArgs a = args_of(d, prec);
    const int nch = cool_chunks_total(a.V), nblk = a.nblk[KIND_COOL];
    bool ok = nblk >= 1 && nblk <= kMaxCoolBlocks;
    for (int p = 0; p < 2 && ok; ++p) {
        std::vector<unsigned char> cnt((size_t)4 * a.V, 0), chunk(nch, 0);
        for (int lb = 0; lb < nblk; ++lb) {
            int c0, c1;
            chunk_range(nch, nblk, lb, c0, c1);
            for (int c = c0; c < c1; ++c) {
                chunk[c]++;
                for (int lane = 0; lane < kBlock; ++lane) {
                    int h, mu;
                    cool_lane(c, lane, h, mu);
                    if (mu < 0 || mu > 3 || h < c * kCoolSites || h >= (c + 1) * kCoolSites) ok = false;
                    if (h >= a.Vh) continue;
                    int of, ob;
                    cool_lane_links(a, p, h, mu, of, ob);
                    if (of < 0 || of >= 4 * a.V || ob < 0 || ob >= 4 * a.V) { ok = false; continue; }
                    cnt[of]++;
                    cnt[ob]++;
                    // of is U_mu(x), starting at the lane's site x; ob is U_mu(x - mu), ending there
                    int m1, p1, h1, m2, p2, h2;
                    link_decompose(a, of, m1, p1, h1);
                    link_decompose(a, ob, m2, p2, h2);
                    const Site sb = site_coords(a, p2, h2);
                    const Site eb = site_move(a, sb, m2, +1);
                    if (m1 != mu || p1 != p || h1 != h || m2 != mu || site_half(a, eb) != h || site_parity(eb) != p)
                        ok = false;
                
                    // the Omega sites of an applying lane (odd site y): y + mu and y - mu are even
                    const Site y = site_coords(a, p, h);
                    if (site_parity(y) != p || site_half(a, y) != h) ok = false;
                    const Site f = site_move(a, y, mu, +1), b = site_move(a, y, mu, -1);
                    if (site_parity(f) != 1 - p || site_parity(b) != 1 - p) ok = false;
                    if (site_half(a, f) >= a.Vh || site_half(a, b) >= a.Vh) ok = false;
                }
            }
        }
        for (int c = 0; c < nch; ++c) ok = ok && chunk[c] == 1;
        for (size_t l = 0; l < cnt.size(); ++l) ok = ok && cnt[l] == 1;
    }
    report(ok, prec ? "cooling lanes own every link once (both parities, mixed-precision block count)"
                    : "cooling lanes own every link once (both parities, FP64 block count)",
           d);
    // the omega kernel deals the same chunks over its own block count
    {
        const int nom = a.nblk[KIND_OMEGA];
        bool ook = nom >= 1 && nom <= nch;
        std::vector<unsigned char> chunk(nch, 0);
        for (int lb = 0; lb < nom && ook; ++lb) {
            int c0, c1;
            chunk_range(nch, nom, lb, c0, c1);
            for (int c = c0; c < c1; ++c) chunk[c]++;
        }
        for (int c = 0; c < nch; ++c) ook = ook && chunk[c] == 1;
        report(ook, prec ? "omega blocks cover every chunk once (mixed-precision block count)"
                         : "omega blocks cover every chunk once (FP64 block count)",
               d);
    }
    // the update: 4V lanes in chunks over the cooling blocks
    std::vector<unsigned char> cnt((size_t)4 * a.V, 0);
    const int nu = (4 * a.V + kBlock - 1) / kBlock;
    for (int lb = 0; lb < nblk; ++lb) {
        int c0, c1;
        chunk_range(nu, nblk, lb, c0, c1);
        for (int c = c0; c < c1; ++c)
            for (int lane = 0; lane < kBlock; ++lane) {
                const int t = c * kBlock + lane;
                if (t < 4 * a.V) cnt[t]++;
            }
    }
    bool uok = true;
    for (size_t l = 0; l < cnt.size(); ++l) uok = uok && cnt[l] == 1;
    // and link_decompose inverts the link offset
    for (int l = 0; l < 4 * a.V && uok; l += 1 + a.V / 4096) {
        int mu, p, h;
        link_decompose(a, l, mu, p, h);
        uok = link_off(a, mu, site_coords(a, p, h)) == l;
    }
    report(uok, "update chunks cover every link once", d);
}

static void check_regions(const int* d)
{
    const RunArgs a = args_of(d);
    bool ok = true;
    for (int kind = 0; kind < 2; ++kind) {
        // drift blocks: (region, mu, parity), 8 per region; clover: (region, plane, parity), 12
        const int per_region = kind == 0 ? 8 : 12;
        const int nreg = (kind == 0 ? a.nblk[KIND_DRIFT] : a.nblk[KIND_PLANE]) / per_region;
        std::vector<int> seen(nreg, 0);
        for (int r = 0; r < nreg; ++r) {
            const int q = xcd_region_order(a, r, nreg);
            if (q < 0 || q >= nreg) { ok = false; continue; }
            seen[q]++;
            if (nreg % kXcds == 0 && q / (nreg / kXcds) != r / (nreg / kXcds)) ok = false;
        }
        for (int r = 0; r < nreg; ++r) ok = ok && seen[r] == 1;
    }
    report(ok, "region order is a permutation within each XCD's share", d);
}

static void check_slots(int total)
{
    const int q = (total + kXcds - 1) / kXcds;
    std::vector<int> seen(kXcds * q, 0);
    bool ok = true;
    for (int w = 0; w < kXcds * q; ++w) {
        const int b = logical_block(w, total);
        if (b < 0 || b >= kXcds * q) { ok = false; continue; }
        seen[b]++;
        if (b < total && b / q != w % kXcds) ok = false;  // XCD w mod 8 takes a contiguous range
    }
    for (int b = 0; b < kXcds * q; ++b) ok = ok && seen[b] == 1;
    char what[96];
    std::snprintf(what, sizeof what, "logical blocks of %d: a bijection of the slots, contiguous per XCD", total);
    report(ok, what, nullptr);
}

static void check_butterfly()
{
    bool ok = true;
    for (int s = 0; s < kButterflyStages; ++s)
        for (int l = 0; l < 64; ++l) {
            const int p = stage_partner(s, l);
            ok = ok && p >= 0 && p < 64 && p != l && stage_partner(s, p) == l;
            ok = ok && p / (2 * stage_span(s)) == l / (2 * stage_span(s));  // within its aligned block
        }
    report(ok, "butterfly stages are involutions within their aligned blocks", nullptr);
    unsigned long long st = 88172645463325252ull;
    auto rnd = [&]() {  // xorshift64, values in [-1, 1) with a wide exponent spread
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        const double u = (double)(st >> 11) * 0x1.0p-53;
        return (2.0 * u - 1.0) * (double)(1ull << (st & 31));
    };
    for (int T = 1; T <= 64; T *= 2) {
        bool tok = true;
        for (int trial = 0; trial < 200; ++trial) {
            double v[64];
            std::vector<int> cnt(64 * 64, 0);  // cnt[lane * 64 + input]: times input entered lane
            for (int l = 0; l < 64; ++l) {
                v[l] = rnd();
                cnt[l * 64 + l] = 1;
            }
            for (int s = 0; s < kButterflyStages; ++s) {
                if (!(T > stage_span(s))) continue;
                double nv[64];
                std::vector<int> nc(64 * 64, 0);
                for (int l = 0; l < 64; ++l) {
                    const int p = stage_partner(s, l);
                    nv[l] = v[l] + v[p];
                    for (int i = 0; i < 64; ++i) nc[l * 64 + i] = cnt[l * 64 + i] + cnt[p * 64 + i];
                }
                std::memcpy(v, nv, sizeof v);
                cnt.swap(nc);
            }
            for (int l = 0; l < 64; ++l) {
                const int g0 = l / T * T;
                tok = tok && std::memcmp(&v[l], &v[g0], sizeof(double)) == 0;
                for (int i = 0; i < 64; ++i) tok = tok && cnt[l * 64 + i] == ((i / T == l / T) ? 1 : 0);
            }
        }
        char what[96];
        std::snprintf(what, sizeof what, "butterfly over groups of %d lanes: every input once, equal bits", T);
        report(tok, what, nullptr);
    }
}

int main()
{
    static const int shapes[][4] = {
        {2, 2, 2, 2},    {4, 4, 4, 4},    {2, 6, 4, 10},   {6, 2, 2, 2},    {4, 4, 4, 6},    {6, 6, 6, 6},
        {8, 8, 8, 8},    {12, 4, 4, 4},   {4, 6, 4, 8},    {8, 8, 8, 16},   {16, 16, 16, 16}, {24, 24, 24, 8},
        {18, 18, 18, 22}, {24, 24, 24, 16}, {32, 32, 32, 16}, {32, 32, 32, 32}, {46, 46, 46, 46}};
    for (const auto& d : shapes) {
        check_cooling(d, 0);
        check_cooling(d, 1);
        check_regions(d);
    }
    for (int total : {1, 7, 8, 9, 64, 100, 512, 1000, 4096, 12345}) check_slots(total);
    check_butterfly();
    std::printf("%s: %d failed\n", g_fail ? "FAIL" : "PASS", g_fail);
    return g_fail ? 1 : 0;
}
