// dl_tune.cpp -- autotuner for the hopping kernel's launch configuration.
//
// Two kernels compete.  The item kernel's tunables are the number of
// right-hand sides a thread carries (1 or 2: links loaded once serve both),
// the workgroup size (64, 128 or 256 sites) and whether the grid is
// persistent (a capped number of workgroups looping over the work items).
// The LDS-link kernel's are the wavefronts per workgroup (1, 2 or 4
// right-hand sides in flight per 64-site block), the wavefronts it allows per
// SIMD (as compiled, 1 or 2: fewer right-hand sides in flight keep more of a
// region's neighbour spinors in L2) and the region size (32, 64 or 128 site
// blocks advancing together on one XCD).  A choice is (kind, nr, bs, grid):
// kind 0 the item kernel with nr right-hand sides per thread, bs sites per
// workgroup and a persistent grid of `grid` workgroups (0: one per item);
// kind 1 the LDS-link kernel with nr wavefronts per workgroup, at most bs
// wavefronts per SIMD (0: as compiled) and regions of `grid` blocks.  The
// first time a (precision, link format, adjoint, epilogue, right-hand sides,
// lattices) combination is launched, each candidate is timed with HIP events
// on the real operands (a hopping launch is idempotent when its output
// aliases no input; the one that updates its y operand in place is timed
// with its output redirected to a scratch field of the same size); a
// candidate replaces the default only if it is 3%
// faster, and the result is kept in memory and in a text cache file
// (DL_TUNE_CACHE, default ~/.cache/dloops/tune_gfx950_v5.txt).
// DL_TUNE=0 disables tuning and uses the default: the LDS-link kernel with 2
// wavefronts, one wavefront per SIMD and regions of 64 blocks where its links
// fit in LDS (FP64 with 12-parameter links: 1 wavefront per block, four
// blocks per CU, regions of 128 blocks), else the item kernel with
// 1 right-hand side per thread and 256 sites per workgroup; DL_TUNE=item and
// DL_TUNE=lds pin those two choices (the latter where the LDS-link kernel
// applies); DL_TUNE=cfg:kind:nr:bs:grid pins one configuration the launcher
// runs (ignored where it cannot run: see launchable below).  The
// variable is read at every lookup.  Tuning never runs while the stream is
// being captured.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <tuple>
#include <vector>

#include "dl_internal.hpp"

namespace dl {

namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int, int>;
const int PERSIST_GRID = 8 * 32 * 8;  // 8 workgroups per CU on 256 CUs

std::mutex g_mu;
std::map<Key, TuneChoice> g_cache;
bool g_loaded = false;

// the lattice part of the key folds every segment's shape into one number
Key make_key(const std::vector<DslashCall> &cs)
{
    const DslashCall &c = cs[0];
    int nrhs = 0;
    long long shape = 0;
    for (const DslashCall &d : cs) {
        nrhs += d.nrhs;
        shape = shape * 1000003LL + ((((long long)d.g.X * 131 + d.g.Y) * 131 + d.g.Z) * 131 + d.g.T) * 7 + d.nrhs;
    }
    const int h1 = (int)(shape & 0x3fffffff), h2 = (int)((shape >> 30) & 0x3fffffff);
    return Key{c.prec, c.recon, c.dag ? 1 : 0, c.epi, nrhs, (int)cs.size(), h1, h2, c.g.T};
}

std::string cache_path()
{
    if (const char *p = std::getenv("DL_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/dloops/tune_gfx950_v5.txt";
}

// DL_TUNE: unset or anything else = tune; "0" = default; "item" / "lds" =
// pinned; "cfg:kind:nr:bs:grid" = that candidate (mode 5, *pin filled in)
int tune_mode(TuneChoice *pin = nullptr)
{
    const char *e = std::getenv("DL_TUNE");
    if (!e) return 0;
    if (std::strcmp(e, "0") == 0) return 1;
    if (std::strcmp(e, "item") == 0) return 2;
    if (std::strcmp(e, "lds") == 0) return 3;
    TuneChoice t;
    if (pin && std::sscanf(e, "cfg:%d:%d:%d:%d", &t.kind, &t.nr, &t.bs, &t.persistent) == 4) {
        *pin = t;
        return 5;
    }
    return 0;
}

// wavefronts per SIMD that the LDS-link kernel's LDS allows with `lanes`
// wavefronts per workgroup (a CU has four SIMDs and LDS_WORKGROUP_BYTES of LDS)
int lds_waves_per_simd(int prec, int recon, int lanes)
{
    return LDS_WORKGROUP_BYTES / lds_link_block_bytes(prec, recon) * lanes / 4;
}

// The candidate set; a cached choice outside it is ignored.  An occupancy cap
// that the LDS already enforces is no separate candidate.
std::vector<TuneChoice> candidates(int prec, int recon)
{
    std::vector<TuneChoice> v;
    for (int nr : {1, 2})
        for (int bs : {64, 128, 256})
            for (int pg : {0, PERSIST_GRID}) v.push_back(TuneChoice{0, nr, bs, pg});
    if (dslash_lds_ok(prec, recon))
        for (int lanes : {1, 2, 4})
            for (int occ : {0, 1, 2})
                if (occ == 0 || lds_waves_per_simd(prec, recon, lanes) > occ)
                    for (int rb : {32, 64, 128}) v.push_back(TuneChoice{1, lanes, occ, rb});
    return v;
}

bool valid_choice(const TuneChoice &t, int prec, int recon)
{
    for (const TuneChoice &c : candidates(prec, recon))
        if (c.kind == t.kind && c.nr == t.nr && c.bs == t.bs && c.persistent == t.persistent) return true;
    return false;
}

// a configuration the launcher runs (DL_TUNE=cfg:... may pin any of them)
bool launchable(const TuneChoice &t, int prec, int recon)
{
    if (t.kind == 0) return (t.nr == 1 || t.nr == 2) && (t.bs == 64 || t.bs == 128 || t.bs == 256) && t.persistent >= 0;
    return t.kind == 1 && dslash_lds_ok(prec, recon) && (t.nr == 1 || t.nr == 2 || t.nr == 4) && t.bs >= 0 &&
           t.bs <= 2 && t.persistent > 0;
}

TuneChoice default_choice(int prec, int recon)
{
    if (!dslash_lds_ok(prec, recon)) return TuneChoice{0, 1, 256, 0};
    // FP64 with its temporal links in registers: one wavefront per block,
    // four blocks per CU, regions of 128 blocks
    if (LDS_TLINK_REGS && prec == P64 && recon == 12) return TuneChoice{1, 1, 0, 128};
    return TuneChoice{1, 2, lds_waves_per_simd(prec, recon, 2) > 1 ? 1 : 0, 64};
}

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    FILE *f = std::fopen(cache_path().c_str(), "r");
    if (!f) return;
    int v[13];
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                       &v[7], &v[8], &v[9], &v[10], &v[11], &v[12]) == 13) {
        const TuneChoice t{v[9], v[10], v[11], v[12]};
        if (valid_choice(t, v[0], v[1])) g_cache[Key{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8]}] = t;
    }
    std::fclose(f);
}

void save_locked(const Key &k, const TuneChoice &t)
{
    std::string path = cache_path();
    std::string dir = path.substr(0, path.find_last_of('/'));
    for (size_t i = 1; i <= dir.size(); ++i)
        if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k), t.kind,
                 t.nr, t.bs, t.persistent);
    std::fclose(f);
}

bool aliases(const std::vector<DslashCall> &cs)
{
    for (const DslashCall &c : cs)
        if (c.out.d == c.in.d || (c.x.d && c.out.d == c.x.d)) return true;
    return false;
}

// calls that write their y operand in place
bool in_place(const std::vector<DslashCall> &cs)
{
    for (const DslashCall &c : cs)
        if (c.y.d && c.out.d == c.y.d) return true;
    return false;
}

}  // namespace

TuneChoice tune_lookup(const std::vector<DslashCall> &c, hipStream_t s)
{
    const TuneChoice dflt = default_choice(c[0].prec, c[0].recon);
    TuneChoice pin;
    const int mode = tune_mode(&pin);
    if (mode == 5 && launchable(pin, c[0].prec, c[0].recon)) return pin;
    if (mode == 2) return TuneChoice{0, 1, 256, 0};
    if (mode == 1 || mode == 3 || aliases(c)) return dflt;
    const Key k = make_key(c);
    std::lock_guard<std::mutex> lk(g_mu);
    if (no_alloc_active()) {
        // a call that must not allocate: a choice already in memory, else the default
        auto it = g_cache.find(k);
        return it != g_cache.end() ? it->second : dflt;
    }
    load_locked();
    auto it = g_cache.find(k);
    if (it != g_cache.end()) return it->second;
    // no timing while a graph is being captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return dflt;

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return dflt;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return dflt;
    }
    // A sample is a run of back-to-back launches spanning at least ~4 ms
    // (one launch of a 288-right-hand-side hop takes a few ms and varies by a
    // few percent from launch to launch); a candidate's time is the better of
    // two samples.  The default goes first and a later candidate must beat
    // the best so far by 3%: near-ties keep the earlier choice, so the result
    // does not wander between equivalent configurations.
    TuneChoice best = dflt;
    float best_ms = 1e30f;
    std::vector<DslashCall> t = c;
    for (DslashCall &d : t) d.live_count = nullptr;
    // in-place calls: candidates write a scratch field instead
    std::vector<DevBuf> scratch;
    if (in_place(c)) {
        try {
            for (DslashCall &d : t) {
                const size_t data = (size_t)d.nrhs * rhs_stride_bytes(d.g.Vh, elem_bytes(d.prec));
                const size_t nrm = d.prec == P16 ? (size_t)d.nrhs * (size_t)d.g.Vh * sizeof(float) : 0;
                scratch.emplace_back(data + nrm);
                d.out.d = scratch.back().p;
                d.out.nrm = nrm ? reinterpret_cast<float *>(static_cast<char *>(scratch.back().p) + data) : nullptr;
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return dflt;
        }
    }
    std::vector<TuneChoice> cands{dflt};
    for (const TuneChoice &cand : candidates(c[0].prec, c[0].recon))
        if (!(cand.kind == dflt.kind && cand.nr == dflt.nr && cand.bs == dflt.bs && cand.persistent == dflt.persistent))
            cands.push_back(cand);
    auto sample = [&](const TuneChoice &cand, int reps) {
        float ms = 0;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) launch_dslash_any(t, cand, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    for (const TuneChoice &cand : cands) {
        launch_dslash_any(t, cand, s);  // warm
        int reps = 1;
        float ms = sample(cand, reps);
        while (ms < 4.0f && reps < 256) {
            reps = ms > 0.0f ? std::min(256, std::max(2 * reps, (int)(reps * 4.5f / ms) + 1)) : 2 * reps;
            ms = sample(cand, reps);
        }
        const float per = std::min(ms, sample(cand, reps)) / reps;
        if (hipGetLastError() == hipSuccess && per < 0.97f * best_ms) {
            best_ms = per;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_cache[k] = best;
    save_locked(k, best);
    return best;
}

}  // namespace dl
