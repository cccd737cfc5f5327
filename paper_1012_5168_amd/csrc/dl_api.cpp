// dl_api.cpp -- the C ABI: handles, validation, the even-odd solver drivers
// (BiCGStab with FP64 reliable updates, truncated CGNR) and the loop
// estimator.  Every step of the computation runs in the library's kernels;
// the host only orders launches, polls convergence flags and moves results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "dl_internal.hpp"

using namespace dl;

// ====================================================================== errors

namespace dl {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace dl

template <typename F>
static int guarded(F &&f)
{
    try {
        g_err.clear();
        return f();
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return DL_ENOMEM;
    } catch (...) {
        g_err = "unexpected internal error";
        return DL_EHIP;
    }
}

// ====================================================================== buffers

namespace dl {

// Device memory cache.  Workspaces of repeated calls have the same sizes, and
// mapping a fresh multi-GB allocation costs about as much as the solve it
// serves, so released buffers are kept per (device, size) and handed out
// again (a cached block serves a request of at least 4/5 of its size).  A
// released block carries an event recorded on the stream of the call that
// released it (every entry point names its stream, see StreamScope); a later
// allocation that takes the block waits on that event, so no kernel still
// reading or writing the block can race with its next user.  Where no call
// stream is known the release synchronises the device instead, as hipFree
// would.  The cached bytes are capped (DL_CACHE_GB, default 64 GB, or
// dl_cache_set_limit; 0 turns the cache off); dl_cache_release frees all of
// it; an allocation that fails releases the cache and tries again.
namespace {
struct CacheEntry {
    void *p;
    hipEvent_t ready;  // recorded after the block's last use (null: the device was synchronised)
};
std::mutex g_cache_mu;
std::multimap<std::pair<int, size_t>, CacheEntry> g_cache_free;
size_t g_cache_bytes = 0;
bool g_cache_limit_set = false;
size_t g_cache_limit = 0;

// the stream of the entry point running on this thread (StreamScope)
thread_local bool t_stream_known = false;
thread_local hipStream_t t_stream = nullptr;

size_t cache_limit_locked()
{
    if (!g_cache_limit_set) {
        const char *e = std::getenv("DL_CACHE_GB");
        const double gb = e ? std::atof(e) : 64.0;
        g_cache_limit = gb > 0 ? (size_t)(gb * 1073741824.0) : (size_t)0;
        g_cache_limit_set = true;
    }
    return g_cache_limit;
}

int current_device()
{
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

void free_entry(const CacheEntry &c)
{
    if (c.ready) {
        (void)hipEventSynchronize(c.ready);
        (void)hipEventDestroy(c.ready);
    }
    (void)hipFree(c.p);
}

// free cached blocks until at most `keep` bytes remain
void cache_trim_locked(size_t keep)
{
    while (g_cache_bytes > keep && !g_cache_free.empty()) {
        auto it = std::prev(g_cache_free.end());  // largest first
        free_entry(it->second);
        g_cache_bytes -= it->first.second;
        g_cache_free.erase(it);
    }
}
}  // namespace

namespace {
thread_local bool t_no_alloc = false;
}

NoAllocScope::NoAllocScope() : prev(t_no_alloc) { t_no_alloc = true; }
NoAllocScope::~NoAllocScope() { t_no_alloc = prev; }
bool no_alloc_active() { return t_no_alloc; }

StreamScope::StreamScope(void *stream) : prev_known(t_stream_known), prev(t_stream)
{
    t_stream_known = true;
    t_stream = static_cast<hipStream_t>(stream);
}

StreamScope::~StreamScope()
{
    t_stream_known = prev_known;
    t_stream = static_cast<hipStream_t>(prev);
}

void DevBuf::alloc(size_t n)
{
    release();
    if (n == 0) return;
    const int dev = current_device();
    CacheEntry hit{nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache_free.lower_bound({dev, n});
        if (it != g_cache_free.end() && it->first.first == dev && it->first.second / 5 * 4 <= n) {
            hit = it->second;
            cap = it->first.second;
            g_cache_bytes -= cap;
            g_cache_free.erase(it);
        }
    }
    if (hit.p) {
        if (hit.ready) {
            // the block's previous user has finished with it
            const hipError_t e = hipEventSynchronize(hit.ready);
            (void)hipEventDestroy(hit.ready);
            if (e != hipSuccess) {
                (void)hipFree(hit.p);
                cap = 0;
                throw Error{DL_EHIP, std::string("waiting for a cached block: ") + hipGetErrorString(e)};
            }
        }
        p = hit.p;
        bytes = n;
        return;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            cache_trim_locked(0);
        }
        e = hipMalloc(&p, n);
    }
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Error{DL_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
    }
    bytes = cap = n;
}

void DevBuf::release() noexcept
{
    if (!p) return;
    bool cached = false;
    size_t limit = 0;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        limit = cache_limit_locked();
        if (g_cache_bytes + cap > limit) limit = 0;
    }
    if (limit > 0) {
        CacheEntry c{p, nullptr};
        bool idle = false;
        if (t_stream_known && !capturing(t_stream)) {
            if (hipEventCreateWithFlags(&c.ready, hipEventDisableTiming) == hipSuccess) {
                if (hipEventRecord(c.ready, t_stream) == hipSuccess) {
                    idle = true;
                } else {
                    (void)hipEventDestroy(c.ready);
                    c.ready = nullptr;
                }
            } else {
                c.ready = nullptr;
            }
        }
        if (!idle && !(t_stream_known && capturing(t_stream))) idle = hipDeviceSynchronize() == hipSuccess;
        if (idle) {
            try {
                std::lock_guard<std::mutex> lk(g_cache_mu);
                if (g_cache_bytes + cap <= cache_limit_locked()) {
                    g_cache_free.insert({{current_device(), cap}, c});
                    g_cache_bytes += cap;
                    cached = true;
                }
            } catch (...) {
                cached = false;
            }
        }
        if (!cached && c.ready) (void)hipEventDestroy(c.ready);
    }
    (void)hipGetLastError();
    if (!cached) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    cap = 0;
}

void HalfField::alloc(int prec_, int64_t nrhs_, int64_t Vh_)
{
    prec = prec_;
    nrhs = nrhs_;
    Vh = Vh_;
    data.alloc((size_t)nrhs * rhs_stride_bytes(Vh, elem_bytes(prec)));
    if (prec == P16)
        nrm.alloc((size_t)nrhs * Vh * sizeof(float));
    else
        nrm.release();
}

Field HalfField::view_rhs(int64_t r) const
{
    Field f;
    f.d = static_cast<char *>(data.p) + (size_t)r * rhs_stride_bytes(Vh, elem_bytes(prec));
    f.nrm = nrm.p ? nrm.as<float>() + r * Vh : nullptr;
    return f;
}

// ====================================================================== profiling

static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfSlot {
    int slot;
    double unit_bytes, fixed_bytes, units_div;
};
struct ProfRec {
    int kind, kind2;
    double bytes;
    hipEvent_t e0, e1;
    std::vector<ProfSlot> slots;
};
static std::vector<ProfRec> g_prof_pending;
static double g_prof_ms[PROF_NKIND], g_prof_bytes[PROF_NKIND];
static int64_t g_prof_n[PROF_NKIND];
// device counters, one per profiled hopping launch and lattice (never destroyed:
// no HIP call runs during static destruction at process exit)
static DevBuf &g_prof_ctr = *new DevBuf;
static TuneChoice g_prof_cfg[PROF_NKIND];  // last profiled hopping configuration per kind
static bool g_prof_cfg_set[PROF_NKIND];
static int g_prof_next = 0;
static const int PROF_SLOTS = 1 << 16;

static void prof_drain_locked();

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

bool prof_on() { return g_prof_on && !no_alloc_active(); }

unsigned *prof_counter()
{
    if (!prof_on()) return nullptr;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_ctr.p) return nullptr;
    if (g_prof_next >= PROF_SLOTS) prof_drain_locked();
    return g_prof_ctr.as<unsigned>() + g_prof_next++;
}

ProfScope::ProfScope(int kind_, double bytes_, hipStream_t s_, int kind2_)
    : kind(kind_), kind2(kind2_), bytes(bytes_), s(s_)
{
    if (!prof_on() || capturing(s)) return;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        e0 = e1 = nullptr;
        return;
    }
    (void)hipEventRecord(e0, s);
}

ProfScope::~ProfScope()
{
    if (!e0) return;
    (void)hipEventRecord(e1, s);
    try {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        ProfRec r{kind, kind2, bytes, e0, e1, {}};
        for (const ProfPart &p : parts)
            if (p.counter)
                r.slots.push_back(
                    {(int)(p.counter - g_prof_ctr.as<unsigned>()), p.unit_bytes, p.fixed_bytes, p.units_div});
        g_prof_pending.push_back(r);
    } catch (...) {
        // out of host memory: this launch goes unrecorded (a destructor must not throw)
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
}

static void prof_drain_locked()
{
    std::vector<unsigned> ctr;
    if (g_prof_ctr.p && g_prof_next > 0) {
        (void)hipDeviceSynchronize();
        ctr.resize(g_prof_next);
        (void)hipMemcpy(ctr.data(), g_prof_ctr.p, sizeof(unsigned) * g_prof_next, hipMemcpyDeviceToHost);
    }
    for (auto &r : g_prof_pending) {
        float ms = 0;
        if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            double by = r.bytes;
            if (!r.slots.empty()) {
                by = 0;
                for (const ProfSlot &ps : r.slots) {
                    const double units = (ps.slot >= 0 && ps.slot < (int)ctr.size()) ? ctr[ps.slot] : 0.0;
                    by += (units > 0 ? ps.fixed_bytes : 0.0) + ps.unit_bytes * units / ps.units_div;
                }
            }
            for (int k : {r.kind, r.kind2}) {
                if (k < 0) continue;
                g_prof_ms[k] += ms;
                g_prof_bytes[k] += by;
                g_prof_n[k] += 1;
            }
        }
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_prof_pending.clear();
    if (g_prof_ctr.p && g_prof_next > 0) {
        (void)hipMemset(g_prof_ctr.p, 0, sizeof(unsigned) * PROF_SLOTS);
        (void)hipDeviceSynchronize();
    }
    g_prof_next = 0;
}

static void prof_drain()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain_locked();
}

// ====================================================================== dslash launch


template <typename S>
void launch_dslash_t(const DslashCall *c, int nseg, int kind, int nr, int bs, int persistent, hipStream_t s);

// algorithmic bytes of one launch: every operand moved once.  Per live
// right-hand side: the input half spinor, the output and the epilogue
// operands; once per launch: the links.
static void dslash_bytes(const DslashCall &c, double &per_rhs, double &links)
{
    const double vh = c.g.Vh, e = (double)elem_bytes(c.prec), nrm = c.prec == P16 ? 4.0 : 0.0;
    const double field = vh * (12 * e + nrm);
    links = vh * 8.0 * (c.recon == 12 ? 6 : 9) * e;
    int nfield = 2;  // in, out
    if (c.epi != EPI_PLAIN) nfield += 1;                             // x
    if (c.epi == EPI_XPAY_DOT || c.epi == EPI_XMY_NRM || c.epi == EPI_XPAY_TS || c.epi == EPI_CG_R) nfield += 1;  // y
    per_rhs = nfield * field;
}

bool dslash_lds_ok(int prec, int recon) { return lds_link_block_bytes(prec, recon) <= LDS_WORKGROUP_BYTES; }

int dslash_block_sites(const DslashCall &c, const TuneChoice &t)
{
    return (t.kind == 1 && dslash_lds_ok(c.prec, c.recon)) ? 64 : t.bs;
}

void launch_dslash_any(const std::vector<DslashCall> &c, const TuneChoice &t, hipStream_t s)
{
    const int n = (int)c.size();
    switch (c[0].prec) {
    case P64: launch_dslash_t<double>(c.data(), n, t.kind, t.nr, t.bs, t.persistent, s); break;
    case P32: launch_dslash_t<float>(c.data(), n, t.kind, t.nr, t.bs, t.persistent, s); break;
    case P16: launch_dslash_t<__half>(c.data(), n, t.kind, t.nr, t.bs, t.persistent, s); break;
    default: launch_dslash_t<__hip_bfloat16>(c.data(), n, t.kind, t.nr, t.bs, t.persistent, s); break;
    }
}

std::vector<int> launch_dslash_batch(const std::vector<DslashCall> &c0, hipStream_t s)
{
    if (c0.empty() || c0.size() > (size_t)MAXSEG) throw Error{DL_EINVAL, "internal: hopping batch size out of range"};
    const TuneChoice t = tune_lookup(c0, s);
    std::vector<DslashCall> c = c0;
    std::vector<int> nblk(c.size());
    double nominal = 0;
    const bool counted = prof_on() && !capturing(s);
    ProfScope ps(PROF_DSLASH, 0.0, s, (c[0].epi == EPI_PLAIN && !c[0].dag) ? PROF_DSLASH_PLAIN : -1);
    for (size_t k = 0; k < c.size(); ++k) {
        double per_rhs, links;
        dslash_bytes(c[k], per_rhs, links);
        nblk[k] = (c[k].g.Vh + dslash_block_sites(c[k], t) - 1) / dslash_block_sites(c[k], t);
        nominal += per_rhs * c[k].nrhs + links;
        c[k].live_count = counted ? prof_counter() : nullptr;
        ps.parts.push_back({c[k].live_count, per_rhs, links, (double)nblk[k]});
    }
    ps.bytes = nominal;
    if (counted) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        TuneChoice used = t;
        if (t.kind == 1 && !dslash_lds_ok(c[0].prec, c[0].recon)) used = TuneChoice{0, 1, 256, 0};
        for (int k : {ps.kind, ps.kind2})
            if (k >= 0 && k < PROF_NKIND) {
                g_prof_cfg[k] = used;
                g_prof_cfg_set[k] = true;
            }
    }
    launch_dslash_any(c, t, s);
    return nblk;
}

int launch_dslash(const DslashCall &c, hipStream_t s) { return launch_dslash_batch({c}, s)[0]; }

}  // namespace dl

// ====================================================================== lattice

dl::Geom dl_lattice_s::geom() const
{
    Geom g;
    g.X = dims[0];
    g.Y = dims[1];
    g.Z = dims[2];
    g.T = dims[3];
    g.Xh = dims[0] / 2;
    g.Vh = (int)Vh;
    g.sY = g.Xh;
    g.sZ = g.Xh * g.Y;
    g.sT = g.Xh * g.Y * g.Z;
    g.tap = tap;
    return g;
}

extern "C" const char *dl_last_error(void) { return g_err.c_str(); }

extern "C" const char *dl_version(void) { return "dloops 0.1 (gfx950)"; }

extern "C" int dl_lattice_create(const int32_t dims[4], int32_t t_antiperiodic, dl_lattice *out)
{
    return guarded([&]() {
        DL_REQUIRE(dims != nullptr && out != nullptr, "dl_lattice_create: null pointer");
        int64_t V = 1;
        for (int mu = 0; mu < 4; ++mu) {
            DL_REQUIRE(dims[mu] >= 2 && dims[mu] % 2 == 0,
                       "dl_lattice_create: every extent must be even and >= 2 (got " + std::to_string(dims[mu]) + ")");
            V *= dims[mu];
        }
        DL_REQUIRE(V <= 0x7fffffff, "dl_lattice_create: volume exceeds 2^31 - 1");
        auto *L = new dl_lattice_s;
        std::memcpy(L->dims, dims, sizeof(L->dims));
        L->tap = t_antiperiodic ? 1 : 0;
        L->V = V;
        L->Vh = V / 2;
        *out = L;
        return DL_OK;
    });
}

extern "C" void dl_lattice_destroy(dl_lattice lat) { delete lat; }

extern "C" int64_t dl_lattice_volume(dl_lattice lat) { return lat ? lat->V : 0; }

// ====================================================================== gauge field

namespace {

// The gauge handle from the links staged on the device as [4][2][9][Vh]
// complex128: each precision in prec_mask converted to its storage format.
dl_gauge gauge_from_stage(const dl_lattice_s &lat, const DevBuf &stage, uint32_t prec_mask, int recon, hipStream_t s)
{
    auto G = std::make_unique<dl_gauge_s>();
    G->lat = lat;
    G->recon = recon;
    G->prec_mask = prec_mask;
    const int64_t Vh = G->lat.Vh;
    const int ne = recon == 12 ? 6 : 9;
    for (int p = 0; p < 4; ++p) {
        if (!(prec_mask & (1u << p))) continue;
        G->links[p].alloc((size_t)4 * 2 * ne * Vh * elem_bytes(p));
        k_links_convert(p, G->links[p].p, ne, stage.as<double>(), Vh, s);
    }
    DL_HIP(hipGetLastError());
    DL_HIP(hipStreamSynchronize(s));
    return G.release();
}

void validate_gauge_args(dl_lattice lat, const void *links, uint32_t prec_mask, int32_t recon, dl_gauge *out,
                         const char *who)
{
    DL_REQUIRE(lat && links && out, std::string(who) + ": null pointer");
    DL_REQUIRE((prec_mask & 0xF) != 0 && (prec_mask & ~0xFu) == 0,
               std::string(who) + ": prec_mask must be a non-empty subset of bits 0..3");
    DL_REQUIRE(recon == 12 || recon == 18, std::string(who) + ": recon must be 12 or 18");
}

}  // namespace

extern "C" int dl_gauge_create(dl_lattice lat, const double *links, uint32_t prec_mask, int32_t recon, void *stream,
                               dl_gauge *out)
{
    return guarded([&]() {
        StreamScope scope(stream);
        validate_gauge_args(lat, links, prec_mask, recon, out, "dl_gauge_create");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom g = lat->geom();
        const int64_t V = lat->V, Vh = lat->Vh;
        // host reorder: canonical [mu][V][3][3] -> [mu][parity][9][Vh]
        std::vector<double> re((size_t)4 * 2 * 9 * Vh * 2);
        for (int64_t i = 0; i < V; ++i) {
            int64_t r = i;
            const int x = (int)(r % g.X);
            r /= g.X;
            const int y = (int)(r % g.Y);
            r /= g.Y;
            const int z = (int)(r % g.Z);
            const int t = (int)(r / g.Z);
            const int par = (x + y + z + t) & 1;
            const int64_t cb = i >> 1;
            for (int mu = 0; mu < 4; ++mu)
                for (int e = 0; e < 9; ++e) {
                    const double *src = links + (((int64_t)mu * V + i) * 9 + e) * 2;
                    double *dst = re.data() + ((((int64_t)mu * 2 + par) * 9 + e) * Vh + cb) * 2;
                    dst[0] = src[0];
                    dst[1] = src[1];
                }
        }
        DevBuf stage(re.size() * sizeof(double));
        DL_HIP(hipMemcpyAsync(stage.p, re.data(), stage.bytes, hipMemcpyHostToDevice, s));
        *out = gauge_from_stage(*lat, stage, prec_mask, recon, s);
        return DL_OK;
    });
}

extern "C" int dl_gauge_create_device(dl_lattice lat, const void *links, uint32_t prec_mask, int32_t recon,
                                      void *stream, dl_gauge *out)
{
    return guarded([&]() {
        StreamScope scope(stream);
        validate_gauge_args(lat, links, prec_mask, recon, out, "dl_gauge_create_device");
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf stage((size_t)4 * 2 * 9 * lat->Vh * 16);
        k_links_reorder(static_cast<const double *>(links), stage.as<double>(), lat->geom(), s);
        *out = gauge_from_stage(*lat, stage, prec_mask, recon, s);
        return DL_OK;
    });
}

extern "C" void dl_gauge_destroy(dl_gauge g) { delete g; }

// ====================================================================== gamma matrices

// Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3 in the chiral basis, as [16][4][4][re,im]
static std::vector<double> gamma_table()
{
    using C = std::complex<double>;
    const C I(0, 1);
    C sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    C gm[4][4][4] = {};
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                gm[k][r][2 + c] = -I * sig[k][r][c];
                gm[k][2 + r][c] = I * sig[k][r][c];
            }
    for (int r = 0; r < 2; ++r) gm[3][r][2 + r] = gm[3][2 + r][r] = 1;
    std::vector<double> out(16 * 32);
    for (int n = 0; n < 16; ++n) {
        C G[4][4] = {};
        for (int a = 0; a < 4; ++a) G[a][a] = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (!((n >> mu) & 1)) continue;
            C H[4][4] = {};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int k = 0; k < 4; ++k) H[a][b] += G[a][k] * gm[mu][k][b];
            std::memcpy(G, H, sizeof(G));
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                out[n * 32 + 2 * (4 * a + b)] = G[a][b].real();
                out[n * 32 + 2 * (4 * a + b) + 1] = G[a][b].imag();
            }
    }
    return out;
}

// ====================================================================== operators

namespace {

struct Ctx {
    dl_gauge G;
    Geom g;
    hipStream_t s;
    const void *links(int prec) const { return G->links[prec].p; }
};

DslashCall dcall(const Ctx &c, int prec, int parity, bool dag, int epi, Field in, Field out, Field x, Field y,
                 double a, int nrhs, double *parts, const int *active)
{
    DslashCall d;
    d.g = c.g;
    d.parity = parity;
    d.prec = prec;
    d.recon = c.G->recon;
    d.dag = dag;
    d.epi = epi;
    d.in = in;
    d.out = out;
    d.x = x;
    d.y = y;
    d.links = c.links(prec);
    d.a = a;
    d.nrhs = nrhs;
    d.partials = parts;
    d.active = active;
    return d;
}

const Field NOF = {nullptr, nullptr};

void check_prec(dl_gauge G, int prec)
{
    DL_REQUIRE(prec >= 0 && prec <= 3, "precision must be one of DL_F64, DL_F32, DL_F16, DL_BF16");
    DL_REQUIRE((G->prec_mask >> prec) & 1, "the gauge handle does not hold links in the requested precision");
}

}  // namespace

namespace {

void validate_apply(dl_gauge G, int32_t op, int32_t prec, const void *in, void *out, int64_t nrhs, const char *who)
{
    DL_REQUIRE(G && in && out, std::string(who) + ": null pointer");
    DL_REQUIRE(nrhs >= 1 && nrhs <= 65535, std::string(who) + ": nrhs must be in [1, 65535]");
    DL_REQUIRE(op >= DL_OP_DHOP && op <= DL_OP_DHOPDAG, std::string(who) + ": unknown operator");
    check_prec(G, prec);
    DL_REQUIRE(in != out, std::string(who) + ": in and out must not overlap");
}

bool schur_op(int op) { return op == DL_OP_MHAT || op == DL_OP_MHATDAG; }

// The launches of dl_apply on packed parity fields: ie / io receive the packed
// input, oe / oo the output, tmp (Schur operators only) the odd-site
// intermediate.  Every field is written before it is read; the odd output of
// a Schur operator is cleared.
void apply_op(const Ctx &c, int op, int prec, double kappa, const void *in, void *out, int n, Field ie, Field io,
              Field oe, Field oo, Field tmp)
{
    const int64_t Vh = c.G->lat.Vh;
    k_pack(prec, ie, 0, static_cast<const double *>(in), c.g, n, c.s);
    k_pack(prec, io, 1, static_cast<const double *>(in), c.g, n, c.s);
    const bool dag = op == DL_OP_MDAG || op == DL_OP_MHATDAG || op == DL_OP_DHOPDAG;
    switch (op) {
    case DL_OP_DHOP:
    case DL_OP_DHOPDAG:
        launch_dslash(dcall(c, prec, 0, dag, EPI_PLAIN, io, oe, NOF, NOF, 1.0, n, nullptr, nullptr), c.s);
        launch_dslash(dcall(c, prec, 1, dag, EPI_PLAIN, ie, oo, NOF, NOF, 1.0, n, nullptr, nullptr), c.s);
        break;
    case DL_OP_M:
    case DL_OP_MDAG:
        launch_dslash(dcall(c, prec, 0, dag, EPI_XPAY, io, oe, ie, NOF, -kappa, n, nullptr, nullptr), c.s);
        launch_dslash(dcall(c, prec, 1, dag, EPI_XPAY, ie, oo, io, NOF, -kappa, n, nullptr, nullptr), c.s);
        break;
    default:  // Schur complement on even sites
        launch_dslash(dcall(c, prec, 1, dag, EPI_PLAIN, ie, tmp, NOF, NOF, 1.0, n, nullptr, nullptr), c.s);
        launch_dslash(dcall(c, prec, 0, dag, EPI_XPAY, tmp, oe, ie, NOF, -kappa * kappa, n, nullptr, nullptr), c.s);
        vec_launch(V_ZERO, prec, {VSeg{{oo, NOF, NOF, NOF, NOF}, nullptr, nullptr, Vh, n, nullptr}}, c.s);
        break;
    }
    k_unpack(prec, oe, 0, static_cast<double *>(out), c.g, n, c.s);
    k_unpack(prec, oo, 1, static_cast<double *>(out), c.g, n, c.s);
    DL_HIP(hipGetLastError());
}

}  // namespace

extern "C" int dl_apply(dl_gauge G, double kappa, int32_t op, int32_t prec, const void *in, void *out, int64_t nrhs,
                        void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        validate_apply(G, op, prec, in, out, nrhs, "dl_apply");
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int n = (int)nrhs;
        const int64_t Vh = G->lat.Vh;
        HalfField ie, io, oe, oo, tmp;
        ie.alloc(prec, n, Vh);
        io.alloc(prec, n, Vh);
        oe.alloc(prec, n, Vh);
        oo.alloc(prec, n, Vh);
        if (schur_op(op)) tmp.alloc(prec, n, Vh);
        apply_op(c, op, prec, kappa, in, out, n, ie.view(), io.view(), oe.view(), oo.view(), tmp.view());
        DL_HIP(hipStreamSynchronize(c.s));
        return DL_OK;
    });
}

// ====================================================================== no-allocation entry

// Scratch of dl_apply_noalloc: the packed parity fields, carved from a static
// device array instead of allocated.  Each GPU the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in for the symbol):
// its device address is looked up once per device with hipGetSymbolAddress,
// with that device current, and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

void *scratch_on_current_device()
{
    int dev = 0;
    DL_HIP(hipGetDevice(&dev));
    DL_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "dl_apply_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        DL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        DL_REQUIRE(ptr != nullptr, "dl_apply_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// bytes of one packed field of n right-hand sides, rounded up to 256
size_t field_span(int prec, int n, int64_t Vh)
{
    const size_t d = (size_t)n * rhs_stride_bytes(Vh, elem_bytes(prec));
    const size_t m = prec == P16 ? (size_t)n * Vh * sizeof(float) : 0;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    return up(d) + up(m);
}

Field carve(char *&p, int prec, int n, int64_t Vh)
{
    const size_t d = ((size_t)n * rhs_stride_bytes(Vh, elem_bytes(prec)) + 255) / 256 * 256;
    Field f{p, nullptr};
    p += d;
    if (prec == P16) {
        f.nrm = reinterpret_cast<float *>(p);
        p += ((size_t)n * Vh * sizeof(float) + 255) / 256 * 256;
    }
    return f;
}

}  // namespace

extern "C" int dl_apply_noalloc(dl_gauge G, double kappa, int32_t op, int32_t prec, const void *in, void *out,
                                int64_t nrhs, void *stream)
{
    return guarded([&]() {
        NoAllocScope na;
        validate_apply(G, op, prec, in, out, nrhs, "dl_apply_noalloc");
        const int n = (int)nrhs;
        const int64_t Vh = G->lat.Vh;
        const int nfield = schur_op(op) ? 5 : 4;
        const size_t need = nfield * field_span(prec, n, Vh);
        DL_REQUIRE(need <= (size_t)DL_NOALLOC_SCRATCH_BYTES,
                   "dl_apply_noalloc: " + std::to_string(nfield) + " packed fields of " + std::to_string(n) +
                       " right-hand sides need " + std::to_string(need) + " bytes, more than the scratch of " +
                       std::to_string((size_t)DL_NOALLOC_SCRATCH_BYTES) + " bytes");
        char *p = static_cast<char *>(scratch_on_current_device());
        Field ie = carve(p, prec, n, Vh), io = carve(p, prec, n, Vh), oe = carve(p, prec, n, Vh),
              oo = carve(p, prec, n, Vh);
        Field tmp = schur_op(op) ? carve(p, prec, n, Vh) : NOF;
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        apply_op(c, op, prec, kappa, in, out, n, ie, io, oe, oo, tmp);
        return DL_OK;
    });
}

// ====================================================================== solvers

namespace {

// Workspace of a batched solve.  Sources b_e, b_o and the FP64 solution x_e,
// x_o live in FP64 for tolerance-driven solves; the Krylov vectors live in
// the iteration precision.
struct SolveWork {
    int n = 0;
    int prec = P64;
    HalfField be, bo, bhat, x64, xo, r64, tmp64;     // FP64 (BiCGStab)
    HalfField r, rh, p, v, t, tmpo, xlo;             // iteration precision
    DevBuf st, act, upd, restart, parts, parts2;
    int nblk_max = 0;

    void alloc_bicg(int prec_, int n_, int64_t Vh)
    {
        prec = prec_;
        n = n_;
        be.alloc(P64, n, Vh);
        bo.alloc(P64, n, Vh);
        bhat.alloc(P64, n, Vh);
        x64.alloc(P64, n, Vh);
        xo.alloc(P64, n, Vh);
        r64.alloc(P64, n, Vh);
        tmp64.alloc(P64, n, Vh);
        r.alloc(prec, n, Vh);
        rh.alloc(prec, n, Vh);
        p.alloc(prec, n, Vh);
        v.alloc(prec, n, Vh);
        t.alloc(prec, n, Vh);
        tmpo.alloc(prec, n, Vh);
        if (prec != P64) xlo.alloc(prec, n, Vh);
        alloc_common(Vh);
    }
    // truncated CGNR in one precision: be, bo, bhat, x(x64 slot), xo, r, p, t(=q), v(=t), tmpo
    void alloc_cgnr(int prec_, int n_, int64_t Vh)
    {
        prec = prec_;
        n = n_;
        be.alloc(prec, n, Vh);
        bo.alloc(prec, n, Vh);
        bhat.alloc(prec, n, Vh);
        x64.alloc(prec, n, Vh);
        xo.alloc(prec, n, Vh);
        r.alloc(prec, n, Vh);
        p.alloc(prec, n, Vh);
        v.alloc(prec, n, Vh);
        t.alloc(prec, n, Vh);
        tmpo.alloc(prec, n, Vh);
        alloc_common(Vh);
    }
    void alloc_common(int64_t Vh)
    {
        nblk_max = (int)((Vh + 63) / 64);
        st.alloc(sizeof(KState) * n);
        act.alloc(sizeof(int) * n);
        upd.alloc(sizeof(int) * n);
        restart.alloc(sizeof(int) * n);
        // partial sums per (right-hand side, site block): up to five per block
        // (the hop that makes t), and a second set that lives across a kernel
        // in between ((rhat, s) of the s update, FP64 residual norms)
        parts.alloc(sizeof(double) * 5 * (size_t)n * nblk_max);
        parts2.alloc(sizeof(double) * 3 * (size_t)n * nblk_max);
    }
    static size_t bytes_bicg(int prec, int64_t Vh)
    {
        size_t f64 = rhs_stride_bytes(Vh, 16), fl = rhs_stride_bytes(Vh, elem_bytes(prec)) + (prec == P16 ? 4 * Vh : 0);
        return 7 * f64 + (prec == P64 ? 6 : 7) * fl + 8 * 8 * ((Vh + 63) / 64) + 256;
    }
    static size_t bytes_cgnr(int prec, int64_t Vh)
    {
        size_t fl = rhs_stride_bytes(Vh, elem_bytes(prec)) + (prec == P16 ? 4 * Vh : 0);
        return 10 * fl + 8 * 8 * ((Vh + 63) / 64) + 256;
    }
};

int parse_poll(const dl_solve_params &prm) { return prm.poll > 0 ? prm.poll : 4; }

// ---- single-segment shorthands

VSeg vs(std::initializer_list<Field> f, int64_t Vh, int n, const int *mask = nullptr, double *parts = nullptr,
        const KState *st = nullptr)
{
    VSeg a;
    int k = 0;
    for (const Field &x : f) a.f[k++] = x;
    for (; k < 5; ++k) a.f[k] = NOF;
    a.st = st;
    a.mask = mask;
    a.Vh = Vh;
    a.nrhs = n;
    a.parts = parts;
    return a;
}

void k_zero(int prec, Field f, int64_t Vh, int n, const int *mask, hipStream_t s)
{
    vec_launch(V_ZERO, prec, {vs({f}, Vh, n, mask)}, s);
}

void k_copy(int prec_dst, Field dst, int prec_src, Field src, int64_t Vh, int n, const int *mask, hipStream_t s)
{
    copy_launch(prec_dst, prec_src, {vs({dst, src}, Vh, n, mask)}, s);
}

// ---- batched solves: one problem per lattice, every step one launch over all of them

struct Prob {
    Ctx c;
    double kappa;
    SolveWork *w;
    int64_t Vh() const { return c.g.Vh; }
    int nb() const { return blas_blocks(c.g.Vh); }
};

template <typename F>
std::vector<VSeg> VS(const std::vector<Prob> &P, F f)
{
    std::vector<VSeg> v;
    for (const Prob &p : P) v.push_back(f(p));
    return v;
}
template <typename F>
std::vector<DslashCall> DS(const std::vector<Prob> &P, F f)
{
    std::vector<DslashCall> v;
    for (const Prob &p : P) v.push_back(f(p));
    return v;
}
// scalar segments with the partials' block count per problem
std::vector<SSeg> SS(const std::vector<Prob> &P, const std::vector<int> &nblk, bool second_parts, const int *(*mask)(
                                                                                                       const Prob &))
{
    std::vector<SSeg> v;
    for (size_t k = 0; k < P.size(); ++k) {
        SolveWork &w = *P[k].w;
        SSeg a;
        a.st = w.st.as<KState>();
        a.act = w.act.as<int>();
        a.upd = w.upd.as<int>();
        a.restart = w.restart.as<int>();
        a.mask = mask ? mask(P[k]) : nullptr;
        a.parts = w.parts.as<double>();
        a.parts2 = second_parts ? w.parts2.as<double>() : nullptr;
        a.nblk = nblk[k];
        a.nrhs = w.n;
        v.push_back(a);
    }
    return v;
}
std::vector<int> blas_nb(const std::vector<Prob> &P)
{
    std::vector<int> v;
    for (const Prob &p : P) v.push_back(p.nb());
    return v;
}
const int *mask_restart(const Prob &p) { return p.w->restart.as<int>(); }

// The launches of one BiCGStab iteration over all problems.  The search
// direction p of this iteration is in place (from the previous iteration's
// fused update, or p = r after a (re)start):
//   v = Mhat p, alpha = rho / (rhat, v);  s = r - alpha v with (rhat, s);
//   t = Mhat s, omega = (t, s) / |t|^2, rho' = (rhat, s) - omega (rhat, t),
//   beta = (rho' / rho)(alpha / omega);
//   x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v) in one
//   pass with |r|^2; then the iteration count, convergence and reliable-update
//   flags.  rho' follows from the linearity of (rhat, .) in r = s - omega t,
//   which lets the p update join the x / r update (twelve field passes of
//   vector kernels per iteration instead of fourteen, for one more read of
//   rhat in the epilogue of the hop that makes t).
void bicg_iteration(const std::vector<Prob> &P, int prec, bool mixed, hipStream_t s)
{
    auto act = [](const Prob &p) { return p.w->act.as<int>(); };
    launch_dslash_batch(DS(P, [&](const Prob &p) {
                            return dcall(p.c, prec, 1, false, EPI_PLAIN, p.w->p.view(), p.w->tmpo.view(), NOF, NOF,
                                         1.0, p.w->n, nullptr, act(p));
                        }),
                        s);
    std::vector<int> nbd = launch_dslash_batch(DS(P, [&](const Prob &p) {
                                                   return dcall(p.c, prec, 0, false, EPI_XPAY_DOT, p.w->tmpo.view(),
                                                                p.w->v.view(), p.w->p.view(), p.w->rh.view(),
                                                                -p.kappa * p.kappa, p.w->n, p.w->parts.as<double>(),
                                                                act(p));
                                               }),
                                               s);
    scalar_launch(S_BICG_ALPHA, SS(P, nbd, false, nullptr), SParams{}, s);
    vec_launch(V_BICG_S, prec, VS(P, [&](const Prob &p) {
                   return vs({p.w->r.view(), p.w->v.view(), p.w->rh.view()}, p.Vh(), p.w->n, act(p),
                             p.w->parts2.as<double>(), p.w->st.as<KState>());
               }),
               s);
    launch_dslash_batch(DS(P, [&](const Prob &p) {
                            return dcall(p.c, prec, 1, false, EPI_PLAIN, p.w->r.view(), p.w->tmpo.view(), NOF, NOF,
                                         1.0, p.w->n, nullptr, act(p));
                        }),
                        s);
    nbd = launch_dslash_batch(DS(P, [&](const Prob &p) {
                                  return dcall(p.c, prec, 0, false, EPI_XPAY_TS, p.w->tmpo.view(), p.w->t.view(),
                                               p.w->r.view(), p.w->rh.view(), -p.kappa * p.kappa, p.w->n,
                                               p.w->parts.as<double>(), act(p));
                              }),
                              s);
    std::vector<SSeg> om = SS(P, nbd, true, nullptr);
    for (size_t k = 0; k < P.size(); ++k) om[k].nblk2 = P[k].nb();
    scalar_launch(S_BICG_OMEGA, om, SParams{}, s);
    vec_launch(V_BICG_XRP, prec, VS(P, [&](const Prob &p) {
                   Field xit = mixed ? p.w->xlo.view() : p.w->x64.view();
                   return vs({xit, p.w->r.view(), p.w->p.view(), p.w->t.view(), p.w->v.view()}, p.Vh(), p.w->n,
                             act(p), p.w->parts.as<double>(), p.w->st.as<KState>());
               }),
               s);
    SParams sp;
    sp.mixed = mixed ? 1 : 0;
    scalar_launch(S_BICG_CHECK, SS(P, blas_nb(P), false, nullptr), sp, s);
}

int count_host(const DevBuf &flags, int n, hipStream_t s, std::vector<int> &h)
{
    h.resize(n);
    DL_HIP(hipMemcpyAsync(h.data(), flags.p, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    int c = 0;
    for (int v : h) c += v != 0;
    return c;
}

int count_all(const std::vector<Prob> &P, bool upd, hipStream_t s)
{
    std::vector<int> h;
    int c = 0;
    for (const Prob &p : P) c += count_host(upd ? p.w->upd : p.w->act, p.w->n, s, h);
    return c;
}

// A stream that graph capture may use: the caller's stream unless it is the
// legacy default stream, else a library stream ordered after it.  The
// caller's stream is ordered after the library stream again by join(), or by
// the destructor when an error unwinds the solve first.
struct CaptureStream {
    hipStream_t user, s;
    hipEvent_t ev = nullptr;
    bool joined = false;
    explicit CaptureStream(hipStream_t u) : user(u), s(u)
    {
        if (u != nullptr) return;
        static hipStream_t own = nullptr;
        static std::mutex mu;
        std::lock_guard<std::mutex> lk(mu);
        if (!own) DL_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        s = own;
        DL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        DL_HIP(hipEventRecord(ev, user));
        DL_HIP(hipStreamWaitEvent(s, ev, 0));
    }
    void join()
    {
        if (s == user || joined) return;
        DL_HIP(hipEventRecord(ev, s));
        DL_HIP(hipStreamWaitEvent(user, ev, 0));
        joined = true;
    }
    CaptureStream(const CaptureStream &) = delete;
    CaptureStream &operator=(const CaptureStream &) = delete;
    ~CaptureStream()
    {
        if (s != user && !joined && ev) {
            (void)hipEventRecord(ev, s);
            (void)hipStreamWaitEvent(user, ev, 0);
        }
        if (ev) (void)hipEventDestroy(ev);
    }
};

// The captured graph of one chunk of iterations.  A capture still open is
// ended and the graph and its executable are destroyed on every exit,
// including an error thrown between the start of a capture and its
// instantiation, so the stream is left usable for the caller.
struct ChunkGraph {
    hipStream_t s = nullptr;
    bool open = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ChunkGraph() = default;
    ChunkGraph(const ChunkGraph &) = delete;
    ChunkGraph &operator=(const ChunkGraph &) = delete;
    void begin(hipStream_t st)
    {
        s = st;
        DL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        open = true;
    }
    void end()
    {
        open = false;  // the stream leaves capture mode whatever EndCapture returns
        DL_HIP(hipStreamEndCapture(s, &graph));
        DL_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    ~ChunkGraph()
    {
        if (open) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
    }
};

// Failure injection for the tests of the error paths: DL_FAULT_INJECT=capture
// makes a graph capture throw after it has begun (read at every capture).
bool fault_injected(const char *where)
{
    const char *e = std::getenv("DL_FAULT_INJECT");
    return e != nullptr && std::strcmp(e, where) == 0;
}

// BiCGStab on the even-site Schur systems of every problem (sources in w.be /
// w.bo, FP64).  Leaves x_e in w.x64, x_o in w.xo and the per right-hand side
// state in w.st.  Iterated vectors in w.prec; below FP64 the iterate is folded
// into the FP64 x and the residual recomputed in FP64 whenever |r| drops by
// delta since the last update (at the poll points).  With use_graph each chunk
// of `poll` iterations after the first is replayed from a captured hipGraph.
void bicgstab_multi(const std::vector<Prob> &P0, const dl_solve_params &prm, hipStream_t user_stream)
{
    std::unique_ptr<CaptureStream> cst;
    if (prm.use_graph) cst.reset(new CaptureStream(user_stream));
    const hipStream_t s = cst ? cst->s : user_stream;
    std::vector<Prob> P = P0;
    for (Prob &p : P) p.c.s = s;
    const int prec = P[0].w->prec;
    const bool mixed = prec != P64;
    const double delta = mixed ? (prm.delta > 0 ? prm.delta : 0.01) : 0.0;
    auto upd = [](const Prob &p) { return (const int *)p.w->upd.as<int>(); };

    // |b|^2 over both parities; bhat = b_e + kappa D_eo b_o
    vec_launch(V_NORM2, P64, VS(P, [&](const Prob &p) {
                   return vs({p.w->be.view()}, p.Vh(), p.w->n, nullptr, p.w->parts.as<double>());
               }),
               s);
    vec_launch(V_NORM2, P64, VS(P, [&](const Prob &p) {
                   return vs({p.w->bo.view()}, p.Vh(), p.w->n, nullptr, p.w->parts2.as<double>());
               }),
               s);
    SParams sp;
    sp.tol2 = prm.tol * prm.tol;
    sp.delta2 = delta * delta;
    sp.maxiter = prm.maxiter;
    scalar_launch(S_BICG_INIT, SS(P, blas_nb(P), true, nullptr), sp, s);
    launch_dslash_batch(DS(P, [&](const Prob &p) {
                            return dcall(p.c, P64, 0, false, EPI_XPAY, p.w->bo.view(), p.w->bhat.view(),
                                         p.w->be.view(), NOF, p.kappa, p.w->n, nullptr, nullptr);
                        }),
                        s);
    vec_launch(V_ZERO, P64, VS(P, [&](const Prob &p) { return vs({p.w->x64.view()}, p.Vh(), p.w->n); }), s);
    if (mixed) vec_launch(V_ZERO, prec, VS(P, [&](const Prob &p) { return vs({p.w->xlo.view()}, p.Vh(), p.w->n); }), s);
    copy_launch(prec, P64, VS(P, [&](const Prob &p) { return vs({p.w->r.view(), p.w->bhat.view()}, p.Vh(), p.w->n); }),
                s);
    copy_launch(prec, prec, VS(P, [&](const Prob &p) { return vs({p.w->rh.view(), p.w->r.view()}, p.Vh(), p.w->n); }),
                s);
    copy_launch(prec, prec, VS(P, [&](const Prob &p) { return vs({p.w->p.view(), p.w->r.view()}, p.Vh(), p.w->n); }),
                s);
    vec_launch(V_DOT, prec, VS(P, [&](const Prob &p) {
                   return vs({p.w->rh.view(), p.w->r.view()}, p.Vh(), p.w->n, nullptr, p.w->parts.as<double>());
               }),
               s);
    SParams sr;
    scalar_launch(S_BICG_RHO, SS(P, blas_nb(P), false, nullptr), sr, s);

    const int poll = parse_poll(prm);
    int it = 0;
    const int cap = prm.maxiter + poll + 8;
    ChunkGraph cg;
    bool first_chunk = true;
    while (it < cap) {
        if (prm.use_graph && !first_chunk) {
            if (!cg.exec) {
                cg.begin(s);
                if (fault_injected("capture")) throw Error{DL_EHIP, "injected fault inside a graph capture"};
                for (int k = 0; k < poll; ++k) bicg_iteration(P, prec, mixed, s);
                cg.end();
            }
            DL_HIP(hipGraphLaunch(cg.exec, s));
            it += poll;
        } else {
            // the first chunk runs eagerly: it tunes every launch shape the graph will use
            for (int k = 0; k < poll; ++k, ++it) bicg_iteration(P, prec, mixed, s);
            first_chunk = false;
        }
        DL_HIP(hipGetLastError());
        // Poll point.  Right-hand sides flagged for a reliable update (converged,
        // out of iterations, or |r| dropped by delta) get their iterate folded
        // into the FP64 x and the FP64 residual bhat - Mhat x recomputed; where
        // the true residual disagrees with a claimed convergence the recursion
        // restarts from it.
        if (count_all(P, true, s) > 0) {
            if (mixed)
                fold_launch(prec, VS(P, [&](const Prob &p) {
                                return vs({p.w->x64.view(), p.w->xlo.view()}, p.Vh(), p.w->n, upd(p));
                            }),
                            s);
            launch_dslash_batch(DS(P, [&](const Prob &p) {
                                    return dcall(p.c, P64, 1, false, EPI_PLAIN, p.w->x64.view(), p.w->tmp64.view(),
                                                 NOF, NOF, 1.0, p.w->n, nullptr, upd(p));
                                }),
                                s);
            std::vector<int> nb64 = launch_dslash_batch(DS(P, [&](const Prob &p) {
                                                            return dcall(p.c, P64, 0, false, EPI_XMY_NRM,
                                                                         p.w->tmp64.view(), p.w->r64.view(),
                                                                         p.w->bhat.view(), p.w->x64.view(),
                                                                         p.kappa * p.kappa, p.w->n,
                                                                         p.w->parts2.as<double>(), upd(p));
                                                        }),
                                                        s);
            // r <- the FP64 residual, p moved by the same difference (p holds
            // r + beta (p - omega v) already) and rho <- (rhat, r) of the new r
            replace_launch(prec, VS(P, [&](const Prob &p) {
                               return vs({p.w->r.view(), p.w->r64.view(), p.w->p.view(), p.w->rh.view()}, p.Vh(),
                                         p.w->n, upd(p), p.w->parts.as<double>());
                           }),
                           s);
            scalar_launch(S_BICG_RESYNC, SS(P, blas_nb(P), false, upd), SParams{}, s);
            // residual norms are in parts2 for this check
            std::vector<SSeg> tr = SS(P, nb64, false, nullptr);
            for (size_t k = 0; k < P.size(); ++k) tr[k].parts = P[k].w->parts2.as<double>();
            scalar_launch(S_TRUE_RES, tr, SParams{}, s);
            // restart from the true residual: rhat = r, p = r
            copy_launch(prec, prec, VS(P, [&](const Prob &p) {
                            return vs({p.w->rh.view(), p.w->r.view()}, p.Vh(), p.w->n, mask_restart(p));
                        }),
                        s);
            copy_launch(prec, prec, VS(P, [&](const Prob &p) {
                            return vs({p.w->p.view(), p.w->r.view()}, p.Vh(), p.w->n, mask_restart(p));
                        }),
                        s);
            vec_launch(V_DOT, prec, VS(P, [&](const Prob &p) {
                           return vs({p.w->rh.view(), p.w->r.view()}, p.Vh(), p.w->n, mask_restart(p),
                                     p.w->parts.as<double>());
                       }),
                       s);
            scalar_launch(S_BICG_RHO, SS(P, blas_nb(P), false, mask_restart), sr, s);
        }
        if (count_all(P, false, s) == 0) break;
    }
    // x_o = b_o + kappa D_oe x_e
    launch_dslash_batch(DS(P, [&](const Prob &p) {
                            return dcall(p.c, P64, 1, false, EPI_XPAY, p.w->x64.view(), p.w->xo.view(), p.w->bo.view(),
                                         NOF, p.kappa, p.w->n, nullptr, nullptr);
                        }),
                        s);
    DL_HIP(hipGetLastError());
    if (cst) cst->join();
}

void bicgstab_batch(const Ctx &c, double kappa, const dl_solve_params &prm, SolveWork &w)
{
    bicgstab_multi({Prob{c, kappa, &w}}, prm, c.s);
}

// Full-lattice FP64 true residual |b - M x|^2 per right-hand side into out[n].
void true_residual_full(const Ctx &c, double kappa, SolveWork &w, std::vector<double> &out)
{
    const int n = w.n;
    double *parts = w.parts.as<double>(), *parts2 = w.parts2.as<double>();
    // r_e = b_e - x_e + kappa D_eo x_o ; r_o = b_o - x_o + kappa D_oe x_e
    int nbd = launch_dslash(dcall(c, P64, 0, false, EPI_XMY_NRM, w.xo.view(), w.r64.view(), w.be.view(), w.x64.view(),
                                  kappa, n, parts, nullptr),
                            c.s);
    launch_dslash(dcall(c, P64, 1, false, EPI_XMY_NRM, w.x64.view(), w.tmp64.view(), w.bo.view(), w.xo.view(), kappa,
                        n, parts2, nullptr),
                  c.s);
    DevBuf sums(sizeof(double) * 2 * n);
    SSeg a;
    a.parts = parts;
    a.nblk = nbd;
    a.nrhs = n;
    a.out = sums.as<double>();
    SParams sp;
    sp.np = 1;
    scalar_launch(S_SUM, {a}, sp, c.s);
    a.parts = parts2;
    a.out = sums.as<double>() + n;
    scalar_launch(S_SUM, {a}, sp, c.s);
    std::vector<double> h(2 * n);
    DL_HIP(hipMemcpyAsync(h.data(), sums.p, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, c.s));
    DL_HIP(hipStreamSynchronize(c.s));
    out.resize(n);
    for (int i = 0; i < n; ++i) out[i] = h[i] + h[n + i];
}

// Truncated CGNR (x0 = 0, exactly `iters` iterations) on the normal equations
// of the even-site Schur system, all in precision w.prec; sources in w.be /
// w.bo (same precision).  x_e -> w.x64 (slot), x_o -> w.xo.
void cgnr_batch(const Ctx &c, double kappa, int iters, SolveWork &w)
{
    const int n = w.n, P = w.prec;
    const int64_t Vh = c.g.Vh;
    const int nb = blas_blocks(Vh);
    KState *st = w.st.as<KState>();
    int *act = w.act.as<int>();
    double *parts = w.parts.as<double>();
    const double k2 = kappa * kappa;
    auto sseg = [&](int nblk) {
        SSeg a;
        a.st = st;
        a.act = act;
        a.parts = parts;
        a.nblk = nblk;
        a.nrhs = n;
        return std::vector<SSeg>{a};
    };
    // bhat = b_e + kappa D_eo b_o ; r = Mhat^+ bhat ; x = 0 ; p = r
    launch_dslash(
        dcall(c, P, 0, false, EPI_XPAY, w.bo.view(), w.bhat.view(), w.be.view(), NOF, kappa, n, nullptr, nullptr),
        c.s);
    launch_dslash(dcall(c, P, 1, true, EPI_PLAIN, w.bhat.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, nullptr),
                  c.s);
    int nbd = launch_dslash(
        dcall(c, P, 0, true, EPI_XPAY_NRM, w.tmpo.view(), w.r.view(), w.bhat.view(), NOF, -k2, n, parts, nullptr), c.s);
    SParams sp;
    sp.maxiter = iters;
    scalar_launch(S_CG_INIT, sseg(nbd), sp, c.s);
    k_zero(P, w.x64.view(), Vh, n, nullptr, c.s);
    k_copy(P, w.p.view(), P, w.r.view(), Vh, n, nullptr, c.s);
    for (int it = 0; it < iters; ++it) {
        // t = Mhat p with |t|^2 = (p, Mhat^+ Mhat p); alpha = |r|^2 / |t|^2
        launch_dslash(dcall(c, P, 1, false, EPI_PLAIN, w.p.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act),
                      c.s);
        nbd = launch_dslash(
            dcall(c, P, 0, false, EPI_XPAY_NRM, w.tmpo.view(), w.t.view(), w.p.view(), NOF, -k2, n, parts, act), c.s);
        scalar_launch(S_CG_ALPHA, sseg(nbd), SParams{}, c.s);
        // q = Mhat^+ t is formed in the epilogue of the adjoint hop and used there at once:
        // r -= alpha q with |r|^2 (q is never stored)
        launch_dslash(dcall(c, P, 1, true, EPI_PLAIN, w.t.view(), w.tmpo.view(), NOF, NOF, 1.0, n, nullptr, act), c.s);
        DslashCall d4 = dcall(c, P, 0, true, EPI_CG_R, w.tmpo.view(), w.r.view(), w.t.view(), w.r.view(), -k2, n, parts,
                              act);
        d4.st = st;
        nbd = launch_dslash(d4, c.s);
        // beta; then x += alpha p and p = r + beta p in one pass (a right-hand side that finishes
        // in this iteration is flagged 2, so it still takes its x update)
        scalar_launch(S_CG_BETA, sseg(nbd), SParams{}, c.s);
        vec_launch(V_CG_P, P, {vs({w.p.view(), w.r.view(), w.x64.view()}, Vh, n, act, nullptr, st)}, c.s);
    }
    launch_dslash(
        dcall(c, P, 1, false, EPI_XPAY, w.x64.view(), w.xo.view(), w.bo.view(), NOF, kappa, n, nullptr, nullptr), c.s);
    DL_HIP(hipGetLastError());
}

void validate_params(const dl_solve_params *prm)
{
    DL_REQUIRE(prm != nullptr, "solve parameters: null pointer");
    DL_REQUIRE(prm->solver == DL_BICGSTAB || prm->solver == DL_CGNR, "solve parameters: unknown solver");
    DL_REQUIRE(prm->prec >= 0 && prm->prec <= 3, "solve parameters: unknown precision");
    if (prm->solver == DL_CGNR) {
        DL_REQUIRE(prm->fixed_iters >= 0, "solve parameters: CGNR needs fixed_iters >= 0");
    } else {
        DL_REQUIRE(prm->fixed_iters == 0, "solve parameters: BiCGStab is tolerance driven (fixed_iters must be 0)");
        DL_REQUIRE(prm->tol > 0 && prm->tol < 1, "solve parameters: tol must be in (0, 1)");
        DL_REQUIRE(prm->maxiter >= 1, "solve parameters: maxiter must be >= 1");
    }
    DL_REQUIRE(prm->delta >= 0 && prm->delta < 1, "solve parameters: delta must be in [0, 1)");
}

size_t workspace_limit()
{
    const char *e = std::getenv("DL_WORKSPACE_GB");
    double gb = e ? std::atof(e) : 160.0;
    if (!(gb > 0)) gb = 160.0;
    return (size_t)(gb * 1e9);
}

int batch_size(size_t per_rhs, int64_t total, int quantum)
{
    int64_t b = (int64_t)(workspace_limit() / std::max<size_t>(per_rhs, 1));
    b = std::min<int64_t>(b, 65535);
    b = std::max<int64_t>(b / quantum * quantum, quantum);
    // as many rounds as the limit needs, of equal size: one workspace (and one
    // cached buffer) then serves every round, instead of a full round and a
    // smaller remainder that the cache cannot serve from the first's buffer
    const int64_t rounds = (total + b - 1) / b;
    const int64_t even = ((total + rounds - 1) / rounds + quantum - 1) / quantum * quantum;
    return (int)std::min<int64_t>(std::min<int64_t>(b, even), total);
}

// Wall time of the parts of a call, for the per-right-hand-side seconds of
// the solve statistics.
struct Stopwatch {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double lap()  // seconds since the previous lap (or since construction)
    {
        const auto t = std::chrono::steady_clock::now();
        const double d = std::chrono::duration<double>(t - t0).count();
        t0 = t;
        return d;
    }
};

// Algorithmic bytes of one right-hand side's field operands in a solve: every
// operand of every kernel the solve runs for it, moved once (the links, which
// the whole batch shares, are not counted).  Per iteration: BiCGStab moves 24
// half fields in the iteration precision (the hops 2 + 4 + 2 + 4, the s
// update 4, the fused x / r / p update 8); the truncated CGNR 16 (four hops
// 2 + 3 + 2 + 4, the last of them forming q and updating r in its epilogue,
// and the fused x and p update 5).  A reliable update moves 9 FP64 half
// fields (2 for the fold, 2 + 4 for the FP64 residual hops, 1 for the
// replacement of r) and 7 in the iteration precision (the fold 2, the
// replacement of r and p with (rhat, r) 5); without iterations below FP64
// there is no fold.  The set-up and the reconstruction of the odd sites move
// 10 FP64 half fields (source norms 2, prepared source 3, zeroed x 1, the copy
// into r 1, reconstruction 3) and 8 in the iteration precision (r, rhat = r,
// p = r, the first dot, zeroed low-precision x).
double solve_bytes(const SolveWork &w, const KState &k, bool cgnr)
{
    const double vh = (double)w.r.Vh;
    const double fb = vh * (12.0 * elem_bytes(w.prec) + (w.prec == P16 ? 4.0 : 0.0));
    if (cgnr) return k.iters * 16.0 * fb + 8.0 * fb;
    const double f8 = vh * 12.0 * 16.0;
    const bool mixed = w.prec != P64;
    const double upd = mixed ? 9.0 * f8 + 7.0 * fb : 7.0 * f8 + 5.0 * fb;
    return k.iters * 24.0 * fb + k.updates * upd + 10.0 * f8 + 8.0 * fb;
}

// Per right-hand side statistics of the solve just finished; `seconds` is the
// solve's share of the wall time since the stopwatch's last lap (the batch's
// time divided by its right-hand sides).
void fill_stats(const SolveWork &w, const std::vector<double> &res2, dl_solve_stats *out, hipStream_t s,
                bool cgnr, Stopwatch &sw, double secs_per_rhs = -1.0)
{
    std::vector<KState> h(w.n);
    DL_HIP(hipMemcpyAsync(h.data(), w.st.p, sizeof(KState) * w.n, hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
    const double secs = secs_per_rhs >= 0 ? secs_per_rhs : sw.lap() / std::max(1, w.n);
    for (int i = 0; i < w.n; ++i) {
        dl_solve_stats &o = out[i];
        o.iters = h[i].iters;
        o.reliable_updates = h[i].updates;
        o.pad = 0;
        const double b2 = h[i].b2;
        o.true_rel_residual = (i < (int)res2.size() && b2 > 0) ? std::sqrt(res2[i] / b2) : 0.0;
        if (h[i].nonfinite)
            o.status = DL_ENAN;
        else if (cgnr || h[i].done)
            o.status = DL_OK;
        else
            o.status = DL_ENOCONV;
        o.seconds = secs;
        o.bytes = solve_bytes(w, h[i], cgnr);
    }
}

}  // namespace

extern "C" int dl_solve(dl_gauge G, double kappa, const dl_solve_params *params, const void *b, void *x, int64_t nrhs,
                        dl_solve_stats *stats, void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && b && x, "dl_solve: null pointer");
        DL_REQUIRE(nrhs >= 1, "dl_solve: nrhs must be >= 1");
        DL_REQUIRE(b != x, "dl_solve: b and x must not overlap");
        validate_params(params);
        const dl_solve_params prm = *params;
        check_prec(G, prm.prec);
        if (prm.solver == DL_BICGSTAB) check_prec(G, P64);
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int64_t Vh = G->lat.Vh, V = G->lat.V;
        const bool cg = prm.solver == DL_CGNR;
        const size_t per = cg ? SolveWork::bytes_cgnr(prm.prec, Vh) : SolveWork::bytes_bicg(prm.prec, Vh);
        const int B = batch_size(per, nrhs, 1);
        int worst = DL_OK;
        Stopwatch sw;
        for (int64_t r0 = 0; r0 < nrhs; r0 += B) {
            const int n = (int)std::min<int64_t>(B, nrhs - r0);
            SolveWork w;
            const double *bsrc = static_cast<const double *>(b) + r0 * V * 24;
            double *xdst = static_cast<double *>(x) + r0 * V * 24;
            std::vector<double> res2;
            if (cg) {
                w.alloc_cgnr(prm.prec, n, Vh);
                k_pack(prm.prec, w.be.view(), 0, bsrc, c.g, n, c.s);
                k_pack(prm.prec, w.bo.view(), 1, bsrc, c.g, n, c.s);
                cgnr_batch(c, kappa, prm.fixed_iters, w);
                k_unpack(prm.prec, w.x64.view(), 0, xdst, c.g, n, c.s);
                k_unpack(prm.prec, w.xo.view(), 1, xdst, c.g, n, c.s);
            } else {
                w.alloc_bicg(prm.prec, n, Vh);
                k_pack(P64, w.be.view(), 0, bsrc, c.g, n, c.s);
                k_pack(P64, w.bo.view(), 1, bsrc, c.g, n, c.s);
                bicgstab_batch(c, kappa, prm, w);
                true_residual_full(c, kappa, w, res2);
                k_unpack(P64, w.x64.view(), 0, xdst, c.g, n, c.s);
                k_unpack(P64, w.xo.view(), 1, xdst, c.g, n, c.s);
            }
            DL_HIP(hipGetLastError());
            DL_HIP(hipStreamSynchronize(c.s));
            std::vector<dl_solve_stats> st(n);
            fill_stats(w, res2, st.data(), c.s, cg, sw);
            for (int i = 0; i < n; ++i) {
                if (stats) stats[r0 + i] = st[i];
                if (st[i].status != DL_OK && worst == DL_OK) worst = st[i].status;
            }
        }
        if (worst != DL_OK) g_err = "dl_solve: at least one right-hand side did not converge";
        return worst;
    });
}

// ====================================================================== loops

namespace {

int dilution_classes(int scheme)
{
    return ((scheme & DL_DIL_SPIN_COLOUR) ? 12 : 1) * ((scheme & DL_DIL_SPIN) ? 4 : 1) *
           ((scheme & DL_DIL_SPIN_EVEN_ODD) ? 2 : 1) * ((scheme & DL_DIL_COLOUR) ? 3 : 1) *
           ((scheme & DL_DIL_CUBIC) ? 8 : 1) * ((scheme & DL_DIL_EVEN_ODD) ? 2 : 1);
}

void validate_sources(const dl_lattice_s &lat, const dl_sources *src)
{
    DL_REQUIRE(src != nullptr, "sources: null pointer");
    DL_REQUIRE(src->kind == DL_SRC_Z2 || src->kind == DL_SRC_POINT, "sources: unknown kind");
    if (src->kind == DL_SRC_POINT) {
        DL_REQUIRE(src->n_noise == 1, "sources: point sources need n_noise = 1");
        DL_REQUIRE(src->point_site >= 0 && src->point_site < lat.V, "sources: point_site outside the lattice");
    } else {
        DL_REQUIRE(src->n_noise >= 1, "sources: n_noise must be >= 1");
        DL_REQUIRE(src->first_noise >= 0, "sources: first_noise must be >= 0");
        DL_REQUIRE((src->scheme & ~127) == 0, "sources: unknown dilution bits");
        DL_REQUIRE(!((src->scheme & DL_DIL_SPIN_COLOUR) &&
                     (src->scheme & (DL_DIL_COLOUR | DL_DIL_SPIN | DL_DIL_SPIN_EVEN_ODD))),
                   "sources: spin-colour dilution excludes the separate spin and colour factors");
        DL_REQUIRE(!((src->scheme & DL_DIL_SPIN) && (src->scheme & DL_DIL_SPIN_EVEN_ODD)),
                   "sources: spin dilution and spin even-odd partitioning exclude each other");
    }
}

int source_classes(const dl_sources *src) { return src->kind == DL_SRC_POINT ? 12 : dilution_classes(src->scheme); }

}  // namespace

extern "C" int64_t dl_sources_count(dl_lattice lat, const dl_sources *src)
{
    int64_t r = DL_EINVAL;
    int rc = guarded([&]() {
        DL_REQUIRE(lat != nullptr, "dl_sources_count: null lattice");
        validate_sources(*lat, src);
        r = (int64_t)src->n_noise * source_classes(src);
        return DL_OK;
    });
    return rc == DL_OK ? r : rc;
}

extern "C" int dl_sources_fill(dl_lattice lat, const dl_sources *src, int64_t first_rhs, int64_t nrhs, void *out,
                               void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(lat && out, "dl_sources_fill: null pointer");
        validate_sources(*lat, src);
        const int ncls = source_classes(src);
        const int64_t total = (int64_t)src->n_noise * ncls;
        DL_REQUIRE(nrhs >= 1 && nrhs <= 65535 && first_rhs >= 0 && first_rhs + nrhs <= total,
                   "dl_sources_fill: right-hand side range outside the description");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom g = lat->geom();
        const int n = (int)nrhs;
        std::vector<int64_t> hnoise(n);
        std::vector<int> hcls(n);
        for (int i = 0; i < n; ++i) {
            hnoise[i] = src->first_noise + (first_rhs + i) / ncls;
            hcls[i] = (int)((first_rhs + i) % ncls);
        }
        DevBuf dnoise(sizeof(int64_t) * n), dcls(sizeof(int) * n);
        DL_HIP(hipMemcpyAsync(dnoise.p, hnoise.data(), dnoise.bytes, hipMemcpyHostToDevice, s));
        DL_HIP(hipMemcpyAsync(dcls.p, hcls.data(), dcls.bytes, hipMemcpyHostToDevice, s));
        SourceSpec ss;
        ss.kind = src->kind;
        ss.scheme = src->kind == DL_SRC_POINT ? 0 : src->scheme;
        ss.seed = src->seed;
        ss.V = lat->V;
        ss.T = lat->dims[3];
        ss.point_site = src->point_site;
        ss.noise = dnoise.as<int64_t>();
        ss.cls = dcls.as<int>();
        HalfField fe, fo;
        fe.alloc(P64, n, lat->Vh);
        fo.alloc(P64, n, lat->Vh);
        k_source(P64, fe.view(), 0, ss, g, n, s);
        k_source(P64, fo.view(), 1, ss, g, n, s);
        k_unpack(P64, fe.view(), 0, static_cast<double *>(out), g, n, s);
        k_unpack(P64, fo.view(), 1, static_cast<double *>(out), g, n, s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(s));
        return DL_OK;
    });
}

namespace {

enum LoopMode { MODE_LOOPS = 0, MODE_DKAPPA = 1, MODE_GRAD = 2 };

void validate_gammas(const int32_t *gammas, int32_t n_gamma)
{
    DL_REQUIRE(gammas != nullptr, "gammas: null pointer");
    DL_REQUIRE(n_gamma >= 1 && n_gamma <= 16, "n_gamma must be in [1, 16]");
    for (int i = 0; i < n_gamma; ++i) DL_REQUIRE(gammas[i] >= 0 && gammas[i] <= 15, "gamma index outside [0, 15]");
}

// A[n][t] = gamma5 sum_g W[n][g][t] Gamma_g^+ for every noise and timeslice, [n][T][4][4] complex
std::vector<double> adjoint_matrices(const std::vector<double> &gtab, const int32_t *gammas, int n_gamma,
                                     const double *W, int T, int n_noise)
{
    std::vector<double> A((size_t)n_noise * T * 32, 0.0);
    const double g5[4] = {1, 1, -1, -1};
    for (int n = 0; n < n_noise; ++n)
        for (int t = 0; t < T; ++t)
            for (int gi = 0; gi < n_gamma; ++gi) {
                const double *w = W + (((size_t)n * n_gamma + gi) * T + t) * 2;
                const double wr = w[0], wi = w[1];
                const double *G = gtab.data() + gammas[gi] * 32;
                double *At = A.data() + ((size_t)n * T + t) * 32;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        // (Gamma^+)_{ab} = conj(Gamma_{ba})
                        const double gr = G[2 * (4 * b + a)], gim = -G[2 * (4 * b + a) + 1];
                        At[2 * (4 * a + b)] += g5[a] * (wr * gr - wi * gim);
                        At[2 * (4 * a + b) + 1] += g5[a] * (wr * gim + wi * gr);
                    }
            }
    return A;
}

// The loop estimator and its derivatives over a batch loop of whole noises.
//   MODE_LOOPS:  out[n][g][t] = sum_d eta^+ P_t Gamma s, s = M^-1 eta
//   MODE_DKAPPA: out[n][g][t] = sum_d eta^+ P_t Gamma u, u = M^-1 D M^-1 eta
//   MODE_GRAD:   grad += d/dU of Re sum conj(W[n]) L[n], using s and the adjoint
//                a = gamma5 M^-1 gamma5 (sum_g W[n] Gamma^+ P_t eta); out (the
//                forward loops) may be null; dout, if set, receives the kappa
//                derivative as in MODE_DKAPPA (a third solve)
// stats: per right-hand side and solve ([nsolve][nrhs]) or null.
// Loop estimates (MODE_LOOPS), their kappa derivative (MODE_DKAPPA) or link
// gradient (MODE_GRAD).  smear_iters > 0 (MODE_LOOPS only): the sources are
// smeared, xi = S eta with S = F^smear_iters, and xi serves at the sink too.
int loops_run(dl_gauge G, double kappa, const dl_sources *src, const dl_solve_params &prm, const int32_t *gammas,
              int n_gamma, int mode, const double *W, double *out_host, double *grad_host, dl_solve_stats *stats,
              hipStream_t stream, double *dout_host = nullptr, double smear_alpha = 0.0, int smear_iters = 0)
{
    Ctx c{G, G->lat.geom(), stream};
    const int64_t Vh = G->lat.Vh, V = G->lat.V;
    const int T = c.g.T;
    const int ncls = source_classes(src);
    const bool cg = prm.solver == DL_CGNR;
    size_t per = (cg ? SolveWork::bytes_cgnr(prm.prec, Vh) : SolveWork::bytes_bicg(prm.prec, Vh)) +
                 (size_t)T * 32 * 8 + 16;
    if (mode == MODE_GRAD) per += 2 * (size_t)rhs_stride_bytes(Vh, 16);  // the stored forward solution
    if (smear_iters > 0) per += 4 * (size_t)rhs_stride_bytes(Vh, 16);    // smeared source and its ping-pong partner
    const int64_t total = (int64_t)src->n_noise * ncls;
    const int nsolve = mode == MODE_LOOPS ? 1 : (mode == MODE_GRAD && dout_host) ? 3 : 2;
    const int B = batch_size(per, total, ncls);
    std::vector<double> gtab = gamma_table();
    DevBuf dgam(gtab.size() * sizeof(double)), dgidx(sizeof(int) * n_gamma), dA, dgrad;
    DevBuf dloops((size_t)src->n_noise * n_gamma * T * 2 * sizeof(double)), ddk;
    if (dout_host) ddk.alloc(dloops.bytes);
    DL_HIP(hipMemcpyAsync(dgam.p, gtab.data(), dgam.bytes, hipMemcpyHostToDevice, c.s));
    DL_HIP(hipMemcpyAsync(dgidx.p, gammas, dgidx.bytes, hipMemcpyHostToDevice, c.s));
    if (mode == MODE_GRAD) {
        std::vector<double> A = adjoint_matrices(gtab, gammas, n_gamma, W, T, src->n_noise);
        dA.alloc(A.size() * sizeof(double));
        DL_HIP(hipMemcpyAsync(dA.p, A.data(), dA.bytes, hipMemcpyHostToDevice, c.s));
        dgrad.alloc((size_t)4 * V * 9 * 16);
        zero_launch(dgrad.p, (int64_t)4 * V * 9, c.s);  // [4][V][9] complex
    }
    int worst = DL_OK;
    Stopwatch sw;
    std::vector<int64_t> hnoise;
    std::vector<int> hcls;
    for (int64_t r0 = 0; r0 < total; r0 += B) {
        const int n = (int)std::min<int64_t>(B, total - r0);
        const int nn = n / ncls;
        hnoise.resize(n);
        hcls.resize(n);
        for (int i = 0; i < n; ++i) {
            hnoise[i] = src->first_noise + (r0 + i) / ncls;
            hcls[i] = (int)((r0 + i) % ncls);
        }
        DevBuf dnoise(sizeof(int64_t) * n), dcls(sizeof(int) * n), dC((size_t)n * T * 32 * sizeof(double));
        DL_HIP(hipMemcpyAsync(dnoise.p, hnoise.data(), dnoise.bytes, hipMemcpyHostToDevice, c.s));
        DL_HIP(hipMemcpyAsync(dcls.p, hcls.data(), dcls.bytes, hipMemcpyHostToDevice, c.s));
        SourceSpec ss;
        ss.kind = src->kind;
        ss.scheme = src->kind == DL_SRC_POINT ? 0 : src->scheme;
        ss.seed = src->seed;
        ss.V = V;
        ss.T = T;
        ss.point_site = src->point_site;
        ss.noise = dnoise.as<int64_t>();
        ss.cls = dcls.as<int>();
        // smeared sources: xi = F^iters eta in FP64, kept for the trace
        HalfField xe, xo, te, to;
        SourceSpec sx = ss;
        if (smear_iters > 0) {
            xe.alloc(P64, n, Vh);
            xo.alloc(P64, n, Vh);
            te.alloc(P64, n, Vh);
            to.alloc(P64, n, Vh);
            k_source(P64, xe.view(), 0, ss, c.g, n, c.s);
            k_source(P64, xo.view(), 1, ss, c.g, n, c.s);
            HalfField *ae = &xe, *ao = &xo, *be = &te, *bo = &to;
            for (int it = 0; it < smear_iters; ++it) {
                k_smear(c.links(P64), G->recon, ae->view(), ao->view(), be->view(), bo->view(), c.g, n, smear_alpha,
                        c.s);
                std::swap(ae, be);
                std::swap(ao, bo);
            }
            sx.kind = SRC_STORED;
            sx.xe = ae->view();
            sx.xo = ao->view();
        }
        auto make_source = [&](int prec, Field be, Field bo) {
            if (smear_iters > 0) {
                k_copy(prec, be, P64, sx.xe, Vh, n, nullptr, c.s);
                k_copy(prec, bo, P64, sx.xo, Vh, n, nullptr, c.s);
            } else {
                k_source(prec, be, 0, ss, c.g, n, c.s);
                k_source(prec, bo, 1, ss, c.g, n, c.s);
            }
        };
        SolveWork w;
        std::vector<std::vector<dl_solve_stats>> st(nsolve, std::vector<dl_solve_stats>(n));
        int sol_prec = P64;
        if (cg) {
            w.alloc_cgnr(prm.prec, n, Vh);
            make_source(prm.prec, w.be.view(), w.bo.view());
            cgnr_batch(c, kappa, prm.fixed_iters, w);
            sol_prec = prm.prec;
            fill_stats(w, {}, st[0].data(), c.s, true, sw);
        } else {
            std::vector<double> res2;
            w.alloc_bicg(prm.prec, n, Vh);
            make_source(P64, w.be.view(), w.bo.view());
            bicgstab_batch(c, kappa, prm, w);
            if (stats) true_residual_full(c, kappa, w, res2);
            fill_stats(w, res2, st[0].data(), c.s, false, sw);
            if (mode == MODE_DKAPPA) {
                // second solve on w = D s (sources are regenerated for the trace)
                launch_dslash(dcall(c, P64, 0, false, EPI_PLAIN, w.xo.view(), w.be.view(), NOF, NOF, 1.0, n, nullptr,
                                    nullptr),
                              c.s);
                launch_dslash(dcall(c, P64, 1, false, EPI_PLAIN, w.x64.view(), w.bo.view(), NOF, NOF, 1.0, n,
                                    nullptr, nullptr),
                              c.s);
                bicgstab_batch(c, kappa, prm, w);
                res2.clear();
                if (stats) true_residual_full(c, kappa, w, res2);
                fill_stats(w, res2, st[1].data(), c.s, false, sw);
            } else if (mode == MODE_GRAD) {
                HalfField se, so;
                se.alloc(P64, n, Vh);
                so.alloc(P64, n, Vh);
                k_copy(P64, se.view(), P64, w.x64.view(), Vh, n, nullptr, c.s);
                k_copy(P64, so.view(), P64, w.xo.view(), Vh, n, nullptr, c.s);
                if (out_host) {
                    k_trace(P64, se.view(), so.view(), ss, c.g, n, dC.as<double>(), c.s);
                    k_gamma_contract(dC.as<double>(), nn, ncls, T, dgam.as<double>(), dgidx.as<int>(), n_gamma,
                                     dloops.as<double>() + (r0 / ncls) * n_gamma * T * 2, c.s);
                }
                if (dout_host) {
                    // kappa derivative: u = M^-1 D s
                    launch_dslash(dcall(c, P64, 0, false, EPI_PLAIN, so.view(), w.be.view(), NOF, NOF, 1.0, n,
                                        nullptr, nullptr),
                                  c.s);
                    launch_dslash(dcall(c, P64, 1, false, EPI_PLAIN, se.view(), w.bo.view(), NOF, NOF, 1.0, n,
                                        nullptr, nullptr),
                                  c.s);
                    bicgstab_batch(c, kappa, prm, w);
                    res2.clear();
                    if (stats) true_residual_full(c, kappa, w, res2);
                    fill_stats(w, res2, st[2].data(), c.s, false, sw);
                    k_trace(P64, w.x64.view(), w.xo.view(), ss, c.g, n, dC.as<double>(), c.s);
                    k_gamma_contract(dC.as<double>(), nn, ncls, T, dgam.as<double>(), dgidx.as<int>(), n_gamma,
                                     ddk.as<double>() + (r0 / ncls) * n_gamma * T * 2, c.s);
                }
                const double *Ab = dA.as<double>();
                k_adjoint_source(w.be.view(), 0, ss, c.g, n, Ab, src->first_noise, c.s);
                k_adjoint_source(w.bo.view(), 1, ss, c.g, n, Ab, src->first_noise, c.s);
                bicgstab_batch(c, kappa, prm, w);
                res2.clear();
                if (stats) true_residual_full(c, kappa, w, res2);
                fill_stats(w, res2, st[1].data(), c.s, false, sw);
                k_link_grad(se.view(), so.view(), w.x64.view(), w.xo.view(), c.g, n, kappa, dgrad.as<double>(),
                            c.s);
                DL_HIP(hipStreamSynchronize(c.s));
            }
        }
        if (mode != MODE_GRAD) {
            k_trace(sol_prec, w.x64.view(), w.xo.view(), sx, c.g, n, dC.as<double>(), c.s);
            k_gamma_contract(dC.as<double>(), nn, ncls, T, dgam.as<double>(), dgidx.as<int>(), n_gamma,
                             dloops.as<double>() + (r0 / ncls) * n_gamma * T * 2, c.s);
        }
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(c.s));
        for (int k = 0; k < nsolve; ++k)
            for (int i = 0; i < n; ++i) {
                if (stats) stats[(int64_t)k * total + r0 + i] = st[k][i];
                if (st[k][i].status != DL_OK && worst == DL_OK) worst = st[k][i].status;
            }
    }
    if (out_host) DL_HIP(hipMemcpyAsync(out_host, dloops.p, dloops.bytes, hipMemcpyDeviceToHost, c.s));
    if (grad_host) DL_HIP(hipMemcpyAsync(grad_host, dgrad.p, dgrad.bytes, hipMemcpyDefault, c.s));
    if (dout_host) DL_HIP(hipMemcpyAsync(dout_host, ddk.p, ddk.bytes, hipMemcpyDeviceToHost, c.s));
    DL_HIP(hipStreamSynchronize(c.s));
    if (worst != DL_OK) g_err = "at least one solve did not converge";
    return worst;
}

void check_solver_for(dl_gauge G, const dl_solve_params &prm)
{
    check_prec(G, prm.prec);
    if (prm.solver == DL_BICGSTAB) check_prec(G, P64);
}

}  // namespace

extern "C" int dl_loops(dl_gauge G, double kappa, const dl_sources *src, const dl_solve_params *params,
                        const int32_t *gammas, int32_t n_gamma, double *loops, dl_solve_stats *stats, void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && loops, "dl_loops: null pointer");
        validate_sources(G->lat, src);
        validate_params(params);
        validate_gammas(gammas, n_gamma);
        check_solver_for(G, *params);
        return loops_run(G, kappa, src, *params, gammas, n_gamma, MODE_LOOPS, nullptr, loops, nullptr, stats,
                         static_cast<hipStream_t>(stream));
    });
}

extern "C" int dl_loops_smeared(dl_gauge G, double kappa, const dl_sources *src, double alpha, int32_t iters,
                                const dl_solve_params *params, const int32_t *gammas, int32_t n_gamma, double *loops,
                                dl_solve_stats *stats, void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && loops, "dl_loops_smeared: null pointer");
        validate_sources(G->lat, src);
        validate_params(params);
        validate_gammas(gammas, n_gamma);
        check_solver_for(G, *params);
        DL_REQUIRE(std::isfinite(alpha) && alpha >= 0, "dl_loops_smeared: alpha must be finite and >= 0");
        DL_REQUIRE(iters >= 0 && iters <= 100000, "dl_loops_smeared: iters must be in [0, 100000]");
        check_prec(G, P64);
        return loops_run(G, kappa, src, *params, gammas, n_gamma, MODE_LOOPS, nullptr, loops, nullptr, stats,
                         static_cast<hipStream_t>(stream), nullptr, alpha, iters);
    });
}

extern "C" int dl_smear(dl_gauge G, double alpha, int32_t iters, const void *in, void *out, int64_t nrhs,
                        void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && in && out, "dl_smear: null pointer");
        DL_REQUIRE(nrhs >= 1 && nrhs <= 65535, "dl_smear: nrhs must be in [1, 65535]");
        DL_REQUIRE(std::isfinite(alpha) && alpha >= 0, "dl_smear: alpha must be finite and >= 0");
        DL_REQUIRE(iters >= 0 && iters <= 100000, "dl_smear: iters must be in [0, 100000]");
        DL_REQUIRE(in != out, "dl_smear: in and out must not overlap");
        check_prec(G, P64);
        Ctx c{G, G->lat.geom(), static_cast<hipStream_t>(stream)};
        const int n = (int)nrhs;
        const int64_t Vh = G->lat.Vh;
        if (iters == 0) {
            // S = 1: the output is the input, bit for bit
            DL_HIP(hipMemcpyAsync(out, in, (size_t)n * G->lat.V * 24 * sizeof(double), hipMemcpyDeviceToDevice, c.s));
            DL_HIP(hipStreamSynchronize(c.s));
            return DL_OK;
        }
        HalfField ae, ao, be, bo;
        ae.alloc(P64, n, Vh);
        ao.alloc(P64, n, Vh);
        be.alloc(P64, n, Vh);
        bo.alloc(P64, n, Vh);
        k_pack(P64, ae.view(), 0, static_cast<const double *>(in), c.g, n, c.s);
        k_pack(P64, ao.view(), 1, static_cast<const double *>(in), c.g, n, c.s);
        HalfField *pe = &ae, *po = &ao, *qe = &be, *qo = &bo;
        for (int it = 0; it < iters; ++it) {
            k_smear(c.links(P64), G->recon, pe->view(), po->view(), qe->view(), qo->view(), c.g, n, alpha, c.s);
            std::swap(pe, qe);
            std::swap(po, qo);
        }
        k_unpack(P64, pe->view(), 0, static_cast<double *>(out), c.g, n, c.s);
        k_unpack(P64, po->view(), 1, static_cast<double *>(out), c.g, n, c.s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipStreamSynchronize(c.s));
        return DL_OK;
    });
}

extern "C" int dl_loops_tsm(dl_gauge G, double kappa, const dl_sources *src, const dl_tsm *tsm,
                            const int32_t *gammas, int32_t n_gamma, double *loops, dl_solve_stats *stats,
                            void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && loops && tsm, "dl_loops_tsm: null pointer");
        validate_sources(G->lat, src);
        DL_REQUIRE(src->kind == DL_SRC_Z2, "dl_loops_tsm: needs noise sources");
        DL_REQUIRE(tsm->n_lp >= 1 && tsm->n_hp >= 1 && (int64_t)tsm->n_lp + tsm->n_hp == src->n_noise,
                   "dl_loops_tsm: n_lp >= 1, n_hp >= 1 and n_lp + n_hp must equal n_noise");
        validate_params(&tsm->lp);
        validate_params(&tsm->hp);
        validate_gammas(gammas, n_gamma);
        check_solver_for(G, tsm->lp);
        check_solver_for(G, tsm->hp);
        const int T = G->lat.dims[3];
        const int ncls = source_classes(src);
        const size_t per_noise = (size_t)n_gamma * T * 2;
        hipStream_t s = static_cast<hipStream_t>(stream);
        // low precision on every noise (LP set, then HP set)
        std::vector<double> lp((size_t)src->n_noise * per_noise);
        int rc1 = loops_run(G, kappa, src, tsm->lp, gammas, n_gamma, MODE_LOOPS, nullptr, lp.data(), nullptr,
                            stats, s);
        // high precision on the HP set
        dl_sources hs = *src;
        hs.first_noise = src->first_noise + tsm->n_lp;
        hs.n_noise = tsm->n_hp;
        std::vector<double> hp((size_t)tsm->n_hp * per_noise);
        int rc2 = loops_run(G, kappa, &hs, tsm->hp, gammas, n_gamma, MODE_LOOPS, nullptr, hp.data(), nullptr,
                            stats ? stats + (int64_t)src->n_noise * ncls : nullptr, s);
        // [LP set, LP] [HP set, HP] [HP set, LP]
        std::memcpy(loops, lp.data(), sizeof(double) * tsm->n_lp * per_noise);
        std::memcpy(loops + tsm->n_lp * per_noise, hp.data(), sizeof(double) * tsm->n_hp * per_noise);
        std::memcpy(loops + (tsm->n_lp + tsm->n_hp) * per_noise, lp.data() + tsm->n_lp * per_noise,
                    sizeof(double) * tsm->n_hp * per_noise);
        const int rc = rc1 != DL_OK ? rc1 : rc2;
        if (rc != DL_OK) g_err = "dl_loops_tsm: at least one solve did not converge";
        return rc;
    });
}

extern "C" int dl_loops_dkappa(dl_gauge G, double kappa, const dl_sources *src, const dl_solve_params *params,
                               const int32_t *gammas, int32_t n_gamma, double *dloops, dl_solve_stats *stats,
                               void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && dloops, "dl_loops_dkappa: null pointer");
        validate_sources(G->lat, src);
        validate_params(params);
        DL_REQUIRE(params->solver == DL_BICGSTAB, "dl_loops_dkappa: needs the tolerance-driven BiCGStab");
        validate_gammas(gammas, n_gamma);
        check_solver_for(G, *params);
        return loops_run(G, kappa, src, *params, gammas, n_gamma, MODE_DKAPPA, nullptr, dloops, nullptr, stats,
                         static_cast<hipStream_t>(stream));
    });
}

extern "C" int dl_loops_link_grad(dl_gauge G, double kappa, const dl_sources *src, const dl_solve_params *params,
                                  const int32_t *gammas, int32_t n_gamma, const double *w, double *grad,
                                  double *loops, double *dloops, double *dF_dkappa, dl_solve_stats *stats,
                                  void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(G && w && grad, "dl_loops_link_grad: null pointer");
        validate_sources(G->lat, src);
        validate_params(params);
        DL_REQUIRE(params->solver == DL_BICGSTAB, "dl_loops_link_grad: needs the tolerance-driven BiCGStab");
        validate_gammas(gammas, n_gamma);
        check_solver_for(G, *params);
        const size_t m = (size_t)src->n_noise * n_gamma * G->lat.dims[3] * 2;
        std::vector<double> dk_own;
        double *dk = dloops;
        if (dF_dkappa && !dk) {
            dk_own.resize(m);
            dk = dk_own.data();
        }
        const int rc = loops_run(G, kappa, src, *params, gammas, n_gamma, MODE_GRAD, w, loops, grad, stats,
                                 static_cast<hipStream_t>(stream), dk);
        if (dF_dkappa) {
            // dF/dkappa = Re sum conj(w) dL/dkappa, in a fixed order
            double acc = 0.0;
            for (size_t k = 0; k < m; k += 2) acc += w[k] * dk[k] + w[k + 1] * dk[k + 1];
            *dF_dkappa = acc;
        }
        return rc;
    });
}

extern "C" int dl_tsm_combine(const double *lp_set_lp, int32_t n_lp, const double *hp_set_hp,
                              const double *hp_set_lp, int32_t n_hp, int32_t n_gamma, int32_t T, double *est,
                              double *var)
{
    return guarded([&]() {
        DL_REQUIRE(lp_set_lp && hp_set_hp && hp_set_lp && est, "dl_tsm_combine: null pointer");
        DL_REQUIRE(n_gamma >= 1 && n_gamma <= 16, "dl_tsm_combine: n_gamma must be in [1, 16]");
        DL_REQUIRE(T >= 1 && T <= 65535, "dl_tsm_combine: T must be in [1, 65535]");
        DL_REQUIRE(n_lp >= 1 && n_hp >= 1, "dl_tsm_combine: both noise sets must be non-empty");
        DL_REQUIRE(!var || (n_lp >= 2 && n_hp >= 2),
                   "dl_tsm_combine: the variance needs at least two noises in each set");
        const size_t m = (size_t)n_gamma * T;
        for (size_t k = 0; k < m; ++k) {
            // mean of the low-precision set and of the high-minus-low corrections
            double lr = 0, li = 0, cr = 0, ci = 0;
            for (int j = 0; j < n_lp; ++j) {
                lr += lp_set_lp[(j * m + k) * 2];
                li += lp_set_lp[(j * m + k) * 2 + 1];
            }
            for (int j = 0; j < n_hp; ++j) {
                cr += hp_set_hp[(j * m + k) * 2] - hp_set_lp[(j * m + k) * 2];
                ci += hp_set_hp[(j * m + k) * 2 + 1] - hp_set_lp[(j * m + k) * 2 + 1];
            }
            lr /= n_lp;
            li /= n_lp;
            cr /= n_hp;
            ci /= n_hp;
            est[2 * k] = lr + cr;
            est[2 * k + 1] = li + ci;
            if (!var) continue;
            // unbiased sample variances of the two means (|z - mean|^2 summed, over n - 1)
            double sl = 0, sc = 0;
            for (int j = 0; j < n_lp; ++j) {
                const double dr = lp_set_lp[(j * m + k) * 2] - lr, di = lp_set_lp[(j * m + k) * 2 + 1] - li;
                sl += dr * dr + di * di;
            }
            for (int j = 0; j < n_hp; ++j) {
                const double dr = hp_set_hp[(j * m + k) * 2] - hp_set_lp[(j * m + k) * 2] - cr;
                const double di = hp_set_hp[(j * m + k) * 2 + 1] - hp_set_lp[(j * m + k) * 2 + 1] - ci;
                sc += dr * dr + di * di;
            }
            var[k] = sl / (n_lp - 1) / n_lp + sc / (n_hp - 1) / n_hp;
        }
        return DL_OK;
    });
}

// ====================================================================== batched lattices

extern "C" int dl_batch_loops(int32_t n_lat, const dl_gauge *gauges, const double *kappas, const dl_sources *srcs,
                              const dl_solve_params *params, const int32_t *gammas, int32_t n_gamma,
                              double *const *loops, dl_solve_stats *const *stats, void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(n_lat >= 1 && n_lat <= MAXSEG, "dl_batch_loops: n_lat must be in [1, 4]");
        DL_REQUIRE(gauges && kappas && srcs && loops, "dl_batch_loops: null pointer");
        validate_params(params);
        DL_REQUIRE(params->solver == DL_BICGSTAB, "dl_batch_loops: needs the tolerance-driven BiCGStab");
        validate_gammas(gammas, n_gamma);
        for (int l = 0; l < n_lat; ++l) {
            DL_REQUIRE(gauges[l] && loops[l], "dl_batch_loops: null gauge or output pointer");
            validate_sources(gauges[l]->lat, &srcs[l]);
            check_solver_for(gauges[l], *params);
        }
        const dl_solve_params prm = *params;
        hipStream_t s = static_cast<hipStream_t>(stream);
        // noises per round, the same for every lattice, so that the round fits the workspace
        size_t per_noise_all = 0;
        int max_noise = 0;
        for (int l = 0; l < n_lat; ++l) {
            const int64_t Vh = gauges[l]->lat.Vh;
            per_noise_all += (SolveWork::bytes_bicg(prm.prec, Vh) + (size_t)gauges[l]->lat.dims[3] * 32 * 8 + 16) *
                             source_classes(&srcs[l]);
            max_noise = std::max(max_noise, srcs[l].n_noise);
        }
        const int kmax = (int)std::max<int64_t>(1, std::min<int64_t>(max_noise, workspace_limit() / per_noise_all));
        const int k = (max_noise + (max_noise + kmax - 1) / kmax - 1) / ((max_noise + kmax - 1) / kmax);  // equal rounds
        std::vector<double> gtab = gamma_table();
        DevBuf dgam(gtab.size() * sizeof(double)), dgidx(sizeof(int) * n_gamma);
        DL_HIP(hipMemcpyAsync(dgam.p, gtab.data(), dgam.bytes, hipMemcpyHostToDevice, s));
        DL_HIP(hipMemcpyAsync(dgidx.p, gammas, dgidx.bytes, hipMemcpyHostToDevice, s));
        std::vector<DevBuf> dloops(n_lat);
        for (int l = 0; l < n_lat; ++l)
            dloops[l].alloc((size_t)srcs[l].n_noise * n_gamma * gauges[l]->lat.dims[3] * 2 * sizeof(double));
        int worst = DL_OK;
        Stopwatch sw;
        for (int n0 = 0; n0 < max_noise; n0 += k) {
            std::vector<std::unique_ptr<SolveWork>> work;
            std::vector<DevBuf> dnoise, dcls, dC;
            std::vector<SourceSpec> spec;
            std::vector<Prob> P;
            std::vector<int> lat_of, r0_of, n_of;
            for (int l = 0; l < n_lat; ++l) {
                const int nn = std::min(k, srcs[l].n_noise - n0);
                if (nn <= 0) continue;
                const int ncls = source_classes(&srcs[l]);
                const int n = nn * ncls;
                dl_gauge G = gauges[l];
                std::vector<int64_t> hn(n);
                std::vector<int> hc(n);
                for (int i = 0; i < n; ++i) {
                    hn[i] = srcs[l].first_noise + n0 + i / ncls;
                    hc[i] = i % ncls;
                }
                dnoise.emplace_back(sizeof(int64_t) * n);
                dcls.emplace_back(sizeof(int) * n);
                dC.emplace_back((size_t)n * G->lat.dims[3] * 32 * sizeof(double));
                DL_HIP(hipMemcpyAsync(dnoise.back().p, hn.data(), dnoise.back().bytes, hipMemcpyHostToDevice, s));
                DL_HIP(hipMemcpyAsync(dcls.back().p, hc.data(), dcls.back().bytes, hipMemcpyHostToDevice, s));
                SourceSpec ss;
                ss.kind = srcs[l].kind;
                ss.scheme = srcs[l].kind == DL_SRC_POINT ? 0 : srcs[l].scheme;
                ss.seed = srcs[l].seed;
                ss.V = G->lat.V;
                ss.T = G->lat.dims[3];
                ss.point_site = srcs[l].point_site;
                ss.noise = dnoise.back().as<int64_t>();
                ss.cls = dcls.back().as<int>();
                spec.push_back(ss);
                work.emplace_back(new SolveWork);
                SolveWork &w = *work.back();
                w.alloc_bicg(prm.prec, n, G->lat.Vh);
                Ctx c{G, G->lat.geom(), s};
                k_source(P64, w.be.view(), 0, ss, c.g, n, s);
                k_source(P64, w.bo.view(), 1, ss, c.g, n, s);
                P.push_back(Prob{c, kappas[l], &w});
                lat_of.push_back(l);
                n_of.push_back(nn);
            }
            bicgstab_multi(P, prm, s);
            DL_HIP(hipStreamSynchronize(s));
            int round_rhs = 0;
            for (const Prob &p : P) round_rhs += p.w->n;
            const double secs_per_rhs = sw.lap() / std::max(1, round_rhs);
            for (size_t q = 0; q < P.size(); ++q) {
                const int l = lat_of[q];
                SolveWork &w = *P[q].w;
                const int ncls = source_classes(&srcs[l]);
                const int T = P[q].c.g.T;
                std::vector<double> res2;
                if (stats && stats[l]) true_residual_full(P[q].c, kappas[l], w, res2);
                k_trace(P64, w.x64.view(), w.xo.view(), spec[q], P[q].c.g, w.n, dC[q].as<double>(), s);
                k_gamma_contract(dC[q].as<double>(), n_of[q], ncls, T, dgam.as<double>(), dgidx.as<int>(), n_gamma,
                                 dloops[l].as<double>() + (size_t)n0 * n_gamma * T * 2, s);
                std::vector<dl_solve_stats> st(w.n);
                fill_stats(w, res2, st.data(), s, false, sw, secs_per_rhs);
                for (int i = 0; i < w.n; ++i) {
                    if (stats && stats[l]) stats[l][(int64_t)n0 * ncls + i] = st[i];
                    if (st[i].status != DL_OK && worst == DL_OK) worst = st[i].status;
                }
            }
            DL_HIP(hipGetLastError());
            DL_HIP(hipStreamSynchronize(s));
        }
        for (int l = 0; l < n_lat; ++l)
            DL_HIP(hipMemcpyAsync(loops[l], dloops[l].p, dloops[l].bytes, hipMemcpyDeviceToHost, s));
        DL_HIP(hipStreamSynchronize(s));
        if (worst != DL_OK) g_err = "dl_batch_loops: at least one solve did not converge";
        return worst;
    });
}

// ====================================================================== correlator

extern "C" int dl_disconnected_correlator(const double *loops_b, const double *loops_a, int32_t n_noise, int32_t T,
                                          int64_t spatial_volume, double *corr, void *stream)
{
    return guarded([&]() {
        StreamScope scope(stream);
        DL_REQUIRE(loops_b && loops_a && corr, "dl_disconnected_correlator: null pointer");
        DL_REQUIRE(n_noise >= 2, "dl_disconnected_correlator: needs at least two noises");
        DL_REQUIRE(T >= 1 && T <= 65535, "dl_disconnected_correlator: T must be in [1, 65535]");
        DL_REQUIRE(spatial_volume >= 1, "dl_disconnected_correlator: spatial volume must be positive");
        DL_REQUIRE((int64_t)n_noise * T <= ((int64_t)1 << 28), "dl_disconnected_correlator: input too large");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t nb = sizeof(double) * 2 * (size_t)n_noise * T, tb = sizeof(double) * 2 * (size_t)T;
        DevBuf db(nb), da(nb), dsb(tb), dsa(tb), dout(tb);
        DL_HIP(hipMemcpyAsync(db.p, loops_b, nb, hipMemcpyHostToDevice, s));
        DL_HIP(hipMemcpyAsync(da.p, loops_a, nb, hipMemcpyHostToDevice, s));
        const double norm = 1.0 / ((double)n_noise * (n_noise - 1)) / ((double)spatial_volume * T);
        k_correlator(db.as<double>(), da.as<double>(), dsb.as<double>(), dsa.as<double>(), n_noise, T, norm,
                     dout.as<double>(), s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipMemcpyAsync(corr, dout.p, tb, hipMemcpyDeviceToHost, s));
        DL_HIP(hipStreamSynchronize(s));
        return DL_OK;
    });
}

extern "C" int dl_eta_prime_fit(const double *d, const double *c_pi, int32_t ncfg, int32_t T, double m_pi,
                                int32_t tmin, int32_t tmax, double *c_eta, double *params, double *errors,
                                double *chi2)
{
    return guarded([&]() {
        eta_prime_fit(d, c_pi, ncfg, T, m_pi, tmin, tmax, c_eta, params, errors, chi2);
        return DL_OK;
    });
}

// ====================================================================== memory

extern "C" int dl_cache_release(void)
{
    return guarded([&]() {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        cache_trim_locked(0);
        return DL_OK;
    });
}

extern "C" int dl_cache_set_limit(uint64_t bytes)
{
    return guarded([&]() {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache_limit = (size_t)bytes;
        g_cache_limit_set = true;
        cache_trim_locked(g_cache_limit);
        return DL_OK;
    });
}

extern "C" uint64_t dl_cache_bytes(void)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return (uint64_t)g_cache_bytes;
}

// ====================================================================== profiling API

extern "C" int dl_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain_locked();
    g_prof_on = false;
    for (int k = 0; k < PROF_NKIND; ++k) {
        g_prof_ms[k] = 0;
        g_prof_bytes[k] = 0;
        g_prof_n[k] = 0;
        g_prof_cfg_set[k] = false;
    }
    if (on) {
        try {
            if (!g_prof_ctr.p) g_prof_ctr.alloc(sizeof(unsigned) * PROF_SLOTS);
            if (hipMemset(g_prof_ctr.p, 0, sizeof(unsigned) * PROF_SLOTS) != hipSuccess) return DL_EHIP;
            if (hipDeviceSynchronize() != hipSuccess) return DL_EHIP;
        } catch (const Error &e) {
            g_err = e.msg;
            return e.code;
        }
        g_prof_next = 0;
        g_prof_on = true;
    }
    return DL_OK;
}

extern "C" int dl_profile_config(int32_t kind, int32_t *cfg)
{
    if ((kind != PROF_DSLASH && kind != PROF_DSLASH_PLAIN) || cfg == nullptr) return DL_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_cfg_set[kind]) {
        for (int i = 0; i < 4; ++i) cfg[i] = -1;
    } else {
        const TuneChoice &t = g_prof_cfg[kind];
        cfg[0] = t.kind;
        cfg[1] = t.nr;
        cfg[2] = t.bs;
        cfg[3] = t.persistent;
    }
    return DL_OK;
}

namespace {
// two HIP events, destroyed on every exit
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EventPair()
    {
        DL_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            throw Error{DL_EHIP, "hipEventCreate failed"};
        }
    }
    ~EventPair()
    {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
};
}  // namespace

extern "C" int dl_stream_probe(const void *src, void *dst, uint64_t bytes, int32_t mode, int32_t reps, void *stream,
                               double *seconds)
{
    return guarded([&]() {
        DL_REQUIRE(src && dst && seconds, "dl_stream_probe: null pointer");
        DL_REQUIRE(mode == 0 || mode == 1, "dl_stream_probe: mode must be 0 (copy) or 1 (read)");
        DL_REQUIRE(reps >= 1, "dl_stream_probe: reps must be at least 1");
        DL_REQUIRE(bytes > 0 && bytes % 16 == 0, "dl_stream_probe: bytes must be a non-zero multiple of 16");
        DL_REQUIRE((uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0,
                   "dl_stream_probe: src and dst must be 16-byte aligned");
        const uintptr_t a0 = (uintptr_t)src, b0 = (uintptr_t)dst;
        const uint64_t span = mode == 0 ? bytes : 131072;
        DL_REQUIRE(a0 + bytes <= b0 || b0 + span <= a0, "dl_stream_probe: src and dst overlap");
        hipStream_t s = static_cast<hipStream_t>(stream);
        EventPair ev;
        DL_HIP(hipEventRecord(ev.e0, s));
        for (int r = 0; r < reps; ++r) stream_launch(mode, src, dst, (int64_t)(bytes / 16), s);
        DL_HIP(hipGetLastError());
        DL_HIP(hipEventRecord(ev.e1, s));
        DL_HIP(hipEventSynchronize(ev.e1));
        float ms = 0.0f;
        DL_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        *seconds = (double)ms * 1e-3 / reps;
        return DL_OK;
    });
}

extern "C" int64_t dl_profile_read(int32_t kind, double *ms, double *bytes)
{
    if (kind < 0 || kind >= PROF_NKIND) return DL_EINVAL;
    prof_drain();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (ms) *ms = g_prof_ms[kind];
    if (bytes) *bytes = g_prof_bytes[kind];
    return g_prof_n[kind];
}
