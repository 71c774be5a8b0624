// C ABI and host runtime of the FS-MLMC library: contexts, gauge upload, work
// plans, the batched BiCGStab driver (FP64 or mixed precision with FP64
// reliable updates, optionally hipGraph-captured), the Frequency-Splitting
// estimator over one or several lattices, the autotuner and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fsmlmc.h"
#include "fs_clover.h"
#include "fs_kernels.h"
#include "fs_probe.h"
#include "fs_shift.h"

using namespace fs;

// ============================================================== errors

// DeGrand-Rossi gamma_1..gamma_4 (g[mu][row][col]); gamma_5 = g1 g2 g3 g4 =
// diag(1, 1, -1, -1).  The stencil's spin projectors encode the same matrices.
void fs::dr_gammas(std::complex<double> g[4][4][4]) {
    using C = std::complex<double>;
    const C I(0, 1);
    const C t[4][4][4] = {
        {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
        {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
        {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
        {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
    };
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) g[m][a][b] = t[m][a][b];
}

namespace {

thread_local std::string g_err = "no error";

struct FsError : std::runtime_error {
    fs_status code;
    FsError(fs_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(fs_status c, const std::string& m) { throw FsError(c, m); }

void hipchk(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            fail(FS_E_OOM, std::string(what) + ": " + hipGetErrorString(e));
        fail(FS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}
#define HC(x) hipchk((x), #x)

template <typename F>
fs_status guard(F&& f) {
    try {
        f();
        return FS_OK;
    } catch (const FsError& e) {
        g_err = e.what();
        return e.code;
    } catch (const ShiftArgError& e) {
        g_err = e.what();
        return FS_E_ARG;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return FS_E_OOM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return FS_E_HIP;
    } catch (...) {
        g_err = "unknown error";
        return FS_E_HIP;
    }
}

// ============================================================== device memory

// Caching device allocator: freed blocks are kept per (device, size) and
// reused, so repeated solves and estimates do not call hipMalloc/hipFree in
// their loops.  Sizes are rounded up to 2 MiB above 1 MiB.  Over the cache
// limit the least recently released blocks go first, so the fields of the
// call just finished stay for the next call of the same shape.
struct Pool {
    struct Block {
        void* p;
        unsigned long long seq;  // release order
    };
    std::recursive_mutex mu;  // several host threads may drive contexts at once
    std::multimap<std::pair<int, size_t>, Block> free_;
    size_t cached = 0;
    size_t cap = 0;
    unsigned long long seq = 0;
    // Cache limit: half the device memory, so that the fields of a large batch
    // (tens of GB) are reused by the next solve of the same shape instead of
    // being released and allocated again, which costs about as much as the
    // solve.  An allocation that would leave less than a reserve of free
    // memory releases the cache first (get), and so does destroying the last
    // context.
    size_t limit() {
        if (!cap) {
            size_t f = 0, t = 0;
            cap = (hipMemGetInfo(&f, &t) == hipSuccess && t > 0) ? t / 2 : ((size_t)8 << 30);
            cap = std::max(cap, (size_t)8 << 30);
        }
        return cap;
    }
    static size_t round(size_t n) {
        if (n <= (1u << 20)) return (n + 255) & ~(size_t)255;
        const size_t g = (size_t)2 << 20;
        return (n + g - 1) / g * g;
    }
    void* get(size_t n, hipError_t* err) {
        std::lock_guard<std::recursive_mutex> lk(mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        auto it = free_.find({dev, n});
        if (it != free_.end()) {
            void* p = it->second.p;
            free_.erase(it);
            cached -= n;
            *err = hipSuccess;
            return p;
        }
        // keep a reserve of free device memory for the runtime (kernel launches,
        // graphs): cached blocks go first
        if (cached > 0) {
            size_t f = 0, t = 0;
            if (hipMemGetInfo(&f, &t) == hipSuccess) {
                const size_t reserve = std::max((size_t)16 << 30, t / 12);
                if (f < n + reserve) trim(0);
            }
        }
        void* p = nullptr;
        *err = hipMalloc(&p, n);
        if (*err != hipSuccess) {
            trim(0);
            *err = hipMalloc(&p, n);
        }
        return *err == hipSuccess ? p : nullptr;
    }
    void put(void* p, size_t n) {
        std::lock_guard<std::recursive_mutex> lk(mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        free_.insert({{dev, n}, Block{p, ++seq}});
        cached += n;
        if (cached > limit()) trim(limit());
    }
    size_t cached_bytes() {
        std::lock_guard<std::recursive_mutex> lk(mu);
        return cached;
    }
    // release cached blocks, least recently released first, until at most
    // `keep` bytes stay cached
    void trim(size_t keep) {
        std::lock_guard<std::recursive_mutex> lk(mu);
        bool synced = false;
        while (cached > keep && !free_.empty()) {
            auto old = free_.begin();
            for (auto it = free_.begin(); it != free_.end(); ++it)
                if (it->second.seq < old->second.seq) old = it;
            if (!synced) {
                (void)hipDeviceSynchronize();
                synced = true;
            }
            (void)hipFree(old->second.p);
            cached -= old->first.second;
            free_.erase(old);
        }
    }
};
int g_live_ctx = 0;  // contexts alive; the device cache is released with the last
std::mutex g_ctx_mu;  // guards g_live_ctx

Pool& pool() {
    static Pool* p = new Pool();  // never destroyed: blocks live until process exit
    return *p;
}

// Device scratch of the allocation-free entry point (fs_apply_dirac_noalloc):
// a fixed array in the code object, one copy per GPU, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (its name is a
// host-side stand-in); it uses the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device when the first
// context is created there.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With the device current: find this device's copy of the scratch array.
void scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;  // no scratch: the entry point reports FS_E_STATE
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return;
    }
    g_scratch_ptr[dev] = p;
}

void* scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { alloc(bytes); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t bytes) {
        release();
        const size_t nb = Pool::round(bytes == 0 ? 16 : bytes);
        hipError_t e;
        p = pool().get(nb, &e);
        hipchk(e, "device allocation");
        n = nb;
    }
    void release() {
        if (p) pool().put(p, n);
        p = nullptr;
        n = 0;
    }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Pinned host staging buffer.
struct HostBuf {
    void* p = nullptr;
    size_t n = 0;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
    void ensure(size_t bytes) {
        if (bytes <= n) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        HC(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        n = bytes;
    }
};

int prec_group_bytes_spinor(int P) { return P == P64 ? 192 : P == P32 ? 96 : 48; }
int prec_link_complex_bytes(int P) { return P == P64 ? 16 : P == P32 ? 8 : 4; }
// Site-major link bytes: 16-byte chunks of the full (9 complex) or, for
// FP32, the two-row (6 complex) form.
int prec_link_site_bytes(int P, bool two_rows) {
    if (two_rows && P == P32) return 48;
    return P == P64 ? 144 : P == P32 ? 80 : 36;
}

// Links whose third row equals the conjugated cross product of the first two
// within this bound are stored in the two-row form: the rebuilt row then
// differs from the stored one by far less than FP32 rounding (6e-8).
constexpr double kSu3RowTol = 1e-9;

// max over links and j of |U_2j - conj(U_0k U_1l - U_0l U_1k)|, (j, k, l)
// cyclic; u is the canonical layout, n_links row-major 3x3 complex matrices.
double su3_row_defect(const double* u, size_t n_links) {
    double worst = 0.0;
    for (size_t i = 0; i < n_links; ++i) {
        const double* m = u + 18 * i;
        for (int j = 0; j < 3; ++j) {
            const int k = (j + 1) % 3, l = (j + 2) % 3;
            const double akr = m[2 * k], aki = m[2 * k + 1], alr = m[2 * l], ali = m[2 * l + 1];
            const double bkr = m[6 + 2 * k], bki = m[7 + 2 * k], blr = m[6 + 2 * l], bli = m[7 + 2 * l];
            const double re = (akr * blr - aki * bli) - (alr * bkr - ali * bki);
            const double im = (akr * bli + aki * blr) - (alr * bki + ali * bkr);
            const double d = std::hypot(m[12 + 2 * j] - re, m[13 + 2 * j] + im);
            if (std::isnan(d)) return d;  // a non-finite entry: "not special unitary"
            if (d > worst) worst = d;
        }
    }
    return worst;
}
int prec_groups(int P) { return P == P64 ? 12 : P == P32 ? 6 : 3; }

// Upper bound on max_links ||U||_2: ||U||_2^2 is the largest eigenvalue of the
// Hermitian U^+ U, which Gershgorin's theorem bounds by its largest absolute
// row sum.  1 up to rounding for unitary links; NaN/Inf propagate.
double link_norm_bound(const double* u, size_t n_links) {
    double worst = 0.0;
    for (size_t i = 0; i < n_links; ++i) {
        const double* m = u + 18 * i;
        for (int a = 0; a < 3; ++a) {
            double row = 0.0;
            for (int b = 0; b < 3; ++b) {
                double re = 0.0, im = 0.0;  // (U^+ U)_ab = sum_k conj(U_ka) U_kb
                for (int k = 0; k < 3; ++k) {
                    const double xr = m[2 * (3 * k + a)], xi = m[2 * (3 * k + a) + 1];
                    const double yr = m[2 * (3 * k + b)], yi = m[2 * (3 * k + b) + 1];
                    re += xr * yr + xi * yi;
                    im += xr * yi - xi * yr;
                }
                row += std::hypot(re, im);
            }
            if (std::isnan(row)) return row;
            if (row > worst) worst = row;
        }
    }
    return std::sqrt(worst);
}

// ============================================================== gamma table

GammaTab make_gamma_tab() {
    using C = std::complex<double>;
    const C I(0, 1);
    C g[4][4][4];
    dr_gammas(g);
    GammaTab t;
    for (int n = 0; n < 16; ++n) {
        C M[4][4] = {};
        for (int a = 0; a < 4; ++a) M[a][a] = 1;
        for (int k = 0; k < 4; ++k) {
            if (!((n >> k) & 1)) continue;
            C R[4][4] = {};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int c = 0; c < 4; ++c) R[a][b] += M[a][c] * g[k][c][b];
            std::memcpy(M, R, sizeof(M));
        }
        for (int a = 0; a < 4; ++a) {
            int col = -1, ph = -1;
            for (int b = 0; b < 4; ++b) {
                if (std::abs(M[a][b]) > 0.5) {
                    col = b;
                    const C v = M[a][b];
                    ph = std::abs(v - C(1, 0)) < 1e-12 ? 0 : std::abs(v - I) < 1e-12 ? 1 : std::abs(v + C(1, 0)) < 1e-12 ? 2 : 3;
                }
            }
            t.perm[n][a] = (int8_t)col;
            t.ph[n][a] = (int8_t)ph;
        }
    }
    return t;
}

}  // namespace

// ============================================================== context

struct TuneEntry {
    int nr = 0, wg = 0, ilp = 0, occ = 0;
    double ms_per_sys = 0;
};

struct fs_ctx_s {
    std::string last_err = "no error";  // message of the last failing call on this context
    int dims[4] = {0, 0, 0, 0};
    int V = 0;
    int tsign = 1;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t instance = 0;
    bool has_gauge = false;
    DevBuf gauge[4];                 // [mu][9][site] per precision
    DevBuf gauge_q[4];               // [mu][site][link_q_bytes] per precision
    DevBuf gauge_q2[4];              // rows 0-1 only, [mu][site][QCR chunks] (FP32 entry only)
    bool two_rows = false;           // gauge_q2 is filled: every link is special unitary
    double su3_defect = 0.0;         // max |U_2j - conj(U_0 x U_1)_j| over the uploaded links
    double link_norm = 1.0;          // upper bound on the spectral norm of every uploaded link
    double c_sw = 0.0;               // clover coefficient (0: the plain Wilson operator)
    DevBuf clv[2];                   // clover term C, [parity][chunk][V/2]: FP64 (36 chunks), FP32 (18)
    double clv_norm = 0.0;           // upper bound on the spectral norm of every block of C
    std::map<int, TuneEntry> tune;   // per precision
    std::map<int, std::array<int, 2>> eo_tune;  // per precision: even-odd stencil variant, residency cap
    HostBuf pinned;
};

struct fs_batch_s {
    std::vector<fs_ctx> ctxs;
};

namespace {

// guard() for calls on a context: a failure's message is also kept on the
// context (fs_last_error(c)); a null context keeps it on the thread only.
template <typename F>
fs_status guard_ctx(fs_ctx c, F&& f) {
    const fs_status st = guard(std::forward<F>(f));
    if (st != FS_OK && c) c->last_err = g_err;
    return st;
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        HC(hipGetDevice(&prev));
        if (prev != dev) HC(hipSetDevice(dev));
    }
    ~DeviceScope() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

// two_rows: the plan's FP32 stencils rebuild row 2.
LatDesc lat_desc(const fs_ctx_s* c, int P, int eo = 0, bool two_rows = false) {
    LatDesc d;
    for (int i = 0; i < 4; ++i) d.L[i] = c->dims[i];
    d.V = c->V;
    d.Vf = eo ? c->V / 2 : c->V;
    d.eo = eo;
    d.tsign = c->tsign;
    d.gauge = c->gauge[P].p;
    d.gauge_q = (two_rows && P == P32) ? c->gauge_q2[P].p : c->gauge_q[P].p;
    d.pty = d.ptz = 0;
    d.clv = (c->c_sw != 0.0 && (P == P64 || P == P32)) ? c->clv[P].p : nullptr;
    return d;
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

bool pow2_ok(int n) { return n >= 1 && n <= 16 && (n & (n - 1)) == 0; }



// ============================================================== plans

// A batch of blocks (each NR systems of one lattice) mapped to workgroups.
struct Plan {
    int nr = 1, lognr = 0, wg = 256, tpw = 1;
    int eo = 0;                       // 1: fields of one parity (V/2 sites per system)
    bool two_rows = false;            // every lattice holds special unitary links (two-row loads)
    int ilp = 0, occ = 0;             // stencil variant and residency cap
    int tl[3] = {0, 0, 0};            // stencil variant 2: log2 tile extents
    int nsys = 0;                     // nblk * nr
    std::vector<BlockDesc> blocks;
    std::vector<int> wg_start;        // nblk + 1  (tile mapping: vector kernels)
    std::vector<int> wg_start_d;      // nblk + 1  (t-column mapping: stencil)
    int tc = 1;                       // t-slices per stencil workgroup
    // one-parity plans: the t-streaming mapping of the FP64 source and
    // reconstruction kernels (the stencil mapping itself when ilp != 2)
    std::vector<int> wg_start_s;
    int tc_s = 1;
    std::vector<std::array<int, 2>> ptile;  // x-pair stencil (ilp 2): TY, TZ per lattice
    std::vector<int> lat_V;           // per lattice
    long long total_slots = 0;
    // device tables
    DevBuf d_blocks, d_wg_start, d_wg_start_d, d_blk_on;
    DevBuf d_lats[4];
    DevBuf d_wg_start_alt;            // alternative start table (hop launches)
    DevBuf d_wg_start_s;              // streaming mapping of one-parity plans

    int max_wg() const {
        return std::max({wg_start.back(), wg_start_d.back(), wg_start_s.empty() ? 0 : wg_start_s.back()});
    }

    // stencil = true: the t-column mapping of the dslash launches (and of the
    // finish kernels that reduce their partial sums).
    // device tables held outside the plan (the allocation-free entry point), or null
    const LatDesc* x_lats = nullptr;
    const BlockDesc* x_blocks = nullptr;
    const int* x_wg_start = nullptr;
    const int* x_wg_start_d = nullptr;

    Work work(int P, bool use_blk_on, bool stencil = false) const {
        Work w;
        w.lats = x_lats ? x_lats : d_lats[P].as<LatDesc>();
        w.blocks = x_blocks ? x_blocks : d_blocks.as<BlockDesc>();
        if (x_wg_start) w.wg_start = stencil ? x_wg_start_d : x_wg_start;
        else w.wg_start = stencil ? d_wg_start_d.as<int>() : d_wg_start.as<int>();
        w.nblk = (int)blocks.size();
        w.total_wg = stencil ? wg_start_d.back() : wg_start.back();
        w.tc = stencil ? tc : 0;
        w.ilp = stencil ? ilp : 0;
        for (int k = 0; k < 3; ++k) w.tl[k] = tl[k];
        w.occ = stencil ? occ : 0;
        w.two_rows = (P == P32 && two_rows) ? 1 : 0;
        w.prow = 1;
        w.vlist = nullptr;
        w.vstart = nullptr;
        w.vcount = nullptr;
        w.tpw = tpw;
        w.wg = wg;
        w.nr = nr;
        w.lognr = lognr;
        w.blk_on = use_blk_on ? d_blk_on.as<int>() : nullptr;
        return w;
    }

    // one-parity plans: the t-streaming mapping (FP64 source and reconstruction)
    Work work_stream(int P) const {
        Work w = work(P, false, true);
        if (eo && ilp == 2) {
            w.wg_start = d_wg_start_s.as<int>();
            w.total_wg = wg_start_s.back();
            w.tc = tc_s;
            w.ilp = 0;
        }
        return w;
    }
};

constexpr int kTargetWG = 4096;  // workgroups per launch to aim for (256 CUs x 16)

// Stencil t-chunks: lanes launched per t-slice are sized to this many times
// the chip's resident capacity at 4 waves per SIMD.
#ifndef FS_TC_OVERSUB
#define FS_TC_OVERSUB 8
#endif

// Tile of the LDS-staged stencil: wg / nr sites as TX x TY x TZ, powers of two,
// each >= 2 and dividing the x/y/z extents of every lattice of the plan; the
// shape with the fewest outside neighbours per site (sum over the axes the
// tile does not span of 2 / T) wins, ties to the longer x extent (contiguous
// in memory).  Returns false if no such shape exists.
static bool choose_tile(int sites, const std::vector<fs_ctx_s*>& lats, int tl[3]) {
    int ls = 0;
    while ((1 << ls) < sites) ++ls;
    if ((1 << ls) != sites) return false;
    double best = 1e30;
    bool found = false;
    for (int a = 1; a <= ls; ++a)
        for (int b = 1; a + b < ls; ++b) {
            const int cz = ls - a - b;
            const int e[3] = {a, b, cz};
            bool ok = true;
            double cost = 0.0;
            for (int k = 0; k < 3 && ok; ++k) {
                bool spans = true;
                for (auto* c : lats) {
                    if (c->dims[k] % (1 << e[k]) != 0) ok = false;
                    if (c->dims[k] != (1 << e[k])) spans = false;
                }
                if (!spans) cost += 2.0 / (1 << e[k]);
            }
            if (!ok) continue;
            cost -= 1e-6 * a;
            if (cost < best) {
                best = cost;
                tl[0] = a;
                tl[1] = b;
                tl[2] = cz;
                found = true;
            }
        }
    return found;
}

// blk_lat[b]: lattice of block b; lats: the contexts of the lattices.
// Work tables for a given list of blocks (each block keeps its system ids and
// field offsets, so a plan over a subset of a batch shares the batch's fields).
// x-pair stencil: at least this many lanes (2 waves per SIMD of the chip),
// else the t-streaming variant, which splits small batches finer
#ifndef FS_PAIR_MIN_LANES
#define FS_PAIR_MIN_LANES (256 * 4 * 2 * 64)
#endif
// resident x-pair workgroups per CU assumed when sizing its t-chunks
#ifndef FS_PAIR_WG_PER_CU
#define FS_PAIR_WG_PER_CU 3
#endif

// Tiles of the x-pair even-odd stencil: per lattice TY x TZ pairs (dividing
// Ly, Lz, each at least 2; the tile spans all Lx/2 pairs of x) so that
// nr * Lx/2 * TY * TZ lanes fit the workgroup; the most lanes win, then the
// fewest reads beyond the tile's y/z faces per output (2/T for an axis the
// tile does not span).  False if no such tile fits.
static bool pair_tiles(int nr, int wg, const std::vector<fs_ctx_s*>& lats, std::vector<std::array<int, 2>>& out) {
    out.clear();
    for (auto* c : lats) {
        const int row = nr * (c->dims[0] / 2);
        if (row > wg || c->dims[0] % 2) return false;
        const int maxyz = wg / row;
        int bt[2] = {0, 0}, best_n = 0;
        double best_cost = 1e30;
        for (int ty = 1; ty <= c->dims[1]; ++ty) {
            if (c->dims[1] % ty) continue;
            if (ty == 1 && c->dims[1] != 1) continue;  // one-pair-thick tiles are not supported
            for (int tz = 2; tz <= c->dims[2] && ty * tz <= maxyz; ++tz) {
                if (c->dims[2] % tz) continue;
                const double cost = (ty < c->dims[1] ? 2.0 / ty : 0.0) + (tz < c->dims[2] ? 2.0 / tz : 0.0);
                if (ty * tz > best_n || (ty * tz == best_n && cost < best_cost)) {
                    best_n = ty * tz;
                    best_cost = cost;
                    bt[0] = ty;
                    bt[1] = tz;
                }
            }
        }
        if (best_n == 0) return false;
        out.push_back({bt[0], bt[1]});
    }
    return true;
}

// The host side of a plan (no device tables): mappings and workgroup counts.
void plan_host(Plan* pl, const std::vector<BlockDesc>& blocks, const std::vector<fs_ctx_s*>& lats, int nr, int wg,
               int ilp, int occ, int eo) {
    pl->nr = nr;
    pl->eo = eo;
    pl->ilp = ilp;
    pl->occ = occ;
    pl->lognr = ilog2(nr);
    if (ilp == 2 && !eo && !choose_tile(wg / nr, lats, pl->tl)) pl->ilp = 0;  // no tile fits: column variant
    pl->wg = wg;
    pl->blocks = blocks;
    const int nblk = (int)blocks.size();
    pl->nsys = nblk * nr;
    for (auto* c : lats) pl->lat_V.push_back(c->V);
    long long tiles_total = 0;
    std::vector<long long> tiles(nblk);
    for (int b = 0; b < nblk; ++b) {
        const long long slots = (long long)(lats[blocks[b].lat]->V >> eo) * nr;
        tiles[b] = (slots + wg - 1) / wg;
        tiles_total += tiles[b];
        pl->total_slots = std::max(pl->total_slots, blocks[b].slot_off + slots);
    }
    pl->tpw = (int)std::max<long long>(1, tiles_total / kTargetWG);
    pl->wg_start.assign(nblk + 1, 0);
    for (int b = 0; b < nblk; ++b) {
        const long long nwg = (tiles[b] + pl->tpw - 1) / pl->tpw;
        if (pl->wg_start[b] + nwg > (1ll << 30)) fail(FS_E_ARG, "batch too large for one launch");
        pl->wg_start[b + 1] = pl->wg_start[b] + (int)nwg;
    }
    // stencil: columns of (xyz, rhs) slots walking t in chunks of tc slices,
    // enough chunks to keep every SIMD busy with ~4 waves even when only 1/8
    // of the blocks still run (the slowest shifts iterate longest, alone)
    {
        long long lanes = 0;
        int Lt_min = 1 << 30;
        for (int b = 0; b < nblk; ++b) {
            const fs_ctx_s* c = lats[blocks[b].lat];
            lanes += (long long)(c->V / c->dims[3]) * nr;
            Lt_min = std::min(Lt_min, c->dims[3]);
        }
        const long long target = (long long)FS_TC_OVERSUB * 256 * 4 * 4 * 64;
        long long nch = std::max<long long>(1, (target + lanes - 1) / std::max<long long>(1, lanes));
        if (!eo) {
            int tcv = (int)std::max<long long>(2, (Lt_min + nch - 1) / nch);
            pl->tc = std::min(tcv, Lt_min);
        } else {  // one-parity fields: tc counts output steps of 2 t-slices
            const int steps = Lt_min / 2;
            pl->tc = std::max(1, std::min(steps, (int)((steps + nch - 1) / nch)));
        }
        pl->wg_start_d.assign(nblk + 1, 0);
        for (int b = 0; b < nblk; ++b) {
            const fs_ctx_s* c = lats[blocks[b].lat];
            long long cnt;
            if (!eo) {
                const long long n3 = (long long)(c->V / c->dims[3]) * nr;
                const long long ntile3 = (n3 + wg - 1) / wg;
                cnt = ntile3 * ((c->dims[3] + pl->tc - 1) / pl->tc);
            } else {  // two parity classes of columns, each walking Lt/2 output steps
                const long long n3 = (long long)(c->V / c->dims[3] / 2) * nr;
                const long long ntile3 = (n3 + wg - 1) / wg;
                cnt = 2 * ntile3 * ((c->dims[3] / 2 + pl->tc - 1) / pl->tc);
            }
            if (pl->wg_start_d[b] + cnt > (1ll << 30)) fail(FS_E_ARG, "batch too large for one launch");
            pl->wg_start_d[b + 1] = pl->wg_start_d[b] + (int)cnt;
        }
    }
    if (eo) {
        pl->wg_start_s = pl->wg_start_d;
        pl->tc_s = pl->tc;
    }
    if (eo && pl->ilp == 2) {
        long long lanes = 0;
        for (int b = 0; b < nblk; ++b) {
            const fs_ctx_s* c = lats[blocks[b].lat];
            lanes += (long long)(c->V / c->dims[3] / 2) * nr;
        }
        if (lanes < FS_PAIR_MIN_LANES || !pair_tiles(nr, wg, lats, pl->ptile)) pl->ilp = 0;
    }
    if (eo && pl->ilp == 2) {
        // x-pair stencil: workgroups of TY x TZ pairs of one block walking
        // chunks of tc t-slices.  Each chunk costs two extra spinor loads per
        // lane (its first input slice and the backward neighbour), and the
        // workgroups run in rounds of the resident count R, so the chunk
        // count minimises (1 + 2/tc) x rounds x R / workgroups.
        long long w1 = 0;  // workgroups of one chunk per block, summed
        int Lt_min = 1 << 30;
        for (int b = 0; b < nblk; ++b) {
            const fs_ctx_s* c = lats[blocks[b].lat];
            const auto& tl = pl->ptile[blocks[b].lat];
            w1 += (long long)(c->dims[1] / tl[0]) * (c->dims[2] / tl[1]);
            Lt_min = std::min(Lt_min, c->dims[3]);
        }
        const long long R = 256ll * FS_PAIR_WG_PER_CU;
        double best = 1e30;
        for (int nch = 1; nch <= 16; ++nch) {
            const int tcv = (Lt_min + nch - 1) / nch;
            if (nch > 1 && tcv < 4) break;
            const long long wgs = w1 * nch;
            const double rounds = (double)((wgs + R - 1) / R);
            const double cost = (1.0 + 2.0 / tcv) * rounds * R / (double)wgs;
            if (cost < best - 1e-9) {
                best = cost;
                pl->tc = tcv;
            }
        }
        for (int b = 0; b < nblk; ++b) {
            const fs_ctx_s* c = lats[blocks[b].lat];
            const auto& tl = pl->ptile[blocks[b].lat];
            const long long cnt =
                (long long)(c->dims[1] / tl[0]) * (c->dims[2] / tl[1]) * ((c->dims[3] + pl->tc - 1) / pl->tc);
            if (pl->wg_start_d[b] + cnt > (1ll << 30)) fail(FS_E_ARG, "batch too large for one launch");
            pl->wg_start_d[b + 1] = pl->wg_start_d[b] + (int)cnt;
        }
    }
    pl->two_rows = !lats.empty();
    for (auto* c : lats) pl->two_rows = pl->two_rows && c->two_rows;
}

std::unique_ptr<Plan> plan_from_blocks(const std::vector<BlockDesc>& blocks, const std::vector<fs_ctx_s*>& lats,
                                       int nr, int wg, hipStream_t s, int ilp, int occ, int eo = 0) {
    auto pl = std::make_unique<Plan>();
    plan_host(pl.get(), blocks, lats, nr, wg, ilp, occ, eo);
    const int nblk = (int)blocks.size();
    const int nb1 = std::max(nblk, 1);
    pl->d_blocks.alloc(sizeof(BlockDesc) * nb1);
    pl->d_wg_start.alloc(sizeof(int) * (nblk + 1));
    pl->d_wg_start_d.alloc(sizeof(int) * (nblk + 1));
    pl->d_blk_on.alloc(sizeof(int) * nb1);
    std::vector<int> ones(nb1, 1);
    if (nblk) HC(hipMemcpyAsync(pl->d_blocks.p, pl->blocks.data(), sizeof(BlockDesc) * nblk, hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(pl->d_wg_start.p, pl->wg_start.data(), sizeof(int) * (nblk + 1), hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(pl->d_wg_start_d.p, pl->wg_start_d.data(), sizeof(int) * (nblk + 1), hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(pl->d_blk_on.p, ones.data(), sizeof(int) * nb1, hipMemcpyHostToDevice, s));
    if (eo) {
        pl->d_wg_start_s.alloc(sizeof(int) * (nblk + 1));
        HC(hipMemcpyAsync(pl->d_wg_start_s.p, pl->wg_start_s.data(), sizeof(int) * (nblk + 1), hipMemcpyHostToDevice,
                          s));
    }
    std::vector<LatDesc> ld[4];
    for (int P = 0; P < 4; ++P) {
        for (size_t k = 0; k < lats.size(); ++k) {
            LatDesc d = lat_desc(lats[k], P, eo, pl->two_rows);
            if (pl->ilp == 2 && eo) {
                d.pty = pl->ptile[k][0];
                d.ptz = pl->ptile[k][1];
            }
            ld[P].push_back(d);
        }
        pl->d_lats[P].alloc(sizeof(LatDesc) * ld[P].size());
        HC(hipMemcpyAsync(pl->d_lats[P].p, ld[P].data(), sizeof(LatDesc) * ld[P].size(), hipMemcpyHostToDevice, s));
    }
    HC(hipStreamSynchronize(s));
    return pl;
}

// A batch of blocks: block b holds systems b*nr .. b*nr+nr-1 of lattice blk_lat[b].
std::unique_ptr<Plan> make_plan(const std::vector<int>& blk_lat, const std::vector<fs_ctx_s*>& lats, int nr, int wg,
                                hipStream_t s, int ilp = 0, int occ = 0, int eo = 0) {
    std::vector<BlockDesc> blocks(blk_lat.size());
    long long off = 0;
    for (size_t b = 0; b < blk_lat.size(); ++b) {
        blocks[b].lat = blk_lat[b];
        blocks[b].sys0 = (int)b * nr;
        blocks[b].slot_off = off;
        off += (long long)(lats[blk_lat[b]]->V >> eo) * nr;
    }
    return plan_from_blocks(blocks, lats, nr, wg, s, ilp, occ, eo);
}

// Residency cap of the t-streaming even-odd stencil (waves per SIMD, 0 =
// none): a sweep of the FP32 hop on the 16^3x32 workload (96 systems) found 3
// fastest at rhs block 4 (0.571 against 0.635 ms uncapped) and no gain at
// other blocks or in FP16.
int eo_occ(int P, int nr) { return (P == P32 && nr == 4) ? 3 : 0; }

// Even-odd stencil configuration of a context for one storage precision:
// variant 0 (t-streaming over one parity class of columns) or 2 (x-pairs
// with LDS sharing), residency cap (-1: the variant's default).  Without a
// setting: x-pairs for FP64, FP32 and FP16 storage (FP16 in its packed form),
// streaming for BF16, whose x-pair Schur launches run at one wave per SIMD.
std::array<int, 2> eo_tuning(const fs_ctx_s* c, int P) {
    auto it = c->eo_tune.find(P);
    if (it != c->eo_tune.end()) return it->second;
    return {P != PBF ? 2 : 0, -1};
}

// The one-parity plan of a full-lattice plan: the same blocks and systems, each
// block holding V/2 sites (even-odd preconditioning).  var, occ as eo_tuning.
std::unique_ptr<Plan> eo_plan_of(const Plan& full, const std::vector<fs_ctx_s*>& lats, hipStream_t s, int P,
                                 int var, int occ) {
    std::vector<BlockDesc> blocks = full.blocks;
    long long off = 0;
    for (auto& bd : blocks) {
        bd.slot_off = off;
        off += (long long)(lats[bd.lat]->V / 2) * full.nr;
    }
    auto pl = plan_from_blocks(blocks, lats, full.nr, full.wg, s, var, std::max(occ, 0), 1);
    if (occ < 0) pl->occ = pl->ilp == 2 ? 0 : eo_occ(P, full.nr);  // launch-time only: no table depends on it
    return pl;
}

// FP64 true residual of a system relative to its source (the full system's
// source under even-odd preconditioning).
double true_rel(const SysState& S) {
    const double d = S.bnorm2 > 0.0 ? S.bnorm2 : S.bb;
    return d > 0.0 ? std::sqrt(S.rr_true / d) : 0.0;
}

// A block-layout field over a whole plan.
struct Field {
    int P = P64;
    DevBuf v, n;
    void alloc(int prec, long long slots) {
        P = prec;
        v.alloc((size_t)slots * prec_group_bytes_spinor(prec));
        if (prec == P16) n.alloc((size_t)slots * sizeof(float));
    }
    Fld f() const {
        Fld r;
        r.v = v.as<uint4>();
        r.n = n.as<float>();
        return r;
    }
};

// ============================================================== solver

// Residual reduction between FP64 reliable updates.  The iterated residual of
// a storage format with unit roundoff u drifts from the true one by ~u/delta;
// the values below were the fastest of a sweep on the 16^3x32 workload (a
// smaller delta means fewer FP64 updates at a slightly higher drift).
double default_delta(int P) { return P == P32 ? 1e-5 : P == P16 ? 0.005 : 0.03; }

struct SolveOpts {
    int P = P64;
    double tol = 1e-10;
    int max_iter = 10000;
    double delta = 0.0;
    int check_every = 8;
    bool use_graph = false;
    bool eo = false;  // even-odd preconditioning
    int eo_var = 0, eo_occ = -1;  // even-odd stencil (eo_tuning)
};

// Multi-shift members carried along a batch's base systems (FP64, full
// lattice): member k of every system solves (A + d[k]) x = b from the base
// system's Krylov space (shifted BiCGStab; launch_ms_scalars).
struct MultiShift {
    int nm = 0;
    std::vector<Field> xs, ps;
    DevBuf d_d, d_state, d_coef;
    MsFields f;
};

// Systems of a plan, with sources in `b` (FP64 block layout) and per-system
// shifts.  On return xhi holds the solutions and `st_host` the final states.
// With even-odd preconditioning the Krylov iteration runs on a one-parity plan
// of the same blocks: sb_ = b_e - D_eo b_o / a, the Schur system S x_e = sb_,
// then x = (x_e, (b_o - D_oe x_e) / a) in xhi.  b, xhi and rhi stay full-lattice.
struct BatchSolver {
    Plan& full;                  // the caller's plan (layout of b, xhi, rhi)
    std::unique_ptr<Plan> eo_pl; // its one-parity plan (even-odd only)
    Plan& pl;                    // the plan the iteration runs on (fields, states, system ids)
    Plan* cur;                   // the blocks still iterating (pl, or a compacted sub-plan)
    std::unique_ptr<Plan> sub;
    std::vector<fs_ctx_s*> lats;
    hipStream_t s;
    SolveOpts o;
    Field b, xhi, rhi, r, p, v, t, xlo;
    Field sb_, sx_, sr_, tmp, tmp64;  // even-odd: FP64 Schur b, x, r; odd-site scratch
    DevBuf d_diag, d_st, d_part, d_flags, d_rkeys, d_rc, d_vl;  // d_rc: shadow-residual code words per slot
    MultiShift* ms = nullptr;  // optional members of a multi-shift solve (FP64, full lattice)
    // clover term: per (lattice, shift) the inverses of C + a at the odd sites
    bool clv = false;
    DevBuf d_inv64, d_inv32, d_off64, d_off32;
    Clv cl64, cl32;
    const Clv& clv_of(int P) const { return P == P64 ? cl64 : cl32; }
    VList vl_run, vl_pend, vl_conv;
    std::vector<SysState> st_host;
    long long dslash_calls = 0;
    size_t part_doubles = 0;
    // doubles of partial sums the launches over plan q may write
    size_t part_need(const Plan& q) const { return (size_t)q.max_wg() * 32 * q.nr; }

    BatchSolver(Plan& plan, const std::vector<fs_ctx_s*>& l, hipStream_t stream, const SolveOpts& opts)
        : full(plan), eo_pl(opts.eo ? eo_plan_of(plan, l, stream, opts.P, opts.eo_var, opts.eo_occ) : nullptr),
          pl(opts.eo ? *eo_pl : plan),
          cur(&pl), lats(l), s(stream), o(opts) {
        int n_clv = 0;
        for (const BlockDesc& bd : pl.blocks) n_clv += lats[bd.lat]->c_sw != 0.0;
        if (n_clv) {
            if (n_clv != (int)pl.blocks.size())
                fail(FS_E_ARG, "a batch mixes lattices with and without the clover term");
            if (!o.eo) fail(FS_E_ARG, "the clover term needs even-odd preconditioning (even_odd = 1)");
            if (o.P != P64 && o.P != P32) fail(FS_E_ARG, "the clover term needs FP64 or FP32 storage");
            clv = true;
        }
        const long long S = pl.total_slots;
        b.alloc(P64, full.total_slots);
        xhi.alloc(P64, full.total_slots);
        rhi.alloc(P64, full.total_slots);
        if (o.eo) {
            for (Field* f : {&sb_, &sx_, &sr_, &tmp64}) f->alloc(P64, S);
            tmp.alloc(o.P, S);
        }
        for (Field* f : {&r, &p, &v, &t, &xlo}) f->alloc(o.P, S);
        d_rc.alloc(sizeof(uint32_t) * (size_t)S);
        d_diag.alloc(sizeof(double) * pl.nsys);
        d_st.alloc(sizeof(SysState) * pl.nsys);
        // partial sums: at most 8 doubles per rhs per workgroup (32 for the hop
        // launches of the bilinears, which callers run over the full-lattice plan)
        part_doubles = std::max(part_need(pl), part_need(full));
        d_part.alloc(sizeof(double) * part_doubles);
        d_flags.alloc(sizeof(int) * 2 * pl.blocks.size());
        const size_t nb = pl.blocks.size();
        d_vl.alloc(sizeof(int) * 3 * (3 * nb + 3));
        int* q = d_vl.as<int>();
        for (VList* v : {&vl_run, &vl_pend, &vl_conv}) {
            v->list = q;
            v->vstart_tile = q + nb;
            v->vstart_sten = q + 2 * nb + 1;
            v->count = q + 3 * nb + 2;
            q += 3 * nb + 3;
        }
        st_host.resize(pl.nsys);
    }

    // diag[sys] = 4 + m0 + sigma; idle marks padding systems; rkeys[sys]: the
    // Z4 stream of the shadow residual (the source's own key for estimator
    // systems, so rhat = r0 = b).
    void setup(const std::vector<double>& diag, const std::vector<char>& idle, const std::vector<NoiseKey>& rkeys) {
        HC(hipMemcpyAsync(d_diag.p, diag.data(), sizeof(double) * pl.nsys, hipMemcpyHostToDevice, s));
        if (clv) setup_clover(diag);
        d_rkeys.alloc(sizeof(NoiseKey) * pl.nsys);
        HC(hipMemcpyAsync(d_rkeys.p, rkeys.data(), sizeof(NoiseKey) * pl.nsys, hipMemcpyHostToDevice, s));
        for (int i = 0; i < pl.nsys; ++i) {
            SysState z;
            std::memset(&z, 0, sizeof(z));
            z.tol2 = o.tol * o.tol;
            z.delta2 = o.delta * o.delta;
            z.max_iter = o.max_iter;
            z.state = idle[i] ? S_IDLE : S_RUN;
            st_host[i] = z;
        }
        HC(hipMemcpyAsync(d_st.p, st_host.data(), sizeof(SysState) * pl.nsys, hipMemcpyHostToDevice, s));
        HC(hipStreamSynchronize(s));  // the host vectors may go out of scope
    }
    // One inverse field per (lattice, 4 + m0 + sigma) of the plan's systems
    // (padding systems included: every system's offset points at a field).
    void setup_clover(const std::vector<double>& diag) {
        std::map<std::pair<int, double>, long long> fld;  // key -> offset in FP32 chunks
        std::vector<std::pair<int, double>> order;
        std::vector<long long> off32(pl.nsys, 0);
        long long tot = 0;
        for (const BlockDesc& bd : pl.blocks)
            for (int r = 0; r < pl.nr; ++r) {
                const int sys = bd.sys0 + r;
                const auto key = std::make_pair(bd.lat, diag[sys]);
                auto it = fld.find(key);
                if (it == fld.end()) {
                    it = fld.emplace(key, tot).first;
                    order.push_back(key);
                    tot += 18ll * (lats[bd.lat]->V / 2);
                }
                off32[sys] = it->second;
            }
        if (order.empty()) return;
        std::vector<long long> off64(off32.size());
        for (size_t i = 0; i < off32.size(); ++i) off64[i] = 2 * off32[i];
        d_inv64.alloc((size_t)tot * 2 * 16);
        if (o.P == P32) d_inv32.alloc((size_t)tot * 16);
        d_off64.alloc(sizeof(long long) * off64.size());
        d_off32.alloc(sizeof(long long) * off32.size());
        HC(hipMemcpyAsync(d_off64.p, off64.data(), sizeof(long long) * off64.size(), hipMemcpyHostToDevice, s));
        HC(hipMemcpyAsync(d_off32.p, off32.data(), sizeof(long long) * off32.size(), hipMemcpyHostToDevice, s));
        DevBuf bad(sizeof(int));
        HC(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        for (const auto& key : order) {
            const fs_ctx_s* c = lats[key.first];
            const int vh = c->V / 2;
            const long long o32 = fld[key];
            launch_clover_invert(c->clv[P64].as<uint4>() + (size_t)36 * vh, vh, key.second,
                                 d_inv64.as<uint4>() + 2 * o32, o.P == P32 ? d_inv32.as<uint4>() + o32 : nullptr,
                                 bad.as<int>(), s);
        }
        HC(hipGetLastError());
        int h_bad = 0;
        HC(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        if (h_bad) fail(FS_E_ARG, "C + 4 + m0 + sigma is singular at an odd site");
        cl64.inv = d_inv64.as<uint4>();
        cl64.off = d_off64.as<long long>();
        cl32.inv = d_inv32.as<uint4>();
        cl32.off = d_off32.as<long long>();
    }
    const NoiseKey* rk() const { return d_rkeys.as<NoiseKey>(); }
    uint32_t* rc() { return d_rc.as<uint32_t>(); }
    // the FP64 fields of the system the iteration solves
    Field& fb() { return o.eo ? sb_ : b; }
    Field& fx() { return o.eo ? sx_ : xhi; }
    Field& fr() { return o.eo ? sr_ : rhi; }

    // out = A in with the fused partial sums of `mode`; A = D + sigma, or the
    // even-odd Schur operator (two launches: the odd-site hop, then S).  `ws` is
    // the stencil mapping the following finish must use.
    void apply(int prec, int mode, const Work& ws, Fld out, Fld in, Fld aux, int mask, Fld scratch) {
        const double* dg = d_diag.as<double>();
        if (!o.eo) {
            launch_dslash(prec, mode, ws, out, in, aux, dg, st(), mask, part(), s, rc());
            return;
        }
        const int hp = mode == D_RESID ? P64 : prec;
        if (clv) {  // the hop's odd-site output times (C_o + a)^-1, then (C_e + a) in - D_eo (.)
            launch_dslash_eo_clv(hp, D_HOP, ws, scratch, in, Fld(), Fld(), dg, st(), mask, part(), s, rc(), 1,
                                 clv_of(hp));
            launch_dslash_eo_clv(hp, mode, ws, out, scratch, in, aux, dg, st(), mask, part(), s, rc(), 0,
                                 clv_of(hp));
            return;
        }
        launch_dslash_eo(hp, D_HOP, ws, scratch, in, Fld(), Fld(), dg, st(), mask, part(), s, rc(), 1);
        launch_dslash_eo(hp, mode, ws, out, scratch, in, aux, dg, st(), mask, part(), s, rc(), 0);
    }

    SysState* st() { return d_st.as<SysState>(); }
    double* part() { return d_part.as<double>(); }
    int* f_run() { return cur->d_blk_on.as<int>(); }
    int* f_pend() { return d_flags.as<int>(); }
    int* f_conv() { return d_flags.as<int>() + pl.blocks.size(); }
    Work with(const Work& w, int* flags) const {
        Work x = w;
        x.blk_on = flags;
        return x;
    }
    // persistent launch over the blocks of list vl (tile or stencil mapping)
    Work listed(const VList& vl, int P, bool stencil) const {
        Work x = cur->work(P, false, stencil);
        x.vlist = vl.list;
        x.vstart = stencil ? vl.vstart_sten : vl.vstart_tile;
        x.vcount = vl.count;
        return x;
    }
    void build_list(const int* flags, const VList& vl) {
        launch_vlist(flags, (int)cur->blocks.size(), cur->d_wg_start.as<int>(), cur->d_wg_start_d.as<int>(), vl, s);
    }

    // One BiCGStab iteration over every running system.  Every launch walks
    // the device-side list of running blocks, so finished blocks cost nothing;
    // the list changes when F_OMEGA (or a resumed reliable update) says so.
    // The t = A s stencil also forms (s, s), (rhat, s) and (rhat, t), so the
    // F_OMEGA finish knows omega, beta and the new residual's (rhat, r) and
    // |r|^2, and one vector kernel updates x, r and p (8 field passes; with
    // s = r - alpha v, 11 per iteration besides the stencils).
    // With in_loop_reliable the FP64 reliable update of the blocks that asked
    // for one follows at once (no host round trip).
    void iteration(bool in_loop_reliable) {
        const Work wr = listed(vl_run, o.P, false), wd = listed(vl_run, o.P, true);
        apply(o.P, D_RHAT, wd, v.f(), p.f(), Fld(), M_RUN, tmp.f());
        launch_finish(F_ALPHA, wd, st(), part(), nullptr, nullptr, s);
        launch_axpy_s(o.P, wr, r.f(), v.f(), st(), s);
        apply(o.P, D_TS, wd, t.f(), r.f(), Fld(), M_RUN, tmp.f());
        launch_finish(F_OMEGA, wd, st(), part(), f_run(), f_pend(), s);
        if (ms) {  // the members' x and p, from s (in r), v and t before the base overwrites them
            launch_ms_scalars(pl.nsys, ms->nm, ms->d_d.as<double>(), st(), ms->d_state.as<MsState>(),
                              ms->d_coef.as<MsCoef>(), s);
            launch_ms_update(wr, ms->nm, r.f(), v.f(), t.f(), ms->f, ms->d_coef.as<MsCoef>(), s);
        }
        build_list(f_run(), vl_run);
        launch_update_xrp(o.P, listed(vl_run, o.P, false), xlo.f(), p.f(), r.f(), t.f(), v.f(), st(), s);
        dslash_calls += 2;
        if (in_loop_reliable) {
            build_list(f_pend(), vl_pend);
            reliable_chain();
        }
    }

    // FP64 reliable update of the blocks in vl_pend: x_hi += x_lo,
    // r_hi = b - (D + sigma) x_hi, then either done or resume with r = r_hi.
    void reliable_chain() {
        const Work wp = listed(vl_pend, o.P, false), wpd = listed(vl_pend, o.P, true);
        const Work wp64d = listed(vl_pend, P64, true);
        launch_fold(o.P, wp, fx().f(), xlo.f(), st(), s);
        apply(P64, D_RESID, wp64d, fr().f(), fx().f(), fb().f(), M_PEND, tmp64.f());
        launch_finish(F_TRUE, wpd, st(), part(), f_conv(), f_pend(), s);  // clears f_pend
        build_list(f_conv(), vl_conv);
        const Work wc = listed(vl_conv, o.P, false);
        launch_convert(o.P, wc, fr().f(), r.f(), rk(), rc(), p.f(), st(), part(), s);
        launch_finish(F_RESUME, wc, st(), part(), f_run(), f_conv(), s);  // clears f_conv
        build_list(f_run(), vl_run);
    }

    // Host-driven variant: mark pending blocks from the states, then the chain.
    void reliable() {
        const Work w = cur->work(o.P, false);
        launch_blk_mask(w, st(), M_PEND, f_pend(), s);
        build_list(f_pend(), vl_pend);
        reliable_chain();
        launch_blk_mask(w, st(), M_RUN, f_run(), s);
        build_list(f_run(), vl_run);
        dslash_calls += 1;
    }

    static bool active_state(int st) {
        return st == S_RUN || st == S_REL || st == S_CHK || st == S_BRK || st == S_MAXIT || st == S_CONV ||
               st == S_RST;
    }

    // Replace the iterating set by the blocks that still have active systems
    // (false: nothing to drop).
    bool compact() {
        std::vector<BlockDesc> keep;
        for (const BlockDesc& bd : cur->blocks) {
            bool any = false;
            for (int r = 0; r < pl.nr; ++r) any |= active_state(st_host[bd.sys0 + r].state);
            if (any) keep.push_back(bd);
        }
        if (keep.empty() || keep.size() == cur->blocks.size()) return false;
        auto np = plan_from_blocks(keep, lats, pl.nr, pl.wg, s, pl.ilp, pl.occ, pl.eo);
        if (part_need(*np) > part_doubles) {
            part_doubles = part_need(*np);
            d_part.alloc(sizeof(double) * part_doubles);
        }
        sub = std::move(np);
        cur = sub.get();
        const Work w = cur->work(o.P, false);
        launch_blk_mask(w, st(), M_RUN, f_run(), s);
        launch_blk_mask(w, st(), M_PEND, f_pend(), s);
        launch_blk_mask(w, st(), M_CONVERT, f_conv(), s);
        build_list(f_run(), vl_run);
        build_list(f_pend(), vl_pend);
        build_list(f_conv(), vl_conv);
        return true;
    }

    void run() {
        if (o.eo) {  // Schur source and the full |b|^2 the tolerance refers to
            // streaming mapping over t; the finish reads that mapping's rows
            const Work wp = pl.work_stream(P64);
            if (clv) {  // sb_ = b_e - D_eo (C_o + a)^-1 b_o
                launch_clover_bo_inv(pl.work(P64, false), full.d_blocks.as<BlockDesc>(), b.f(), tmp64.f(), cl64, s);
                launch_eo_prep_clv(wp, full.d_blocks.as<BlockDesc>(), b.f(), tmp64.f(), sb_.f(),
                                   d_diag.as<double>(), part(), s);
            } else {
                launch_eo_prep(wp, full.d_blocks.as<BlockDesc>(), b.f(), sb_.f(), d_diag.as<double>(), part(), s);
            }
            launch_finish(F_BNORM, wp, st(), part(), nullptr, nullptr, s);
        }
        launch_init(o.P, pl.work(o.P, false), fb().f(), fx().f(), xlo.f(), fr().f(), r.f(), rk(), rc(), p.f(), part(),
                    s);
        launch_finish(F_INIT, pl.work(o.P, false), st(), part(), f_run(), nullptr, s);
        {
            const Work w = cur->work(o.P, false);
            launch_blk_mask(w, st(), M_PEND, f_pend(), s);  // all zero at start
            launch_blk_mask(w, st(), M_CONVERT, f_conv(), s);
        }
        build_list(f_run(), vl_run);
        // reduced precision: reliable updates inside every iteration; FP64:
        // the only FP64 check is at convergence, driven from the host.
        const bool in_loop = o.P != P64;
        const int k = std::max(1, o.check_every);
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        auto drop_graph = [&]() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
        };
        auto capture = [&]() {
            HC(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < k; ++i) iteration(in_loop);
            dslash_calls -= 2 * k;
            HC(hipStreamEndCapture(s, &graph));
            HC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        };
        const long long cap = (long long)o.max_iter * 4 + 64;  // host-side bound on chunks
        long long chunks = 0;
        try {
            if (o.use_graph) capture();
            while (true) {
                if (exec) {
                    HC(hipGraphLaunch(exec, s));
                    dslash_calls += 2 * k;
                } else {
                    for (int i = 0; i < k; ++i) iteration(in_loop);
                }
                HC(hipMemcpyAsync(st_host.data(), d_st.p, sizeof(SysState) * pl.nsys, hipMemcpyDeviceToHost, s));
                HC(hipStreamSynchronize(s));
                int n_run = 0, n_pend = 0;
                for (const auto& x : st_host) {
                    if (x.state == S_RUN) ++n_run;
                    else if (x.state == S_REL || x.state == S_CHK || x.state == S_BRK || x.state == S_MAXIT) ++n_pend;
                }
                if (n_pend > 0) reliable();
                if (n_pend == 0 && n_run == 0) break;
                // re-plan the stencil chunks once a good part of the blocks has finished
                int n_active_blk = 0;
                for (const BlockDesc& bd : cur->blocks) {
                    bool any = false;
                    for (int r = 0; r < pl.nr; ++r) any |= active_state(st_host[bd.sys0 + r].state);
                    n_active_blk += any;
                }
                if (cur->blocks.size() >= 4 && n_active_blk <= (int)(0.6 * cur->blocks.size())) {
                    if (n_pend > 0) {
                        HC(hipMemcpyAsync(st_host.data(), d_st.p, sizeof(SysState) * pl.nsys, hipMemcpyDeviceToHost, s));
                        HC(hipStreamSynchronize(s));
                    }
                    if (compact() && exec) {
                        drop_graph();
                        capture();
                    }
                }
                if (++chunks > cap) fail(FS_E_HIP, "solver driver did not terminate");
            }
        } catch (...) {
            drop_graph();
            throw;
        }
        drop_graph();
        if (o.eo && clv)
            launch_eo_post_clv(pl.work_stream(P64), full.d_blocks.as<BlockDesc>(), b.f(), sx_.f(), xhi.f(),
                               d_diag.as<double>(), cl64, s);
        else if (o.eo)
            launch_eo_post(pl.work_stream(P64), full.d_blocks.as<BlockDesc>(), b.f(), sx_.f(), xhi.f(),
                           d_diag.as<double>(), s);
        HC(hipMemcpyAsync(st_host.data(), d_st.p, sizeof(SysState) * pl.nsys, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
    }
};


// ============================================================== argument checks

void check_ctx(fs_ctx c, bool need_gauge = true) {
    if (!c) fail(FS_E_ARG, "null context");
    if (need_gauge && !c->has_gauge) fail(FS_E_STATE, "no gauge field uploaded");
}

void check_prec(int P) {
    if (P < 0 || P > 3) fail(FS_E_ARG, "invalid precision");
}

// The clover term is kept in FP64 and FP32 only.
void check_clover_prec(const fs_ctx_s* c, int P) {
    if (c->c_sw != 0.0 && P != P64 && P != P32) fail(FS_E_ARG, "the clover term needs FP64 or FP32 storage");
}

void check_eo(bool eo, const fs_ctx_s* c) {
    if (!eo) return;
    for (int i = 0; i < 4; ++i)
        if (c->dims[i] % 2) fail(FS_E_ARG, "even-odd preconditioning needs every extent even");
}

// Copy n bytes of a user buffer to a fresh device buffer.
DevBuf to_device(const void* src, size_t n, int is_device, hipStream_t s) {
    DevBuf d(n);
    HC(hipMemcpyAsync(d.p, src, n, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    return d;
}

void from_device(void* dst, const DevBuf& d, size_t n, int is_device, hipStream_t s) {
    HC(hipMemcpyAsync(dst, d.p, n, is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
}

// Untuned rhs block: 4 for FP64 and FP32 (FP32 at 8 ran at half the rate on
// the uneven 8^3x16 ... 24^3x48 batch, 147 against 314 solves/s), 8 for FP16
// and BF16 (FP16: 370 and 380 solves/s at 8 and 4).
int tuned_nr(fs_ctx c, int P, int n_sys) {
    auto it = c->tune.find(P);
    int nr = it != c->tune.end() ? it->second.nr : (P == P64 || P == P32 ? 4 : 8);
    while (nr > 1 && nr > n_sys) nr >>= 1;
    return nr;
}
int tuned_wg(fs_ctx c, int P) {
    auto it = c->tune.find(P);
    return it != c->tune.end() ? it->second.wg : 256;
}
int tuned_ilp(fs_ctx c, int P) {
    auto it = c->tune.find(P);
    return it != c->tune.end() ? it->second.ilp : 1;
}
int tuned_occ(fs_ctx c, int P) {
    auto it = c->tune.find(P);
    return it != c->tune.end() ? it->second.occ : 0;
}

// ============================================================== estimator

struct EstSys {
    int inst, level, sample;
    double sigma;
    bool is_x, g5;
};

struct EstResult {
    std::vector<double> stats;   // per instance [L+1][16][P+1][4]
    std::vector<double> samples; // per instance [L+1][N][16][P+1][2]
    std::vector<double> level_res;  // per instance [L+1] worst relative true residual
    std::vector<double> bound;   // per instance [L+1][N]: bound on |X_s - X_s^exact| / ||Gamma Omega_p||
    fs_est_report rep;
    bool noconv = false;
};

// Lower bound on the smallest singular value of D + sigma: D + sigma =
// (4 + m0 + sigma) - H with H = sum_mu H_mu, and H_mu psi = P_- U_mu Pi_mu psi
// + P_+ Pi_mu^-1 U_mu^+ psi with P_-+ = (1 -+ g_mu)/2 orthogonal projectors
// commuting with the colour and site maps, so ||H_mu psi||^2 <= u^2
// (||P_- psi||^2 + ||P_+ psi||^2) = u^2 ||psi||^2 for links of norm <= u.
// With the clover term, D + sigma = (4 + m0 + sigma) + C - H and ||C|| is at
// most the largest absolute row sum of its blocks (clv_norm).
double smin_lower(const fs_ctx_s* c, double m0, double sigma) {
    return 4.0 + m0 + sigma - 4.0 * c->link_norm - c->clv_norm;
}

// C of the context's links at its c_sw (FP64 and FP32 copies) and its norm bound.
void build_clover(fs_ctx_s* c) {
    static const SigmaTab tab = make_sigma_tab();
    const size_t vh = (size_t)c->V / 2;
    c->clv[P64].alloc((size_t)2 * 36 * vh * 16);
    c->clv[P32].alloc((size_t)2 * 18 * vh * 16);
    DevBuf nb(sizeof(unsigned long long));
    HC(hipMemsetAsync(nb.p, 0, sizeof(unsigned long long), c->stream));
    launch_clover_build(lat_desc(c, P64), c->c_sw, tab, c->clv[P64].as<uint4>(), c->clv[P32].as<uint4>(),
                        nb.as<unsigned long long>(), c->stream);
    HC(hipGetLastError());
    unsigned long long bits = 0;
    HC(hipMemcpyAsync(&bits, nb.p, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    HC(hipStreamSynchronize(c->stream));
    double nrm;
    std::memcpy(&nrm, &bits, sizeof(nrm));
    if (!std::isfinite(nrm)) fail(FS_E_ARG, "the clover term is not finite (links not finite?)");
    c->clv_norm = nrm;
}

// One batched pass over a set of (instance, level, sample) units.  For each
// unit level l < L: an x-system at sigma_{l+1} and a y-system at sigma_l on
// g5 z; level L: one x-system.  x- and y-blocks are paired rhs by rhs.
void run_units(const std::vector<fs_ctx_s*>& ctxs, const fs_est_params* prm, const std::vector<double>& sigma,
               const std::vector<std::array<int, 3>>& units, int nr, int wg, hipStream_t s, EstResult& res,
               int n_noise) {
    const bool want_bound = prm->report_fp64_error != 0;
    const int L = (int)sigma.size() - 1;
    const int P1 = prm->p_max + 1;
    // group units by (inst, level) into blocks of nr samples
    std::vector<int> blk_lat;
    std::vector<EstSys> sysv;  // per system slot
    std::vector<std::pair<int, int>> pairs;  // (x-block, y-block or -1)
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (auto& u : units) groups[{u[0], u[1]}].push_back(u[2]);
    for (auto& kv : groups) {
        const int inst = kv.first.first, l = kv.first.second;
        const auto& smp = kv.second;
        for (size_t c0 = 0; c0 < smp.size(); c0 += nr) {
            const int xb = (int)blk_lat.size();
            blk_lat.push_back(inst);
            for (int r = 0; r < nr; ++r) {
                EstSys e{inst, l, -1, l < L ? sigma[l + 1] : sigma[L], true, false};
                if (c0 + r < smp.size()) e.sample = smp[c0 + r];
                sysv.push_back(e);
            }
            int yb = -1;
            if (l < L) {
                yb = (int)blk_lat.size();
                blk_lat.push_back(inst);
                for (int r = 0; r < nr; ++r) {
                    EstSys e{inst, l, -1, sigma[l], false, true};
                    if (c0 + r < smp.size()) e.sample = smp[c0 + r];
                    sysv.push_back(e);
                }
            }
            pairs.push_back({xb, yb});
        }
    }
    const int Pst = prm->solve.storage;
    auto pl = make_plan(blk_lat, ctxs, nr, wg, s, tuned_ilp(ctxs[0], Pst), tuned_occ(ctxs[0], Pst));
    SolveOpts o;
    o.P = prm->solve.storage;
    o.tol = prm->solve.tol;
    o.max_iter = prm->solve.max_iter;
    o.delta = o.P == P64 ? 0.0 : (prm->solve.reliable_delta > 0 ? prm->solve.reliable_delta : default_delta(o.P));
    o.check_every = prm->solve.check_every > 0 ? prm->solve.check_every : 8;
    o.use_graph = prm->solve.use_graph != 0;
    o.eo = prm->solve.even_odd != 0;
    o.eo_var = eo_tuning(ctxs[0], o.P)[0];
    o.eo_occ = eo_tuning(ctxs[0], o.P)[1];
    BatchSolver bs(*pl, ctxs, s, o);
    const int nsys = pl->nsys;
    std::vector<double> diag(nsys);
    std::vector<char> idle(nsys);
    std::vector<NoiseKey> keys(nsys);
    for (int i = 0; i < nsys; ++i) {
        const EstSys& e = sysv[i];
        diag[i] = 4.0 + prm->solve.m0 + e.sigma;
        idle[i] = e.sample < 0;
        NoiseKey k;
        std::memset(&k, 0, sizeof(k));
        k.seed = prm->seed;
        k.instance = ctxs[e.inst]->instance;
        k.level = prm->shared_noise ? 0u : (uint32_t)e.level;  // shared: z_s of level 0 on every level
        k.sample = (uint64_t)std::max(0, e.sample);
        k.g5 = e.g5 ? 1 : 0;
        k.pad = e.sample < 0 ? 1 : 0;
        keys[i] = k;
    }
    bs.setup(diag, idle, keys);
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * nsys, 0, s);
    launch_noise_block(P64, pl->work(P64, false), bs.b.f(), d_keys.as<NoiseKey>(), s);
    bs.run();
    res.rep.dslash_calls += bs.dslash_calls;
    const int nblk = (int)blk_lat.size();

    // error bound of every sample: ||x~||^2 of every system from the spin
    // correlation of the solution with itself (p = 0, each block paired with
    // itself; the trace over spins is the squared norm), FP64 true residuals
    // from the solver states
    if (want_bound) {
        std::vector<int> ys(2 * nblk, 0);
        for (int b2 = 0; b2 < nblk; ++b2) ys[2 * b2] = b2;
        DevBuf d_ys = to_device(ys.data(), sizeof(int) * 2 * nblk, 0, s);
        const Work wn = pl->work(P64, false);
        DevBuf d_N(sizeof(double) * (size_t)nsys * 32);
        launch_hop_reduce(wn, 0, Fld(), bs.xhi.f(), bs.xhi.f(), Fld(), d_ys.as<int>(), bs.part(), s);
        launch_hop_finish(wn, bs.part(), d_N.as<double>(), 1, 0, s);
        std::vector<double> hN((size_t)nsys * 32);
        HC(hipMemcpyAsync(hN.data(), d_N.p, sizeof(double) * hN.size(), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        auto norm = [&](int sys) {
            const double* m = &hN[(size_t)sys * 32];
            return std::sqrt(std::max(0.0, m[0] + m[10] + m[20] + m[30]));  // sum_a M_aa
        };
        auto err = [&](int sys, int inst, double sg) {
            const double lo = smin_lower(ctxs[inst], prm->solve.m0, sg);
            const double r = std::sqrt(std::max(0.0, bs.st_host[sys].rr_true));
            return lo > 0.0 ? r / lo : std::numeric_limits<double>::infinity();
        };
        for (auto& pr : pairs)
            for (int r = 0; r < nr; ++r) {
                const int sx = pr.first * nr + r;
                const EstSys& e = sysv[sx];
                if (e.sample < 0) continue;
                const double ex = err(sx, e.inst, e.sigma);
                double bnd;
                if (pr.second < 0) {  // last level: y = z exactly
                    const SysState& S = bs.st_host[sx];
                    bnd = std::sqrt(S.bnorm2 > 0.0 ? S.bnorm2 : S.bb) * ex;
                } else {
                    const int sy = pr.second * nr + r;
                    const double ey = err(sy, e.inst, sigma[e.level]);
                    const double c = std::fabs(sigma[e.level + 1] - sigma[e.level]);
                    bnd = c * (norm(sy) * ex + ey * (norm(sx) + ex));
                }
                res.bound[((size_t)e.inst * (L + 1) + e.level) * n_noise + e.sample] = bnd;
            }
    }

    // bilinears: hop launches over x-blocks only (y-blocks get no workgroups)
    std::vector<int> yb(2 * nblk, -1), hop_start(nblk + 1, 0);
    std::vector<char> is_x(nblk, 0);
    for (auto& pr : pairs) {
        is_x[pr.first] = 1;
        yb[2 * pr.first] = pr.second;
        yb[2 * pr.first + 1] = pr.second >= 0 ? 1 : 0;
    }
    for (int b = 0; b < nblk; ++b)
        hop_start[b + 1] = hop_start[b] + (is_x[b] ? pl->wg_start[b + 1] - pl->wg_start[b] : 0);
    DevBuf d_hop_start = to_device(hop_start.data(), sizeof(int) * (nblk + 1), 0, s);
    DevBuf d_yb = to_device(yb.data(), sizeof(int) * 2 * nblk, 0, s);
    Work wh = pl->work(P64, false);
    wh.wg_start = d_hop_start.as<int>();
    wh.total_wg = hop_start.back();
    DevBuf d_M(sizeof(double) * (size_t)nsys * P1 * 32);
    Field phi1;
    phi1.alloc(P64, pl->total_slots);
    // ping-pong: p=0 reads xhi; then phi in rhi / phi1
    Fld cur = bs.xhi.f();
    for (int p = 0; p <= prm->p_max; ++p) {
        Fld out = (p % 2 == 1) ? bs.rhi.f() : phi1.f();
        launch_hop_reduce(wh, p, out, cur, bs.xhi.f(), bs.b.f(), d_yb.as<int>(), bs.part(), s);
        launch_hop_finish(wh, bs.part(), d_M.as<double>(), P1, p, s);
        if (p > 0) cur = out;
    }
    // contraction into the per-sample estimates
    std::vector<XMap> xm(nsys);
    for (int i = 0; i < nsys; ++i) {
        const EstSys& e = sysv[i];
        XMap m;
        std::memset(&m, 0, sizeof(m));
        m.level = (e.is_x && e.sample >= 0) ? e.level : -1;
        m.sample = std::max(0, e.sample);
        m.g5 = e.level < L ? 1 : 0;
        m.coef = e.level < L ? sigma[e.level + 1] - sigma[e.level] : 1.0;
        xm[i] = m;
    }
    // one X array per instance: contract per instance with masked maps
    static const GammaTab gt = make_gamma_tab();
    const size_t xsz = (size_t)(L + 1) * n_noise * 16 * P1 * 2;
    for (size_t inst = 0; inst < ctxs.size(); ++inst) {
        std::vector<XMap> xi = xm;
        bool any = false;
        for (int i = 0; i < nsys; ++i) {
            if (sysv[i].inst != (int)inst) xi[i].level = -1;
            any |= xi[i].level >= 0;
        }
        if (!any) continue;
        DevBuf d_xm = to_device(xi.data(), sizeof(XMap) * nsys, 0, s);
        DevBuf d_X(sizeof(double) * xsz);
        HC(hipMemcpyAsync(d_X.p, res.samples.data() + inst * xsz, sizeof(double) * xsz, hipMemcpyHostToDevice, s));
        launch_gamma_contract(d_M.as<double>(), P1, nsys, d_xm.as<XMap>(), gt, d_X.as<double>(), n_noise, s);
        HC(hipMemcpyAsync(res.samples.data() + inst * xsz, d_X.p, sizeof(double) * xsz, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
    }
    for (int i = 0; i < nsys; ++i) {
        const EstSys& e = sysv[i];
        const SysState& S = bs.st_host[i];
        if (e.sample < 0) continue;
        res.rep.systems += 1;
        res.rep.iterations += S.iters;
        res.rep.reliable_updates += S.n_rel;
        const double rel = true_rel(S);
        double& lr = res.level_res[(size_t)e.inst * (L + 1) + e.level];
        lr = std::max(lr, rel);
        res.rep.max_rel_residual = std::max(res.rep.max_rel_residual, rel);
        if (S.state != S_DONE) res.noconv = true;
    }
}

// FS estimate with probing and full spin-colour dilution (paper Background,
// Probing; Sec. 3.1 and 3.4).  Each sample s of level l uses D = 12 c sources:
// the Z4 vector of key (seed, instance, l, s) restricted to one probing colour
// j and one spin-colour component a.  A spin-diluted source is a g5
// eigenvector (g5 z = s_a z), so y_l = (D + sigma_l)^-dagger z = s_a g5 x' with
// x' = (D + sigma_l)^-1 z: level l < L solves each source at sigma_l and
// sigma_{l+1}, level L at sigma_L.  Systems are grouped per (level, role), the
// D sources of a sample consecutive, so an x-block and its y-block hold the
// same sources.  The shadow residual of every system is the undiluted Z4
// vector of its key, whose inner product with the source is the source's norm.
// Per-system estimates are summed over the D sources in a fixed order.
void probed_impl(fs_ctx_s* c, const fs_est_params* prm, const double* sigma_in, int L, const int32_t* colours,
                 int n_col, fs_level_stat* out, double* samples_out, fs_est_report* report) {
    if (!prm || !sigma_in || !out || !colours) fail(FS_E_ARG, "null argument");
    if (L < 0) fail(FS_E_ARG, "L must be >= 0");
    if (prm->hpe_order != 0) fail(FS_E_ARG, "hpe_order applies to fs_sample_variances only");
    if (prm->solve.multi_shift != 0) fail(FS_E_ARG, "multi_shift applies to fs_solve_shifted only");
    if (prm->n_noise < 1) fail(FS_E_ARG, "n_noise must be >= 1");
    if (prm->p_max < 0 || prm->p_max >= c->dims[2]) fail(FS_E_ARG, "p_max must be in [0, Lz)");
    check_prec(prm->solve.storage);
    check_eo(prm->solve.even_odd != 0, c);
    if (!(prm->solve.tol > 0)) fail(FS_E_ARG, "tol must be > 0");
    if (prm->solve.max_iter < 1) fail(FS_E_ARG, "max_iter must be >= 1");
    if (prm->solve.rhs_block != 0 && !pow2_ok(prm->solve.rhs_block)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
    if (n_col < 1 || n_col > 4096) fail(FS_E_ARG, "n_colours must be in 1..4096");
    std::vector<double> sigma(sigma_in, sigma_in + L + 1);
    if (sigma[0] != 0.0) fail(FS_E_ARG, "sigma[0] must be 0");
    for (int l = 0; l < L; ++l)
        if (!(sigma[l + 1] > sigma[l])) fail(FS_E_ARG, "sigma must be strictly increasing");
    const long long V = (long long)c->dims[0] * c->dims[1] * c->dims[2] * c->dims[3];
    std::vector<uint16_t> col16(V);
    std::vector<char> seen(n_col, 0);
    for (long long i = 0; i < V; ++i) {
        if (colours[i] < 0 || colours[i] >= n_col) fail(FS_E_ARG, "colour out of range");
        col16[i] = (uint16_t)colours[i];
        seen[colours[i]] = 1;
    }
    for (int j = 0; j < n_col; ++j)
        if (!seen[j]) fail(FS_E_ARG, "every colour must hold at least one site");
    auto t0 = std::chrono::steady_clock::now();
    DeviceScope ds(c->device);
    hipStream_t s = c->stream;
    const int N = prm->n_noise, P1 = prm->p_max + 1, P = prm->solve.storage, D = 12 * n_col;
    const long long per_group = (long long)N * D;
    const int nr = prm->solve.rhs_block ? prm->solve.rhs_block : tuned_nr(c, P, (int)std::min<long long>(per_group, 1 << 20));
    const int nbg = (int)((per_group + nr - 1) / nr);  // blocks per (level, role) group
    // groups: level l: x (shift sigma_{l+1}, or sigma_L on the last level), then y (sigma_l) for l < L
    std::vector<int> gx(L + 1), gy(L + 1, -1);
    int ngroups = 0;
    for (int l = 0; l <= L; ++l) {
        gx[l] = ngroups++;
        if (l < L) gy[l] = ngroups++;
    }
    const long long nblk_ll = (long long)ngroups * nbg;
    if (nblk_ll * nr > (1ll << 24)) fail(FS_E_ARG, "too many diluted systems for one batch");
    const int nblk = (int)nblk_ll;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, P), s, tuned_ilp(c, P), tuned_occ(c, P));
    const int nsys = pl->nsys;
    std::vector<double> diag(nsys);
    std::vector<char> idle(nsys);
    std::vector<NoiseKey> keys(nsys), rkeys(nsys);
    std::vector<XMap> xm(nsys);
    std::vector<int> sys_level(nsys, -1);
    for (int l = 0; l <= L; ++l)
        for (int role = 0; role < 2; ++role) {
            const int g = role == 0 ? gx[l] : gy[l];
            if (g < 0) continue;
            const double shift = role == 0 ? sigma[l < L ? l + 1 : L] : sigma[l];
            for (long long q = 0; q < (long long)nbg * nr; ++q) {
                const int sys = (int)((long long)g * nbg * nr + q);
                const bool real = q < per_group;
                const int smp = real ? (int)(q / D) : 0, d = real ? (int)(q % D) : 0;
                diag[sys] = 4.0 + prm->solve.m0 + shift;
                idle[sys] = !real;
                NoiseKey k;
                std::memset(&k, 0, sizeof(k));
                k.seed = prm->seed;
                k.instance = c->instance;
                k.level = (uint32_t)l;
                k.sample = (uint64_t)smp;
                k.pad = real ? 0 : 1;
                rkeys[sys] = k;  // shadow residual: the undiluted Z4 vector
                k.dil = 1 + d;
                keys[sys] = k;
                XMap mp;
                std::memset(&mp, 0, sizeof(mp));
                mp.level = -1;
                if (role == 0 && real) {
                    const int a = d % 12;
                    const double sa = (a / 3) < 2 ? 1.0 : -1.0;  // g5 eigenvalue of the source's spin
                    mp.level = sys;  // one slot per system; summed over the D sources below
                    mp.sample = 0;
                    mp.g5 = l < L ? 1 : 0;
                    mp.coef = l < L ? (sigma[l + 1] - sigma[l]) * sa : 1.0;
                    sys_level[sys] = l;
                }
                xm[sys] = mp;
            }
        }
    SolveOpts o;
    o.P = P;
    o.tol = prm->solve.tol;
    o.max_iter = prm->solve.max_iter;
    o.delta = P == P64 ? 0.0 : (prm->solve.reliable_delta > 0 ? prm->solve.reliable_delta : default_delta(P));
    o.check_every = prm->solve.check_every > 0 ? prm->solve.check_every : 8;
    o.use_graph = prm->solve.use_graph != 0;
    o.eo = prm->solve.even_odd != 0;
    o.eo_var = eo_tuning(c, o.P)[0];
    o.eo_occ = eo_tuning(c, o.P)[1];
    BatchSolver bs(*pl, lats, s, o);
    bs.setup(diag, idle, rkeys);
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * nsys, 0, s);
    DevBuf d_col = to_device(col16.data(), sizeof(uint16_t) * V, 0, s);
    launch_noise_block(P64, pl->work(P64, false), bs.b.f(), d_keys.as<NoiseKey>(), s, d_col.as<uint16_t>());
    bs.run();

    // bilinears: x-blocks only, paired with the y-block of the same sources (or their own source on level L)
    static const GammaTab gt = make_gamma_tab();
    std::vector<int> yb(2 * nblk, -1), hop_start(nblk + 1, 0);
    for (int l = 0; l <= L; ++l)
        for (int b = 0; b < nbg; ++b) {
            const int xb = gx[l] * nbg + b;
            if (l < L) {
                yb[2 * xb] = gy[l] * nbg + b;
                yb[2 * xb + 1] = 1;
            }
        }
    std::vector<char> is_x_group(ngroups, 0);
    for (int l = 0; l <= L; ++l) is_x_group[gx[l]] = 1;
    for (int b = 0; b < nblk; ++b)
        hop_start[b + 1] = hop_start[b] + (is_x_group[b / nbg] ? pl->wg_start[b + 1] - pl->wg_start[b] : 0);
    DevBuf d_hop_start = to_device(hop_start.data(), sizeof(int) * (nblk + 1), 0, s);
    DevBuf d_yb = to_device(yb.data(), sizeof(int) * 2 * nblk, 0, s);
    DevBuf d_xm = to_device(xm.data(), sizeof(XMap) * nsys, 0, s);
    Work wh = pl->work(P64, false);
    wh.wg_start = d_hop_start.as<int>();
    wh.total_wg = hop_start.back();
    DevBuf d_M(sizeof(double) * (size_t)nsys * P1 * 32);
    Field phi1;
    phi1.alloc(P64, pl->total_slots);
    Fld cur = bs.xhi.f();
    for (int p = 0; p <= prm->p_max; ++p) {
        Fld outf = (p % 2 == 1) ? bs.rhi.f() : phi1.f();
        launch_hop_reduce(wh, p, outf, cur, bs.xhi.f(), bs.b.f(), d_yb.as<int>(), bs.part(), s);
        launch_hop_finish(wh, bs.part(), d_M.as<double>(), P1, p, s);
        if (p > 0) cur = outf;
    }
    DevBuf d_Y(sizeof(double) * 2 * (size_t)nsys * 16 * P1);
    launch_gamma_contract(d_M.as<double>(), P1, nsys, d_xm.as<XMap>(), gt, d_Y.as<double>(), 1, s);
    std::vector<int> g0((size_t)(L + 1) * N);
    for (int l = 0; l <= L; ++l)
        for (int smp = 0; smp < N; ++smp) g0[(size_t)l * N + smp] = gx[l] * nbg * nr + smp * D;
    DevBuf d_g0 = to_device(g0.data(), sizeof(int) * g0.size(), 0, s);
    const size_t xsz = (size_t)(L + 1) * N * 16 * P1 * 2;
    DevBuf d_X(sizeof(double) * xsz);
    launch_dilution_sum(d_Y.as<double>(), P1, d_g0.as<int>(), (L + 1) * N, D, d_X.as<double>(), s);
    DevBuf d_st(sizeof(double) * (size_t)(L + 1) * 16 * P1 * 4);
    launch_level_stats(d_X.as<double>(), L + 1, N, P1, d_st.as<double>(), s);
    std::vector<double> stv((size_t)(L + 1) * 16 * P1 * 4), X(xsz);
    HC(hipMemcpyAsync(stv.data(), d_st.p, sizeof(double) * stv.size(), hipMemcpyDeviceToHost, s));
    HC(hipMemcpyAsync(X.data(), d_X.p, sizeof(double) * xsz, hipMemcpyDeviceToHost, s));
    HC(hipGetLastError());
    HC(hipStreamSynchronize(s));

    fs_est_report rep;
    std::memset(&rep, 0, sizeof(rep));
    std::vector<double> level_res(L + 1, 0.0);
    bool noconv = false;
    for (int l = 0; l <= L; ++l)
        for (int role = 0; role < 2; ++role) {
            const int g = role == 0 ? gx[l] : gy[l];
            if (g < 0) continue;
            for (long long q = 0; q < per_group; ++q) {
                const SysState& S = bs.st_host[(size_t)g * nbg * nr + q];
                rep.systems += 1;
                rep.iterations += S.iters;
                rep.reliable_updates += S.n_rel;
                const double rel = true_rel(S);
                level_res[l] = std::max(level_res[l], rel);
                rep.max_rel_residual = std::max(rep.max_rel_residual, rel);
                if (S.state != S_DONE) noconv = true;
            }
        }
    rep.dslash_calls = bs.dslash_calls;
    const uint16_t mask = prm->gamma_mask ? prm->gamma_mask : 0xffff;
    for (int l = 0; l <= L; ++l)
        for (int n = 0; n < 16; ++n)
            for (int p = 0; p < P1; ++p) {
                fs_level_stat& ostat = out[((size_t)l * 16 + n) * P1 + p];
                std::memset(&ostat, 0, sizeof(ostat));
                if (!((mask >> n) & 1)) continue;
                const double* d = &stv[(((size_t)l * 16 + n) * P1 + p) * 4];
                ostat.tr_re = d[0];
                ostat.tr_im = d[1];
                ostat.var_paper = d[2];
                ostat.var_unbiased = d[3];
                ostat.n = N;
                ostat.max_rel_residual = level_res[l];
            }
    if (samples_out) std::memcpy(samples_out, X.data(), sizeof(double) * xsz);
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    if (noconv) throw FsError(FS_E_NOCONV, "a shifted solve did not reach tol (outputs are filled)");
}

// Variance sampling (paper Sec. 3.1, "Sampling the Variance").  One Z4
// vector per sample, shared by every sampling shift (noise level field
// kSamplingLevel); per shift s_i an x-system on z and a y-system on g5 z,
// solved in one batch.  The hop/bilinear chain then runs once per pairing:
// pass 0 pairs each x-block with its own source (V_L(s_i)), pass q >= 1 pairs
// the x-blocks of s_j, j >= q-1, with the y-blocks of s_{q-1} holding the same
// samples (Vbar_l(s_{q-1}, s_j)).  Slot order: singles i, then pairs (i, j).
constexpr uint32_t kSamplingLevel = 0xFFFFFFFFu;

void sampling_multishift(fs_ctx_s* c, const fs_solve_params* prm, const std::vector<double>& sh, int nch, int nr,
                         BatchSolver& bs, const std::vector<NoiseKey>& keys);

void sampling_impl(fs_ctx_s* c, const fs_est_params* prm, const double* sh_in, int m, fs_level_stat* single,
                   fs_level_stat* pair, double* samples_out, double* iters_out, fs_est_report* report) {
    if (!prm || !sh_in || !single || !pair) fail(FS_E_ARG, "null argument");
    if (m < 1 || m > 16) fail(FS_E_ARG, "m must be in 1..16");
    if (prm->n_noise < 2) fail(FS_E_ARG, "n_noise must be >= 2");
    if (prm->p_max < 0 || prm->p_max >= c->dims[2]) fail(FS_E_ARG, "p_max must be in [0, Lz)");
    check_prec(prm->solve.storage);
    check_eo(prm->solve.even_odd != 0, c);
    if (!(prm->solve.tol > 0)) fail(FS_E_ARG, "tol must be > 0");
    if (prm->solve.max_iter < 1) fail(FS_E_ARG, "max_iter must be >= 1");
    if (prm->solve.rhs_block != 0 && !pow2_ok(prm->solve.rhs_block)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
    if (prm->hpe_order < 0 || prm->hpe_order > 16) fail(FS_E_ARG, "hpe_order must be in 0..16");
    if (prm->solve.multi_shift) {
        if (prm->solve.storage != P64) fail(FS_E_ARG, "multi-shift solves run in FP64 storage");
        if (prm->solve.even_odd) fail(FS_E_ARG, "multi-shift solves need even_odd = 0");
        if (c->c_sw != 0.0) fail(FS_E_ARG, "multi-shift solves use the plain operator (no clover term)");
    }
    std::vector<double> sh(sh_in, sh_in + m);
    if (sh[0] != 0.0) fail(FS_E_ARG, "shifts[0] must be 0");
    for (int i = 0; i + 1 < m; ++i)
        if (!(sh[i + 1] > sh[i])) fail(FS_E_ARG, "shifts must be strictly increasing");
    auto t0 = std::chrono::steady_clock::now();
    DeviceScope ds(c->device);
    hipStream_t s = c->stream;
    const int N = prm->n_noise, P1 = prm->p_max + 1, P = prm->solve.storage;
    const int nr = prm->solve.rhs_block ? prm->solve.rhs_block : tuned_nr(c, P, N);
    const int nch = (N + nr - 1) / nr;
    const int nslot = m + m * (m + 1) / 2;
    auto slot_pair = [&](int i, int j) { return m + i * m - i * (i - 1) / 2 + (j - i); };
    // blocks: x(i, ch) = 2 (i nch + ch), y(i, ch) = x + 1
    const int nblk = 2 * m * nch;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, P), s, tuned_ilp(c, P), tuned_occ(c, P));
    const int nsys = pl->nsys;
    std::vector<double> diag(nsys);
    std::vector<char> idle(nsys);
    std::vector<NoiseKey> keys(nsys);
    std::vector<int> smp(nsys);
    for (int b = 0; b < nblk; ++b) {
        const int i = (b / 2) / nch, ch = (b / 2) % nch;
        const bool is_y = b & 1;
        for (int r = 0; r < nr; ++r) {
            const int sys = b * nr + r;
            const int k = ch * nr + r;
            smp[sys] = k < N ? k : -1;
            diag[sys] = 4.0 + prm->solve.m0 + sh[i];
            idle[sys] = k >= N;
            NoiseKey key;
            std::memset(&key, 0, sizeof(key));
            key.seed = prm->seed;
            key.instance = c->instance;
            key.level = kSamplingLevel;
            key.sample = (uint64_t)(k < N ? k : 0);
            key.g5 = is_y ? 1 : 0;
            key.pad = k < N ? 0 : 1;
            keys[sys] = key;
        }
    }
    SolveOpts o;
    o.P = P;
    o.tol = prm->solve.tol;
    o.max_iter = prm->solve.max_iter;
    o.delta = P == P64 ? 0.0 : (prm->solve.reliable_delta > 0 ? prm->solve.reliable_delta : default_delta(P));
    o.check_every = prm->solve.check_every > 0 ? prm->solve.check_every : 8;
    o.use_graph = prm->solve.use_graph != 0;
    o.eo = prm->solve.even_odd != 0;
    o.eo_var = eo_tuning(c, o.P)[0];
    o.eo_occ = eo_tuning(c, o.P)[1];
    BatchSolver bs(*pl, lats, s, o);
    bs.setup(diag, idle, keys);
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * nsys, 0, s);
    launch_noise_block(P64, pl->work(P64, false), bs.b.f(), d_keys.as<NoiseKey>(), s);
    if (prm->solve.multi_shift) sampling_multishift(c, &prm->solve, sh, nch, nr, bs, keys);
    else bs.run();

    // bilinears, one pass per pairing
    static const GammaTab gt = make_gamma_tab();
    const size_t xsz = (size_t)nslot * N * 16 * P1 * 2;
    std::vector<double> X(xsz, 0.0);
    DevBuf d_X = to_device(X.data(), sizeof(double) * xsz, 0, s);
    DevBuf d_M(sizeof(double) * (size_t)nsys * P1 * 32);
    Field phi1;
    phi1.alloc(P64, pl->total_slots);
    // hopping parameter expansion of the singles: w = (H/a)^k x for the x-blocks
    // of shifts with m0 + s > 0 (x elsewhere), H = a - (D + s): k rounds of the
    // stencil with a zero diagonal (giving -H w) and a scale by -1/a
    Field whpe;
    {
        std::vector<BlockDesc> eb;
        for (int b = 0; b < nblk; b += 2)
            if (prm->hpe_order > 0 && prm->solve.m0 + sh[(b / 2) / nch] > 0.0) eb.push_back(pl->blocks[b]);
        if (!eb.empty()) {
            whpe.alloc(P64, pl->total_slots);
            HC(hipMemcpyAsync(whpe.v.p, bs.xhi.v.p, whpe.v.n < bs.xhi.v.n ? whpe.v.n : bs.xhi.v.n,
                              hipMemcpyDeviceToDevice, s));
            auto sp = plan_from_blocks(eb, lats, nr, pl->wg, s, pl->ilp, pl->occ, 0);
            std::vector<double> zero(nsys, 0.0), coef(nsys);
            for (int i = 0; i < nsys; ++i) coef[i] = -1.0 / diag[i];
            DevBuf d_zero = to_device(zero.data(), sizeof(double) * nsys, 0, s);
            DevBuf d_coef = to_device(coef.data(), sizeof(double) * nsys, 0, s);
            // with the clover term the factor is A^-1 = (C + a)^-1 at every site (the
            // generalized expansion): inverse blocks of both parities per eligible shift
            DevBuf d_inv, d_off;
            Clv cfull;
            if (c->c_sw != 0.0) {
                const int vh = c->V / 2;
                std::vector<long long> off(nsys, 0);
                std::map<double, long long> fld;
                for (const BlockDesc& bd : eb)
                    for (int r = 0; r < nr; ++r) {
                        const int sys = bd.sys0 + r;
                        auto it = fld.find(diag[sys]);
                        if (it == fld.end()) it = fld.emplace(diag[sys], (long long)fld.size() * 72 * vh).first;
                        off[sys] = it->second;
                    }
                d_inv.alloc((size_t)fld.size() * 72 * vh * 16);
                DevBuf bad(sizeof(int));
                HC(hipMemsetAsync(bad.p, 0, sizeof(int), s));
                for (const auto& kv : fld)
                    for (int par = 0; par < 2; ++par)
                        launch_clover_invert(c->clv[P64].as<uint4>() + (size_t)par * 36 * vh, vh, kv.first,
                                             d_inv.as<uint4>() + kv.second + (size_t)par * 36 * vh, nullptr,
                                             bad.as<int>(), s);
                int h_bad = 0;
                HC(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
                HC(hipStreamSynchronize(s));
                if (h_bad) fail(FS_E_ARG, "C + 4 + m0 + s is singular at a site");
                d_off = to_device(off.data(), sizeof(long long) * nsys, 0, s);
                cfull.inv = d_inv.as<uint4>();
                cfull.off = d_off.as<long long>();
            }
            for (int it = 0; it < prm->hpe_order; ++it) {
                launch_dslash(P64, D_PLAIN, sp->work(P64, false, true), phi1.f(), whpe.f(), Fld(),
                              d_zero.as<double>(), nullptr, M_ALL, nullptr, s);
                if (c->c_sw != 0.0) launch_clover_inv_full(sp->work(P64, false), whpe.f(), phi1.f(), cfull, s);
                else launch_scale_sys(sp->work(P64, false), whpe.f(), phi1.f(), d_coef.as<double>(), s);
            }
            HC(hipGetLastError());
            HC(hipStreamSynchronize(s));  // the tables die with this scope
        }
    }
    for (int q = 0; q <= m; ++q) {
        const int iy = q - 1;
        std::vector<int> yb(2 * nblk, -1), hop_start(nblk + 1, 0);
        std::vector<XMap> xm(nsys);
        for (int b = 0; b < nblk; ++b) {
            const int j = (b / 2) / nch, ch = (b / 2) % nch;
            const bool part_of = !(b & 1) && (q == 0 || j >= iy);
            if (part_of && q > 0) {
                yb[2 * b] = 2 * (iy * nch + ch) + 1;
                yb[2 * b + 1] = 1;
            }
            hop_start[b + 1] = hop_start[b] + (part_of ? pl->wg_start[b + 1] - pl->wg_start[b] : 0);
            for (int r = 0; r < nr; ++r) {
                const int sys = b * nr + r;
                XMap mp;
                std::memset(&mp, 0, sizeof(mp));
                mp.level = (part_of && smp[sys] >= 0) ? (q == 0 ? j : slot_pair(iy, j)) : -1;
                mp.sample = std::max(0, smp[sys]);
                mp.g5 = q > 0 ? 1 : 0;
                mp.coef = 1.0;
                xm[sys] = mp;
            }
        }
        DevBuf d_hop_start = to_device(hop_start.data(), sizeof(int) * (nblk + 1), 0, s);
        DevBuf d_yb = to_device(yb.data(), sizeof(int) * 2 * nblk, 0, s);
        DevBuf d_xm = to_device(xm.data(), sizeof(XMap) * nsys, 0, s);
        Work wh = pl->work(P64, false);
        wh.wg_start = d_hop_start.as<int>();
        wh.total_wg = hop_start.back();
        Fld cur = (q == 0 && whpe.v.p) ? whpe.f() : bs.xhi.f();
        for (int p = 0; p <= prm->p_max; ++p) {
            Fld outf = (p % 2 == 1) ? bs.rhi.f() : phi1.f();
            launch_hop_reduce(wh, p, outf, cur, bs.xhi.f(), bs.b.f(), d_yb.as<int>(), bs.part(), s);
            launch_hop_finish(wh, bs.part(), d_M.as<double>(), P1, p, s);
            if (p > 0) cur = outf;
        }
        launch_gamma_contract(d_M.as<double>(), P1, nsys, d_xm.as<XMap>(), gt, d_X.as<double>(), N, s);
        HC(hipStreamSynchronize(s));  // the host tables above die with this scope
    }
    // statistics per slot
    DevBuf d_st(sizeof(double) * (size_t)nslot * 16 * P1 * 4);
    launch_level_stats(d_X.as<double>(), nslot, N, P1, d_st.as<double>(), s);
    std::vector<double> stv((size_t)nslot * 16 * P1 * 4);
    HC(hipMemcpyAsync(stv.data(), d_st.p, sizeof(double) * stv.size(), hipMemcpyDeviceToHost, s));
    HC(hipMemcpyAsync(X.data(), d_X.p, sizeof(double) * xsz, hipMemcpyDeviceToHost, s));
    HC(hipGetLastError());
    HC(hipStreamSynchronize(s));
    fs_est_report rep;
    std::memset(&rep, 0, sizeof(rep));
    bool noconv = false;
    std::vector<double> it_sum(m, 0.0);
    for (int i = 0; i < nsys; ++i) {
        if (smp[i] < 0) continue;
        const SysState& S = bs.st_host[i];
        it_sum[(i / nr / 2) / nch] += S.iters;
        rep.systems += 1;
        rep.iterations += S.iters;
        rep.reliable_updates += S.n_rel;
        const double rel = true_rel(S);
        rep.max_rel_residual = std::max(rep.max_rel_residual, rel);
        if (S.state != S_DONE) noconv = true;
    }
    rep.dslash_calls = bs.dslash_calls;
    const uint16_t mask = prm->gamma_mask ? prm->gamma_mask : 0xffff;
    auto fill = [&](fs_level_stat& ostat, int slot, int n, int p) {
        std::memset(&ostat, 0, sizeof(ostat));
        if (slot < 0 || !((mask >> n) & 1)) return;
        const double* d = &stv[(((size_t)slot * 16 + n) * P1 + p) * 4];
        ostat.tr_re = d[0];
        ostat.tr_im = d[1];
        ostat.var_paper = d[2];
        ostat.var_unbiased = d[3];
        ostat.n = N;
        ostat.max_rel_residual = rep.max_rel_residual;
    };
    for (int i = 0; i < m; ++i)
        for (int n = 0; n < 16; ++n)
            for (int p = 0; p < P1; ++p) {
                fill(single[((size_t)i * 16 + n) * P1 + p], i, n, p);
                for (int j = 0; j < m; ++j)
                    fill(pair[(((size_t)i * m + j) * 16 + n) * P1 + p], j >= i ? slot_pair(i, j) : -1, n, p);
            }
    if (samples_out) std::memcpy(samples_out, X.data(), sizeof(double) * xsz);
    if (iters_out)
        for (int i = 0; i < m; ++i) iters_out[i] = it_sum[i] / (2.0 * N);
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    if (noconv) throw FsError(FS_E_NOCONV, "a shifted solve did not reach tol (outputs are filled)");
}

void estimate_impl(const std::vector<fs_ctx_s*>& ctxs, const fs_est_params* prm, const double* sigma_in, int L,
                   fs_level_stat* out, double* samples_out, fs_est_report* report) {
    if (!prm || !sigma_in || !out) fail(FS_E_ARG, "null argument");
    if (L < 0) fail(FS_E_ARG, "L must be >= 0");
    if (prm->p_max < 0) fail(FS_E_ARG, "p_max must be >= 0");
    if (prm->hpe_order != 0) fail(FS_E_ARG, "hpe_order applies to fs_sample_variances only");
    if (prm->solve.multi_shift != 0) fail(FS_E_ARG, "multi_shift applies to fs_solve_shifted only");
    // samples per level: n_level[l], or n_noise for every level
    std::vector<int> Nl(L + 1);
    for (int l = 0; l <= L; ++l) {
        const int n = prm->n_level ? prm->n_level[l] : prm->n_noise;
        if (n < 1 || n > (1 << 24)) fail(FS_E_ARG, prm->n_level ? "n_level[l] must be in 1..2^24" : "n_noise must be >= 1");
        Nl[l] = n;
    }
    check_prec(prm->solve.storage);
    if (!(prm->solve.tol > 0)) fail(FS_E_ARG, "tol must be > 0");
    if (prm->solve.max_iter < 1) fail(FS_E_ARG, "max_iter must be >= 1");
    std::vector<double> sigma(sigma_in, sigma_in + L + 1);
    if (sigma[0] != 0.0) fail(FS_E_ARG, "sigma[0] must be 0");
    for (int l = 0; l < L; ++l)
        if (!(sigma[l + 1] > sigma[l])) fail(FS_E_ARG, "sigma must be strictly increasing");
    for (auto* c : ctxs) {
        check_ctx(c);
        if (prm->p_max >= c->dims[2]) fail(FS_E_ARG, "p_max must be < Lz");
        check_eo(prm->solve.even_odd != 0, c);
        if (c->device != ctxs[0]->device) fail(FS_E_ARG, "batch contexts must share a device");
    }
    if (prm->solve.rhs_block != 0 && !pow2_ok(prm->solve.rhs_block)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
    auto t0 = std::chrono::steady_clock::now();
    fs_ctx_s* c0 = ctxs[0];
    DeviceScope ds(c0->device);
    hipStream_t s = c0->stream;
    const int N = *std::max_element(Nl.begin(), Nl.end());  // sample slots per level
    const int P1 = prm->p_max + 1;
    const bool report_err = prm->report_fp64_error != 0;
    EstResult res;
    std::memset(&res.rep, 0, sizeof(res.rep));
    const size_t xsz = (size_t)(L + 1) * N * 16 * P1 * 2;
    res.samples.assign(xsz * ctxs.size(), 0.0);
    res.level_res.assign((size_t)(L + 1) * ctxs.size(), 0.0);
    if (report_err) res.bound.assign((size_t)(L + 1) * N * ctxs.size(), 0.0);
    const int P = prm->solve.storage;
    if (!prm->solve.batched) {
        // plain path: one system at a time, NR = 1
        for (size_t i = 0; i < ctxs.size(); ++i)
            for (int l = 0; l <= L; ++l)
                for (int smp = 0; smp < Nl[l]; ++smp) {
                    std::vector<fs_ctx_s*> one{ctxs[i]};
                    EstResult r1;
                    std::memset(&r1.rep, 0, sizeof(r1.rep));
                    r1.samples.assign(xsz, 0.0);
                    r1.level_res.assign(L + 1, 0.0);
                    if (report_err) r1.bound.assign((size_t)(L + 1) * N, 0.0);
                    run_units(one, prm, sigma, {{0, l, smp}}, 1, tuned_wg(ctxs[i], P), s, r1, N);
                    for (size_t k = 0; k < xsz; ++k) res.samples[i * xsz + k] += r1.samples[k];
                    for (size_t k = 0; k < r1.bound.size(); ++k) res.bound[i * (L + 1) * N + k] += r1.bound[k];
                    for (int k = 0; k <= L; ++k)
                        res.level_res[i * (L + 1) + k] = std::max(res.level_res[i * (L + 1) + k], r1.level_res[k]);
                    res.rep.systems += r1.rep.systems;
                    res.rep.iterations += r1.rep.iterations;
                    res.rep.reliable_updates += r1.rep.reliable_updates;
                    res.rep.dslash_calls += r1.rep.dslash_calls;
                    res.rep.max_rel_residual = std::max(res.rep.max_rel_residual, r1.rep.max_rel_residual);
                    res.noconv |= r1.noconv;
                }
    } else {
        int nr = prm->solve.rhs_block ? prm->solve.rhs_block : tuned_nr(c0, P, N);
        const int wg = tuned_wg(c0, P);
        // memory budget per pass: fields per system ~ (4 FP64 + 6 low) spinors.
        // Free memory counts the blocks the allocator holds for reuse, so the
        // budget, and with it the passes, do not depend on what earlier calls
        // left cached.
        size_t bytes_per_site_sys = 4 * 192 + 6 * (size_t)prec_group_bytes_spinor(P) + (P == P16 ? 24 : 0);
        size_t free_b = 0, total_b = 0;
        HC(hipMemGetInfo(&free_b, &total_b));
        if (prm->pass_bytes < 0) fail(FS_E_ARG, "pass_bytes must be >= 0");
        const size_t budget = prm->pass_bytes > 0 ? (size_t)prm->pass_bytes
                                                  : std::min<size_t>((free_b + pool().cached_bytes()) / 2,
                                                                     (size_t)96 << 30);
        // units in chunks of nr samples of one (instance, level): the rhs blocks
        struct Chunk {
            int c;  // chunk index within its (instance, level)
            std::vector<std::array<int, 3>> units;
        };
        std::vector<Chunk> chunks;
        size_t total_need = 0;
        int max_nch = 1;
        for (int l = 0; l <= L; ++l)
            for (size_t i = 0; i < ctxs.size(); ++i) {
                const int nch = (Nl[l] + nr - 1) / nr;
                max_nch = std::max(max_nch, nch);
                for (int c = 0; c < nch; ++c) {
                    Chunk ch{c, {}};
                    for (int smp = c * nr; smp < std::min(Nl[l], (c + 1) * nr); ++smp) ch.units.push_back({(int)i, l, smp});
                    total_need += (size_t)ctxs[i]->V * bytes_per_site_sys * nr * (l < L ? 2 : 1);
                    chunks.push_back(std::move(ch));
                }
            }
        // Passes of equal make-up, so that every pass, and the next call of the
        // same shape, reuses the same field sizes: with d passes dividing the
        // chunks per (instance, level), pass k takes the chunks c = k mod d of
        // every one; more passes than that deal the chunks round-robin.
        const int need_pass =
            (int)std::min<size_t>(chunks.size(), std::max<size_t>(1, (total_need + budget - 1) / budget));
        int d = need_pass;
        while (d <= max_nch && max_nch % d) ++d;
        const bool by_index = d <= max_nch;
        if (!by_index) d = need_pass;
        for (int k = 0; k < d; ++k) {
            std::vector<std::array<int, 3>> units;
            for (size_t j = 0; j < chunks.size(); ++j)
                if ((by_index ? chunks[j].c : (int)j) % d == k)
                    units.insert(units.end(), chunks[j].units.begin(), chunks[j].units.end());
            if (!units.empty()) run_units(ctxs, prm, sigma, units, nr, wg, s, res, N);
        }
    }
    // deviation from the plain FP64 path: the same estimate (same noise) solved in FP64
    std::vector<double> t64, scale64;
    if (report_err && P != P64) {
        fs_est_params p64 = *prm;
        p64.solve.storage = FS_F64;
        p64.solve.batched = 1;
        p64.report_fp64_error = 0;
        std::vector<fs_level_stat> o64((size_t)ctxs.size() * (L + 1) * 16 * P1);
        std::vector<double> x64(xsz * ctxs.size());
        estimate_impl(ctxs, &p64, sigma_in, L, o64.data(), x64.data(), nullptr);
        t64.assign((size_t)ctxs.size() * (L + 1) * 16 * P1 * 2, 0.0);
        scale64.assign((size_t)ctxs.size() * (L + 1) * 16 * P1, 0.0);
        for (size_t i = 0; i < ctxs.size(); ++i)
            for (int l = 0; l <= L; ++l)
                for (int n = 0; n < 16; ++n)
                    for (int p = 0; p < P1; ++p) {
                        const size_t q = (((size_t)i * (L + 1) + l) * 16 + n) * P1 + p;
                        t64[2 * q] = o64[q].tr_re;
                        t64[2 * q + 1] = o64[q].tr_im;
                        double a = 0.0;
                        for (int smp = 0; smp < Nl[l]; ++smp) {
                            const size_t o = i * xsz + 2 * ((((size_t)l * N + smp) * 16 + n) * P1 + p);
                            a += std::hypot(x64[o], x64[o + 1]);
                        }
                        scale64[q] = a / Nl[l];
                    }
    }
    // level statistics from the per-sample estimates (device, FP64, fixed order)
    DevBuf d_nl = to_device(Nl.data(), sizeof(int) * (L + 1), 0, s);
    for (size_t i = 0; i < ctxs.size(); ++i) {
        DevBuf d_X = to_device(res.samples.data() + i * xsz, sizeof(double) * xsz, 0, s);
        DevBuf d_st(sizeof(double) * (size_t)(L + 1) * 16 * P1 * 4);
        launch_level_stats(d_X.as<double>(), L + 1, N, P1, d_st.as<double>(), s, d_nl.as<int>());
        std::vector<double> stv((size_t)(L + 1) * 16 * P1 * 4);
        HC(hipMemcpyAsync(stv.data(), d_st.p, sizeof(double) * stv.size(), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        const uint16_t mask = prm->gamma_mask ? prm->gamma_mask : 0xffff;
        const double u = ctxs[i]->link_norm;
        for (int l = 0; l <= L; ++l) {
            double bmax = 0.0;
            if (report_err)
                for (int smp = 0; smp < Nl[l]; ++smp) {
                    const double bv = res.bound[((size_t)i * (L + 1) + l) * N + smp];
                    bmax = (std::isnan(bv) || bv > bmax) ? bv : bmax;
                }
            for (int n = 0; n < 16; ++n)
                for (int p = 0; p < P1; ++p) {
                    const size_t q = ((size_t)i * (L + 1) + l) * 16 * P1 + (size_t)n * P1 + p;
                    fs_level_stat& o = out[q];
                    std::memset(&o, 0, sizeof(o));
                    if (!((mask >> n) & 1)) continue;
                    const double* d = &stv[(((size_t)l * 16 + n) * P1 + p) * 4];
                    o.tr_re = d[0];
                    o.tr_im = d[1];
                    o.var_paper = d[2];
                    o.var_unbiased = d[3];
                    o.n = Nl[l];
                    o.max_rel_residual = res.level_res[i * (L + 1) + l];
                    if (report_err) {
                        o.err_bound = bmax * std::pow(std::max(u, 1.0), p);  // ||Gamma_n Omega_p|| <= u^p
                        if (!t64.empty()) {
                            const double dr = o.tr_re - t64[2 * q], di = o.tr_im - t64[2 * q + 1];
                            const double sc = scale64[q] > 0.0 ? scale64[q] : 1.0;
                            o.fp64_rel_err = std::hypot(dr, di) / sc;
                        }
                    }
                }
        }
        if (samples_out) std::memcpy(samples_out + i * xsz, res.samples.data() + i * xsz, sizeof(double) * xsz);
    }
    res.rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = res.rep;
    if (res.noconv) throw FsError(FS_E_NOCONV, "a shifted solve did not reach tol (outputs are filled)");
}

// ============================================================== dslash timing

// Link reals the stencil reads per site (4 directions): 72, or 48 when the
// FP32 quad-shared loads (rhs blocks of 4 or more) take the two-row form.
double link_reals_per_site(int P, int nr, bool two_rows) {
    return (two_rows && P == P32 && nr >= 4) ? 48.0 : 72.0;
}

double dslash_bytes(int P, long long V, int n_sys, int nr, bool two_rows) {
    const double ws = P == P64 ? 8 : P == P32 ? 4 : 2;
    const double wg = ws;
    double per_sys = 48.0 * ws + (P == P16 ? 8.0 : 0.0);
    const long long nblk = (n_sys + nr - 1) / nr;
    return (double)V * (per_sys * n_sys + link_reals_per_site(P, nr, two_rows) * wg * nblk);
}

double time_dslash_impl(fs_ctx c, int P, int n_sys, int nr, int wg, int ilp, int occ, int n_launch) {
    hipStream_t s = c->stream;
    const int nblk = (n_sys + nr - 1) / nr;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto pl = make_plan(blk_lat, lats, nr, wg, s, ilp, occ);
    Field in, out;
    in.alloc(P, pl->total_slots);
    out.alloc(P, pl->total_slots);
    std::vector<NoiseKey> keys(pl->nsys);
    for (int i = 0; i < pl->nsys; ++i) {
        std::memset(&keys[i], 0, sizeof(NoiseKey));
        keys[i].seed = 12345;
        keys[i].sample = (uint64_t)i;
    }
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * keys.size(), 0, s);
    // Z4 noise input in the storage precision (out gets a copy so both are valid)
    launch_noise_block(P, pl->work(P, false), in.f(), d_keys.as<NoiseKey>(), s);
    launch_noise_block(P, pl->work(P, false), out.f(), d_keys.as<NoiseKey>(), s);
    std::vector<double> diag(pl->nsys, 4.1);
    DevBuf d_diag = to_device(diag.data(), sizeof(double) * diag.size(), 0, s);
    HC(hipStreamSynchronize(s));
    const Work w = pl->work(P, false, true);
    for (int i = 0; i < 3; ++i)
        launch_dslash(P, D_PLAIN, w, out.f(), in.f(), Fld(), d_diag.as<double>(), nullptr, M_ALL, nullptr, s);
    hipEvent_t e0, e1;
    HC(hipEventCreate(&e0));
    HC(hipEventCreate(&e1));
    HC(hipEventRecord(e0, s));
    for (int i = 0; i < n_launch; ++i)
        launch_dslash(P, D_PLAIN, w, (i & 1) ? in.f() : out.f(), (i & 1) ? out.f() : in.f(), Fld(),
                      d_diag.as<double>(), nullptr, M_ALL, nullptr, s);
    HC(hipEventRecord(e1, s));
    HC(hipEventSynchronize(e1));
    float ms = 0;
    HC(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / n_launch;
}

// Algorithmic bytes of one even-odd hop launch (one parity out): per output
// site and system 24 reals in and 24 out (+ FP16 scales); every link of the
// lattice once per block of nr systems (each link joins an even and an odd
// site), 18 reals, or 12 in the two-row form.
double dslash_eo_bytes(int P, long long V, int n_sys, int nr, bool two_rows) {
    const double w = P == P64 ? 8 : P == P32 ? 4 : 2;
    const double per_sys = 48.0 * w + (P == P16 ? 8.0 : 0.0);
    const long long nblk = (n_sys + nr - 1) / nr;
    return (double)(V / 2) * per_sys * n_sys + (double)V * link_reals_per_site(P, nr, two_rows) * w * nblk;
}

double time_dslash_eo_impl(fs_ctx c, int P, int n_sys, int nr, int var, int occ, int n_launch,
                           std::vector<float>* each = nullptr) {
    hipStream_t s = c->stream;
    const int nblk = (n_sys + nr - 1) / nr;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto full = make_plan(blk_lat, lats, nr, 256, s, 0, 0, 0);
    auto pl = eo_plan_of(*full, lats, s, P, var, occ);
    Field in, out;
    in.alloc(P, pl->total_slots);
    out.alloc(P, pl->total_slots);
    std::vector<NoiseKey> keys(pl->nsys);
    for (int i = 0; i < pl->nsys; ++i) {
        std::memset(&keys[i], 0, sizeof(NoiseKey));
        keys[i].seed = 12345;
        keys[i].sample = (uint64_t)i;
    }
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * keys.size(), 0, s);
    launch_noise_block(P, pl->work(P, false), in.f(), d_keys.as<NoiseKey>(), s);
    launch_noise_block(P, pl->work(P, false), out.f(), d_keys.as<NoiseKey>(), s);
    std::vector<double> diag(pl->nsys, 4.1);
    DevBuf d_diag = to_device(diag.data(), sizeof(double) * diag.size(), 0, s);
    HC(hipStreamSynchronize(s));
    const Work w = pl->work(P, false, true);
    auto hop = [&](int i) {  // odd sites from even ones, then back
        launch_dslash_eo(P, D_HOP, w, (i & 1) ? in.f() : out.f(), (i & 1) ? out.f() : in.f(), Fld(), Fld(),
                         d_diag.as<double>(), nullptr, M_ALL, nullptr, s, nullptr, (i & 1) ? 0 : 1);
    };
    for (int i = 0; i < 3; ++i) hop(i);
    hipEvent_t e0, e1;
    HC(hipEventCreate(&e0));
    HC(hipEventCreate(&e1));
    if (each) {  // every launch timed on its own (for medians)
        each->resize(n_launch);
        for (int i = 0; i < n_launch; ++i) {
            HC(hipEventRecord(e0, s));
            hop(i);
            HC(hipEventRecord(e1, s));
            HC(hipEventSynchronize(e1));
            HC(hipEventElapsedTime(&(*each)[i], e0, e1));
        }
    }
    HC(hipEventRecord(e0, s));
    for (int i = 0; i < n_launch; ++i) hop(i);
    HC(hipEventRecord(e1, s));
    HC(hipEventSynchronize(e1));
    float ms = 0;
    HC(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / n_launch;
}

// Work tables of a plan of nblk equal blocks of one lattice, written on the
// device (the allocation-free entry point keeps them in its scratch area).
__global__ void k_uniform_tables(BlockDesc* blocks, int* wg_start, int* wg_start_d, LatDesc* lats, double* diag,
                                 int* sys_map, int nblk, int nr, long long slots_per_block, int nwg_tile,
                                 int nwg_sten, LatDesc ld, double dg, int n_rhs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) lats[0] = ld;
    if (i <= nblk) {
        wg_start[i] = i * nwg_tile;
        wg_start_d[i] = i * nwg_sten;
    }
    if (i < nblk) {
        BlockDesc b;
        b.lat = 0;
        b.sys0 = i * nr;
        b.slot_off = (long long)i * slots_per_block;
        blocks[i] = b;
    }
    if (i < nblk * nr) {
        diag[i] = dg;
        sys_map[i] = i < n_rhs ? i : -1;
    }
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// fs_apply_dirac with every device buffer carved out of the scratch area.
void apply_dirac_noalloc(fs_ctx c, double m0, double sigma, int storage, const double* in, double* out, int n_rhs) {
    check_ctx(c);
    check_prec(storage);
    check_clover_prec(c, storage);
    if (!in || !out) fail(FS_E_ARG, "null buffer");
    if (n_rhs < 1) fail(FS_E_ARG, "n_rhs must be >= 1");
    DeviceScope ds(c->device);
    char* base = static_cast<char*>(scratch_of(c->device));
    if (!base) fail(FS_E_STATE, "no scratch area on this device");
    hipStream_t s = c->stream;
    const int nr = tuned_nr(c, storage, n_rhs);
    const int nblk = (n_rhs + nr - 1) / nr;
    std::vector<fs_ctx_s*> lats{c};
    std::vector<BlockDesc> blocks(nblk);
    for (int b = 0; b < nblk; ++b) {
        blocks[b].lat = 0;
        blocks[b].sys0 = b * nr;
        blocks[b].slot_off = (long long)b * c->V * nr;
    }
    Plan pl;
    plan_host(&pl, blocks, lats, nr, tuned_wg(c, storage), tuned_ilp(c, storage), tuned_occ(c, storage), 0);
    // scratch layout: tables, then the two block-layout fields (and FP16 scales)
    const int nsys = pl.nsys;
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off += align256(n);
        return o;
    };
    const size_t o_blocks = take(sizeof(BlockDesc) * nblk), o_ws = take(sizeof(int) * (nblk + 1)),
                 o_wsd = take(sizeof(int) * (nblk + 1)), o_lat = take(sizeof(LatDesc)),
                 o_diag = take(sizeof(double) * nsys), o_map = take(sizeof(int) * nsys);
    const size_t fbytes = (size_t)pl.total_slots * prec_group_bytes_spinor(storage);
    const size_t nbytes = storage == P16 ? (size_t)pl.total_slots * sizeof(float) : 0;
    const size_t o_fi = take(fbytes), o_fo = take(fbytes), o_ni = take(nbytes), o_no = take(nbytes);
    if (off > kScratchBytes)
        fail(FS_E_ARG, "input too large for the allocation-free scratch (" + std::to_string(off >> 20) +
                           " MiB needed, 64 MiB available)");
    pl.x_blocks = reinterpret_cast<const BlockDesc*>(base + o_blocks);
    pl.x_wg_start = reinterpret_cast<const int*>(base + o_ws);
    pl.x_wg_start_d = reinterpret_cast<const int*>(base + o_wsd);
    pl.x_lats = reinterpret_cast<const LatDesc*>(base + o_lat);
    const double* diag = reinterpret_cast<const double*>(base + o_diag);
    const int* sys_map = reinterpret_cast<const int*>(base + o_map);
    Fld fi, fo;
    fi.v = reinterpret_cast<uint4*>(base + o_fi);
    fo.v = reinterpret_cast<uint4*>(base + o_fo);
    if (storage == P16) {
        fi.n = reinterpret_cast<float*>(base + o_ni);
        fo.n = reinterpret_cast<float*>(base + o_no);
    }
    const int n_items = std::max(nblk + 1, nsys);
    hipLaunchKernelGGL(k_uniform_tables, dim3((n_items + 255) / 256), dim3(256), 0, s, (BlockDesc*)(base + o_blocks),
                       (int*)(base + o_ws), (int*)(base + o_wsd), (LatDesc*)(base + o_lat), (double*)(base + o_diag),
                       (int*)(base + o_map), nblk, nr, (long long)c->V * nr, pl.wg_start[1], pl.wg_start_d[1],
                       lat_desc(c, storage, 0, pl.two_rows), 4.0 + m0 + sigma, n_rhs);
    const long long stride = 24ll * c->V;
    launch_pack(storage, pl.work(storage, false), fi, in, stride, sys_map, s);
    launch_dslash(storage, D_PLAIN, pl.work(storage, false, true), fo, fi, Fld(), diag, nullptr, M_ALL, nullptr, s);
    if (c->c_sw != 0.0) launch_clover_add(storage, pl.work(storage, false), fo, fi, s);
    launch_unpack(storage, pl.work(storage, false), out, fo, stride, sys_map, s);
    HC(hipGetLastError());
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HC(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone) HC(hipStreamSynchronize(s));
}

// One application of the even-odd Schur operator as the solver issues it (the
// D_oe hop into odd-site scratch, then S with the fused (t, s), (t, t) partial
// sums), averaged over n_launch applications on n_sys systems.
double time_eo_apply_impl(fs_ctx c, int P, int n_sys, int nr, int var, int occ, int n_launch) {
    hipStream_t s = c->stream;
    const int nblk = (n_sys + nr - 1) / nr;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto full = make_plan(blk_lat, lats, nr, 256, s, 0, 0, 0);
    auto pl = eo_plan_of(*full, lats, s, P, var, occ);
    Field in, tmp, out;
    in.alloc(P, pl->total_slots);
    tmp.alloc(P, pl->total_slots);
    out.alloc(P, pl->total_slots);
    std::vector<NoiseKey> keys(pl->nsys);
    for (int i = 0; i < pl->nsys; ++i) {
        std::memset(&keys[i], 0, sizeof(NoiseKey));
        keys[i].seed = 12345;
        keys[i].sample = (uint64_t)i;
    }
    DevBuf d_keys = to_device(keys.data(), sizeof(NoiseKey) * keys.size(), 0, s);
    launch_noise_block(P, pl->work(P, false), in.f(), d_keys.as<NoiseKey>(), s);
    DevBuf d_rc(sizeof(uint32_t) * (size_t)pl->total_slots);
    launch_rhat_codes(pl->work(P, false), d_keys.as<NoiseKey>(), d_rc.as<uint32_t>(), s);
    std::vector<double> diag(pl->nsys, 4.1);
    DevBuf d_diag = to_device(diag.data(), sizeof(double) * diag.size(), 0, s);
    // the Schur launch's partial sums read each system's state (all "running")
    // and its shadow residual's code words
    std::vector<SysState> sts(pl->nsys);
    std::memset(sts.data(), 0, sizeof(SysState) * sts.size());
    DevBuf d_st = to_device(sts.data(), sizeof(SysState) * sts.size(), 0, s);
    DevBuf d_part(sizeof(double) * (size_t)pl->max_wg() * 8 * nr);
    HC(hipStreamSynchronize(s));
    const Work w = pl->work(P, false, true);
    auto apply = [&]() {
        launch_dslash_eo(P, D_HOP, w, tmp.f(), in.f(), Fld(), Fld(), d_diag.as<double>(), d_st.as<SysState>(), M_ALL,
                         nullptr, s, d_rc.as<uint32_t>(), 1);
        launch_dslash_eo(P, D_TS, w, out.f(), tmp.f(), in.f(), Fld(), d_diag.as<double>(), d_st.as<SysState>(),
                         M_ALL, d_part.as<double>(), s, d_rc.as<uint32_t>(), 0);
    };
    for (int i = 0; i < 2; ++i) apply();
    hipEvent_t e0, e1;
    HC(hipEventCreate(&e0));
    HC(hipEventCreate(&e1));
    HC(hipEventRecord(e0, s));
    for (int i = 0; i < n_launch; ++i) apply();
    HC(hipEventRecord(e1, s));
    HC(hipEventSynchronize(e1));
    float ms = 0;
    HC(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / n_launch;
}

// Multi-shift core: the systems of plan pl (one lattice, FP64, unpreconditioned)
// solved at every shift of `shifts` from one Krylov space each: batched
// BiCGStab on shifts[base] (the smallest) with the others carried along as
// members (launch_ms_scalars).  fill_b(bs) writes the sources into bs.b;
// consume(k, x_k, states_k) receives each shift's solutions (plan layout) and
// the states with their FP64 true residuals (rr_true; state S_DONE where the
// residual meets tol and the base converged, else S_FAIL).
template <class FillB, class Consume>
void ms_core(fs_ctx_s* c, const fs_solve_params* prm, const std::vector<double>& shifts, Plan& pl,
             const std::vector<char>& idle, const std::vector<NoiseKey>& rkeys, FillB&& fill_b, Consume&& consume) {
    hipStream_t s = c->stream;
    const int n_shift = (int)shifts.size();
    int base = 0;
    for (int k = 1; k < n_shift; ++k)
        if (shifts[k] < shifts[base]) base = k;
    std::vector<int> member;
    std::vector<double> dsh;
    for (int k = 0; k < n_shift; ++k)
        if (k != base) {
            member.push_back(k);
            dsh.push_back(shifts[k] - shifts[base]);
        }
    const int nm = (int)member.size();
    const int nsys = pl.nsys;
    const int nblk = (int)pl.blocks.size();
    SolveOpts o;
    o.P = P64;
    o.tol = prm->tol;
    o.max_iter = prm->max_iter;
    o.delta = 0.0;
    o.check_every = prm->check_every > 0 ? prm->check_every : 8;
    o.use_graph = prm->use_graph != 0;
    o.eo = false;
    std::vector<fs_ctx_s*> lats{c};
    BatchSolver bs(pl, lats, s, o);
    bs.setup(std::vector<double>(nsys, 4.0 + prm->m0 + shifts[base]), idle, rkeys);
    fill_b(bs);
    // members: x = 0, p = b, recurrence state zeta = tau = alpha_prev = 1, beta_prev = 0
    MultiShift ms;
    ms.nm = nm;
    ms.xs.resize(nm);
    ms.ps.resize(nm);
    std::memset(&ms.f, 0, sizeof(ms.f));
    const size_t fbytes = (size_t)pl.total_slots * prec_group_bytes_spinor(P64);
    for (int j = 0; j < nm; ++j) {
        ms.xs[j].alloc(P64, pl.total_slots);
        ms.ps[j].alloc(P64, pl.total_slots);
        HC(hipMemsetAsync(ms.xs[j].v.p, 0, fbytes, s));
        HC(hipMemcpyAsync(ms.ps[j].v.p, bs.b.v.p, fbytes, hipMemcpyDeviceToDevice, s));
        ms.f.x[j] = ms.xs[j].v.as<uint4>();
        ms.f.p[j] = ms.ps[j].v.as<uint4>();
    }
    if (nm > 0) {  // a single shift is the plain batched solve
        std::vector<MsState> st0((size_t)nsys * nm);
        for (auto& m : st0) {
            std::memset(&m, 0, sizeof(m));
            m.zp[0] = m.z[0] = m.tau[0] = m.ap[0] = 1.0;
        }
        ms.d_d = to_device(dsh.data(), sizeof(double) * nm, 0, s);
        ms.d_state = to_device(st0.data(), sizeof(MsState) * st0.size(), 0, s);
        ms.d_coef.alloc(sizeof(MsCoef) * st0.size());
        bs.ms = &ms;
    }
    bs.run();
    bs.ms = nullptr;
    std::vector<MsState> msh((size_t)nsys * nm);
    if (nm > 0) {
        HC(hipMemcpyAsync(msh.data(), ms.d_state.p, sizeof(MsState) * msh.size(), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
    }
    // true residuals of every solution: r = b - (D + sigma_k) x in FP64 and |r|^2
    Field rtmp;
    rtmp.alloc(P64, pl.total_slots);
    const Work wsten = pl.work(P64, false, true);
    DevBuf flags1(sizeof(int) * std::max(nblk, 1)), flags2(sizeof(int) * std::max(nblk, 1));
    for (int k = 0; k < n_shift; ++k) {
        const int j = k == base ? -1 : (int)(std::find(member.begin(), member.end(), k) - member.begin());
        Fld xk = j < 0 ? bs.xhi.f() : ms.xs[j].f();
        std::vector<double> dk(nsys, 4.0 + prm->m0 + shifts[k]);
        std::vector<SysState> sk(bs.st_host);
        for (int i = 0; i < nsys; ++i)
            if (!idle[i]) sk[i].state = S_CHK;
        DevBuf d_dk = to_device(dk.data(), sizeof(double) * nsys, 0, s);
        DevBuf d_sk = to_device(sk.data(), sizeof(SysState) * nsys, 0, s);
        launch_dslash(P64, D_RESID, wsten, rtmp.f(), xk, bs.b.f(), d_dk.as<double>(), d_sk.as<SysState>(), M_ALL,
                      bs.part(), s, bs.rc());
        launch_finish(F_TRUE, wsten, d_sk.as<SysState>(), bs.part(), flags1.as<int>(), flags2.as<int>(), s);
        HC(hipGetLastError());
        HC(hipMemcpyAsync(sk.data(), d_sk.p, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        for (int i = 0; i < nsys; ++i) {
            if (idle[i]) continue;
            const SysState& B0 = bs.st_host[i];
            sk[i].state = (true_rel(sk[i]) <= prm->tol && B0.state == S_DONE) ? S_DONE : S_FAIL;
            sk[i].iters = j < 0 ? B0.iters : msh[(size_t)i * nm + j].iters;  // the member's own Krylov steps
            sk[i].n_rel = B0.n_rel;
            sk[i].restarts = B0.restarts;
        }
        consume(k, xk, sk);
        HC(hipStreamSynchronize(s));  // consume's host tables may die with its scope
    }
}

// The sampling solves by ms_core: per chunk of nr samples one x-family (source z)
// and one y-family (source g5 z) solved at every sampling shift from one Krylov
// space; the solutions go to the blocks of the sampling plan (x(i, ch) =
// 2 (i nch + ch), y = x + 1) in bs.xhi, and their states to bs.st_host.
void sampling_multishift(fs_ctx_s* c, const fs_solve_params* prm, const std::vector<double>& sh, int nch, int nr,
                         BatchSolver& bs, const std::vector<NoiseKey>& keys) {
    hipStream_t s = c->stream;
    std::vector<int> blk_lat(2 * nch, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, P64), s, tuned_ilp(c, P64), tuned_occ(c, P64));
    const int nsys = pl->nsys;  // the shift-0 systems of the sampling plan, in the same order
    std::vector<NoiseKey> k0(keys.begin(), keys.begin() + nsys);
    std::vector<char> idle(nsys);
    for (int i = 0; i < nsys; ++i) idle[i] = k0[i].pad != 0;
    DevBuf d_k0 = to_device(k0.data(), sizeof(NoiseKey) * nsys, 0, s);
    const size_t blk_bytes = (size_t)Tr<P64>::G * 16 * (size_t)c->V * nr;
    ms_core(
        c, prm, sh, *pl, idle, k0,
        [&](BatchSolver& b2) { launch_noise_block(P64, pl->work(P64, false), b2.b.f(), d_k0.as<NoiseKey>(), s); },
        [&](int k, Fld xk, const std::vector<SysState>& sk) {
            for (int bb = 0; bb < 2 * nch; ++bb) {
                const int ch = bb / 2, f = bb % 2;
                const int bf = 2 * (k * nch + ch) + f;  // block of the sampling plan
                HC(hipMemcpyAsync(reinterpret_cast<char*>(bs.xhi.v.p) + (size_t)bs.pl.blocks[bf].slot_off * Tr<P64>::G * 16,
                                  reinterpret_cast<const char*>(xk.v) + (size_t)pl->blocks[bb].slot_off * Tr<P64>::G * 16,
                                  blk_bytes, hipMemcpyDeviceToDevice, s));
                for (int r = 0; r < nr; ++r) bs.st_host[(size_t)bf * nr + r] = sk[(size_t)bb * nr + r];
            }
        });
}

// X[s][r] = (D + sigma_s)^-1 B[r] by ms_core; dB, dX device, canonical; stats as
// fs_solve_shifted.  Returns the worst status.
fs_status ms_solve(fs_ctx_s* c, const fs_solve_params* prm, const double* sigma, int n_shift, const DevBuf& dB,
                   int n_rhs, DevBuf& dX, fs_solve_stats* stats) {
    hipStream_t s = c->stream;
    const int nr = prm->batched ? (prm->rhs_block ? prm->rhs_block : tuned_nr(c, P64, n_rhs)) : 1;
    const int nblk = (n_rhs + nr - 1) / nr;
    std::vector<int> blk_lat(nblk, 0);
    std::vector<fs_ctx_s*> lats{c};
    auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, P64), s, tuned_ilp(c, P64), tuned_occ(c, P64));
    const int nsys = pl->nsys;
    std::vector<char> idle(nsys);
    std::vector<int> src(nsys);
    std::vector<NoiseKey> rkeys(nsys);
    for (int i = 0; i < nsys; ++i) {
        idle[i] = i >= n_rhs;
        src[i] = i < n_rhs ? i : -1;
        std::memset(&rkeys[i], 0, sizeof(NoiseKey));
        rkeys[i].seed = 0x5A4E4F4953452121ull;
        rkeys[i].instance = 0x40000001u;
        rkeys[i].sample = (uint64_t)(i < n_rhs ? i : 0);
        rkeys[i].pad = idle[i] ? 1 : 0;
    }
    DevBuf d_src = to_device(src.data(), sizeof(int) * nsys, 0, s);
    fs_status worst = FS_OK;
    ms_core(
        c, prm, std::vector<double>(sigma, sigma + n_shift), *pl, idle, rkeys,
        [&](BatchSolver& bs) {
            launch_pack(P64, pl->work(P64, false), bs.b.f(), dB.as<double>(), 24ll * c->V, d_src.as<int>(), s);
        },
        [&](int k, Fld xk, const std::vector<SysState>& sk) {
            std::vector<int> dst(nsys);
            for (int i = 0; i < nsys; ++i) dst[i] = i < n_rhs ? k * n_rhs + i : -1;
            DevBuf d_dst = to_device(dst.data(), sizeof(int) * nsys, 0, s);
            launch_unpack(P64, pl->work(P64, false), dX.as<double>(), xk, 24ll * c->V, d_dst.as<int>(), s);
            HC(hipGetLastError());
            HC(hipStreamSynchronize(s));
            for (int i = 0; i < n_rhs; ++i) {
                const fs_status code = sk[i].state == S_DONE ? FS_OK : FS_E_NOCONV;
                if (code != FS_OK) worst = code;
                if (stats) {
                    fs_solve_stats& o2 = stats[k * n_rhs + i];
                    o2.iters = sk[i].iters;
                    o2.reliable_updates = sk[i].n_rel;
                    o2.status = code;
                    o2.restarts = sk[i].restarts;
                    o2.true_rel_residual = true_rel(sk[i]);
                }
            }
        });
    return worst;
}


}  // namespace

// ============================================================== C ABI

extern "C" {

const char* fs_version(void) { return "fsmlmc 0.1 (gfx950)"; }

int32_t fs_struct_sizes(int64_t* out, int32_t n) {
    const int64_t sz[] = {(int64_t)sizeof(fs_solve_params), (int64_t)sizeof(fs_solve_stats),
                          (int64_t)sizeof(fs_est_params),   (int64_t)sizeof(fs_level_stat),
                          (int64_t)sizeof(fs_total_stat),   (int64_t)sizeof(fs_est_report),
                          (int64_t)sizeof(fs_shift_model)};
    const int32_t count = (int32_t)(sizeof(sz) / sizeof(sz[0]));
    if (out)
        for (int32_t i = 0; i < std::min(n, count); ++i) out[i] = sz[i];
    return count;
}

const char* fs_last_error(fs_ctx c) { return c ? c->last_err.c_str() : g_err.c_str(); }

fs_status fs_create(fs_ctx* out, const int32_t dims[4], int32_t t_antiperiodic, int32_t device, void* hip_stream) {
    return guard([&] {
        if (!out || !dims) fail(FS_E_ARG, "null argument");
        *out = nullptr;
        long long V = 1;
        for (int i = 0; i < 4; ++i) {
            if (dims[i] < 2) fail(FS_E_ARG, "every lattice extent must be >= 2");
            V *= dims[i];
        }
        // one direction of FP64 links (nine complex planes) is addressed with
        // 32-bit offsets
        if (144ll * V >= (1ll << 32)) fail(FS_E_ARG, "lattice too large (over 29.8M sites)");
        int ndev = 0;
        HC(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) fail(FS_E_ARG, "invalid device ordinal");
        auto c = std::make_unique<fs_ctx_s>();
        for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
        c->V = (int)V;
        c->tsign = t_antiperiodic ? -1 : 1;
        c->device = device;
        DeviceScope ds(device);
        scratch_init(device);
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            HC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        *out = c.release();
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        ++g_live_ctx;
    });
}

fs_status fs_destroy(fs_ctx c) {
    return guard([&] {
        if (!c) return;
        {
            DeviceScope ds(c->device);
            (void)hipStreamSynchronize(c->stream);
            for (auto& g : c->gauge) g.release();
            for (auto& g : c->gauge_q) g.release();
            for (auto& g : c->gauge_q2) g.release();
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
        }
        delete c;
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        if (--g_live_ctx <= 0) {
            g_live_ctx = 0;
            pool().trim(0);
        }
    });
}

fs_status fs_set_instance(fs_ctx c, uint32_t instance) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        c->instance = instance;
    });
}

fs_status fs_upload_gauge(fs_ctx c, const double* links, int32_t is_device) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        if (!links) fail(FS_E_ARG, "null links");
        DeviceScope ds(c->device);
        const size_t n = sizeof(double) * 18 * 4 * (size_t)c->V;
        DevBuf src = to_device(links, n, is_device, c->stream);
        if (is_device) {
            std::vector<double> h(n / sizeof(double));
            from_device(h.data(), src, n, 0, c->stream);
            c->su3_defect = su3_row_defect(h.data(), (size_t)4 * c->V);
            c->link_norm = link_norm_bound(h.data(), (size_t)4 * c->V);
        } else {
            c->su3_defect = su3_row_defect(links, (size_t)4 * c->V);
            c->link_norm = link_norm_bound(links, (size_t)4 * c->V);
        }
        c->two_rows = c->su3_defect <= kSu3RowTol;
        for (int P = 0; P < 4; ++P) {
            c->gauge[P].alloc((size_t)4 * 9 * c->V * prec_link_complex_bytes(P));
            launch_gauge_convert(P, c->gauge[P].p, src.as<double>(), c->V, c->stream);
            c->gauge_q[P].alloc((size_t)4 * c->V * prec_link_site_bytes(P, false));
            launch_gauge_convert_q(P, c->gauge_q[P].p, src.as<double>(), c->V, false, c->stream);
            if (c->two_rows && P == P32) {
                c->gauge_q2[P].alloc((size_t)4 * c->V * prec_link_site_bytes(P, true));
                launch_gauge_convert_q(P, c->gauge_q2[P].p, src.as<double>(), c->V, true, c->stream);
            } else {
                c->gauge_q2[P].release();
            }
        }
        HC(hipStreamSynchronize(c->stream));
        c->has_gauge = true;
        if (c->c_sw != 0.0) build_clover(c);
    });
}

fs_status fs_set_clover(fs_ctx c, double c_sw) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        if (!std::isfinite(c_sw)) fail(FS_E_ARG, "c_sw must be finite");
        if (c_sw != 0.0 && (c->dims[0] % 2 || c->dims[1] % 2 || c->dims[2] % 2 || c->dims[3] % 2))
            fail(FS_E_ARG, "the clover term needs even extents (even-odd layout)");
        DeviceScope ds(c->device);
        c->c_sw = c_sw;
        if (c_sw == 0.0) {
            c->clv[P64].release();
            c->clv[P32].release();
            c->clv_norm = 0.0;
            return;
        }
        try {
            build_clover(c);
        } catch (...) {
            c->c_sw = 0.0;
            c->clv_norm = 0.0;
            throw;
        }
    });
}

fs_status fs_gauge_info(fs_ctx c, int32_t* two_rows, double* su3_defect) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        if (two_rows) *two_rows = c->two_rows ? 1 : 0;
        if (su3_defect) *su3_defect = c->su3_defect;
    });
}

fs_status fs_apply_dirac(fs_ctx c, double m0, double sigma, fs_prec storage, const double* in, double* out,
                         int32_t n_rhs, int32_t is_device) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        check_prec(storage);
        check_clover_prec(c, storage);
        if (!in || !out) fail(FS_E_ARG, "null buffer");
        if (n_rhs < 1) fail(FS_E_ARG, "n_rhs must be >= 1");
        DeviceScope ds(c->device);
        hipStream_t s = c->stream;
        // the tuned (or set) rhs block and work-group size; a last partial
        // block is padded with zero systems
        const int nr = tuned_nr(c, storage, n_rhs);
        const int nblk = (n_rhs + nr - 1) / nr;
        std::vector<int> blk_lat(nblk, 0);
        std::vector<fs_ctx_s*> lats{c};
        auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, storage), s, tuned_ilp(c, storage), tuned_occ(c, storage));
        std::vector<int> sys_map(pl->nsys);
        for (int i = 0; i < pl->nsys; ++i) sys_map[i] = i < n_rhs ? i : -1;
        DevBuf d_map = to_device(sys_map.data(), sizeof(int) * sys_map.size(), 0, s);
        const size_t nb = sizeof(double) * 24 * (size_t)c->V * n_rhs;
        DevBuf din = to_device(in, nb, is_device, s);
        DevBuf dout(nb);
        Field fi, fo;
        fi.alloc(storage, pl->total_slots);
        fo.alloc(storage, pl->total_slots);
        const long long stride = 24ll * c->V;
        launch_pack(storage, pl->work(storage, false), fi.f(), din.as<double>(), stride, d_map.as<int>(), s);
        std::vector<double> diag(pl->nsys, 4.0 + m0 + sigma);
        DevBuf d_diag = to_device(diag.data(), sizeof(double) * diag.size(), 0, s);
        launch_dslash(storage, D_PLAIN, pl->work(storage, false, true), fo.f(), fi.f(), Fld(), d_diag.as<double>(),
                      nullptr, M_ALL, nullptr, s);
        if (c->c_sw != 0.0) launch_clover_add(storage, pl->work(storage, false), fo.f(), fi.f(), s);
        launch_unpack(storage, pl->work(storage, false), dout.as<double>(), fo.f(), stride, d_map.as<int>(), s);
        HC(hipGetLastError());
        from_device(out, dout, nb, is_device, s);
    });
}

fs_status fs_apply_dirac_noalloc(fs_ctx c, double m0, double sigma, fs_prec storage, const double* in, double* out,
                                 int32_t n_rhs) {
    return guard_ctx(c, [&] { apply_dirac_noalloc(c, m0, sigma, storage, in, out, n_rhs); });
}

fs_status fs_z4_noise(fs_ctx c, uint64_t seed, uint32_t instance, uint32_t level, uint64_t sample, double* out,
                      int32_t is_device) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        if (!out) fail(FS_E_ARG, "null buffer");
        DeviceScope ds(c->device);
        const size_t nb = sizeof(double) * 24 * (size_t)c->V;
        DevBuf d(nb);
        NoiseKey k;
        std::memset(&k, 0, sizeof(k));
        k.seed = seed;
        k.instance = instance;
        k.level = level;
        k.sample = sample;
        launch_noise_canonical(d.as<double>(), c->V, k, c->stream);
        HC(hipGetLastError());
        from_device(out, d, nb, is_device, c->stream);
    });
}

fs_status fs_displace(fs_ctx c, int32_t p, const double* in, double* out, int32_t is_device) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        if (!in || !out) fail(FS_E_ARG, "null buffer");
        if (p < 0) fail(FS_E_ARG, "p must be >= 0");
        DeviceScope ds(c->device);
        const size_t nb = sizeof(double) * 24 * (size_t)c->V;
        DevBuf a = to_device(in, nb, is_device, c->stream);
        DevBuf b(nb);
        const LatDesc ld = lat_desc(c, P64);
        for (int k = 0; k < p; ++k) {
            launch_displace_canonical(b.as<double>(), a.as<double>(), c->gauge[P64].as<double>(), ld, c->stream);
            std::swap(a, b);
        }
        HC(hipGetLastError());
        from_device(out, a, nb, is_device, c->stream);
    });
}

fs_status fs_bilinear(fs_ctx c, int32_t p_max, const double* y, const double* x, double* out, int32_t is_device) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        if (!y || !x || !out) fail(FS_E_ARG, "null buffer");
        if (p_max < 0 || p_max >= c->dims[2]) fail(FS_E_ARG, "p_max must be in [0, Lz)");
        DeviceScope ds(c->device);
        hipStream_t s = c->stream;
        const int P1 = p_max + 1;
        std::vector<int> blk_lat{0, 0};  // block 0: x, block 1: y (no workgroups in hop launches)
        std::vector<fs_ctx_s*> lats{c};
        auto pl = make_plan(blk_lat, lats, 1, 256, s);
        const size_t nb = sizeof(double) * 24 * (size_t)c->V;
        DevBuf dx = to_device(x, nb, is_device, s);
        DevBuf dy = to_device(y, nb, is_device, s);
        Field fx, f1, f2;
        fx.alloc(P64, pl->total_slots);
        f1.alloc(P64, pl->total_slots);
        f2.alloc(P64, pl->total_slots);
        std::vector<int> map_x{0, -2}, map_y{-2, 0};
        DevBuf dmx = to_device(map_x.data(), sizeof(int) * 2, 0, s);
        DevBuf dmy = to_device(map_y.data(), sizeof(int) * 2, 0, s);
        launch_pack(P64, pl->work(P64, false), fx.f(), dx.as<double>(), 0, dmx.as<int>(), s);
        launch_pack(P64, pl->work(P64, false), fx.f(), dy.as<double>(), 0, dmy.as<int>(), s);
        std::vector<int> hop_start{0, pl->wg_start[1], pl->wg_start[1]};
        DevBuf d_hs = to_device(hop_start.data(), sizeof(int) * 3, 0, s);
        std::vector<int> yb{1, 0, -1, 0};
        DevBuf d_yb = to_device(yb.data(), sizeof(int) * 4, 0, s);
        Work wh = pl->work(P64, false);
        wh.wg_start = d_hs.as<int>();
        wh.total_wg = hop_start.back();
        DevBuf d_part(sizeof(double) * (size_t)pl->wg_start.back() * 32);
        DevBuf d_M(sizeof(double) * 2 * P1 * 32);
        Fld cur = fx.f();
        for (int p = 0; p <= p_max; ++p) {
            Fld o = (p % 2 == 1) ? f1.f() : f2.f();
            launch_hop_reduce(wh, p, o, cur, fx.f(), Fld(), d_yb.as<int>(), d_part.as<double>(), s);
            launch_hop_finish(wh, d_part.as<double>(), d_M.as<double>(), P1, p, s);
            if (p > 0) cur = o;
        }
        std::vector<XMap> xm(2);
        std::memset(xm.data(), 0, sizeof(XMap) * 2);
        xm[0].level = 0;
        xm[0].coef = 1.0;
        xm[1].level = -1;
        DevBuf d_xm = to_device(xm.data(), sizeof(XMap) * 2, 0, s);
        static const GammaTab gt = make_gamma_tab();
        DevBuf d_X(sizeof(double) * 16 * P1 * 2);
        launch_gamma_contract(d_M.as<double>(), P1, 2, d_xm.as<XMap>(), gt, d_X.as<double>(), 1, s);
        HC(hipGetLastError());
        // X layout [n][p] -> out [p][n]
        std::vector<double> X(16 * P1 * 2);
        HC(hipMemcpyAsync(X.data(), d_X.p, sizeof(double) * X.size(), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        std::vector<double> o(16 * P1 * 2);
        for (int n = 0; n < 16; ++n)
            for (int p = 0; p < P1; ++p) {
                o[2 * (p * 16 + n)] = X[2 * (n * P1 + p)];
                o[2 * (p * 16 + n) + 1] = X[2 * (n * P1 + p) + 1];
            }
        if (is_device) {
            HC(hipMemcpyAsync(out, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, s));
            HC(hipStreamSynchronize(s));
        } else {
            std::memcpy(out, o.data(), sizeof(double) * o.size());
        }
    });
}

fs_status fs_solve_shifted(fs_ctx c, const fs_solve_params* prm, const double* sigma, int32_t n_shift, const double* B,
                           int32_t n_rhs, double* X, int32_t is_device, fs_solve_stats* stats) {
    fs_status worst = FS_OK;
    fs_status st = guard_ctx(c, [&] {
        check_ctx(c);
        if (!prm || !sigma || !B || !X) fail(FS_E_ARG, "null argument");
        if (n_shift < 1 || n_rhs < 1) fail(FS_E_ARG, "n_shift and n_rhs must be >= 1");
        check_prec(prm->storage);
        if (!(prm->tol > 0)) fail(FS_E_ARG, "tol must be > 0");
        if (prm->max_iter < 1) fail(FS_E_ARG, "max_iter must be >= 1");
        if (prm->rhs_block != 0 && !pow2_ok(prm->rhs_block)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
        check_eo(prm->even_odd != 0, c);
        if (prm->multi_shift) {
            if (prm->storage != P64) fail(FS_E_ARG, "multi-shift solves run in FP64 storage");
            if (prm->even_odd)
                fail(FS_E_ARG, "multi-shift solves need even_odd = 0 (Schur complements of different shifts "
                               "share no Krylov space)");
            if (n_shift > MS_MAX + 1) fail(FS_E_ARG, "at most 17 shifts per multi-shift solve");
            if (c->c_sw != 0.0) fail(FS_E_ARG, "multi-shift solves use the plain operator (no clover term)");
        }
        DeviceScope ds(c->device);
        hipStream_t s = c->stream;
        const size_t nb1 = sizeof(double) * 24 * (size_t)c->V;
        DevBuf dB = to_device(B, nb1 * n_rhs, is_device, s);
        DevBuf dX(nb1 * n_rhs * n_shift);
        if (prm->multi_shift) {
            worst = ms_solve(c, prm, sigma, n_shift, dB, n_rhs, dX, stats);
            from_device(X, dX, nb1 * n_rhs * n_shift, is_device, s);
            return;
        }
        const int P = prm->storage;
        SolveOpts o;
        o.P = P;
        o.tol = prm->tol;
        o.max_iter = prm->max_iter;
        o.delta = P == P64 ? 0.0 : (prm->reliable_delta > 0 ? prm->reliable_delta : default_delta(P));
        o.check_every = prm->check_every > 0 ? prm->check_every : 8;
        o.use_graph = prm->use_graph != 0;
        o.eo = prm->even_odd != 0;
        o.eo_var = eo_tuning(c, P)[0];
        o.eo_occ = eo_tuning(c, P)[1];
        std::vector<fs_ctx_s*> lats{c};
        // groups: (shift, rhs range) solved together
        std::vector<std::vector<std::pair<int, int>>> passes;  // each pass: list of (shift, rhs)
        int nr = 1;
        if (prm->batched) {
            nr = prm->rhs_block ? prm->rhs_block : tuned_nr(c, P, n_rhs);
            std::vector<std::pair<int, int>> all;
            for (int sh = 0; sh < n_shift; ++sh)
                for (int r = 0; r < n_rhs; ++r) all.push_back({sh, r});
            passes.push_back(all);
        } else {
            for (int sh = 0; sh < n_shift; ++sh)
                for (int r = 0; r < n_rhs; ++r) passes.push_back({{sh, r}});
        }
        for (auto& pass : passes) {
            // blocks: per shift, rhs chunks of nr
            std::vector<int> blk_lat;
            std::vector<int> sys_src, sys_dst;
            std::vector<double> diag;
            std::vector<char> idle;
            std::map<int, std::vector<int>> by_shift;
            for (auto& pr : pass) by_shift[pr.first].push_back(pr.second);
            for (auto& kv : by_shift) {
                const auto& rr = kv.second;
                for (size_t c0 = 0; c0 < rr.size(); c0 += nr) {
                    blk_lat.push_back(0);
                    for (int q = 0; q < nr; ++q) {
                        const bool ok = c0 + q < rr.size();
                        sys_src.push_back(ok ? rr[c0 + q] : -1);
                        sys_dst.push_back(ok ? kv.first * n_rhs + rr[c0 + q] : -1);
                        diag.push_back(4.0 + prm->m0 + sigma[kv.first]);
                        idle.push_back(!ok);
                    }
                }
            }
            auto pl = make_plan(blk_lat, lats, nr, tuned_wg(c, P), s, tuned_ilp(c, P), tuned_occ(c, P));
            BatchSolver bs(*pl, lats, s, o);
            // shadow residuals: one fixed Z4 stream per system (sources are arbitrary)
            std::vector<NoiseKey> rkeys(pl->nsys);
            for (int i = 0; i < pl->nsys; ++i) {
                std::memset(&rkeys[i], 0, sizeof(NoiseKey));
                rkeys[i].seed = 0x5A4E4F4953452121ull;
                rkeys[i].instance = 0x40000000u;
                rkeys[i].sample = (uint64_t)(sys_dst[i] < 0 ? 0 : sys_dst[i]);
                rkeys[i].pad = idle[i] ? 1 : 0;
            }
            bs.setup(diag, idle, rkeys);
            DevBuf d_src = to_device(sys_src.data(), sizeof(int) * sys_src.size(), 0, s);
            DevBuf d_dst = to_device(sys_dst.data(), sizeof(int) * sys_dst.size(), 0, s);
            launch_pack(P64, pl->work(P64, false), bs.b.f(), dB.as<double>(), 24ll * c->V, d_src.as<int>(), s);
            bs.run();
            launch_unpack(P64, pl->work(P64, false), dX.as<double>(), bs.xhi.f(), 24ll * c->V, d_dst.as<int>(), s);
            HC(hipGetLastError());
            for (int i = 0; i < pl->nsys; ++i) {
                if (sys_dst[i] < 0) continue;
                const SysState& S = bs.st_host[i];
                fs_status code = S.state == S_DONE ? FS_OK : FS_E_NOCONV;
                if (code != FS_OK) worst = code;
                if (stats) {
                    fs_solve_stats& o2 = stats[sys_dst[i]];
                    o2.iters = S.iters;
                    o2.reliable_updates = S.n_rel;
                    o2.status = code;
                    o2.restarts = S.restarts;
                    o2.true_rel_residual = true_rel(S);
                }
            }
        }
        from_device(X, dX, nb1 * n_rhs * n_shift, is_device, s);
    });
    if (st != FS_OK) return st;
    if (worst != FS_OK) {
        g_err = "some systems did not reach tol";
        c->last_err = g_err;
    }
    return worst;
}

fs_status fs_estimate(fs_ctx c, const fs_est_params* prm, const double* sigma, int32_t L, fs_level_stat* out,
                      double* samples_out, fs_est_report* report) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        estimate_impl({c}, prm, sigma, L, out, samples_out, report);
    });
}

fs_status fs_sample_variances(fs_ctx c, const fs_est_params* prm, const double* shifts, int32_t m,
                              fs_level_stat* single, fs_level_stat* pair, double* samples_out,
                              double* iters_out, fs_est_report* report) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        sampling_impl(c, prm, shifts, m, single, pair, samples_out, iters_out, report);
    });
}

// ------------------------------------------------------------------ shift selection

fs_status fs_eval_grid(const double* s_hat, int32_t m, double* s_out, int32_t cap, int32_t* n_out) {
    return guard([&] {
        if (!s_hat || !s_out || !n_out) fail(FS_E_ARG, "null argument");
        if (m < 2 || m > 16) fail(FS_E_ARG, "m must be in 2..16");
        if (s_hat[0] != 0.0) fail(FS_E_ARG, "s_hat[0] must be 0");
        for (int i = 0; i + 1 < m; ++i)
            if (!(s_hat[i + 1] > s_hat[i]) || !std::isfinite(s_hat[i + 1]))
                fail(FS_E_ARG, "s_hat must be strictly increasing");
        const std::vector<double> g = paper_eval_grid(s_hat, m);
        if ((int)g.size() > cap) fail(FS_E_ARG, "output capacity too small");
        std::copy(g.begin(), g.end(), s_out);
        *n_out = (int32_t)g.size();
    });
}

fs_status fs_shift_tables(const fs_shift_model* model, double* v_pair_eval, double* v_single_eval, double* r_eval) {
    return guard([&] {
        if (!model) fail(FS_E_ARG, "null model");
        const ShiftTables T = shift_tables(*model);
        if (v_pair_eval) std::copy(T.vp.begin(), T.vp.end(), v_pair_eval);
        if (v_single_eval) std::copy(T.vs.begin(), T.vs.end(), v_single_eval);
        if (r_eval) std::copy(T.r.begin(), T.r.end(), r_eval);
    });
}

namespace {

void level_terms(const ShiftTables& T, const std::vector<int>& id, double* v_levels, double* c_levels) {
    const int L = (int)id.size() - 1, n = T.n;
    for (int l = 0; l <= L; ++l) {
        const bool last = l == L;
        if (v_levels) v_levels[l] = last ? T.vs[id[l]] : T.vp[(size_t)id[l] * n + id[l + 1]];
        if (c_levels) c_levels[l] = last ? T.r[id[l]] : T.r[id[l]] + T.r[id[l + 1]];
    }
}

}  // namespace

fs_status fs_select_shifts(const fs_shift_model* model, int32_t L, int32_t* idx, double* c_fs, double* v_levels,
                           double* c_levels) {
    return guard([&] {
        if (!model || !idx || !c_fs) fail(FS_E_ARG, "null argument");
        const ShiftTables T = shift_tables(*model);
        if (L < 0 || L > T.n - 1) fail(FS_E_ARG, "L must be in 0..n-1");
        std::vector<int> id(L + 1);
        const double c = shift_select_dp(T, L, id.data());
        for (int l = 0; l <= L; ++l) idx[l] = id[l];
        *c_fs = c;
        level_terms(T, id, v_levels, c_levels);
    });
}

fs_status fs_sweep_shifts(fs_ctx c, const fs_shift_model* model, int32_t L, int32_t* idx, double* c_fs, double* ms) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        if (!model || !idx || !c_fs) fail(FS_E_ARG, "null argument");
        if (L < 1 || L > kSweepMaxL) fail(FS_E_ARG, "L must be in 1..8 for the sweep");
        if (model->n > kSweepMaxN) fail(FS_E_ARG, "n must be <= 88 for the sweep");
        const ShiftTables T = shift_tables(*model);
        const int n = T.n;
        if (L > n - 1) fail(FS_E_ARG, "L must be <= n-1");
        constexpr int BW = kSweepMaxL + 1;
        std::vector<uint64_t> binom((size_t)(kSweepMaxN + 1) * BW, 0);
        for (int a = 0; a <= kSweepMaxN; ++a) {
            binom[(size_t)a * BW] = 1;
            for (int b = 1; b < BW && a > 0; ++b) binom[(size_t)a * BW + b] = binom[(size_t)(a - 1) * BW + b - 1] +
                                                                             binom[(size_t)(a - 1) * BW + b];
        }
        auto C = [&](int a, int b) { return binom[(size_t)a * BW + b]; };
        if (C(n - 1, L) > (1ull << 40)) fail(FS_E_ARG, "too many combinations for the sweep");
        const uint64_t n_prefix = C(n - 2, L - 1);  // prefixes from {1..n-2}: each has a last index above it
        const uint64_t max_threads = 1024ull * 256;
        const uint64_t per = (n_prefix + max_threads - 1) / max_threads;
        const int grid = (int)((n_prefix + per * 256 - 1) / (per * 256));
        DeviceScope ds(c->device);
        hipStream_t s = c->stream;
        DevBuf d_w = to_device(T.w.data(), sizeof(double) * n * n, 0, s);
        DevBuf d_u = to_device(T.u.data(), sizeof(double) * n, 0, s);
        DevBuf d_b = to_device(binom.data(), sizeof(uint64_t) * binom.size(), 0, s);
        DevBuf d_pc(sizeof(double) * grid), d_pk(sizeof(uint64_t) * grid), d_oc(sizeof(double)),
            d_ok(sizeof(uint64_t));
        hipEvent_t e0, e1;
        HC(hipEventCreate(&e0));
        HC(hipEventCreate(&e1));
        HC(hipEventRecord(e0, s));
        launch_shift_sweep(L, d_w.as<double>(), d_u.as<double>(), d_b.as<uint64_t>(), n, n_prefix, per, grid,
                           d_pc.as<double>(), d_pk.as<uint64_t>(), s);
        launch_sweep_reduce(d_pc.as<double>(), d_pk.as<uint64_t>(), grid, d_oc.as<double>(), d_ok.as<uint64_t>(), s);
        HC(hipEventRecord(e1, s));
        HC(hipGetLastError());
        double best = 0.0;
        uint64_t key = 0;
        HC(hipMemcpyAsync(&best, d_oc.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HC(hipMemcpyAsync(&key, d_ok.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        float t = 0.f;
        HC(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (!std::isfinite(best)) fail(FS_E_HIP, "sweep found no finite cost");
        // decode: lexicographic prefix rank, then the last index
        uint64_t r = key >> 7;
        const int K = L - 1, M = n - 2;
        std::vector<int> id(L + 1, 0);
        for (int p = 0, x = 1; p < K; ++p) {
            while (r >= C(M - x, K - 1 - p)) {
                r -= C(M - x, K - 1 - p);
                ++x;
            }
            id[p + 1] = x++;
        }
        id[L] = (int)(key & 127);
        for (int l = 0; l <= L; ++l) idx[l] = id[l];
        *c_fs = best * best;
        if (ms) *ms = t;
    });
}

fs_status fs_probing_colours(const int32_t dims[4], int32_t p, int32_t k, int32_t* colours, int32_t* n_colours) {
    return guard([&] {
        if (!dims || !colours || !n_colours) fail(FS_E_ARG, "null argument");
        int d[4];
        long long V = 1;
        for (int i = 0; i < 4; ++i) {
            if (dims[i] < 2) fail(FS_E_ARG, "every extent must be >= 2");
            d[i] = dims[i];
            V *= dims[i];
        }
        if (V > (1ll << 26)) fail(FS_E_ARG, "lattice too large for the colouring");
        if (p < 0 || p >= dims[2]) fail(FS_E_ARG, "p must be in [0, Lz)");
        if (k < 0 || k > 16) fail(FS_E_ARG, "k must be in 0..16");
        int nc = 0;
        const std::vector<int32_t> col = probing_colours(d, p, k, &nc);
        std::copy(col.begin(), col.end(), colours);
        *n_colours = nc;
    });
}

fs_status fs_estimate_probed(fs_ctx c, const fs_est_params* prm, const double* sigma, int32_t L,
                             const int32_t* colours, int32_t n_colours, fs_level_stat* out, double* samples_out,
                             fs_est_report* report) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        probed_impl(c, prm, sigma, L, colours, n_colours, out, samples_out, report);
    });
}

fs_status fs_batch_create(fs_batch* out, const fs_ctx* ctxs, int32_t n) {
    return guard([&] {
        if (!out || !ctxs || n < 1) fail(FS_E_ARG, "invalid batch");
        *out = nullptr;
        auto b = std::make_unique<fs_batch_s>();
        for (int i = 0; i < n; ++i) {
            check_ctx(ctxs[i]);
            if (ctxs[i]->device != ctxs[0]->device) fail(FS_E_ARG, "batch contexts must share a device");
            b->ctxs.push_back(ctxs[i]);
        }
        *out = b.release();
    });
}

fs_status fs_batch_estimate(fs_batch b, const fs_est_params* prm, const double* sigma, int32_t L, fs_level_stat* out,
                            double* samples_out, fs_est_report* report) {
    return guard([&] {
        if (!b) fail(FS_E_ARG, "null batch");
        std::vector<fs_ctx_s*> v(b->ctxs.begin(), b->ctxs.end());
        estimate_impl(v, prm, sigma, L, out, samples_out, report);
    });
}

fs_status fs_level_totals(const fs_level_stat* levels, int32_t L, int32_t p_max, fs_total_stat* out) {
    return guard([&] {
        if (!levels || !out) fail(FS_E_ARG, "null argument");
        if (L < 0 || p_max < 0) fail(FS_E_ARG, "L and p_max must be >= 0");
        const int P1 = p_max + 1;
        for (int n = 0; n < 16; ++n)
            for (int p = 0; p < P1; ++p) {
                fs_total_stat t;
                std::memset(&t, 0, sizeof(t));
                for (int l = 0; l <= L; ++l) {
                    const fs_level_stat& v = levels[((size_t)l * 16 + n) * P1 + p];
                    if (v.n <= 0) continue;  // Gamma_n not requested
                    t.tr_re += v.tr_re;
                    t.tr_im += v.tr_im;
                    t.v_fs += v.var_paper / (double)v.n;
                    t.v_fs_unbiased += v.var_unbiased / (double)v.n;
                    t.v_total += v.var_paper;
                    t.v_total_unbiased += v.var_unbiased;
                    t.err_bound += v.err_bound;
                }
                out[(size_t)n * P1 + p] = t;
            }
    });
}

fs_status fs_optimal_samples(const double* v_levels, const double* c_levels, int32_t L, double eps2, int32_t n_min,
                             int32_t* n_out, double* mu_out) {
    return guard([&] {
        if (!v_levels || !c_levels || !n_out) fail(FS_E_ARG, "null argument");
        if (L < 0) fail(FS_E_ARG, "L must be >= 0");
        if (!(eps2 > 0) || !std::isfinite(eps2)) fail(FS_E_ARG, "eps2 must be > 0");
        if (n_min < 1) fail(FS_E_ARG, "n_min must be >= 1");
        double sum = 0.0;
        for (int l = 0; l <= L; ++l) {
            if (!(v_levels[l] >= 0) || !std::isfinite(v_levels[l])) fail(FS_E_ARG, "V_l must be finite and >= 0");
            if (!(c_levels[l] > 0) || !std::isfinite(c_levels[l])) fail(FS_E_ARG, "C_l must be finite and > 0");
            sum += std::sqrt(v_levels[l] * c_levels[l]);
        }
        const double mu = sum / eps2;  // Lagrange multiplier of eq. num_samples
        std::vector<int32_t> n(L + 1);
        for (int l = 0; l <= L; ++l) {
            const double x = std::ceil(mu * std::sqrt(v_levels[l] / c_levels[l]));
            if (!(x <= (double)(1 << 24))) fail(FS_E_ARG, "a sample count exceeds 2^24");
            n[l] = std::max<int32_t>(n_min, (int32_t)x);
        }
        std::copy(n.begin(), n.end(), n_out);
        if (mu_out) *mu_out = mu;
    });
}

fs_status fs_batch_destroy(fs_batch b) {
    return guard([&] { delete b; });
}

fs_status fs_time_dslash(fs_ctx c, fs_prec storage, int32_t n_sys, int32_t rhs_block, int32_t wg, int32_t ilp,
                         int32_t occ, int32_t n_launch, double* avg_ms, double* bytes) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        check_prec(storage);
        if (n_sys < 1 || n_launch < 1) fail(FS_E_ARG, "n_sys and n_launch must be >= 1");
        int nr = rhs_block ? rhs_block : tuned_nr(c, storage, n_sys);
        if (!pow2_ok(nr)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
        int w = wg ? wg : tuned_wg(c, storage);
        if (w != 64 && w != 128 && w != 256) fail(FS_E_ARG, "wg must be 64, 128 or 256");
        if (ilp > 2) fail(FS_E_ARG, "ilp must be -1, 0, 1 or 2");
        const int il = ilp < 0 ? tuned_ilp(c, storage) : ilp;
        const int oc = occ < 0 ? tuned_occ(c, storage) : occ;
        if (oc > 8) fail(FS_E_ARG, "occ must be <= 8");
        DeviceScope ds(c->device);
        const double ms = time_dslash_impl(c, storage, n_sys, nr, w, il, oc, n_launch);
        if (avg_ms) *avg_ms = ms;
        if (bytes) *bytes = dslash_bytes(storage, c->V, n_sys, nr, c->two_rows);
    });
}

fs_status fs_time_dslash_eo(fs_ctx c, fs_prec storage, int32_t n_sys, int32_t rhs_block, int32_t occ,
                            int32_t n_launch, double* avg_ms, double* bytes) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        check_prec(storage);
        check_eo(true, c);
        if (n_sys < 1 || n_launch < 1) fail(FS_E_ARG, "n_sys and n_launch must be >= 1");
        const int nr = rhs_block ? rhs_block : tuned_nr(c, storage, n_sys);
        if (!pow2_ok(nr)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
        DeviceScope ds(c->device);
        if (occ > 8) fail(FS_E_ARG, "occ must be -1 (the solver's choice) or 0..8");
        const auto et = eo_tuning(c, storage);
        const double ms = time_dslash_eo_impl(c, storage, n_sys, nr, et[0], occ < 0 ? et[1] : occ, n_launch);
        if (avg_ms) *avg_ms = ms;
        if (bytes) *bytes = dslash_eo_bytes(storage, c->V, n_sys, nr, c->two_rows);
    });
}

fs_status fs_time_dslash_eo_each(fs_ctx c, fs_prec storage, int32_t n_sys, int32_t rhs_block, int32_t n_launch,
                                 float* ms_each, double* bytes) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        check_prec(storage);
        check_eo(true, c);
        if (n_sys < 1 || n_launch < 1 || !ms_each) fail(FS_E_ARG, "n_sys, n_launch >= 1 and ms_each needed");
        const int nr = rhs_block ? rhs_block : tuned_nr(c, storage, n_sys);
        if (!pow2_ok(nr)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
        DeviceScope ds(c->device);
        const auto et = eo_tuning(c, storage);
        std::vector<float> each;
        time_dslash_eo_impl(c, storage, n_sys, nr, et[0], et[1], n_launch, &each);
        std::copy(each.begin(), each.end(), ms_each);
        if (bytes) *bytes = dslash_eo_bytes(storage, c->V, n_sys, nr, c->two_rows);
    });
}

fs_status fs_set_eo_tuning(fs_ctx c, fs_prec storage, int32_t variant, int32_t occ) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        check_prec(storage);
        if (variant != 0 && variant != 2) fail(FS_E_ARG, "even-odd variant must be 0 or 2");
        if (occ < -1 || occ > 8) fail(FS_E_ARG, "occ must be in -1..8");
        c->eo_tune[storage] = {variant, occ};
    });
}

fs_status fs_time_copy(fs_ctx c, uint64_t bytes, int32_t n_launch, double* avg_ms) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        if (bytes < 16 || n_launch < 1 || !avg_ms) fail(FS_E_ARG, "invalid copy size or count");
        DeviceScope ds(c->device);
        const size_t n16 = bytes / 16;
        DevBuf a(n16 * 16), b(n16 * 16);
        HC(hipMemsetAsync(a.p, 0, n16 * 16, c->stream));
        launch_copy(b.as<uint4>(), a.as<uint4>(), n16, c->stream);
        hipEvent_t e0, e1;
        HC(hipEventCreate(&e0));
        HC(hipEventCreate(&e1));
        HC(hipEventRecord(e0, c->stream));
        for (int i = 0; i < n_launch; ++i)
            launch_copy((i & 1) ? a.as<uint4>() : b.as<uint4>(), (i & 1) ? b.as<uint4>() : a.as<uint4>(), n16,
                        c->stream);
        HC(hipEventRecord(e1, c->stream));
        HC(hipEventSynchronize(e1));
        float ms = 0;
        HC(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_ms = (double)ms / n_launch;
    });
}

fs_status fs_set_tuning(fs_ctx c, fs_prec storage, int32_t rhs_block, int32_t wg, int32_t variant, int32_t occ) {
    return guard_ctx(c, [&] {
        check_ctx(c, false);
        check_prec(storage);
        if (!pow2_ok(rhs_block)) fail(FS_E_ARG, "rhs_block must be 1,2,4,8,16");
        if (wg != 64 && wg != 128 && wg != 256) fail(FS_E_ARG, "wg must be 64, 128 or 256");
        if (variant < 0 || variant > 2) fail(FS_E_ARG, "variant must be 0, 1 or 2");
        if (occ < 0 || occ > 8) fail(FS_E_ARG, "occ must be in 0..8");
        TuneEntry e;
        e.nr = rhs_block;
        e.wg = wg;
        e.ilp = variant;
        e.occ = occ;
        c->tune[storage] = e;
    });
}

fs_status fs_autotune(fs_ctx c, fs_prec storage, int32_t n_sys, const char* cache_path, int32_t* best_rhs_block,
                      int32_t* best_wg) {
    return guard_ctx(c, [&] {
        check_ctx(c);
        check_prec(storage);
        if (n_sys < 1) fail(FS_E_ARG, "n_sys must be >= 1");
        DeviceScope ds(c->device);
        hipDeviceProp_t prop;
        HC(hipGetDeviceProperties(&prop, c->device));
        std::string arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
        // batches above 96 systems behave like 96: the resident set is bounded by the chip
        const int n_tune = std::min(n_sys, 96);
        int cls = 1;
        while (cls < n_tune) cls <<= 1;
        std::ostringstream key;
        key << arch << " " << c->dims[0] << " " << c->dims[1] << " " << c->dims[2] << " " << c->dims[3] << " "
            << (int)storage << " " << cls;
        TuneEntry best;
        bool found = false;
        if (cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                if (line.rfind(key.str() + " ", 0) == 0) {
                    std::istringstream ls(line.substr(key.str().size()));
                    TuneEntry e;
                    if (ls >> e.nr >> e.wg >> e.ilp >> e.occ >> e.ms_per_sys && pow2_ok(e.nr) && e.ilp >= 0 && e.ilp <= 2 &&
                        (e.wg == 64 || e.wg == 128 || e.wg == 256) && e.occ >= 0 && e.occ <= 8) {
                        best = e;
                        found = true;
                    }
                }
            }
        }
        if (!found) {
            best.ms_per_sys = 1e30;
            for (int nr : {1, 2, 4, 8, 16}) {
                if (nr > n_tune) break;
                for (int wg : {64, 128, 256})
                    for (int ilp : {0, 1, 2})
                        for (int occ : {0, 1, 2, 4}) {
                            const double ms = time_dslash_impl(c, storage, n_tune, nr, wg, ilp, occ, 8) / n_tune;
                            if (ms < best.ms_per_sys) {
                                best.ms_per_sys = ms;
                                best.nr = nr;
                                best.wg = wg;
                                best.ilp = ilp;
                                best.occ = occ;
                            }
                        }
            }
            if (cache_path) {
                std::ofstream outf(cache_path, std::ios::app);
                outf << key.str() << " " << best.nr << " " << best.wg << " " << best.ilp << " " << best.occ << " "
                     << best.ms_per_sys << "\n";
            }
        }
        c->tune[storage] = best;
        // the even-odd operator of the same rhs block: stencil variant and
        // residency cap, timed as the solver applies it (hop + Schur launch)
        bool eo_ok = true;
        for (int i = 0; i < 4; ++i) eo_ok = eo_ok && c->dims[i] % 2 == 0;
        if (eo_ok) {
            std::ostringstream ekey;
            ekey << "eo " << key.str() << " " << best.nr;
            std::array<int, 2> eb{-1, -1};
            if (cache_path) {
                std::ifstream in(cache_path);
                std::string line;
                while (std::getline(in, line)) {
                    if (line.rfind(ekey.str() + " ", 0) == 0) {
                        std::istringstream ls(line.substr(ekey.str().size()));
                        int v = -1, o = -2;
                        if (ls >> v >> o && (v == 0 || v == 2) && o >= -1 && o <= 8) eb = {v, o};
                    }
                }
            }
            if (eb[0] < 0) {
                double bt = 1e30;
                for (int v : {0, 2})
                    for (int o : {-1, 0, 2, 3, 4}) {
                        const double ms = time_eo_apply_impl(c, storage, n_tune, best.nr, v, o, 6);
                        if (ms < bt) {
                            bt = ms;
                            eb = {v, o};
                        }
                    }
                if (cache_path) {
                    std::ofstream outf(cache_path, std::ios::app);
                    outf << ekey.str() << " " << eb[0] << " " << eb[1] << " " << bt / n_tune << "\n";
                }
            }
            c->eo_tune[storage] = eb;
        }
        if (best_rhs_block) *best_rhs_block = best.nr;
        if (best_wg) *best_wg = best.wg;
    });
}

}  // extern "C"
