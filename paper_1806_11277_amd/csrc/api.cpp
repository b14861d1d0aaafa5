// C ABI of the elastic Helmholtz hybrid MG/DD solver (declared in include/ehh.h).
//
// Host side: validation, the multigrid hierarchy per (sub)domain, the cycle
// sequencing of Algorithm 1 (recursive; one call = V, two = W), the domain
// decomposition around it (section 4, Algorithm 2) and the flexible GMRES loop.
// Every arithmetic step runs in the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include <cxxabi.h>
#include <dlfcn.h>

#include <functional>

#include "ehh.h"
#include "internal.hpp"
#include "launchlog.hpp"
#include "batch.hpp"

// ------------------------------------------------------------------ launch log
// On for the calling thread only, while ehh_profile_precondition runs one
// preconditioner application; the other threads' launches are never recorded.
namespace ehh {
namespace {
struct LogRec {
    const void* kernel;
    LaunchBytes bytes;
    LaunchAgain again;
};
thread_local bool t_log_on = false;
thread_local std::vector<LogRec> t_log;
}  // namespace
thread_local bool t_batch_on = false;
thread_local std::vector<BatchRec> t_batch;
bool launch_log_on() { return t_log_on; }
bool batch_recording() { return t_batch_on; }
void batch_record(BatchRec&& r) { t_batch.push_back(std::move(r)); }
void launch_log_add(const void* kernel, LaunchBytes bytes, LaunchAgain again) {
    t_log.push_back(LogRec{kernel, bytes, std::move(again)});
}
}  // namespace ehh

using namespace ehh;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(EHH_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                      \
    do {                               \
        int32_t s_ = (expr);           \
        if (s_ != EHH_OK) return s_;   \
    } while (0)

// Optional injected allocation failure, for testing the OOM path:
// EHH_FAIL_ALLOC_AFTER=k makes the device allocation that follows k successful
// ones fail, once; the count restarts whenever the variable's value changes
// (read at every allocation), so one process can inject a failure at each
// allocation point in turn.
std::mutex g_inject_mutex;
std::string g_inject_value;
long g_alloc_count = 0;
bool injected_failure() {
    const char* s = std::getenv("EHH_FAIL_ALLOC_AFTER");
    std::lock_guard<std::mutex> l(g_inject_mutex);
    const std::string v = s ? s : "";
    if (v != g_inject_value) {
        g_inject_value = v;
        g_alloc_count = 0;
    }
    if (v.empty()) return false;
    const long lim = std::atol(v.c_str());
    return lim >= 0 && g_alloc_count++ == lim;
}

// Device memory cache.  A setup-solve-destroy cycle would otherwise pay
// hipMalloc for every buffer and hipFree, which waits for the whole device, for
// every release.  Released blocks are kept per device and size class (powers of
// two up to 2 MiB, then multiples of 2 MiB) and handed to later allocations of
// the same class.  The cache holds at most EHH_CACHE_MB MiB (default 32768), is
// emptied for a device when hipMalloc fails there, and
// ehh_release_cached_memory() hands it back to the driver.  A block enters the
// cache only once the device has finished the work queued before its release
// (the callers synchronise the device first).
class BlockCache {
  public:
    static BlockCache& get() {
        static BlockCache c;
        return c;
    }
    static size_t size_class(size_t b) {
        const size_t g = size_t(1) << 21;
        if (b > g) return (b + g - 1) / g * g;
        size_t c = 512;
        while (c < b) c <<= 1;
        return c;
    }
    void* take(int dev, size_t cls) {
        std::lock_guard<std::mutex> l(m_);
        auto it = free_.find({dev, cls});
        if (it == free_.end() || it->second.empty()) return nullptr;
        void* p = it->second.back();
        it->second.pop_back();
        cached_ -= cls;
        return p;
    }
    // false: the cache is full, the caller frees the block
    bool put(int dev, size_t cls, void* p) {
        std::lock_guard<std::mutex> l(m_);
        if (cached_ + cls > cap_) return false;
        free_[{dev, cls}].push_back(p);
        cached_ += cls;
        return true;
    }
    // frees the cached blocks of device dev (every device for dev < 0)
    void trim(int dev) {
        std::vector<std::pair<int, void*>> out;
        {
            std::lock_guard<std::mutex> l(m_);
            for (auto& kv : free_) {
                if (dev >= 0 && kv.first.first != dev) continue;
                for (void* p : kv.second) out.emplace_back(kv.first.first, p);
                cached_ -= kv.first.second * kv.second.size();
                kv.second.clear();
            }
        }
        if (out.empty()) return;
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto& dp : out) {
            (void)hipSetDevice(dp.first);
            (void)hipFree(dp.second);
        }
        (void)hipSetDevice(cur);
    }

  private:
    BlockCache() {
        const char* v = std::getenv("EHH_CACHE_MB");
        cap_ = (size_t)(v ? std::atol(v) : 32768L) << 20;
    }
    std::mutex m_;
    std::map<std::pair<int, size_t>, std::vector<void*>> free_;
    size_t cached_ = 0;
    size_t cap_ = 0;
};

// EHH_LOG=1 prints the setup phases with their durations to stderr.
bool log_enabled() {
    static bool v = [] {
        const char* s = std::getenv("EHH_LOG");
        return s && std::atoi(s) != 0;
    }();
    return v;
}
struct PhaseLog {
    hipStream_t s;
    std::chrono::steady_clock::time_point t0;
    explicit PhaseLog(hipStream_t st) : s(st), t0(std::chrono::steady_clock::now()) {}
    void mark(const char* what) {
        if (!log_enabled()) return;
        (void)hipStreamSynchronize(s);
        const auto t1 = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[ehh] %-40s %9.2f ms\n", what,
                     std::chrono::duration<double, std::milli>(t1 - t0).count());
        std::fflush(stderr);
        t0 = t1;
    }
};

struct Level {
    Geo g{};
    bool fine = false;
    int tune_relax = 0, tune_apply = 0;   // source groups per launch (autotuner; 0: heuristic)
    double damping = 0.0;       // Vanka damping of the displacement rows
    double damping_p = 0.0;     // and of the pressure row
    double* coef64 = nullptr;   // fine: mu, dinv, rho, gam planes; coarse: stencil
    float* coef32 = nullptr;
    void* b = nullptr;          // right-hand side of this level (levels >= 1)
    void* e = nullptr;          // correction of this level (levels >= 1)
    void* t = nullptr;          // half-sweep ping-pong / residual
    // stored row coefficients of the two colours' half-sweeps (cycle precision)
    void* sp_re[2] = {nullptr, nullptr};
    void* sp_im[2] = {nullptr, nullptr};
    int64_t sp_lanes = 0;
    void* rp_re = nullptr;      // stored rows of the residual
    void* rp_im = nullptr;
    bool sp_half = false;       // the rows above hold FP16 values scaled by 1 / sp_scale
    float sp_scale = 1.0f;
};

// DD as the coarsest-grid solver: the boxes (subdomains) of a hierarchy's
// coarsest level, ordered by colour, each with the dense inverse of the
// coarsest operator restricted to it.
struct CoarseBox {
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int colour = 0;
    Geo g{};                    // the box's own grid
    double* inv = nullptr;
    double* sym = nullptr;
    int64_t base = 0;           // first local unknown in the box numbering
};
struct CoarseDD {
    std::vector<CoarseBox> box;
    std::vector<int> col_begin;  // box index where colour c starts (ncol + 1 entries)
    int* idx = nullptr;          // device: map, bsub, bn (int) in one block
    int64_t* bbase = nullptr;    // device: first local unknown of each box
    double* wgt = nullptr;       // device: inverse owner count per coarsest unknown (one colour)
    int64_t ntot = 0;            // local unknowns of all boxes
    bool active() const { return !box.empty(); }
    // idx holds map (ntot), bsub (ntot) and bn (one per box) back to back
    BoxMap view() const { return BoxMap{idx, idx + ntot, bbase, idx + 2 * ntot}; }
};

struct Sub {
    int origin[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    int pad_lo[3] = {0, 0, 0}, pad_hi[3] = {0, 0, 0}, nloc[3] = {1, 1, 1};
    int colour = 0;
    std::vector<Level> lev;
    double* inv = nullptr;      // dense inverse of the coarsest operator
    double* sym = nullptr;      // its lower 64 x 64 tiles, packed (few right-hand sides)
    void* r0 = nullptr;         // local level-0 right-hand side / correction (DD or FP32)
    void* e0 = nullptr;
    CoarseDD cdd;               // DD as the coarsest solver (empty: dense inverse)
    // its FP64 workspaces: right-hand side and iterate (complex64 cycle), residual,
    // and the boxes' local right-hand sides and corrections
    double *cdd_r = nullptr, *cdd_e = nullptr, *cdd_t = nullptr, *cdd_lr = nullptr, *cdd_le = nullptr;
    double* coarse_ws = nullptr;   // partial sums of the split coarse apply (one per subdomain: the
                                   // coarse applies of several subdomains may run in one launch)
};

}  // namespace

struct ehh_ctx {
    ehh_problem_t prob{};
    ehh_options_t opt{};
    int device = 0;             // the device current at setup, which holds every buffer
    int dim = 2;
    Geo gg{};
    double mu_bar = 1, rho_bar = 1, omega_nd = 1;
    double* fine64 = nullptr;
    std::vector<Sub> subs;
    bool dd = false;
    int* cnt_dev = nullptr;
    const int* cnt_cell[3] = {nullptr, nullptr, nullptr};
    const int* cnt_face[3] = {nullptr, nullptr, nullptr};
    int ws_rhs = 0;
    // Krylov workspace
    int kr_rhs = 0;
    double *V = nullptr, *Z = nullptr, *w = nullptr, *R = nullptr, *H = nullptr, *cs = nullptr, *g = nullptr;
    double *hcol = nullptr, *hcol2 = nullptr, *nrm2 = nullptr, *bnorm = nullptr, *est = nullptr, *y = nullptr;
    double *partial = nullptr, *scal = nullptr;
    int *active = nullptr, *ncols = nullptr;
    double* host_pinned = nullptr;
    // g, scal, active and ncols live in one device block, rst_dev, mirrored by
    // the pinned host block rst_host, so that a restart sends them with one
    // asynchronous copy
    void* rst_dev = nullptr;
    char* rst_host = nullptr;
    // conjugated right-hand sides of the adjoint solve
    int adj_rhs = 0;
    double* adjb = nullptr;
    // device buffers of the handle: pointer, device and size class (BlockCache)
    struct Block {
        void* p;
        int dev;
        size_t cls;
    };
    std::vector<Block> allocs;
    // one captured graph per Arnoldi step j for the current batch size
    int graph_rhs = 0;
    std::vector<hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;

    ~ehh_ctx() {
        clear_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        std::vector<int> devs;
        for (const Block& b : allocs)
            if (std::find(devs.begin(), devs.end(), b.dev) == devs.end()) devs.push_back(b.dev);
        for (int d : devs) sync_device(d);
        for (const Block& b : allocs) give_back(b);
        if (host_pinned) (void)hipHostFree(host_pinned);
        if (rst_host) (void)hipHostFree(rst_host);
    }
    // waits for the work queued on device d (the buffers' device, which need not
    // be the current one)
    static void sync_device(int d) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != d) (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
        if (cur != d) (void)hipSetDevice(cur);
    }
    static void give_back(const Block& b) {
        if (!BlockCache::get().put(b.dev, b.cls, b.p)) (void)hipFree(b.p);
    }
    void clear_graphs() {
        for (hipGraphExec_t e : graphs)
            if (e) (void)hipGraphExecDestroy(e);
        graphs.clear();
        graph_rhs = 0;
    }

    int32_t alloc(void** p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        if (injected_failure()) return fail(EHH_ERR_OOM, "injected allocation failure");
        int dev = 0;
        (void)hipGetDevice(&dev);
        const size_t cls = BlockCache::size_class(bytes);
        *p = BlockCache::get().take(dev, cls);
        if (!*p) {
            hipError_t e = hipMalloc(p, cls);
            if (e != hipSuccess) {   // return the cached blocks to the driver and try once more
                (void)hipGetLastError();
                BlockCache::get().trim(dev);
                e = hipMalloc(p, cls);
            }
            if (e != hipSuccess) {
                *p = nullptr;
                (void)hipGetLastError();
                return fail(EHH_ERR_OOM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
            }
        }
        allocs.push_back(Block{*p, dev, cls});
        return EHH_OK;
    }
    void release(void* p) {
        if (!p) return;
        auto it = std::find_if(allocs.begin(), allocs.end(), [p](const Block& b) { return b.p == p; });
        if (it == allocs.end()) {
            (void)hipFree(p);
            return;
        }
        const Block b = *it;
        allocs.erase(it);
        sync_device(b.dev);   // work queued before the release may still read the block
        give_back(b);
    }
    int bits() const { return opt.precond_bits; }
};

namespace {

template <typename T> const T* coef_of(const Level& L);
template <> const double* coef_of<double>(const Level& L) { return L.coef64; }
template <> const float* coef_of<float>(const Level& L) { return L.coef32; }

template <typename T> LevelDesc<T> level_desc(const ehh_ctx* c, const Level& L, double alpha) {
    LevelDesc<T> d{};
    d.g = L.g;
    d.fine = L.fine;
    d.tune_relax = L.tune_relax;
    d.tune_apply = L.tune_apply;
    const T* base = coef_of<T>(L);
    if (L.fine) {
        const int64_t n = L.g.ncell;
        d.f = FineCoef<T>{base, base + n, base + 2 * n, base + 3 * n, (T)(c->omega_nd * c->omega_nd), (T)alpha};
    } else {
        if (L.g.dim == 2)
            d.s = stencil_view<2, T>(L.g, base);
        else
            d.s = stencil_view<3, T>(L.g, base);
        const bool mine = (sizeof(T) == 4) == (c->bits() == 32);   // rows are kept in the cycle precision
        if (mine && L.sp_lanes)
            for (int col = 0; col < 2; ++col) {
                d.sp.re[col] = (const T*)L.sp_re[col];
                d.sp.im[col] = (const T*)L.sp_im[col];
            }
        d.sp.lanes = L.sp_lanes;
        if (mine && L.rp_re) {
            d.sp.rre = (const T*)L.rp_re;
            d.sp.rim = (const T*)L.rp_im;
        }
        d.sp.half = mine && L.sp_half;
        d.sp.scale = L.sp_scale;
    }
    return d;
}

int64_t stencil_size(const Geo& g) { return g.dim == 2 ? stencil_reals<2>(g) : stencil_reals<3>(g); }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// --------------------------------------------------------------- workspaces
int32_t ensure_ws(ehh_ctx* c, int nrhs) {
    if (nrhs <= c->ws_rhs) return EHH_OK;
    c->clear_graphs();
    // a growth that fails part way leaves no capacity behind, so that the next
    // call allocates again instead of using released buffers
    c->ws_rhs = 0;
    const size_t es = c->bits() == 32 ? sizeof(float) : sizeof(double);
    for (Sub& S : c->subs) {
        for (size_t l = 0; l < S.lev.size(); ++l) {
            Level& L = S.lev[l];
            const size_t bytes = es * 2 * (size_t)L.g.N * nrhs;
            c->release(L.b);
            c->release(L.e);
            c->release(L.t);
            L.b = L.e = L.t = nullptr;
            CHK(c->alloc(&L.t, bytes));
            if (l > 0) {
                CHK(c->alloc(&L.b, bytes));
                CHK(c->alloc(&L.e, bytes));
            }
        }
        c->release(S.r0);
        c->release(S.e0);
        S.r0 = S.e0 = nullptr;
        const size_t b0 = es * 2 * (size_t)S.lev[0].g.N * nrhs;
        CHK(c->alloc(&S.r0, b0));
        CHK(c->alloc(&S.e0, b0));
        for (double** p : {&S.cdd_r, &S.cdd_e, &S.cdd_t, &S.cdd_lr, &S.cdd_le}) {
            c->release(*p);
            *p = nullptr;
        }
        if (S.cdd.active()) {
            const size_t bc = sizeof(double) * 2 * (size_t)S.lev.back().g.N * nrhs;
            const size_t bl = sizeof(double) * 2 * (size_t)S.cdd.ntot * nrhs;
            CHK(c->alloc((void**)&S.cdd_r, bc));
            CHK(c->alloc((void**)&S.cdd_e, bc));
            CHK(c->alloc((void**)&S.cdd_t, bc));
            CHK(c->alloc((void**)&S.cdd_lr, bl));
            CHK(c->alloc((void**)&S.cdd_le, bl));
        }
    }
    // the split depends on the batch size: cover every batch up to nrhs
    for (Sub& S : c->subs) {
        size_t cw = 0;
        for (int q = 1; q <= nrhs; ++q) {
            if (S.cdd.active())
                for (const CoarseBox& B : S.cdd.box) cw = std::max(cw, coarse_ws_doubles(B.g.N, q));
            else
                cw = std::max(cw, coarse_ws_doubles(S.lev.back().g.N, q));
        }
        c->release(S.coarse_ws);
        S.coarse_ws = nullptr;
        if (cw) CHK(c->alloc((void**)&S.coarse_ws, sizeof(double) * cw));
    }
    c->ws_rhs = nrhs;
    return EHH_OK;
}

// bytes of the restart block: g (2 nrhs (m + 1) doubles), scal (nrhs doubles),
// active and ncols (nrhs ints each)
size_t restart_block_bytes(int nrhs, int m) {
    return sizeof(double) * (2 * (size_t)nrhs * (m + 1) + nrhs) + 2 * sizeof(int) * (size_t)nrhs;
}

int32_t ensure_krylov(ehh_ctx* c, int nrhs) {
    if (nrhs <= c->kr_rhs) return EHH_OK;
    c->clear_graphs();
    c->kr_rhs = 0;   // as in ensure_ws: a failed growth leaves no capacity
    const int m = c->opt.restart;
    const size_t vec = 2 * (size_t)c->gg.N * nrhs * sizeof(double);
    double** bufs[] = {&c->V, &c->Z, &c->w, &c->R, &c->H, &c->cs, &c->hcol, &c->hcol2, &c->nrm2,
                       &c->bnorm, &c->est, &c->y, &c->partial};
    for (double** b : bufs) {
        c->release(*b);
        *b = nullptr;
    }
    c->release(c->rst_dev);
    c->rst_dev = nullptr;
    c->g = c->scal = nullptr;
    c->active = c->ncols = nullptr;
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    c->host_pinned = nullptr;
    if (c->rst_host) (void)hipHostFree(c->rst_host);
    c->rst_host = nullptr;
    const int nb = krylov_blocks(c->gg.N);
    CHK(c->alloc((void**)&c->V, vec * (m + 1)));
    CHK(c->alloc((void**)&c->Z, vec * m));
    CHK(c->alloc((void**)&c->w, vec));
    CHK(c->alloc((void**)&c->R, vec));
    CHK(c->alloc((void**)&c->H, sizeof(double) * 2 * (size_t)nrhs * m * (m + 1)));
    CHK(c->alloc((void**)&c->cs, sizeof(double) * 3 * (size_t)nrhs * m));
    CHK(c->alloc((void**)&c->hcol, sizeof(double) * 2 * (size_t)nrhs * (m + 1)));
    CHK(c->alloc((void**)&c->hcol2, sizeof(double) * 2 * (size_t)nrhs * (m + 1)));
    CHK(c->alloc((void**)&c->nrm2, sizeof(double) * nrhs));
    CHK(c->alloc((void**)&c->bnorm, sizeof(double) * nrhs));
    CHK(c->alloc((void**)&c->est, sizeof(double) * nrhs));
    CHK(c->alloc((void**)&c->y, sizeof(double) * 2 * (size_t)nrhs * m));
    CHK(c->alloc((void**)&c->partial, sizeof(double) * (size_t)nb * nrhs * (m + 1) * 2));
    const size_t rst_bytes = restart_block_bytes(nrhs, m);
    CHK(c->alloc(&c->rst_dev, rst_bytes));
    c->g = (double*)c->rst_dev;
    c->scal = c->g + 2 * (size_t)nrhs * (m + 1);
    c->active = (int*)(c->scal + nrhs);
    c->ncols = c->active + nrhs;
    hipError_t e = hipHostMalloc((void**)&c->host_pinned, sizeof(double) * 4 * nrhs);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->rst_host, rst_bytes);
    if (e != hipSuccess) {
        return fail(EHH_ERR_OOM, "hipHostMalloc failed");
    }
    c->kr_rhs = nrhs;
    return EHH_OK;
}

// ------------------------------------------------------------------- the cycle
// The coarsest solve: e = A_c^{-1} b by the dense inverse, or one sweep of the
// coarsest level's DD (section 4), in FP64, from e = 0 (zero_init) or continuing
// from e (a W-cycle's second call).
template <typename T>
int32_t coarse_solve(ehh_ctx* c, Sub& S, const T* b, T* e, bool zero_init, int nrhs, hipStream_t s) {
    Level& L = S.lev.back();
    const int64_t Nc = L.g.N;
    if (!S.cdd.active()) {
        HIPCHK(launch_coarse_apply<T>(S.inv, S.sym, Nc, b, e, nrhs, S.coarse_ws, s));
        return EHH_OK;
    }
    const CoarseDD& D = S.cdd;
    const BoxMap M = D.view();
    const double* r;
    double* z;
    if constexpr (std::is_same<T, double>::value) {
        r = b;
        z = e;
    } else {
        HIPCHK(launch_cast_f2d(b, S.cdd_r, 2 * Nc * nrhs, s));
        if (!zero_init) HIPCHK(launch_cast_f2d(e, S.cdd_e, 2 * Nc * nrhs, s));
        r = S.cdd_r;
        z = S.cdd_e;
    }
    if (zero_init) HIPCHK(launch_zero(z, sizeof(double) * 2 * (size_t)Nc * nrhs, s));
    const LevelDesc<double> A = level_desc<double>(c, L, c->prob.shift);
    const bool one = c->opt.coarse_dd_colors == 1;
    const int ncol = one ? 1 : (int)D.col_begin.size() - 1;
    for (int col = 0; col < ncol; ++col) {
        const int b0 = one ? 0 : D.col_begin[col], b1 = one ? (int)D.box.size() : D.col_begin[col + 1];
        const double* src = r;
        if (!(col == 0 && zero_init)) {   // the residual left by the previous colours
            HIPCHK(launch_apply<double>(A, z, r, S.cdd_t, nrhs, s));
            src = S.cdd_t;
        }
        const int64_t j0 = D.box[b0].base, j1 = b1 < (int)D.box.size() ? D.box[b1].base : D.ntot;
        HIPCHK(launch_box_gather(M, j0, j1, src, Nc, S.cdd_lr, nrhs, s));
        for (int bi = b0; bi < b1; ++bi) {
            const CoarseBox& B = D.box[bi];
            const size_t off = 2 * (size_t)nrhs * B.base;
            HIPCHK(launch_coarse_apply<double>(B.inv, B.sym, B.g.N, S.cdd_lr + off, S.cdd_le + off, nrhs,
                                               S.coarse_ws, s));
        }
        if (one)   // the boxes overlap: one scatter per box, in turn
            for (int bi = b0; bi < b1; ++bi) {
                const int64_t k0 = D.box[bi].base, k1 = bi + 1 < (int)D.box.size() ? D.box[bi + 1].base : D.ntot;
                HIPCHK(launch_box_scatter(M, k0, k1, S.cdd_le, D.wgt, Nc, z, nrhs, s));
            }
        else       // the boxes of one colour are disjoint
            HIPCHK(launch_box_scatter(M, j0, j1, S.cdd_le, nullptr, Nc, z, nrhs, s));
    }
    if constexpr (!std::is_same<T, double>::value) HIPCHK(launch_cast_d2f(z, e, 2 * Nc * nrhs, s));
    return EHH_OK;
}

template <typename T>
int32_t cycle(ehh_ctx* c, Sub& S, int l, const T* b, T* e, bool zero_init, int nrhs, hipStream_t s,
              const T* rsrc = nullptr, const Geo* gsrc = nullptr, double* z64 = nullptr, bool* wrote64 = nullptr) {
    // z64 (level 0 of a complex64 cycle): where the kernels allow it, the last
    // half-sweep writes its result there in FP64 (*wrote64 set) instead of to e
    // rsrc: the finer level's residual (grid gsrc) when b = P^T rsrc is still to be
    // formed; the first half-sweep then forms and writes it (zero_init, nu1 >= 1)
    Level& L = S.lev[l];
    const int nl = (int)S.lev.size();
    if (l == nl - 1) return coarse_solve<T>(c, S, b, e, zero_init, nrhs, s);
    const LevelDesc<T> D = level_desc<T>(c, L, c->prob.shift);
    const int econ = c->opt.vanka == 0;
    T* t = (T*)L.t;
    bool have = !zero_init;
    for (int it = 0; it < c->opt.nu1; ++it) {
        if (it == 0 && rsrc)
            HIPCHK(launch_relax_restrict<T>(D, Damp{L.damping, L.damping_p}, econ, *gsrc, rsrc, (T*)b, t, nrhs, s));
        else
            HIPCHK(launch_relax<T>(D, 0, Damp{L.damping, L.damping_p}, econ, b, have ? e : nullptr, t, nrhs, s));
        HIPCHK(launch_relax<T>(D, 1, Damp{L.damping, L.damping_p}, econ, b, t, e, nrhs, s));
        have = true;
    }
    Level& C = S.lev[l + 1];
    // the restriction to a coarser level that is not the coarsest is fused into
    // that level's first half-sweep where its kernels allow it
    const bool fuse = l + 1 < nl - 1 && c->opt.nu1 >= 1 &&
                      relax_restrict_supported<T>(level_desc<T>(c, C, c->prob.shift), L.g, nrhs);
    if (have) {
        bool done = false;   // C.b = P^T (b - A e) in one launch where the kernels allow it
        if (!fuse) HIPCHK(launch_residual_restrict<T>(D, C.g, e, b, (T*)C.b, nrhs, s, &done));
        if (!done) {
            HIPCHK(launch_apply<T>(D, e, b, t, nrhs, s));   // t = b - A e
            if (!fuse) HIPCHK(launch_restrict<T>(L.g, C.g, t, (T*)C.b, nrhs, s));
        }
    } else {
        HIPCHK(launch_zero(e, sizeof(T) * 2 * (size_t)L.g.N * nrhs, s));
        if (!fuse) HIPCHK(launch_restrict<T>(L.g, C.g, b, (T*)C.b, nrhs, s));
    }
    const T* rfine = have ? (const T*)t : b;
    // gamma_c recursive calls (V: 1, W: 2); an exact coarsest solve would repeat
    // the same result in a second call, a DD coarsest solve continues from it.
    const bool exact_next = l + 1 == nl - 1 && !S.cdd.active();
    const int ncall = (exact_next || l < c->opt.cycle_level) ? 1 : c->opt.cycle;
    for (int k = 0; k < ncall; ++k)
        CHK(cycle<T>(c, S, l + 1, (const T*)C.b, (T*)C.e, k == 0, nrhs, s, (k == 0 && fuse) ? rfine : nullptr,
                     &L.g));
    HIPCHK(launch_prolong<T>(L.g, C.g, (const T*)C.e, e, nrhs, s));
    for (int it = 0; it < c->opt.nu2; ++it) {
        HIPCHK(launch_relax<T>(D, 0, Damp{L.damping, L.damping_p}, econ, b, e, t, nrhs, s));
        bool done = false;
        if constexpr (std::is_same<T, float>::value) {
            if (z64 && it == c->opt.nu2 - 1)
                HIPCHK(launch_relax_to64(D, Damp{L.damping, L.damping_p}, econ, b, t, z64, nrhs, s, &done));
        }
        if (done)
            *wrote64 = true;
        else
            HIPCHK(launch_relax<T>(D, 1, Damp{L.damping, L.damping_p}, econ, b, t, e, nrhs, s));
    }
    return EHH_OK;
}

SubMap submap(const ehh_ctx* c, const Sub& S) {
    SubMap m{};
    m.dim = c->dim;
    for (int a = 0; a < 3; ++a) {
        m.origin[a] = S.origin[a];
        m.lo[a] = S.lo[a];
        m.hi[a] = S.hi[a];
        m.cnt_cell[a] = c->cnt_cell[a];
        m.cnt_face[a] = c->cnt_face[a];
    }
    return m;
}

// Runs fn(S) for every subdomain of subs with the kernel launches recorded, then
// launches position k of every subdomain's launch sequence as one batch launch
// (the same step of all subdomains in one launch over a flat (subdomain, block)
// list).  The sequences coincide when the subdomains' levels take the same
// kernels; where they do not, every subdomain's steps are launched on their own.
int32_t run_batched(ehh_ctx* c, const std::vector<Sub*>& subs, const std::function<int32_t(Sub&)>& fn,
                    hipStream_t s) {
    if (subs.size() == 1 || !c->opt.dd_batch) {
        for (Sub* S : subs) CHK(fn(*S));
        return EHH_OK;
    }
    std::vector<std::vector<BatchRec>> seq(subs.size());
    for (size_t i = 0; i < subs.size(); ++i) {
        t_batch.clear();
        t_batch_on = true;
        const int32_t st = fn(*subs[i]);
        t_batch_on = false;
        seq[i].swap(t_batch);
        if (st != EHH_OK) return st;
    }
    bool same = true;
    for (const auto& q : seq) {
        if (q.size() != seq[0].size()) {
            same = false;
            break;
        }
        for (size_t k = 0; k < q.size() && same; ++k)
            same = q[k].kernel == seq[0][k].kernel && q[k].block.x == seq[0][k].block.x &&
                   q[k].shmem == seq[0][k].shmem;
    }
    if (!same) {
        for (const auto& q : seq)
            for (const BatchRec& r : q) {
                const BatchRec* one = &r;
                HIPCHK(r.launch(&one, 1, s));
            }
        return EHH_OK;
    }
    std::vector<const BatchRec*> recs;
    for (size_t k = 0; k < seq[0].size(); ++k)
        for (size_t i0 = 0; i0 < seq.size(); i0 += kMaxBatch) {
            recs.clear();
            for (size_t i = i0; i < seq.size() && i < i0 + kMaxBatch; ++i) recs.push_back(&seq[i][k]);
            HIPCHK(recs[0]->launch(recs.data(), (int)recs.size(), s));
        }
    return EHH_OK;
}

// z = M^{-1} v (FP64 global vectors).
// v_in_r0: the complex64 copy of v is already in the cycle's input buffer
// (written by the scaling that produced v).
template <typename T>
int32_t precondition_t(ehh_ctx* c, const double* v, double* z, int nrhs, hipStream_t s, bool v_in_r0) {
    const Geo& gg = c->gg;
    if (!c->dd) {
        Sub& S = c->subs[0];
        if (std::is_same<T, double>::value) {
            return cycle<T>(c, S, 0, (const T*)v, (T*)z, true, nrhs, s);
        }
        if (!v_in_r0) HIPCHK(launch_cast_d2f(v, (float*)S.r0, 2 * gg.N * nrhs, s));
        bool wrote = false;
        CHK(cycle<T>(c, S, 0, (const T*)S.r0, (T*)S.e0, true, nrhs, s, nullptr, nullptr, z, &wrote));
        if (!wrote) HIPCHK(launch_cast_f2d((const float*)S.e0, z, 2 * gg.N * nrhs, s));
        return EHH_OK;
    }
    HIPCHK(launch_zero(z, sizeof(double) * 2 * (size_t)gg.N * nrhs, s));
    if (c->opt.dd_colors == 1) {
        std::vector<Sub*> all;
        for (Sub& S : c->subs) all.push_back(&S);
        // the gathers and cycles of all subdomains in batch launches; the averaging
        // scatters one subdomain at a time, their extents overlapping
        CHK(run_batched(c, all, [&](Sub& S) -> int32_t {
            HIPCHK(launch_dd_gather<T>(gg, S.lev[0].g, submap(c, S), v, (T*)S.r0, nrhs, s));
            return cycle<T>(c, S, 0, (const T*)S.r0, (T*)S.e0, true, nrhs, s);
        }, s));
        for (Sub& S : c->subs)
            HIPCHK(launch_dd_scatter<T>(gg, S.lev[0].g, submap(c, S), (const T*)S.e0, z, nrhs, 1, s));
        return EHH_OK;
    }
    // Algorithm 2: colours in turn, each from the residual of the unshifted operator
    int ncol = 0;
    for (const Sub& S : c->subs) ncol = std::max(ncol, S.colour + 1);
    LevelDesc<double> A{};
    A.g = gg;
    A.fine = true;
    const int64_t n = gg.ncell;
    A.f = FineCoef<double>{c->fine64, c->fine64 + n, c->fine64 + 2 * n, c->fine64 + 3 * n,
                           c->omega_nd * c->omega_nd, 0.0};
    for (int col = 0; col < ncol; ++col) {
        std::vector<Sub*> mine;
        for (Sub& S : c->subs)
            if (S.colour == col) mine.push_back(&S);
        // every subdomain of the colour takes its residual before any of them
        // adds its correction: the merged launches keep that order (all gathers,
        // then each cycle step, then all scatters, the colour's extents disjoint)
        CHK(run_batched(c, mine, [&](Sub& S) -> int32_t {
            const SubMap m = submap(c, S);
            if (col == 0)   // z = 0: the local residual is v itself
                HIPCHK(launch_dd_gather<T>(gg, S.lev[0].g, m, v, (T*)S.r0, nrhs, s));
            else            // local residual of the unshifted operator on the extent only
                HIPCHK(launch_dd_gather_res<T>(gg, S.lev[0].g, m, A.f, v, z, (T*)S.r0, nrhs, s));
            CHK(cycle<T>(c, S, 0, (const T*)S.r0, (T*)S.e0, true, nrhs, s));
            HIPCHK(launch_dd_scatter<T>(gg, S.lev[0].g, m, (const T*)S.e0, z, nrhs, 0, s));
            return EHH_OK;
        }, s));
    }
    return EHH_OK;
}

int32_t precondition_any(ehh_ctx* c, const double* v, double* z, int nrhs, hipStream_t s, bool v_in_r0 = false) {
    CHK(ensure_ws(c, nrhs));
    return c->bits() == 32 ? precondition_t<float>(c, v, z, nrhs, s, v_in_r0)
                           : precondition_t<double>(c, v, z, nrhs, s, false);
}

// FP32 copy of the Krylov vector for the complex64 cycle, written by the
// scaling kernel (global preconditioner only; with subdomains the gather casts).
float* krylov_copy32(ehh_ctx* c) { return (c->bits() == 32 && !c->dd) ? (float*)c->subs[0].r0 : nullptr; }

// ------------------------------------------------------------------ validation
int32_t check_problem(const ehh_problem_t* p, const ehh_options_t* o) {
    if (!p || !o) return fail(EHH_ERR_INVALID, "null problem or options");
    if (p->dim != 2 && p->dim != 3) return fail(EHH_ERR_INVALID, "dim must be 2 or 3");
    for (int a = 0; a < p->dim; ++a) {
        if (p->n[a] < 2 || p->n[a] > (1 << 20)) return fail(EHH_ERR_INVALID, "each n[a] must be in [2, 2^20]");
        if (p->abl_cells[a] < 0 || p->abl_cells[a] > p->n[a]) return fail(EHH_ERR_INVALID, "abl_cells out of range");
    }
    if (!(p->h > 0) || !(p->omega > 0) || !(p->shift >= 0) || !(p->abl_max >= 0) || !(p->atten0 >= 0) ||
        !std::isfinite(p->h) || !std::isfinite(p->omega) || !std::isfinite(p->shift) || !std::isfinite(p->abl_max) ||
        !std::isfinite(p->atten0))
        return fail(EHH_ERR_INVALID, "h, omega > 0 and shift, abl_max, atten0 >= 0 (finite) required");
    if (!(p->mu_bar >= 0) || !(p->rho_bar >= 0) || !std::isfinite(p->mu_bar) || !std::isfinite(p->rho_bar))
        return fail(EHH_ERR_INVALID, "mu_bar, rho_bar must be finite and >= 0 (0 = media means)");
    if (o->levels < 1 || o->levels > EHH_MAX_LEVELS) return fail(EHH_ERR_INVALID, "levels out of range");
    if (o->cycle != 1 && o->cycle != 2) return fail(EHH_ERR_INVALID, "cycle must be 1 (V) or 2 (W)");
    if (o->cycle_level < 0 || o->cycle_level >= EHH_MAX_LEVELS) return fail(EHH_ERR_INVALID, "cycle_level out of range");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 8 || o->nu2 > 8) return fail(EHH_ERR_INVALID, "nu1, nu2 in [0, 8]");
    if (o->vanka != 0 && o->vanka != 1) return fail(EHH_ERR_INVALID, "vanka must be 0 or 1");
    if (o->precond_bits != 32 && o->precond_bits != 64) return fail(EHH_ERR_INVALID, "precond_bits must be 32 or 64");
    if (o->coarse_bits != 16 && o->coarse_bits != 32) return fail(EHH_ERR_INVALID, "coarse_bits must be 16 or 32");
    if (o->coarse_bits == 16 && o->precond_bits != 32)
        return fail(EHH_ERR_INVALID, "coarse_bits = 16 needs the complex64 cycle (precond_bits = 32)");
    if (o->restart < 1 || o->restart > EHH_MAX_RESTART) return fail(EHH_ERR_INVALID, "restart out of range");
    for (int a = 0; a < p->dim; ++a)
        if (o->coarse_dd_parts[a] < 1) return fail(EHH_ERR_INVALID, "coarse_dd_parts must be >= 1");
    if (o->coarse_dd_overlap < 0) return fail(EHH_ERR_INVALID, "coarse_dd_overlap >= 0");
    if (o->coarse_dd_colors != 0 && o->coarse_dd_colors != 1) return fail(EHH_ERR_INVALID, "coarse_dd_colors must be 0 or 1");
    if (o->dd_batch != 0 && o->dd_batch != 1) return fail(EHH_ERR_INVALID, "dd_batch must be 0 or 1");
    if (o->reorth != 0 && o->reorth != 1) return fail(EHH_ERR_INVALID, "reorth must be 0 or 1");
    for (int a = 0; a < p->dim; ++a)
        if (o->dd_parts[a] < 1 || o->dd_parts[a] > p->n[a]) return fail(EHH_ERR_INVALID, "dd_parts out of range");
    if (o->dd_overlap < 0 || o->dd_pad < 0) return fail(EHH_ERR_INVALID, "dd_overlap, dd_pad >= 0");
    if (o->dd_colors != 0 && o->dd_colors != 1) return fail(EHH_ERR_INVALID, "dd_colors must be 0 or 1");
    for (int l = 0; l < o->levels - 1; ++l) {
        if (!(o->damping[l] > 0 && o->damping[l] <= 2)) return fail(EHH_ERR_INVALID, "damping must be in (0, 2]");
        if (!(o->damping_p[l] >= 0 && o->damping_p[l] <= 2))
            return fail(EHH_ERR_INVALID, "damping_p must be in (0, 2] (0: as damping)");
    }
    return EHH_OK;
}

// Subdomain extents per axis: core = n / parts, overlap split around the cut,
// absorbing padding on interior sides only.
void make_subdomains(ehh_ctx* c) {
    const int d = c->dim;
    int parts[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) parts[a] = c->opt.dd_parts[a];
    const int ov = c->opt.dd_overlap, pad = c->opt.dd_pad;
    const int nz = d == 3 ? parts[2] : 1;
    for (int pz = 0; pz < nz; ++pz)
        for (int py = 0; py < parts[1]; ++py)
            for (int px = 0; px < parts[0]; ++px) {
                Sub S;
                const int idx[3] = {px, py, pz};
                for (int a = 0; a < 3; ++a) {
                    if (a >= d) {
                        S.lo[a] = 0;
                        S.hi[a] = 1;
                        S.nloc[a] = 1;
                        continue;
                    }
                    const int n = c->prob.n[a], P = parts[a], p = idx[a];
                    const int core = n / P;
                    int lo = std::max(0, p * core - ov / 2);
                    int hi = p < P - 1 ? std::min(n, (p + 1) * core + (ov - ov / 2)) : n;
                    if (p == 0) lo = 0;
                    S.lo[a] = lo;
                    S.hi[a] = hi;
                    S.pad_lo[a] = lo > 0 ? pad : 0;
                    S.pad_hi[a] = hi < n ? pad : 0;
                    S.origin[a] = lo - S.pad_lo[a];
                    S.nloc[a] = hi - lo + S.pad_lo[a] + S.pad_hi[a];
                }
                S.colour = (px % 2) + 2 * (py % 2) + 4 * (pz % 2);
                c->subs.push_back(std::move(S));
            }
}


// FP16 storage of a Galerkin level's stored rows (coarse_bits = 16, section 3
// of the paper suggests half precision for the coarse data): every row array
// is divided by one power-of-two scale that brings the largest modulus to
// about 2^14, rounded to FP16, and the FP32 arrays are released.
int32_t rows_to_half(ehh_ctx* c, Level& Q, int NT, int NF, int64_t lanes, hipStream_t s) {
    const int64_t N = Q.g.N;
    void** arrs[6] = {&Q.sp_re[0], &Q.sp_im[0], &Q.sp_re[1], &Q.sp_im[1], &Q.rp_re, &Q.rp_im};
    const int64_t cnt[6] = {NT * lanes, NF * lanes, NT * lanes, NF * lanes, NT * N, NF * N};
    unsigned* mx = nullptr;
    CHK(c->alloc((void**)&mx, sizeof(unsigned)));
    HIPCHK(hipMemsetAsync(mx, 0, sizeof(unsigned), s));
    for (int a = 0; a < 6; ++a) HIPCHK(launch_absmax_bits((const float*)*arrs[a], cnt[a], mx, s));
    unsigned bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, mx, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    c->release(mx);
    float amax = 0.0f;
    std::memcpy(&amax, &bits, sizeof(float));
    if (!std::isfinite(amax)) return fail(EHH_ERR_BREAKDOWN, "non-finite coarse-level coefficient");
    const float scale = amax > 0.0f ? std::ldexp(1.0f, std::ilogb(amax) - 14) : 1.0f;
    for (int a = 0; a < 6; ++a) {
        void* h = nullptr;
        CHK(c->alloc(&h, sizeof(uint16_t) * cnt[a]));
        HIPCHK(launch_to_half((const float*)*arrs[a], h, cnt[a], 1.0f / scale, s));
        HIPCHK(hipStreamSynchronize(s));
        c->release(*arrs[a]);
        *arrs[a] = h;
    }
    Q.sp_half = true;
    Q.sp_scale = scale;
    return EHH_OK;
}

// Dense inverse of the operator of a stencil-format level (grid g, FP64 stencil
// st) and its lower 64 x 64 tiles packed.
int32_t build_dense_inverse(ehh_ctx* c, const Geo& g, const double* st, double** inv_out, double** sym_out,
                            hipStream_t s) {
    const int64_t nc = g.N;
    if ((double)nc * nc * 16.0 > 2.4e10)
        return fail(EHH_ERR_UNSUPPORTED, "coarsest grid too large for a dense inverse (24 GB)");
    double* inv0 = nullptr;
    CHK(c->alloc((void**)&inv0, sizeof(double) * 2 * nc * nc));
    HIPCHK(launch_dense_assemble(g, st, inv0, s));
    int* piv = nullptr;
    CHK(c->alloc((void**)&piv, sizeof(int) * (nc + 1)));
    HIPCHK(launch_dense_invert(inv0, nc, piv, piv + nc, s));
    std::vector<int> hp(nc + 1);
    HIPCHK(hipMemcpyAsync(hp.data(), piv, sizeof(int) * (nc + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hp[nc]) {
        c->release(piv);
        c->release(inv0);
        return fail(EHH_ERR_BREAKDOWN, "singular coarsest operator");
    }
    // A^{-1} = (Pi A)^{-1} Pi: column q[k] of A^{-1} is column k of the result,
    // with q the row order after the interchanges.
    std::vector<int> q(nc), qinv(nc);
    for (int64_t k = 0; k < nc; ++k) q[k] = (int)k;
    for (int64_t k = 0; k < nc; ++k) std::swap(q[k], q[hp[k]]);
    for (int64_t k = 0; k < nc; ++k) qinv[q[k]] = (int)k;
    HIPCHK(hipMemcpyAsync(piv, qinv.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
    double* inv = nullptr;
    CHK(c->alloc((void**)&inv, sizeof(double) * 2 * nc * nc));
    HIPCHK(launch_permute_columns(inv0, inv, nc, piv, s));
    HIPCHK(hipStreamSynchronize(s));
    c->release(inv0);
    double* sym = nullptr;
    CHK(c->alloc((void**)&sym, sizeof(double) * 2 * 64 * 64 * sym_tiles(nc)));
    HIPCHK(launch_pack_sym(inv, nc, sym, s));
    c->release(piv);
    *inv_out = inv;
    *sym_out = sym;
    return EHH_OK;
}

// Boxes (subdomains) of the coarsest level gc with their index maps and the
// dense inverses of the restricted operators (DD as the coarsest solver).
// Extents per axis as for the fine subdomains without padding: core n / parts,
// the overlap split around each cut; colour = parity of the box index per axis.
int32_t build_coarse_dd(ehh_ctx* c, Sub& S, const Geo& gc, const double* stc, hipStream_t s) {
    const int d = c->dim, ov = c->opt.coarse_dd_overlap;
    int parts[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
        parts[a] = c->opt.coarse_dd_parts[a];
        if (parts[a] > gc.n[a]) return fail(EHH_ERR_INVALID, "coarse_dd_parts exceeds the coarsest grid");
        if (parts[a] > 1 && gc.n[a] / parts[a] <= ov)
            return fail(EHH_ERR_INVALID, "coarse_dd_overlap must be smaller than a coarsest subdomain's core");
    }
    CoarseDD& D = S.cdd;
    std::vector<CoarseBox> boxes;
    for (int pz = 0; pz < parts[2]; ++pz)
        for (int py = 0; py < parts[1]; ++py)
            for (int px = 0; px < parts[0]; ++px) {
                CoarseBox B;
                const int idx[3] = {px, py, pz};
                int nb[3] = {1, 1, 1};
                for (int a = 0; a < d; ++a) {
                    const int n = gc.n[a], P = parts[a], p = idx[a], core = n / P;
                    B.lo[a] = p == 0 ? 0 : std::max(0, p * core - ov / 2);
                    B.hi[a] = p < P - 1 ? std::min(n, (p + 1) * core + (ov - ov / 2)) : n;
                    nb[a] = B.hi[a] - B.lo[a];
                }
                B.colour = (px % 2) + 2 * (py % 2) + 4 * (pz % 2);
                B.g = make_geo(d, nb);
                boxes.push_back(B);
            }
    std::stable_sort(boxes.begin(), boxes.end(),
                     [](const CoarseBox& a, const CoarseBox& b) { return a.colour < b.colour; });
    D.box = boxes;
    D.col_begin.clear();
    int64_t base = 0;
    for (size_t i = 0; i < D.box.size(); ++i) {
        if (i == 0 || D.box[i].colour != D.box[i - 1].colour) D.col_begin.push_back((int)i);
        D.box[i].base = base;
        base += D.box[i].g.N;
    }
    D.col_begin.push_back((int)D.box.size());
    D.ntot = base;
    // index maps (host) and owner counts
    const int nbox = (int)D.box.size();
    std::vector<int> hidx(2 * D.ntot + nbox);
    std::vector<int64_t> hbase(nbox);
    std::vector<int> cnt(gc.N, 0);
    for (int b = 0; b < nbox; ++b) {
        const CoarseBox& B = D.box[b];
        hbase[b] = B.base;
        hidx[2 * D.ntot + b] = (int)B.g.N;
        for (int64_t t = 0; t < B.g.N; ++t) {
            int k = 0;
            while (k < 3 && t >= B.g.off[k + 1]) ++k;
            if (k >= d) k = 3;
            const int64_t li = t - B.g.off[k];
            int p[3] = {0, 0, 0};
            int64_t gi;
            if (d == 2) {
                if (k == 3) cell_pos<2>(B.g, li, p);
                else face_pos<2>(B.g, k, li, p);
                for (int a = 0; a < 2; ++a) p[a] += B.lo[a];
                gi = k == 3 ? gc.off[3] + cell_idx<2>(gc, p) : gc.off[k] + face_idx<2>(gc, k, p);
            } else {
                if (k == 3) cell_pos<3>(B.g, li, p);
                else face_pos<3>(B.g, k, li, p);
                for (int a = 0; a < 3; ++a) p[a] += B.lo[a];
                gi = k == 3 ? gc.off[3] + cell_idx<3>(gc, p) : gc.off[k] + face_idx<3>(gc, k, p);
            }
            hidx[B.base + t] = (int)gi;
            hidx[D.ntot + B.base + t] = b;
            cnt[gi] += 1;
        }
    }
    std::vector<double> hw(gc.N);
    for (int64_t i = 0; i < gc.N; ++i) {
        if (cnt[i] == 0) return fail(EHH_ERR_INVALID, "coarsest-level subdomains leave an unknown uncovered");
        hw[i] = 1.0 / cnt[i];
    }
    CHK(c->alloc((void**)&D.idx, sizeof(int) * hidx.size()));
    CHK(c->alloc((void**)&D.bbase, sizeof(int64_t) * nbox));
    CHK(c->alloc((void**)&D.wgt, sizeof(double) * gc.N));
    HIPCHK(hipMemcpyAsync(D.idx, hidx.data(), sizeof(int) * hidx.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(D.bbase, hbase.data(), sizeof(int64_t) * nbox, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(D.wgt, hw.data(), sizeof(double) * gc.N, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    // each box's restricted operator, inverted
    for (CoarseBox& B : D.box) {
        double* stb = nullptr;
        CHK(c->alloc((void**)&stb, sizeof(double) * stencil_size(B.g)));
        HIPCHK(launch_zero(stb, sizeof(double) * stencil_size(B.g), s));
        HIPCHK(launch_box_stencil(gc, stc, B.g, stb, B.lo, s));
        CHK(build_dense_inverse(c, B.g, stb, &B.inv, &B.sym, s));
        c->release(stb);
    }
    return EHH_OK;
}

int32_t build_hierarchy(ehh_ctx* c, Sub& S, const double* lam, const double* mu, const double* rho,
                        const double* gam, hipStream_t s) {
    const int L = c->opt.levels;
    S.lev.resize(L);
    int n[3] = {S.nloc[0], S.nloc[1], S.nloc[2]};
    for (int l = 0; l < L; ++l) {
        if (l > 0)
            for (int a = 0; a < c->dim; ++a) {
                if (n[a] % 2) return fail(EHH_ERR_INVALID, "(sub)domain size not divisible by 2^(levels-1)");
                n[a] /= 2;
            }
        for (int a = 0; a < c->dim; ++a)
            if (n[a] < 2) return fail(EHH_ERR_INVALID, "coarsest grid must keep at least 2 cells per axis");
        S.lev[l].g = make_geo(c->dim, n);
        S.lev[l].fine = l == 0;
        S.lev[l].damping = l < L - 1 ? c->opt.damping[l] : 0.0;
        S.lev[l].damping_p = l < L - 1 ? (c->opt.damping_p[l] > 0 ? c->opt.damping_p[l] : c->opt.damping[l]) : 0.0;
    }
    // level 0 coefficients
    Level& L0 = S.lev[0];
    if (!c->dd) {
        L0.coef64 = c->fine64;
    } else {
        CHK(c->alloc((void**)&L0.coef64, sizeof(double) * 4 * L0.g.ncell));
        FineCoefParams p{};
        p.dim = c->dim;
        for (int a = 0; a < 3; ++a) {
            p.n_glob[a] = c->gg.n[a];
            p.n_loc[a] = L0.g.n[a];
            p.origin[a] = S.origin[a];
            p.pad_lo[a] = S.pad_lo[a];
            p.pad_hi[a] = S.pad_hi[a];
            p.abl[a] = a < c->dim ? c->prob.abl_cells[a] : 0;
        }
        p.abl_max = c->prob.abl_max;
        p.gam0 = c->prob.atten0 / c->prob.omega;
        p.inv_omega = 1.0 / c->prob.omega;
        p.mu_bar = c->mu_bar;
        p.rho_bar = c->rho_bar;
        HIPCHK(launch_fine_coef(p, lam, mu, rho, gam, L0.coef64, s));
    }
    PhaseLog lg(s);
    const int64_t n0 = L0.g.ncell;
    const FineCoef<double> fc{L0.coef64, L0.coef64 + n0, L0.coef64 + 2 * n0, L0.coef64 + 3 * n0,
                              c->omega_nd * c->omega_nd, c->prob.shift};
    // stencil of level 0 (temporary), Galerkin levels, dense coarsest
    double* st0 = nullptr;
    CHK(c->alloc((void**)&st0, sizeof(double) * stencil_size(L0.g)));
    HIPCHK(launch_materialise(L0.g, fc, st0, s));
    const double* prev = st0;
    for (int l = 1; l < L; ++l) {
        Level& C = S.lev[l];
        CHK(c->alloc((void**)&C.coef64, sizeof(double) * stencil_size(C.g)));
        HIPCHK(launch_galerkin(S.lev[l - 1].g, prev, C.g, C.coef64, s));
        prev = C.coef64;
        lg.mark("galerkin level");
    }
    const Level& Lc = S.lev[L - 1];
    const double* stc = L == 1 ? st0 : Lc.coef64;
    bool cdd = false;
    for (int a = 0; a < c->dim; ++a) cdd = cdd || c->opt.coarse_dd_parts[a] > 1;
    if (cdd)
        CHK(build_coarse_dd(c, S, Lc.g, stc, s));
    else
        CHK(build_dense_inverse(c, Lc.g, stc, &S.inv, &S.sym, s));
    lg.mark(cdd ? "coarsest-level subdomain inverses" : "coarsest inverse");
    c->release(st0);
    if (c->bits() == 32) {
        for (int l = 0; l < L; ++l) {
            Level& Q = S.lev[l];
            if (l == 0 && !c->dd) continue;   // shares the global FP32 copy (set by the caller)
            const int64_t cnt = Q.fine ? 4 * Q.g.ncell : stencil_size(Q.g);
            CHK(c->alloc((void**)&Q.coef32, sizeof(float) * cnt));
            HIPCHK(launch_cast_d2f(Q.coef64, Q.coef32, cnt, s));
        }
    }
    // stored rows of the Galerkin levels, built once in the cycle precision
    for (int l = 1; l < L - 1; ++l) {
        Level& Q = S.lev[l];
        if (!stored_plan_wanted(Q.g, Q.fine)) continue;
        const int64_t lanes = stored_plan_lanes(Q.g);
        const size_t es = c->bits() == 32 ? sizeof(float) : sizeof(double);
        const int NT = stored_terms(Q.g.dim), NF = stored_imag_terms(Q.g.dim);
        for (int col = 0; col < 2; ++col) {
            CHK(c->alloc(&Q.sp_re[col], es * NT * lanes));
            CHK(c->alloc(&Q.sp_im[col], es * NF * lanes));
            if (c->bits() == 32)
                HIPCHK(launch_build_plans<float>(level_desc<float>(c, Q, c->prob.shift), col,
                                                 (float*)Q.sp_re[col], (float*)Q.sp_im[col], s));
            else
                HIPCHK(launch_build_plans<double>(level_desc<double>(c, Q, c->prob.shift), col,
                                                  (double*)Q.sp_re[col], (double*)Q.sp_im[col], s));
        }
        Q.sp_lanes = lanes;
        const int64_t N = Q.g.N;
        CHK(c->alloc(&Q.rp_re, es * NT * N));
        CHK(c->alloc(&Q.rp_im, es * NF * N));
        if (c->bits() == 32)
            HIPCHK(launch_build_row_plans<float>(level_desc<float>(c, Q, c->prob.shift), (float*)Q.rp_re,
                                                 (float*)Q.rp_im, s));
        else
            HIPCHK(launch_build_row_plans<double>(level_desc<double>(c, Q, c->prob.shift),
                                                  (double*)Q.rp_re, (double*)Q.rp_im, s));
        if (c->opt.coarse_bits == 16) CHK(rows_to_half(c, Q, NT, NF, lanes, s));
    }
    return EHH_OK;
}

// Memory the runtime knows as device memory (read in place by the setup
// kernels); anything else is host memory and is copied first.
bool is_device_pointer(const void* p) {
    hipPointerAttribute_t a{};
    const hipError_t e = hipPointerGetAttributes(&a, p);
    (void)hipGetLastError();   // unregistered host memory may report an error here
    return e == hipSuccess && a.type == hipMemoryTypeDevice;
}

int32_t setup_impl(ehh_ctx* c, const double* lam_h, const double* mu_h, const double* rho_h,
                   const double* gam_h, hipStream_t s) {
    const ehh_problem_t& P = c->prob;
    c->dim = P.dim;
    int n[3] = {P.n[0], P.n[1], P.dim == 3 ? P.n[2] : 1};
    c->gg = make_geo(P.dim, n);
    // media in host memory are copied to the device for the setup kernels (the
    // copies are released at the end of the setup: the operator keeps its own
    // nondimensional planes); media already in device memory are read in place
    const int64_t ncell0 = c->gg.ncell;
    const double* src[4] = {lam_h, mu_h, rho_h, gam_h};
    const double* dev[4] = {nullptr, nullptr, nullptr, nullptr};
    int nhost = 0;
    for (int a = 0; a < 4; ++a) {
        if (!src[a]) continue;
        if (is_device_pointer(src[a])) dev[a] = src[a];
        else ++nhost;
    }
    double* media = nullptr;
    if (nhost) CHK(c->alloc((void**)&media, sizeof(double) * nhost * ncell0));
    for (int a = 0, h = 0; a < 4; ++a) {
        if (!src[a] || dev[a]) continue;
        double* d = media + (int64_t)h++ * ncell0;
        HIPCHK(hipMemcpyAsync(d, src[a], sizeof(double) * ncell0, hipMemcpyHostToDevice, s));
        dev[a] = d;
    }
    const double* lam = dev[0];
    const double* mu = dev[1];
    const double* rho = dev[2];
    const double* gam = dev[3];
    // media means and physical check
    const int nb = media_check_blocks(c->gg.ncell);
    double* part = nullptr;
    CHK(c->alloc((void**)&part, sizeof(double) * (3 * nb + 4)));
    HIPCHK(launch_media_check(lam, mu, rho, gam, c->gg.ncell, part, nb, part + 3 * nb, s));
    double sums[4];
    HIPCHK(hipMemcpyAsync(sums, part + 3 * nb, sizeof(sums), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    c->release(part);
    if (sums[2] > 0) return fail(EHH_ERR_BREAKDOWN, "media contain non-finite or non-physical values");
    c->mu_bar = sums[0] / (double)c->gg.ncell;
    if (!(c->mu_bar > 0)) c->mu_bar = sums[3] / (double)c->gg.ncell;
    c->rho_bar = sums[1] / (double)c->gg.ncell;
    if (P.mu_bar > 0) c->mu_bar = P.mu_bar;      // caller-fixed units (e.g. across model updates)
    if (P.rho_bar > 0) c->rho_bar = P.rho_bar;
    if (!(c->mu_bar > 0) || !(c->rho_bar > 0)) return fail(EHH_ERR_BREAKDOWN, "degenerate media means");
    c->omega_nd = P.omega * P.h * std::sqrt(c->rho_bar / c->mu_bar);
    // global fine coefficients (the unshifted operator of the outer solve)
    CHK(c->alloc((void**)&c->fine64, sizeof(double) * 4 * c->gg.ncell));
    FineCoefParams fp{};
    fp.dim = P.dim;
    for (int a = 0; a < 3; ++a) {
        fp.n_glob[a] = n[a];
        fp.n_loc[a] = n[a];
        fp.abl[a] = a < P.dim ? P.abl_cells[a] : 0;
    }
    fp.abl_max = P.abl_max;
    fp.gam0 = P.atten0 / P.omega;
    fp.inv_omega = 1.0 / P.omega;
    fp.mu_bar = c->mu_bar;
    fp.rho_bar = c->rho_bar;
    HIPCHK(launch_fine_coef(fp, lam, mu, rho, gam, c->fine64, s));
    // subdomains
    c->dd = false;
    for (int a = 0; a < P.dim; ++a) c->dd = c->dd || c->opt.dd_parts[a] > 1;
    if (c->dd) {
        make_subdomains(c);
        // owner counts per axis
        std::vector<int> host;
        int offc[3], offf[3];
        for (int a = 0; a < 3; ++a) {
            offc[a] = (int)host.size();
            const int na = a < P.dim ? n[a] : 1;
            for (int x = 0; x < na; ++x) {
                int cnt = 0;
                std::vector<std::pair<int, int>> seen;
                for (const Sub& S : c->subs) {
                    std::pair<int, int> r{S.lo[a], S.hi[a]};
                    if (std::find(seen.begin(), seen.end(), r) != seen.end()) continue;
                    seen.push_back(r);
                    if (x >= S.lo[a] && x < S.hi[a]) ++cnt;
                }
                host.push_back(std::max(cnt, 1));
            }
            offf[a] = (int)host.size();
            for (int f = 0; f <= na; ++f) {
                int cnt = 0;
                std::vector<std::pair<int, int>> seen;
                for (const Sub& S : c->subs) {
                    std::pair<int, int> r{S.lo[a], S.hi[a]};
                    if (std::find(seen.begin(), seen.end(), r) != seen.end()) continue;
                    seen.push_back(r);
                    if (f > S.lo[a] && f < S.hi[a]) ++cnt;
                }
                host.push_back(std::max(cnt, 1));
            }
        }
        CHK(c->alloc((void**)&c->cnt_dev, sizeof(int) * host.size()));
        HIPCHK(hipMemcpyAsync(c->cnt_dev, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int a = 0; a < 3; ++a) {
            c->cnt_cell[a] = c->cnt_dev + offc[a];
            c->cnt_face[a] = c->cnt_dev + offf[a];
        }
    } else {
        Sub S;
        for (int a = 0; a < 3; ++a) {
            S.hi[a] = n[a];
            S.nloc[a] = n[a];
        }
        c->subs.push_back(std::move(S));
    }
    float* fine32 = nullptr;
    if (c->bits() == 32 && !c->dd) {
        CHK(c->alloc((void**)&fine32, sizeof(float) * 4 * c->gg.ncell));
        HIPCHK(launch_cast_d2f(c->fine64, fine32, 4 * c->gg.ncell, s));
    }
    for (Sub& S : c->subs) {
        CHK(build_hierarchy(c, S, lam, mu, rho, gam, s));
        if (fine32) S.lev[0].coef32 = fine32;
    }
    HIPCHK(hipStreamSynchronize(s));
    c->release(media);
    return EHH_OK;
}

int32_t check_handle(ehh_handle_t h) {
    if (!h) return fail(EHH_ERR_INVALID, "null handle");
    return EHH_OK;
}

int32_t level_of(ehh_ctx* c, int sub, int level, Sub** S, Level** L) {
    if (sub < 0 || sub >= (int)c->subs.size()) return fail(EHH_ERR_INVALID, "subdomain index out of range");
    Sub& Sr = c->subs[sub];
    if (level < 0 || level >= (int)Sr.lev.size()) return fail(EHH_ERR_INVALID, "level out of range");
    *S = &Sr;
    *L = &Sr.lev[level];
    return EHH_OK;
}

// The preconditioned vectors Z are kept in FP32 where the complex64 cycle runs
// on the whole grid (no domain decomposition, whose averaging sums in FP64):
// they are then exactly the cycle's output, and the FGMRES product and the
// solution update read them at half the bytes.
bool z_in_fp32(const ehh_ctx* c, const LevelDesc<double>& A) {
    return c->bits() == 32 && !c->dd && apply_x32_supported(A);
}

// z32 = M^{-1} v by the complex64 cycle on the whole grid, written in FP32
// (v_in_r0: the cycle's input copy of v is already in place).
int32_t precondition_f32(ehh_ctx* c, const double* v, float* z32, int nrhs, hipStream_t s, bool v_in_r0) {
    CHK(ensure_ws(c, nrhs));
    Sub& S = c->subs[0];
    if (!v_in_r0) HIPCHK(launch_cast_d2f(v, (float*)S.r0, 2 * c->gg.N * nrhs, s));
    return cycle<float>(c, S, 0, (const float*)S.r0, z32, true, nrhs, s);
}

// One Arnoldi step j of flexible GMRES for every right-hand side, enqueued
// without any host synchronisation (so that it can be captured in a graph):
// Z_j = M^{-1} V_j, w = A Z_j, classical Gram-Schmidt (reorthogonalised where
// needed), |w|, the Givens rotation and the residual estimate, V_{j+1} = w / |w|.
int32_t enqueue_iter(ehh_ctx* c, const LevelDesc<double>& A, int j, int nrhs, hipStream_t s) {
    const int m = c->opt.restart;
    const int64_t N = c->gg.N;
    double* Vj = c->V + (size_t)j * nrhs * 2 * N;
    float* v32 = krylov_copy32(c);
    if (z_in_fp32(c, A)) {
        float* Zj = (float*)c->Z + (size_t)j * nrhs * 2 * N;
        CHK(precondition_f32(c, Vj, Zj, nrhs, s, v32 != nullptr));
        HIPCHK(launch_apply_x32(A, Zj, c->w, nrhs, s));
    } else {
        double* Zj = c->Z + (size_t)j * nrhs * 2 * N;
        CHK(precondition_any(c, Vj, Zj, nrhs, s, v32 != nullptr));
        HIPCHK(launch_apply<double>(A, Zj, nullptr, c->w, nrhs, s));
    }
    // classical Gram-Schmidt, reorthogonalised where one pass is not enough,
    // V_{j+1} = the normalised result; then the Givens step
    double* Vn = c->V + (size_t)(j + 1) * nrhs * 2 * N;
    HIPCHK(launch_orthogonalise(c->V, j + 1, c->w, N, nrhs, c->partial, c->hcol, c->hcol2, m, c->nrm2, Vn, v32,
                                c->opt.reorth == 1, s));
    HIPCHK(launch_givens(c->H, c->cs, c->g, c->hcol, c->hcol2, c->nrm2, j, m, nrhs, c->active, c->est, c->bnorm, s));
    return EHH_OK;
}

bool graphs_enabled() {
    const char* v = std::getenv("EHH_GRAPHS");
    return !(v && std::atoi(v) == 0);
}

// Capture the m Arnoldi steps of the current batch size into executable graphs.
int32_t build_graphs(ehh_ctx* c, const LevelDesc<double>& A, int nrhs) {
    c->clear_graphs();
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    for (int j = 0; j < c->opt.restart; ++j) {
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        const int32_t st = enqueue_iter(c, A, j, nrhs, c->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (st != EHH_OK) {
            if (g) (void)hipGraphDestroy(g);
            c->clear_graphs();
            return st;
        }
        if (e != hipSuccess) {
            c->clear_graphs();
            return fail(EHH_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            c->clear_graphs();
            return fail(EHH_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        c->graphs.push_back(ex);
    }
    c->graph_rhs = nrhs;
    return EHH_OK;
}

// The demangled name of a kernel's host stub without namespace, return type and
// parameter list (as kernel traces print it), e.g. "k_relax_st2d<double, false, false>".
std::string kernel_name(const void* k) {
    Dl_info info{};
    if (!dladdr(k, &info) || !info.dli_sname) return "unknown";
    int st = 0;
    char* d = abi::__cxa_demangle(info.dli_sname, nullptr, nullptr, &st);
    std::string n = (st == 0 && d) ? d : info.dli_sname;
    std::free(d);
    if (n.compare(0, 5, "void ") == 0) n = n.substr(5);
    for (size_t p = n.find("ehh::"); p != std::string::npos; p = n.find("ehh::")) n.erase(p, 5);
    // a batch kernel's first template argument is its argument pack: left out
    const size_t pk = n.find("_batch<Pack<");
    if (pk != std::string::npos) {
        size_t i = pk + 7, depth = 0;
        for (; i < n.size(); ++i) {
            if (n[i] == '<') ++depth;
            else if (n[i] == '>' && --depth == 0) break;
        }
        size_t j = i + 1;
        while (j < n.size() && (n[j] == ',' || n[j] == ' ')) ++j;
        n.erase(pk + 7, j - (pk + 7));
    }
    int depth = 0;
    for (size_t i = 0; i < n.size(); ++i) {
        if (n[i] == '<') ++depth;
        else if (n[i] == '>') --depth;
        else if (n[i] == '(' && depth == 0) return n.substr(0, i);
    }
    return n;
}

// Time `reps` rounds of the recorded launches (each preceded by the eviction
// write when evict is given) replayed from a graph on the caller's stream;
// with_kernel = false times the eviction writes alone.
int32_t time_replay(ehh_ctx* c, const std::vector<const LogRec*>& recs, int reps, void* evict, int64_t evict_bytes,
                    bool with_kernel, hipStream_t s, double* ms) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < reps; ++r)
        for (const LogRec* rec : recs) {
            if (evict) (void)launch_zero(evict, (size_t)evict_bytes, c->cap_stream);
            if (with_kernel) rec->again(c->cap_stream, nullptr, nullptr);
        }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (ec != hipSuccess) return fail(EHH_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(EHH_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 1e300;
    if (e == hipSuccess) e = hipGraphLaunch(ex, s);   // warm-up replay
    for (int t = 0; t < 3 && e == hipSuccess; ++t) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = hipGraphLaunch(ex, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        if (e == hipSuccess) best = std::min(best, (double)f);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGraphExecDestroy(ex);
    if (e != hipSuccess) return fail(EHH_ERR_HIP, std::string("timed replay: ") + hipGetErrorString(e));
    *ms = best;
    return EHH_OK;
}

// The whole log replayed in order on stream s, each launch between its own start
// and stop events (recorded by the dispatch itself), once untimed and then reps
// times: every launch finds the caches as the launches before it in the
// application left them, as inside a solve.  sum_ms[i]: the durations of
// launch i summed over the reps.
int32_t time_in_order(const std::vector<LogRec>& log, int reps, hipStream_t s, std::vector<double>& sum_ms) {
    const size_t n = log.size();
    sum_ms.assign(n, 0.0);
    std::vector<hipEvent_t> ev(2 * n, nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < 2 * n && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        for (size_t i = 0; i < n; ++i) log[i].again(s, ev[2 * i], ev[2 * i + 1]);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (size_t i = 0; i < n && e == hipSuccess && r > 0; ++i) {
            float f = 0.0f;
            e = hipEventElapsedTime(&f, ev[2 * i], ev[2 * i + 1]);
            sum_ms[i] += f;
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(EHH_ERR_HIP, std::string("in-order replay: ") + hipGetErrorString(e));
    return EHH_OK;
}

}  // namespace

// ======================================================================= C ABI
namespace {
// Best of three timings of `reps` back-to-back calls of f on stream s [ms].
template <class F> int32_t time_calls(hipStream_t s, int reps, F&& f, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int32_t st = EHH_OK;
    for (int w = 0; w < 2 && st == EHH_OK; ++w) st = f();   // warm-up
    for (int t = 0; t < 3 && st == EHH_OK; ++t) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == EHH_OK; ++r) st = f();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float f_ms = 0.0f;
        (void)hipEventElapsedTime(&f_ms, e0, e1);
        best = std::min(best, (double)f_ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return st;
}

template <typename T> int32_t autotune_t(ehh_ctx* c, int nrhs, hipStream_t s) {
    Sub& S = c->subs[0];
    const int L = (int)S.lev.size();
    const int econ = c->opt.vanka == 0;
    const int cand[] = {0, 1, 2, 4, 8, 16, 32, 64};
    for (int l = 0; l < L; ++l) {
        Level& Q = S.lev[l];
        const size_t bytes = sizeof(T) * 2 * (size_t)Q.g.N * nrhs;
        T* b = (T*)(l == 0 ? S.r0 : Q.b);
        T* e = (T*)(l == 0 ? S.e0 : Q.e);
        T* t = (T*)Q.t;
        HIPCHK(launch_zero(b, bytes, s));
        HIPCHK(launch_zero(e, bytes, s));
        for (int kind = 0; kind < 2; ++kind) {
            if (kind == 0 && l == L - 1) continue;   // the coarsest level is not relaxed
            int& knob = kind == 0 ? Q.tune_relax : Q.tune_apply;
            double best = 1e300;
            int pick = 0;
            for (int g : cand) {
                if (g > nrhs) break;
                knob = g;
                const LevelDesc<T> D = level_desc<T>(c, Q, c->prob.shift);
                double ms = 0.0;
                if (kind == 0)
                    CHK(time_calls(s, 8, [&]() -> int32_t {
                        HIPCHK(launch_relax<T>(D, 0, Damp{Q.damping, Q.damping_p}, econ, b, e, t, nrhs, s));
                        return EHH_OK;
                    }, &ms));
                else
                    CHK(time_calls(s, 8, [&]() -> int32_t {
                        HIPCHK(launch_apply<T>(D, e, b, t, nrhs, s));
                        return EHH_OK;
                    }, &ms));
                // another shape must beat the heuristic one by 2 % to replace it
                if (g == 0 || ms < 0.98 * best) {
                    if (g == 0 || ms < best) pick = g;
                    best = std::min(best, ms);
                }
            }
            knob = pick;
        }
    }
    for (Sub& O : c->subs)
        for (int l = 0; l < L && l < (int)O.lev.size(); ++l) {
            O.lev[l].tune_relax = S.lev[l].tune_relax;
            O.lev[l].tune_apply = S.lev[l].tune_apply;
        }
    return EHH_OK;
}
}  // namespace

extern "C" {

void ehh_default_options(ehh_options_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->levels = 3;
    o->cycle = 1;
    o->nu1 = o->nu2 = 1;
    o->vanka = 1;
    o->precond_bits = 64;
    o->coarse_bits = 32;
    o->coarse_dd_parts[0] = o->coarse_dd_parts[1] = o->coarse_dd_parts[2] = 1;
    o->coarse_dd_overlap = 2;
    o->coarse_dd_colors = 0;
    o->dd_batch = 1;
    o->restart = 5;
    o->dd_parts[0] = o->dd_parts[1] = o->dd_parts[2] = 1;
    o->dd_colors = 1;
    const double d[EHH_MAX_LEVELS] = {0.75, 0.5, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25};
    for (int l = 0; l < EHH_MAX_LEVELS; ++l) o->damping[l] = d[l];
}

int32_t ehh_setup_operator(const ehh_problem_t* problem, const double* lambda, const double* mu, const double* rho,
                           const double* gamma, const ehh_options_t* options, void* stream, ehh_handle_t* out) {
    if (!out) return fail(EHH_ERR_INVALID, "null output handle");
    *out = nullptr;
    CHK(check_problem(problem, options));
    if (!lambda || !mu || !rho) return fail(EHH_ERR_INVALID, "null media pointer");
    ehh_ctx* c = new ehh_ctx();
    c->prob = *problem;
    c->opt = *options;
    (void)hipGetDevice(&c->device);
    if (c->prob.dim == 2) {
        c->prob.n[2] = 1;
        c->prob.abl_cells[2] = 0;
        c->opt.dd_parts[2] = 1;
        c->opt.coarse_dd_parts[2] = 1;
    }
    int32_t st = setup_impl(c, lambda, mu, rho, gamma, as_stream(stream));
    if (st != EHH_OK) {
        (void)hipStreamSynchronize(as_stream(stream));
        delete c;
        return st;
    }
    // the address of this device's scratch array for ehh_coarse_solve_noalloc
    // (taken once per device; a failure here only disables that entry point,
    // which then reports it)
    (void)noalloc_scratch_init(c->device);
    (void)hipGetLastError();
    *out = c;
    return EHH_OK;
}

void ehh_destroy(ehh_handle_t h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

void ehh_release_cached_memory(void) { BlockCache::get().trim(-1); }

int32_t ehh_vector_layout(ehh_handle_t h, int64_t counts[4], int64_t* stride) {
    CHK(check_handle(h));
    if (!counts || !stride) return fail(EHH_ERR_INVALID, "null output");
    for (int k = 0; k < 4; ++k) counts[k] = h->gg.cnt[k];
    *stride = 2 * h->gg.N;
    return EHH_OK;
}

int32_t ehh_scaling(ehh_handle_t h, double out[3]) {
    CHK(check_handle(h));
    if (!out) return fail(EHH_ERR_INVALID, "null output");
    out[0] = h->mu_bar;
    out[1] = h->rho_bar;
    out[2] = h->omega_nd;
    return EHH_OK;
}

int32_t ehh_apply(ehh_handle_t h, int32_t shifted, const double* x, double* y, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    if (!x || !y || x == y || nrhs < 1) return fail(EHH_ERR_INVALID, "ehh_apply: bad vectors or nrhs");
    LevelDesc<double> A{};
    A.g = h->gg;
    A.fine = true;
    const int64_t n = h->gg.ncell;
    A.f = FineCoef<double>{h->fine64, h->fine64 + n, h->fine64 + 2 * n, h->fine64 + 3 * n,
                           h->omega_nd * h->omega_nd, shifted ? h->prob.shift : 0.0};
    HIPCHK(launch_apply<double>(A, x, nullptr, y, nrhs, as_stream(stream)));
    return EHH_OK;
}

int32_t ehh_vcycle(ehh_handle_t h, int32_t sub, const void* r, void* e, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, 0, &S, &L));
    if (!r || !e || r == e || nrhs < 1) return fail(EHH_ERR_INVALID, "ehh_vcycle: bad vectors or nrhs");
    CHK(ensure_ws(h, nrhs));
    if (h->bits() == 32) return cycle<float>(h, *S, 0, (const float*)r, (float*)e, true, nrhs, as_stream(stream));
    return cycle<double>(h, *S, 0, (const double*)r, (double*)e, true, nrhs, as_stream(stream));
}

int32_t ehh_precondition(ehh_handle_t h, const double* v, double* z, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    if (!v || !z || v == z || nrhs < 1) return fail(EHH_ERR_INVALID, "ehh_precondition: bad vectors or nrhs");
    return precondition_any(h, v, z, nrhs, as_stream(stream));
}

int32_t ehh_solve(ehh_handle_t h, const double* b, double* x, int32_t nrhs, double tol, int32_t maxit,
                  ehh_stats_t* stats, void* stream) {
    CHK(check_handle(h));
    if (!b || !x || b == x || nrhs < 1 || !(tol > 0) || maxit < 1)
        return fail(EHH_ERR_INVALID, "ehh_solve: bad vectors, nrhs, tol or maxit");
    hipStream_t s = as_stream(stream);
    ehh_ctx* c = h;
    CHK(ensure_ws(c, nrhs));
    CHK(ensure_krylov(c, nrhs));
    const int m = c->opt.restart;
    const int64_t N = c->gg.N;
    const size_t vb = sizeof(double) * 2 * (size_t)N;
    double* hp = c->host_pinned;
    // pinned mirror of the restart block, at the offsets of its device copy
    // (laid out for the batch size it was allocated for, possibly larger)
    char* const hb = c->rst_host;
    double* hg = (double*)hb;
    double* hs = (double*)(hb + ((char*)c->scal - (char*)c->g));
    int* ha = (int*)(hb + ((char*)c->active - (char*)c->g));
    int* hn = (int*)(hb + ((char*)c->ncols - (char*)c->g));
    LevelDesc<double> A{};
    A.g = c->gg;
    A.fine = true;
    const int64_t nc = c->gg.ncell;
    A.f = FineCoef<double>{c->fine64, c->fine64 + nc, c->fine64 + 2 * nc, c->fine64 + 3 * nc,
                           c->omega_nd * c->omega_nd, 0.0};

    const bool use_graphs = graphs_enabled();
    if (use_graphs && c->graph_rhs != nrhs) CHK(build_graphs(c, A, nrhs));
    std::vector<double> bnorm(nrhs), beta(nrhs), est(nrhs, 1.0), fin_est(nrhs, 1.0);
    std::vector<int> active(nrhs, 0), iters(nrhs, 0), ncols(nrhs, 0), done_flag(nrhs, 0);
    std::vector<std::vector<double>> hist(nrhs);
    HIPCHK(launch_norm2(b, N, nrhs, c->partial, c->nrm2, s));
    HIPCHK(hipMemcpyAsync(hp, c->nrm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemsetAsync(x, 0, vb * nrhs, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
        bnorm[r] = std::sqrt(hp[r]);
        if (!std::isfinite(bnorm[r])) return fail(EHH_ERR_BREAKDOWN, "non-finite right-hand side");
    }
    HIPCHK(hipMemcpyAsync(c->bnorm, bnorm.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
    int it = 0;
    bool first = true;
    bool breakdown = false;
    std::vector<double> g0(2 * (size_t)nrhs * (m + 1));
    std::vector<double> inv_beta(nrhs);
    while (true) {
        // true residual R = b - A x
        if (first) {
            HIPCHK(hipMemcpyAsync(c->R, b, vb * nrhs, hipMemcpyDeviceToDevice, s));
            for (int r = 0; r < nrhs; ++r) beta[r] = bnorm[r];
        } else {
            HIPCHK(launch_apply<double>(A, x, b, c->R, nrhs, s));
            HIPCHK(launch_norm2(c->R, N, nrhs, c->partial, c->nrm2, s));
            HIPCHK(hipMemcpyAsync(hp, c->nrm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int r = 0; r < nrhs; ++r) beta[r] = std::sqrt(hp[r]);
        }
        first = false;
        int nact = 0;
        for (int r = 0; r < nrhs; ++r) {
            if (!std::isfinite(beta[r])) breakdown = true;
            active[r] = bnorm[r] > 0 && beta[r] > tol * bnorm[r] && std::isfinite(beta[r]);
            if (bnorm[r] > 0) fin_est[r] = beta[r] / bnorm[r];
            nact += active[r];
        }
        if (breakdown || nact == 0 || it >= maxit) break;
        std::fill(g0.begin(), g0.end(), 0.0);
        for (int r = 0; r < nrhs; ++r) {
            g0[2 * (size_t)r * (m + 1)] = beta[r];
            inv_beta[r] = active[r] ? 1.0 / beta[r] : 0.0;
            ncols[r] = 0;
        }
        // g, scal and active in one copy from the pinned mirror (the stream has
        // been synchronised since the mirror was last read)
        std::memcpy(hg, g0.data(), sizeof(double) * g0.size());
        std::memcpy(hs, inv_beta.data(), sizeof(double) * nrhs);
        std::memcpy(ha, active.data(), sizeof(int) * nrhs);
        HIPCHK(hipMemcpyAsync(c->g, hb, (char*)c->ncols - (char*)c->g, hipMemcpyHostToDevice, s));
        HIPCHK(launch_scale(c->R, c->V, N, nrhs, c->scal, 0, s, krylov_copy32(c)));
        int j = 0;
        for (j = 0; j < m; ++j) {
            if (use_graphs)
                HIPCHK(hipGraphLaunch(c->graphs[j], s));
            else
                CHK(enqueue_iter(c, A, j, nrhs, s));
            HIPCHK(hipMemcpyAsync(hp, c->est, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ++it;
            bool changed = false;
            int left = 0;
            for (int r = 0; r < nrhs; ++r) {
                if (!active[r]) continue;
                iters[r] += 1;
                const double e = hp[r];
                hist[r].push_back(e);
                fin_est[r] = e;
                if (!std::isfinite(e)) {
                    breakdown = true;
                    active[r] = 0;
                    ncols[r] = j;
                    changed = true;
                    continue;
                }
                if (e <= tol) {
                    active[r] = 0;
                    ncols[r] = j + 1;
                    changed = true;
                    continue;
                }
                ++left;
            }
            if (log_enabled() && it % 10 == 0) {
                double worst = 0.0;
                for (int r = 0; r < nrhs; ++r)
                    if (active[r]) worst = std::max(worst, hp[r]);
                std::fprintf(stderr, "[ehh] iteration %d: %d active, worst estimate %.3e\n", it, left, worst);
                std::fflush(stderr);
            }
            if (left == 0 || it >= maxit || breakdown) break;
            if (changed) {
                std::memcpy(ha, active.data(), sizeof(int) * nrhs);
                HIPCHK(hipMemcpyAsync(c->active, ha, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
            }
        }
        const int done_cols = std::min(j + 1, m);
        for (int r = 0; r < nrhs; ++r)
            if (active[r]) ncols[r] = done_cols;
        std::memcpy(hn, ncols.data(), sizeof(int) * nrhs);
        HIPCHK(hipMemcpyAsync(c->ncols, hn, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        if (z_in_fp32(c, A))
            HIPCHK(launch_update_x(c->H, c->g, (const float*)c->Z, x, N, nrhs, m, c->ncols, c->y, s));
        else
            HIPCHK(launch_update_x(c->H, c->g, c->Z, x, N, nrhs, m, c->ncols, c->y, s));
        if (breakdown) break;
    }
    // final true residuals
    HIPCHK(launch_apply<double>(A, x, b, c->R, nrhs, s));
    HIPCHK(launch_norm2(c->R, N, nrhs, c->partial, c->nrm2, s));
    HIPCHK(hipMemcpyAsync(hp, c->nrm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t status = EHH_OK;
    for (int r = 0; r < nrhs; ++r) {
        const double tr = bnorm[r] > 0 ? std::sqrt(hp[r]) / bnorm[r] : 0.0;
        int32_t st = EHH_OK;
        if (!std::isfinite(tr) || breakdown) st = EHH_ERR_BREAKDOWN;
        else if (tr > tol) st = EHH_NOT_CONVERGED;
        if (stats) {
            stats[r].status = st;
            stats[r].iters = iters[r];
            stats[r].rel_res_est = fin_est[r];
            stats[r].rel_res_true = tr;
            const auto& hh = hist[r];
            const int warm = 5;
            if ((int)hh.size() > warm + 1 && hh[warm] > 0 && hh.back() > 0)
                stats[r].conv_factor = std::pow(hh.back() / hh[warm], 1.0 / (double)(hh.size() - 1 - warm));
            else
                stats[r].conv_factor = NAN;
        }
        if (st == EHH_ERR_BREAKDOWN) status = EHH_ERR_BREAKDOWN;
        else if (st == EHH_NOT_CONVERGED && status == EHH_OK) status = EHH_NOT_CONVERGED;
    }
    if (status == EHH_ERR_BREAKDOWN) g_err = "non-finite residual in the Krylov iteration";
    else if (status == EHH_NOT_CONVERGED) g_err = "maxit reached before tol";
    return status;
}

int32_t ehh_solve_adjoint(ehh_handle_t h, const double* g, double* y, int32_t nrhs, double tol, int32_t maxit,
                          ehh_stats_t* stats, void* stream) {
    CHK(check_handle(h));
    if (!g || !y || g == y || nrhs < 1 || !(tol > 0) || maxit < 1)
        return fail(EHH_ERR_INVALID, "ehh_solve_adjoint: bad vectors, nrhs, tol or maxit");
    hipStream_t s = as_stream(stream);
    ehh_ctx* c = h;
    if (nrhs > c->adj_rhs) {
        c->release(c->adjb);
        c->adjb = nullptr;
        c->adj_rhs = 0;
        CHK(c->alloc((void**)&c->adjb, sizeof(double) * 2 * (size_t)c->gg.N * nrhs));
        c->adj_rhs = nrhs;
    }
    // A^H = conj(A) because A^T = A: A^H y = g  <=>  A conj(y) = conj(g)
    HIPCHK(launch_conj(g, c->adjb, c->gg.N, nrhs, s));
    const int32_t st = ehh_solve(h, c->adjb, y, nrhs, tol, maxit, stats, stream);
    if (st == EHH_OK || st == EHH_NOT_CONVERGED || st == EHH_ERR_BREAKDOWN)
        HIPCHK(launch_conj(y, y, c->gg.N, nrhs, s));
    return st;
}

int32_t ehh_media_gradient(ehh_handle_t h, const double* y, const double* x, int32_t nrhs, double* grad_lambda,
                           double* grad_mu, double* grad_rho, int32_t accumulate, void* stream) {
    CHK(check_handle(h));
    if (!y || !x || nrhs < 1 || !grad_lambda || !grad_mu || !grad_rho || grad_lambda == grad_mu ||
        grad_mu == grad_rho || grad_lambda == grad_rho || (accumulate != 0 && accumulate != 1))
        return fail(EHH_ERR_INVALID, "ehh_media_gradient: bad vectors, nrhs or accumulate flag");
    HIPCHK(launch_media_gradient(h->gg, h->fine64, h->omega_nd * h->omega_nd, y, x, nrhs, h->mu_bar, h->rho_bar,
                                 grad_lambda, grad_mu, grad_rho, accumulate, as_stream(stream)));
    return EHH_OK;
}

int32_t ehh_num_subdomains(ehh_handle_t h) { return h ? (int32_t)h->subs.size() : 0; }

int32_t ehh_subdomain_info(ehh_handle_t h, int32_t sub, int32_t n_local[3], int32_t origin[3], int32_t lo[3],
                           int32_t hi[3]) {
    CHK(check_handle(h));
    if (sub < 0 || sub >= (int)h->subs.size()) return fail(EHH_ERR_INVALID, "subdomain index out of range");
    const Sub& S = h->subs[sub];
    for (int a = 0; a < 3; ++a) {
        if (n_local) n_local[a] = S.nloc[a];
        if (origin) origin[a] = S.origin[a];
        if (lo) lo[a] = S.lo[a];
        if (hi) hi[a] = S.hi[a];
    }
    return EHH_OK;
}

int32_t ehh_level_info(ehh_handle_t h, int32_t sub, int32_t level, int32_t n[3], int64_t counts[4], int64_t* stride) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, level, &S, &L));
    for (int a = 0; a < 3; ++a)
        if (n) n[a] = L->g.n[a];
    for (int k = 0; k < 4; ++k)
        if (counts) counts[k] = L->g.cnt[k];
    if (stride) *stride = 2 * L->g.N;
    return EHH_OK;
}

int32_t ehh_level_apply(ehh_handle_t h, int32_t sub, int32_t level, const void* x, void* y, int32_t nrhs,
                        void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, level, &S, &L));
    if (!x || !y || x == y || nrhs < 1) return fail(EHH_ERR_INVALID, "bad vectors or nrhs");
    if (h->bits() == 32)
        HIPCHK(launch_apply<float>(level_desc<float>(h, *L, h->prob.shift), (const float*)x, nullptr, (float*)y, nrhs,
                                   as_stream(stream)));
    else
        HIPCHK(launch_apply<double>(level_desc<double>(h, *L, h->prob.shift), (const double*)x, nullptr, (double*)y,
                                    nrhs, as_stream(stream)));
    return EHH_OK;
}

int32_t ehh_level_relax(ehh_handle_t h, int32_t sub, int32_t level, int32_t colour, const void* b, const void* e_in,
                        void* e_out, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, level, &S, &L));
    if (level == (int)S->lev.size() - 1) return fail(EHH_ERR_INVALID, "the coarsest level is not relaxed");
    if (!b || !e_out || e_in == e_out || b == e_out || (colour != 0 && colour != 1) || nrhs < 1)
        return fail(EHH_ERR_INVALID, "bad vectors, colour or nrhs");
    const int econ = h->opt.vanka == 0;
    if (h->bits() == 32)
        HIPCHK(launch_relax<float>(level_desc<float>(h, *L, h->prob.shift), colour, Damp{L->damping, L->damping_p},
                                   econ, (const float*)b,
                                   (const float*)e_in, (float*)e_out, nrhs, as_stream(stream)));
    else
        HIPCHK(launch_relax<double>(level_desc<double>(h, *L, h->prob.shift), colour, Damp{L->damping, L->damping_p},
                                    econ,
                                    (const double*)b, (const double*)e_in, (double*)e_out, nrhs, as_stream(stream)));
    return EHH_OK;
}

int32_t ehh_level_restrict(ehh_handle_t h, int32_t sub, int32_t level, const void* b, const void* e, void* rc,
                           int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, level, &S, &L));
    if (level == (int)S->lev.size() - 1) return fail(EHH_ERR_INVALID, "no coarser level");
    if (!b || !e || !rc || nrhs < 1) return fail(EHH_ERR_INVALID, "bad vectors or nrhs");
    CHK(ensure_ws(h, nrhs));
    hipStream_t s = as_stream(stream);
    const Geo& gc = S->lev[level + 1].g;
    bool done = false;
    if (h->bits() == 32) {
        const LevelDesc<float> D = level_desc<float>(h, *L, h->prob.shift);
        HIPCHK(launch_residual_restrict<float>(D, gc, (const float*)e, (const float*)b, (float*)rc, nrhs, s, &done));
        if (!done) {
            HIPCHK(launch_apply<float>(D, (const float*)e, (const float*)b, (float*)L->t, nrhs, s));
            HIPCHK(launch_restrict<float>(L->g, gc, (const float*)L->t, (float*)rc, nrhs, s));
        }
    } else {
        const LevelDesc<double> D = level_desc<double>(h, *L, h->prob.shift);
        HIPCHK(launch_residual_restrict<double>(D, gc, (const double*)e, (const double*)b, (double*)rc, nrhs, s,
                                                &done));
        if (!done) {
            HIPCHK(launch_apply<double>(D, (const double*)e, (const double*)b, (double*)L->t, nrhs, s));
            HIPCHK(launch_restrict<double>(L->g, gc, (const double*)L->t, (double*)rc, nrhs, s));
        }
    }
    return EHH_OK;
}

int32_t ehh_level_prolong(ehh_handle_t h, int32_t sub, int32_t level, const void* ec, void* e, int32_t nrhs,
                          void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    CHK(level_of(h, sub, level, &S, &L));
    if (level == (int)S->lev.size() - 1) return fail(EHH_ERR_INVALID, "no coarser level");
    if (!ec || !e || nrhs < 1) return fail(EHH_ERR_INVALID, "bad vectors or nrhs");
    const Geo& gc = S->lev[level + 1].g;
    if (h->bits() == 32)
        HIPCHK(launch_prolong<float>(L->g, gc, (const float*)ec, (float*)e, nrhs, as_stream(stream)));
    else
        HIPCHK(launch_prolong<double>(L->g, gc, (const double*)ec, (double*)e, nrhs, as_stream(stream)));
    return EHH_OK;
}

int32_t ehh_coarse_solve(ehh_handle_t h, int32_t sub, const void* r, void* e, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    Sub* S;
    Level* L;
    if (sub < 0 || sub >= (int)h->subs.size()) return fail(EHH_ERR_INVALID, "subdomain index out of range");
    CHK(level_of(h, sub, (int)h->subs[sub].lev.size() - 1, &S, &L));
    if (!r || !e || r == e || nrhs < 1) return fail(EHH_ERR_INVALID, "bad vectors or nrhs");
    CHK(ensure_ws(h, nrhs));   // sizes the coarse-apply workspace for nrhs
    if (h->bits() == 32) return coarse_solve<float>(h, *S, (const float*)r, (float*)e, true, nrhs, as_stream(stream));
    return coarse_solve<double>(h, *S, (const double*)r, (double*)e, true, nrhs, as_stream(stream));
}

int32_t ehh_profile_precondition(ehh_handle_t h, const double* v, double* z, int32_t nrhs, int32_t reps, void* evict,
                                 int64_t evict_bytes, ehh_kernel_time_t* out, int32_t cap, int32_t* count,
                                 void* stream) {
    CHK(check_handle(h));
    if (!v || !z || v == z || nrhs < 1 || reps < 1 || !out || cap < 1 || !count || evict_bytes < 0 ||
        (evict && evict_bytes % 4) || (!evict && evict_bytes))
        return fail(EHH_ERR_INVALID, "ehh_profile_precondition: bad vectors, nrhs, reps, eviction buffer or output");
    hipStream_t s = as_stream(stream);
    CHK(ensure_ws(h, nrhs));
    t_log.clear();
    t_log_on = true;
    const int32_t st = precondition_any(h, v, z, nrhs, s);
    t_log_on = false;
    std::vector<LogRec> log;
    log.swap(t_log);
    CHK(st);
    HIPCHK(hipStreamSynchronize(s));
    // kernels in order of their first launch, each with its launches in order
    std::vector<const void*> order;
    std::map<const void*, std::vector<const LogRec*>> groups;
    for (const LogRec& r : log) {
        auto& gv = groups[r.kernel];
        if (gv.empty()) order.push_back(r.kernel);
        gv.push_back(&r);
    }
    std::vector<double> seq_ms;
    CHK(time_in_order(log, reps, s, seq_ms));
    std::map<const void*, double> seq_sum;
    for (size_t i = 0; i < log.size(); ++i) seq_sum[log[i].kernel] += seq_ms[i];
    int32_t k = 0;
    for (const void* kern : order) {
        if (k >= cap) break;
        const auto& recs = groups[kern];
        double t_all = 0.0, t_evict = 0.0, t_warm = 0.0;
        CHK(time_replay(h, recs, reps, evict, evict_bytes, true, s, &t_all));
        if (evict) CHK(time_replay(h, recs, reps, evict, evict_bytes, false, s, &t_evict));
        CHK(time_replay(h, recs, reps, nullptr, 0, true, s, &t_warm));
        ehh_kernel_time_t& o = out[k++];
        std::memset(&o, 0, sizeof(o));
        const std::string nm = kernel_name(kern);
        std::strncpy(o.kernel, nm.c_str(), sizeof(o.kernel) - 1);
        o.launches = (int32_t)recs.size();
        o.avg_us = std::max(t_all - t_evict, 0.0) * 1e3 / ((double)reps * recs.size());
        o.avg_us_warm = t_warm * 1e3 / ((double)reps * recs.size());
        o.avg_us_seq = seq_sum[kern] * 1e3 / ((double)reps * recs.size());
        for (const LogRec* r : recs) {
            o.bytes += r->bytes.mine / recs.size();
            o.bytes_model += r->bytes.model / recs.size();
        }
    }
    *count = k;
    return EHH_OK;
}


int32_t ehh_autotune(ehh_handle_t h, int32_t nrhs, int32_t* table, int32_t len, void* stream) {
    CHK(check_handle(h));
    const int L = (int)h->subs[0].lev.size();
    if (nrhs < 1 || !table || len < 2 * L) return fail(EHH_ERR_INVALID, "ehh_autotune: nrhs >= 1, table of 2 x levels");
    hipStream_t s = as_stream(stream);
    CHK(ensure_ws(h, nrhs));
    h->clear_graphs();
    for (Sub& S : h->subs)
        for (Level& Q : S.lev) Q.tune_relax = Q.tune_apply = 0;
    CHK(h->bits() == 32 ? autotune_t<float>(h, nrhs, s) : autotune_t<double>(h, nrhs, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int l = 0; l < L; ++l) {
        table[2 * l] = h->subs[0].lev[l].tune_relax;
        table[2 * l + 1] = h->subs[0].lev[l].tune_apply;
    }
    return EHH_OK;
}

int32_t ehh_set_tuning(ehh_handle_t h, const int32_t* table, int32_t len) {
    CHK(check_handle(h));
    const int L = (int)h->subs[0].lev.size();
    if (!table || len != 2 * L) return fail(EHH_ERR_INVALID, "ehh_set_tuning: table of 2 x levels entries");
    for (int i = 0; i < len; ++i)
        if (table[i] < 0 || table[i] > 4096) return fail(EHH_ERR_INVALID, "ehh_set_tuning: entries in [0, 4096]");
    h->clear_graphs();
    for (Sub& S : h->subs)
        for (int l = 0; l < L && l < (int)S.lev.size(); ++l) {
            S.lev[l].tune_relax = table[2 * l];
            S.lev[l].tune_apply = table[2 * l + 1];
        }
    return EHH_OK;
}

int32_t ehh_coarse_solve_noalloc(ehh_handle_t h, int32_t sub, const void* r, void* e, int32_t nrhs, void* stream) {
    CHK(check_handle(h));
    if (sub < 0 || sub >= (int)h->subs.size()) return fail(EHH_ERR_INVALID, "subdomain index out of range");
    if (!r || !e || r == e || nrhs < 1) return fail(EHH_ERR_INVALID, "bad vectors or nrhs");
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != h->device) return fail(EHH_ERR_INVALID, "the handle's device must be current");
    double* scratch = noalloc_scratch(h->device);
    if (!scratch) {
        const hipError_t ie = noalloc_scratch_init(h->device);
        if (ie != hipSuccess) return fail(EHH_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(ie));
        scratch = noalloc_scratch(h->device);
    }
    const Sub& S = h->subs[sub];
    if (S.cdd.active())
        return fail(EHH_ERR_UNSUPPORTED, "ehh_coarse_solve_noalloc: the coarsest level is solved by domain "
                                         "decomposition, whose workspaces would have to be allocated");
    const int64_t n = S.lev.back().g.N;
    const size_t need = coarse_ws_doubles(n, nrhs);
    if (need > (size_t)kNoallocScratchDoubles)
        return fail(EHH_ERR_UNSUPPORTED, "ehh_coarse_solve_noalloc: " + std::to_string(n) + " unknowns x " +
                                             std::to_string(nrhs) + " right-hand sides need " +
                                             std::to_string(need) + " doubles of scratch; the array holds " +
                                             std::to_string(kNoallocScratchDoubles));
    if (h->bits() == 32)
        HIPCHK(launch_coarse_apply<float>(S.inv, S.sym, n, (const float*)r, (float*)e, nrhs, scratch,
                                          as_stream(stream)));
    else
        HIPCHK(launch_coarse_apply<double>(S.inv, S.sym, n, (const double*)r, (double*)e, nrhs, scratch,
                                           as_stream(stream)));
    return EHH_OK;
}

const char* ehh_last_error(void) { return g_err.c_str(); }

}  // extern "C"
