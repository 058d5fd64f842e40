// amrmg_state.hpp -- host-side state of libamrmg shared by its C-ABI source
// files (amrmg_api.cpp, amrmg_build.cpp, amrmg_particles.cpp,
// amrmg_solver.cpp): error reporting, grow-only device and pinned buffers,
// the device copy of the merged hierarchy metadata with the solve workspace
// (DevState), per-launch profiling, and the context behind amrmg_ctx.
// Internal to the library; no torch types, no oracle code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "amrmg.h"
#include "amrmg_hier.hpp"
#include "amrmg_kernels.hpp"
#include "amrmg_noalloc.hpp"

using namespace amrmg;

// record the message behind the status for amrmg_last_error (thread-local)
// and return the status
amrmg_status fail(amrmg_status s, const std::string &m);

#define HIP_TRY(x)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(AMRMG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// ---------------------------------------------------------------------------
// grow-only device and pinned host buffers (allocation happens only when a
// hierarchy outgrows its predecessor, so regrids do not reallocate)
// ---------------------------------------------------------------------------
struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t c = n + n / 4 + 4096;
        hipError_t e = hipMalloc(&p, c);
        if (e == hipSuccess) cap = c;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    ~DBuf() { release(); }
};

// host memory the device writes and the host polls (coherent, mapped)
struct CBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc(&p, n, hipHostMallocCoherent | hipHostMallocMapped);
        if (e == hipSuccess) {
            cap = n;
            std::memset(p, 0, n);
        }
        return e;
    }
    ~CBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

struct PBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t c = n + n / 4 + 4096;
        hipError_t e = hipHostMalloc(&p, c);
        if (e == hipSuccess) cap = c;
        return e;
    }
    ~PBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

// Packs host arrays into one pinned staging buffer and one device buffer
// with a single host-to-device copy.
struct Packer {
    struct Item {
        const void *src;
        size_t bytes, off;
        void **dst;
    };
    std::vector<Item> items;
    size_t total = 0;
    template <class V>
    void add(const std::vector<V> &v, V **dst)
    {
        add_raw(v.data(), sizeof(V) * v.size(), (void **)dst);
    }
    void add_raw(const void *src, size_t bytes, void **dst)
    {
        items.push_back({src, bytes, total, dst});
        total += align256(bytes ? bytes : 1);
    }
    amrmg_status run(DBuf &dev, PBuf &stage, hipStream_t st)
    {
        HIP_TRY(stage.ensure(total));
        HIP_TRY(dev.ensure(total));
        for (auto &it : items) {
            if (it.bytes) std::memcpy((char *)stage.p + it.off, it.src, it.bytes);
            *it.dst = (char *)dev.p + it.off;
        }
        HIP_TRY(hipMemcpyAsync(dev.p, stage.p, total, hipMemcpyHostToDevice, st));
        return AMRMG_OK;
    }
};

#define ST_TRY(x)                                \
    do {                                         \
        amrmg_status s_ = (x);                   \
        if (s_ != AMRMG_OK) return s_;           \
    } while (0)

// ---------------------------------------------------------------------------
// device copy of merged metadata plus the solve workspace
// ---------------------------------------------------------------------------
struct DevState {
    Meta meta;
    DevMeta M{};
    DBuf metabuf;
    PBuf stage;
    // brick tables built on the device (org, nbr, child, ... and the scan
    // scratch); per-level counts come back through bsum
    DBuf brickbuf;
    CBuf bsum;
    unsigned bseq = 0;
    int n_amr = 0, amr_first = 0, n_reflux = 0;  // AMR bricks (list d_amr), update list length
    int32_t *d_reflux = nullptr, *d_amr = nullptr;
    int2 *d_ranges = nullptr;  // brick range of each AMR level of each problem
    std::vector<int> range_prob, range_amr;
    int4 *d_jobs = nullptr;
    int njobs = 0;
    size_t cg_doubles = 0;
    CoarseJob *d_cjobs = nullptr;
    int n_cg = 0;  // problems whose coarsest grid is solved by CG
    // direct solves of the coarsest grids: tables, jobs, work lists, scratch
    double *d_dtab = nullptr;
    DirectJob *d_djobs = nullptr;
    int2 *d_planes = nullptr, *d_groups = nullptr;
    int n_planes = 0, n_groups = 0, direct_maxdim = 0;
    int n_djobs = 0;
    DirectJob djob0{};  // host copy of the job when there is one
    size_t dw_doubles = 0;
    double *dw = nullptr;
    int kc = 0;  // levels 0..kc of every problem run in the one-workgroup coarse cycle
    // per-level pointer tables: phi[ne], rho[ne], rout[ne], E[3 ne]
    DBuf ptrbuf;
    PBuf ptrstage;
    double **d_phi = nullptr, **d_rho = nullptr, **d_E = nullptr, **d_rout = nullptr;
    std::vector<double *> h_phi, h_rho, h_E, h_rout;
    // workspace
    DBuf ws_own;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int ws_prec = -1;
    void *e = nullptr, *r = nullptr, *et = nullptr, *cpe = nullptr;
    double *cpphi = nullptr, *part = nullptr, *dnorm = nullptr;
    double *ffs = nullptr;  // fine sums of coarse-fine faces, 96 per brick
    double *phib = nullptr, *rhob = nullptr;  // FP64 phi and rho in brick layout during a solve
    double *cgw = nullptr;
    int *cgit = nullptr;
    int cg_threads = 1024;
    PBuf h_normbuf;
    double *h_norm = nullptr;
    // norms of each outer iteration, published by the norms kernel: values,
    // then a sequence number; the device keeps the count at d_seqc
    CBuf pubbuf;
    double *h_pub = nullptr;
    unsigned *h_seq = nullptr, *d_seqc = nullptr;
    unsigned seq = 0;
    // AMR-level brick maps with global brick ids of the first problem (views
    // into the map pool)
    std::vector<int32_t *> d_bmap;
    // face data generated on the device: gbc, cf_pat, cf_idx, error flag
    DBuf facebuf;
    int *d_face_err = nullptr;
    PBuf h_face_err;
    // captured outer iteration (V-cycle, phi update, FP64 residual, norms)
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;
    int meta_gen = 0;
    hipStream_t cap_stream = nullptr;  // capture needs a stream other than the null stream
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        gkey.clear();
    }
    ~DevState()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};
// ---------------------------------------------------------------------------
// per-launch event timing of selected kernel classes
// ---------------------------------------------------------------------------
struct Prof {
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int cls;
        size_t ev;  // index of the start event; end = ev + 1
        double bytes;
    };
    std::vector<Rec> recs;
    double tot_ms[AMRMG_K_NCLASS] = {}, tot_bytes[AMRMG_K_NCLASS] = {};
    int64_t tot_n[AMRMG_K_NCLASS] = {};
    // per-launch (ms, bytes) of each class, the first kMaxKept launches
    static constexpr size_t kMaxKept = 65536;
    std::vector<std::pair<double, double>> kept[AMRMG_K_NCLASS];
    size_t pending = (size_t)-1;
    int pending_cls = -1;

    bool on(int cls) const { return (mask >> cls) & 1; }
    void begin(int cls)
    {
        pending = (size_t)-1;
        if (!on(cls)) return;
        if (used + 2 > pool.size()) flush();
        if (used + 2 > pool.size()) return;
        pending = used;
        pending_cls = cls;
        set_launch_timing(pool[used], pool[used + 1]);
        used += 2;
    }
    void end(int cls, double bytes)
    {
        if (pending == (size_t)-1 || pending_cls != cls) return;
        if (launch_timing_pending()) {  // the launcher launched nothing
            set_launch_timing(nullptr, nullptr);
            used -= 2;
        } else {
            recs.push_back({cls, pending, bytes});
        }
        pending = (size_t)-1;
    }
    // fold the recorded launches into the totals (waits for them)
    void flush()
    {
        for (const auto &r : recs) {
            float e = 0.f;
            if (hipEventSynchronize(pool[r.ev + 1]) == hipSuccess &&
                hipEventElapsedTime(&e, pool[r.ev], pool[r.ev + 1]) == hipSuccess) {
                tot_ms[r.cls] += e;
                tot_bytes[r.cls] += r.bytes;
                tot_n[r.cls] += 1;
                if (kept[r.cls].size() < kMaxKept) kept[r.cls].emplace_back((double)e, r.bytes);
            }
        }
        recs.clear();
        used = 0;
    }
    void reset(uint32_t m)
    {
        mask = m;
        used = 0;
        recs.clear();
        for (int c = 0; c < AMRMG_K_NCLASS; ++c) tot_ms[c] = tot_bytes[c] = 0.0, tot_n[c] = 0, kept[c].clear();
        if (m && pool.empty()) {
            pool.resize(1 << 12);
            for (auto &e : pool) (void)hipEventCreate(&e);
        }
    }
    ~Prof()
    {
        for (auto &e : pool) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct amrmg_ctx {
    amrmg_params P{};
    std::vector<double> mono;
    hipStream_t st = nullptr;
    Problem prob;
    bool built = false;
    DevState ds;
    // scratch of the tagging passes of build_hierarchy
    DBuf tag_marks, tag_scratch, tag_geom, tag_fields, tag_bits;
    PBuf tag_stage, tag_host;
    // spatial visiting order of the particles (a performance hint for the
    // deposit; any order gives the same sums up to rounding)
    DBuf sort_scratch, sort_vals;  // the sort's work space; the order and its inverse
    DBuf sorted;  // the particles of the last build in visiting order (charges, x, y, z)
    uint32_t *perm = nullptr;
    uint32_t *iperm = nullptr;  // its inverse (perm[iperm[p]] == p)
    int64_t perm_n = -1;
    // E of a gather in visiting order (one double4 per particle), before it
    // is written in the caller's order
    DBuf gather_rec;
    DBuf dep_count;
    // what the last build keeps for amrmg_deposit_built: the charge of each
    // level it deposited for tagging (caller's layout), the particle count
    // and position type of the ordered copy, and its count of particles
    // outside the domain (device, valid when level 0 was deposited)
    std::vector<DBuf> lev_rho;
    std::vector<char> lev_rho_ok;
    int64_t built_n = -1;
    int built_pos = -1;
    DBuf built_nout;
    void *user_ws = nullptr;
    size_t user_ws_bytes = 0;
    int generation = 0;
    // batch cache (kept by the first context of a batch)
    std::vector<amrmg_ctx *> batch_ctx;
    std::vector<int> batch_gen;
    DevState *batch = nullptr;
    Prof prof;
    // the device of the context's stream, and two events made on it at
    // creation for the timing of amrmg_solve_noalloc (which makes none)
    int device = -1;
    hipEvent_t ev_solve[2] = {nullptr, nullptr};
    ~amrmg_ctx()
    {
        delete batch;
        for (auto &e : ev_solve)
            if (e) (void)hipEventDestroy(e);
    }
};

struct SolveOpts {
    int precision, smoother, nu1, nu2, norm_p, max_iters;
    double omega, bottom_rtol, inv_eps0;
};

// amrmg_build.cpp: upload the merged metadata of probs into D (one copy),
// build the brick tables and face data on the device
amrmg_status upload_meta(DevState &D, hipStream_t st, const std::vector<const Problem *> &probs, bool direct);

// amrmg_particles.cpp
bool big_tile(const amrmg_ctx *ctx, int level);
DepLevel dep_level(const Problem &P, const HostLevel &L, const int32_t *bmap);
amrmg_status compute_order(amrmg_ctx *ctx, int pos_dtype, const void *x, const void *y, const void *z,
                           const double *q, int64_t n, bool copy, const void **xs, const void **ys,
                           const void **zs, const double **qs);

// amrmg_solver.cpp: workspace bytes of a solve on D, and carving the
// workspace (the caller's buffer user, else the library's own)
size_t ws_need(const DevState &D, int prec);
amrmg_status ensure_ws(DevState &D, int prec, void *user, size_t user_bytes);
