// C ABI and host driver of the MI355X Stokes Schur-complement solver.
//
// The outer loop is Algorithm 1 of Pimanov et al. (arXiv 2307.05266, Sec. 3.1)
// written as standard preconditioned CG on S p = g (residual r = g - S p),
// with S d = B A^{-1} B^T d applied through an inner Jacobi-PCG solve with A
// and, for the SIMPLE preconditioner (eq. schur_uzawa_prec), z = Shat^+ r by an
// inner Jacobi-PCG solve with Shat = B diag(A)^{-1} B^T (Sec. 3.2).  Inner
// loops keep their scalars on the device; the host only polls a small state
// block every few iterations.  Outer scalars are formed on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/stokes.h"
#include "geometry.h"
#include "kernels.h"
#include "mg.h"

using namespace stokes;

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return STOKES_E_DEVICE;   \
    } while (0)

#define ST_TRY(expr)                                    \
    do {                                                \
        stokes_status _s = (expr);                      \
        if (_s < 0) return _s;                          \
    } while (0)

namespace {

constexpr int kMaxN = 800;
using GraphKey = std::array<uintptr_t, 8>;
constexpr int kCompBlocks = 256;

// kinds of timed kernels and their algorithmic bytes per voxel (FP64)
enum { kTimeADir = 0, kTimeAStencil = 1, kTimeAUpdate = 2, kTimeSDir = 3, kTimeSStencil = 4, kTimeSUpdate = 5,
       kTimeMgARestrict = 6, kTimeMgASmooth = 7, kTimeMgSRestrict = 8, kTimeMgSSmooth = 9,
       kTimeAUpdRestrict = 10, kTimeSUpdRestrict = 11, kTimeADirStencil = 12, kTimeSDirStencil = 13,
       kTimeSUpdRestrictPipe = 14, kTimeMgSSmoothPipe = 15, kTimeSDirStencilPipe = 16, kTimeKinds = 17 };
// A dir     : r, d read (3 planes each), code byte read; d written
// A stencil : d read, code byte read; q written
// A update  : x, d, r, q read, code byte read; x, r written
// S dir     : r, inverse diagonal, d read; d written
// S stencil : d read, code byte read; q written
// S update  : inverse diagonal, x, d, r, q read; x, r written
// multigrid, level 0 (1/8 of a value per voxel for the level-1 vector):
// A restriction   : b (3 planes), code byte read; level-1 b written
// A smoothing     : b (3 planes), code byte, level-1 x read; y (3 planes) written
// S restriction   : b, inverse diagonal, code byte read; level-1 b written
// S smoothing     : b, inverse diagonal, code byte, level-1 x read; y written
// A update + restriction: x, r, d, q read (3 planes), code byte; x, r written, level-1 b written
// S update + restriction: inverse diagonal, x, r, d, q read, code byte; x, r written, level-1 b written
// A direction + stencil: z, d read (3 planes), code byte; d, q written (3 planes)
// S direction + stencil: z, d read, code byte; d, q written
// the FP64 SIMPLE solve's software-pipelined forms (option mg_pipe):
// S update + restriction: x, r, d, q read, 16-bit code; x, r written, level-1 b written
// S smoothing: b, 16-bit code, level-1 x read; y written
// S direction + stencil: z, d read, 16-bit code; d, q written
constexpr double kBytesPerCell[kTimeKinds] = {9 * 8 + 1,     6 * 8 + 1,         18 * 8 + 1,    4 * 8,
                                              2 * 8 + 1,     7 * 8,             3 * 8 + 1 + 3, 6 * 8 + 1 + 3,
                                              2 * 8 + 1 + 1, 3 * 8 + 1 + 1,     18 * 8 + 1 + 3, 7 * 8 + 1 + 1,
                                              12 * 8 + 1,    4 * 8 + 1,         6 * 8 + 2 + 1, 2 * 8 + 2 + 1,
                                              4 * 8 + 2};

}  // namespace

// tiled coarse-level sweeps: 1 024 blocks (measured: 256 left the 64^3 and 128^3
// levels latency-bound, 2 048 and 4 096 gain nothing more)
constexpr int kMgLevelBlocksDefault = 1024;

struct stokes_ctx {
    int N = 0;
    int64_t n3 = 0;
    double force[3] = {0, 0, 0};
    unsigned setup_flags = 0;
    hipStream_t stream = nullptr;
    int device = 0;                // the device current at setup
    // batched context (stokes_setup_batch): nbatch members of one size, member
    // m's buffers at m * bstride bytes from member 0's (a plain context: 1, 0)
    int nbatch = 1;
    size_t bstride = 0;
    bool batch_api = false;        // set up by stokes_setup_batch (any member count)
    char* slab = nullptr;          // batched: the members' common allocation
    size_t slab_used = 0;          // bytes of member 0's part handed out so far
    struct Member {
        int64_t nfluid_in = 0, nfluid = 0, nsurf = 0;
        int ncomp_all = 0, ncomp_kept = 0;
        int64_t nface[3] = {0, 0, 0};
    };
    std::vector<Member> member;    // per member (plain: one)
    std::vector<stokes_report> mrep;        // per member: report of the last solve
    std::vector<std::vector<double>> mhist; // per member: history of the last solve
    std::vector<int> m_it, m_status;        // per member: last inner solve's iterations, status
    double* noalloc_scratch = nullptr;  // this device's copy of `scratch` (stokes_apply_device_noalloc)

    // geometry summary
    int64_t nfluid_in = 0, nfluid = 0, nsurf = 0;
    int ncomp_all = 0, ncomp_kept = 0;
    int64_t nface[3] = {0, 0, 0};

    Sweep sw{};
    Sweep sw32{};           // the FP32 inner solves' sweep
    int wpr = 0;            // bitmask words per x-row

    // device memory
    uint32_t* bits = nullptr;
    uint8_t* code = nullptr;
    uint16_t* label = nullptr;     // only with more than one component
    double* comp_count = nullptr;  // [K]
    double* comp_part = nullptr;   // [kCompBlocks][K]
    double* proj_part = nullptr;   // [kMaxBlocks] partials of the one-component projection
    double* comp_mean = nullptr;   // [K]
    double *fx = nullptr, *fr = nullptr, *fq = nullptr, *u = nullptr;  // faces
    double* fd = nullptr;                                               // faces, inner direction
    double *p = nullptr, *r = nullptr, *zs = nullptr, *d = nullptr, *q = nullptr;  // cells
    double *sr = nullptr, *sq = nullptr, *invdS = nullptr;                         // cells (SIMPLE solve)
    uint16_t* code2 = nullptr;     // lower and upper face states of every voxel (k_code2)
    double* sd = nullptr;                                                          // cells, inner direction
    // FP32 inner-solve vectors of the mixed-precision path (allocated on first use)
    float *fx32 = nullptr, *fr32 = nullptr, *fd32 = nullptr, *fq32 = nullptr;     // faces
    float *zs32 = nullptr, *sr32 = nullptr, *sd32 = nullptr, *sq32 = nullptr;     // cells
    float* invdS32 = nullptr;
    // multigrid hierarchies: the SIMPLE matrix (one plane) and A (three planes)
    struct MgHier {
        int levels = 0;                // 0: none (odd size or tiny box)
        int nb = 1, kind = 0;
        std::vector<MgGrid> grid;      // [0..levels]
        std::vector<Sweep> sweep;      // [0..levels]: sweeps of the tiled level kernels (side >= 64)
        // w: level 1 only, the residual of the first visit of a two-visit cycle
        struct Lev64 { double *D, *Wx, *Wy, *Wz, *b, *x, *y, *w; };
        struct Lev32 { float *D, *Wx, *Wy, *Wz, *b, *x, *y, *w; };
        std::vector<Lev64> l64;        // [1..levels]
        std::vector<Lev32> l32;        // FP32 vectors; D, Wx, Wy, Wz point into c32
        // the coarse operators in FP32, read by the cycle in both precisions
        struct LevC { float *D, *Wx, *Wy, *Wz; };
        std::vector<LevC> c32;         // [1..levels]
        double* z = nullptr;           // fine level: output of the cycle
        float* z32 = nullptr;
        double* r2 = nullptr;          // fine level: second residual buffer of the fused update
        float* r2_32 = nullptr;
        double* d2 = nullptr;          // fine level: second direction buffer of the fused direction + stencil
        float* d2_32 = nullptr;
    };
    MgHier mgS, mgA;
    int use_mg = 1;                    // SIMPLE inner solve: 1 multigrid-PCG, 0 Jacobi-PCG
    int use_mg_A = 1;                  // inner solve with A: 1 multigrid-PCG, 0 Jacobi-PCG
    double mg_omega = 0.9, mg_scale = 1.7, mg_scale_A = 1.5;   // coarse-correction scale: SIMPLE matrix, A
    double mg_scale_deep = 0.0;    // SIMPLE matrix: scale of the corrections into levels >= 2 (0: mg_scale)
    double mg_deep_auto = 0.0;     // the same, chosen by prepare_two_visits (0: none)
    // multigrid solves: direction fused with the stencil (measured: a gain for
    // the SIMPLE matrix; about even for A, whose fused sweep loads z and d at
    // the ring points of three planes)
    int fuse_dir_A = 0, fuse_dir_S = 1;
    int mg_pipe = 1;
    int mg_coarse_sweeps = 8;
    // coarse-level smoother: 0 damped Jacobi; 1 red-black Gauss-Seidel below the
    // tiled size; 2 red-black Gauss-Seidel on every coarse level but the coarsest
    int mg_coarse_gs = 1;
    int mg_level_blocks = kMgLevelBlocksDefault;   // target blocks of a tiled coarse-level sweep
    // visits of level 1 per cycle of the SIMPLE matrix: 0 (auto) two where level
    // 1 has a side of at least kMgTwoVisitMinSide, 1 never, 2 wherever level 1 is
    // tiled; never where level 1 is the coarsest or smooths by Gauss-Seidel
    int mg_visits = 0;
    int mg_two_ok = 0;             // auto mode: 0 not yet estimated, 1 two visits, -1 one
    double mg_lambda1 = 0.0;       // the estimate of the largest eigenvalue of B_1 A_1
    CgState* cg = nullptr;         // [0] A, [1] SIMPLE
    double* part = nullptr;        // [kNumSlots][kMaxBlocks] partials of the inner loops
    double* dpart = nullptr;       // [kMaxBlocks][3] partials of host-side sums
    std::vector<std::pair<void*, size_t>> allocations;
    int64_t device_bytes = 0;
    bool async_alloc = false;      // allocations ordered on `stream` (stokes_setup_on_stream)
    stokes_allocator ext_alloc{};  // caller's allocator (stokes_setup_with_allocator), else all NULL
    int progress = 0;              // > 0: report every n-th outer iteration on stderr
    std::chrono::steady_clock::time_point t_solve0;
    CgState* host_state = nullptr; // pinned
    double* host_part = nullptr;   // pinned [3 * kMaxBlocks]
    int sweep_blocks = 1024;
    // mixed precision: FP32 inner solves, FP64 outer flexible CG with FP64
    // true-residual refinement
    int precision = 0;             // 0: FP64 throughout, 1: mixed
    double eps_A32 = 1e-5, eps_S32 = 1e-5;   // FP32 inner tolerances
    double cycle_rtol = 1e-4;      // residual reduction per defect-correction cycle
    double eps_refine = 1e-12;     // FP64 velocity refinement tolerance
    int max_refine = 12;
    // g counts as zero below zero_rhs_factor * eps * sqrt(f . u0) (rhs_floor)
    double zero_rhs_factor = 1000.0;

    // options
    double eps_A = 1e-12, eps_S = 1e-12;
    int max_outer = 5000, max_inner = 100000;
    int stop_prec = 0, check_every = 0, true_velocity = 0;
    int timing = 0;                // 0: off; n: time every n-th iteration of each inner solve
    int64_t timing_seen[2] = {};   // iterations seen per inner solve (0: A, 1: SIMPLE)
    bool time_iter = false;        // the iteration being launched is a timed one
    // captured inner iterations (HIP graphs), keyed by solver variant and vectors
    int use_graphs = 1;
    hipStream_t cap_stream = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;

    // adaptive polling
    int last_it[2] = {0, 0};

    // results
    bool have_solution = false;
    stokes_report rep{};
    std::vector<double> hist;

    // kernel timing: event pairs around the inner-loop kernels, by kind
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    double timing_ms[kTimeKinds] = {};
    int64_t timing_launches[kTimeKinds] = {};
};

namespace {

Sweep make_sweep(int N, int target_blocks) {
    Sweep s{};
    s.N = N;
    s.N2 = N * N;
    s.n3 = N * N * N;
    // x-extent of a column: 64 unless 32 wastes fewer idle lanes at the row end
    const int waste64 = (N + 63) / 64 * 64 - N, waste32 = (N + 31) / 32 * 32 - N;
    s.bxlog = (N >= 64 && waste64 <= waste32) ? 6 : 5;
    const int bx = 1 << s.bxlog, by = kBlock >> s.bxlog;
    s.gx = (N + bx - 1) / bx;
    s.gy = (N + by - 1) / by;
    const int cols = s.gx * s.gy;
    int gz = std::max(1, std::min(N, (target_blocks + cols - 1) / cols));
    s.lz = (N + gz - 1) / gz;
    // even N: even z-runs, so the multigrid restriction pairs planes within a block
    if (N % 2 == 0 && (s.lz & 1)) ++s.lz;
    s.gz = (N + s.lz - 1) / s.lz;
    s.nblk = s.gx * s.gy * s.gz;
    s.nbatch = 1;
    s.active = 1u;
    s.bstride = 0;
    return s;
}

// Sweep of the FP32 inner solves: their kernels hold about half the registers
// of the FP64 ones and keep twice the waves per SIMD, so they run over up to
// twice the blocks, as long as a block's z-run keeps at least 8 planes (the
// first and last plane of a run are loaded twice).
Sweep make_sweep32(int N, int target_blocks) {
    const Sweep s = make_sweep(N, target_blocks);
    const int cols = s.gx * s.gy;
    const int t = std::min(2 * target_blocks, std::max(target_blocks, cols * std::max(1, N / 8)));
    return make_sweep(N, std::min(t, kMaxBlocks));
}

// the sweep of an inner solve in precision T (one for all its kernels)
const Sweep& inner_sweep(const stokes_ctx* c, double) { return c->sw; }
const Sweep& inner_sweep(const stokes_ctx* c, float) { return c->sw32; }

// Every device buffer of a context comes from here: the caller's allocator
// when one was given, else stream-ordered allocation for contexts set up on a
// stream (concurrent contexts never wait on each other's allocations), else
// hipMalloc.  Each buffer is cleared on the context's stream, so no kernel
// depends on what the memory held before (a caching allocator hands back
// used memory).
template <class T>
stokes_status dev_alloc(stokes_ctx* c, T** ptr, size_t count) {
    void* m = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (c->slab) {
        // batched: member 0's buffer at the next 256-byte boundary of its part
        // of the slab; every member has its own at the same offset
        const size_t off = (c->slab_used + 255) & ~(size_t)255;
        if (off + bytes > c->bstride) return STOKES_E_NOMEM;
        c->slab_used = off + bytes;
        m = c->slab + off;
        HIP_TRY(hipMemset2DAsync(m, c->bstride, 0, bytes, (size_t)c->nbatch, c->stream));
        *ptr = static_cast<T*>(m);
        return STOKES_OK;
    }
    if (c->ext_alloc.alloc) {
        m = c->ext_alloc.alloc(bytes, (void*)c->stream, c->ext_alloc.user);
        if (!m) return STOKES_E_NOMEM;
    } else {
        const hipError_t e = c->async_alloc ? hipMallocAsync(&m, bytes, c->stream) : hipMalloc(&m, bytes);
        if (e != hipSuccess) return STOKES_E_NOMEM;
    }
    c->allocations.push_back({m, bytes});
    c->device_bytes += (int64_t)bytes;
    HIP_TRY(hipMemsetAsync(m, 0, bytes, c->stream));
    *ptr = static_cast<T*>(m);
    return STOKES_OK;
}

void release(stokes_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->ext_alloc.alloc) {
        // the caller's allocator may hand the memory to other work at once
        (void)(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
        for (auto& a : c->allocations) c->ext_alloc.free(a.first, a.second, (void*)c->stream, c->ext_alloc.user);
    } else {
        for (auto& a : c->allocations)
            (void)(c->async_alloc ? hipFreeAsync(a.first, c->stream) : hipFree(a.first));
        if (c->async_alloc && c->stream) (void)hipStreamSynchronize(c->stream);
    }
    c->allocations.clear();
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_part) (void)hipHostFree(c->host_part);
    c->host_state = nullptr;
    c->host_part = nullptr;
}

dim3 grid_of(const Sweep& s) { return dim3((unsigned)s.nblk, (unsigned)s.nbatch); }

// bit mask of members 0 .. B-1
unsigned all_members_of(int B) { return B >= 32 ? 0xFFFFFFFFu : ((1u << B) - 1u); }

// the same scalar for member 0 (plain contexts)
MemberScalars ms1(double v) {
    MemberScalars m{};
    m.v[0] = v;
    return m;
}

// The members' copy of a sweep (grid y = member, their buffers bstride apart).
Sweep member_sweep(const stokes_ctx* c, Sweep s) {
    s.nbatch = c->nbatch;
    s.bstride = c->bstride;
    s.active = all_members_of(c->nbatch);
    return s;
}


// ---- inner solves -----------------------------------------------------------
// With kernel timing on, every `timing`-th iteration of an inner solve runs
// eagerly with each of its kernels bracketed by HIP events (the others are
// untimed, or replayed as a graph), so the events barely perturb the run they
// measure; the open flag tells time_end whether to close.
stokes_status time_begin(stokes_ctx* c, int kind, bool* open) {
    *open = false;
    if (!c->timing || !c->time_iter) return STOKES_OK;
    *open = true;
    if (c->ev_used + 2 > c->ev.size()) {
        for (int q = 0; q < 512; ++q) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            c->ev.push_back(e);
            c->ev_kind.push_back(0);
        }
    }
    c->ev_kind[c->ev_used] = kind;
    HIP_TRY(hipEventRecord(c->ev[c->ev_used], c->stream));
    return STOKES_OK;
}

stokes_status time_end(stokes_ctx* c, bool open) {
    if (!open) return STOKES_OK;
    HIP_TRY(hipEventRecord(c->ev[c->ev_used + 1], c->stream));
    c->ev_used += 2;
    return STOKES_OK;
}

stokes_status collect_timing(stokes_ctx* c) {
    if (c->ev_used == 0) return STOKES_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t q = 0; q + 1 < c->ev_used; q += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[q], c->ev[q + 1]));
        c->timing_ms[c->ev_kind[q]] += ms;
        c->timing_launches[c->ev_kind[q]] += 1;
    }
    c->ev_used = 0;
    return STOKES_OK;
}

// Inner-CG state of every member (host_state[m]).
stokes_status read_states(stokes_ctx* c, int which) {
    if (c->nbatch == 1)
        HIP_TRY(hipMemcpyAsync(c->host_state, c->cg + which, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    else
        HIP_TRY(hipMemcpy2DAsync(c->host_state, sizeof(CgState), c->cg + which, c->bstride, sizeof(CgState),
                                 (size_t)c->nbatch, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STOKES_OK;
}

int first_batch(stokes_ctx* c, int which) {
    if (c->check_every > 0) return c->check_every;
    return c->last_it[which] > 0 ? std::max(1, c->last_it[which]) : 16;
}

int next_batch(stokes_ctx* c) { return c->check_every > 0 ? c->check_every : 4; }

// Inner solves in the value type T (double, or float on the mixed path).
template <class T>
struct InnerA {
    T *x, *r, *d, *q;
};
template <class T>
struct InnerS {
    T *x, *r, *d, *q;
    const T* invd;
};

InnerA<double> bufA64(stokes_ctx* c) { return {c->fx, c->fr, c->fd, c->fq}; }
InnerA<float> bufA32(stokes_ctx* c) { return {c->fx32, c->fr32, c->fd32, c->fq32}; }
InnerS<double> bufS64(stokes_ctx* c) { return {c->zs, c->sr, c->sd, c->sq, c->invdS}; }
InnerS<float> bufS32(stokes_ctx* c) { return {c->zs32, c->sr32, c->sd32, c->sq32, c->invdS32}; }

// ---- iteration driver ---------------------------------------------------------
// An inner solve launches the same sequence every iteration (the iteration
// index lives in the device state), so the sequence is captured once per
// context and vector set as a HIP graph and replayed; the host polls the device
// state between batches.  Captures run on a private stream (the context's
// stream may be the legacy null stream, which cannot capture); the graph is
// launched on the context's stream.
void drop_graphs(stokes_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

template <class Body>
stokes_status capture_graph(stokes_ctx* c, Body& body, hipGraphExec_t* out) {
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipStream_t keep = c->stream;
    c->stream = c->cap_stream;
    const stokes_status st = body();
    c->stream = keep;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (st != STOKES_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != STOKES_OK ? st : STOKES_E_DEVICE;
    }
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return ei == hipSuccess ? STOKES_OK : STOKES_E_DEVICE;
}

// Run inner-CG iterations of solve `which` (0: A, 1: SIMPLE) until the device
// state says done.  body(parity) launches one iteration; iterations go in
// pairs (parity 0 then 1: the fused multigrid update alternates its two
// residual buffers), so a graph holds one pair and a batch is rounded up to
// whole pairs (iterations queued after convergence return at once).  key
// identifies the launch sequence (solver variant and vectors) for the cache.
template <class Body>
stokes_status run_inner(stokes_ctx* c, int which, const GraphKey& key, Body body, int* iters, int* status) {
    auto pair = [&body]() -> stokes_status {
        ST_TRY(body(0));
        return body(1);
    };
    hipGraphExec_t g = nullptr;
    if (c->use_graphs) {
        auto it = c->graphs.find(key);
        if (it != c->graphs.end()) {
            g = it->second;
        } else {
            ST_TRY(capture_graph(c, pair, &g));
            c->graphs[key] = g;
        }
    }
    int batch = first_batch(c, which);
    const int B = c->nbatch;
    for (;;) {
        for (int t = 0; t < (batch + 1) / 2; ++t) {
            c->time_iter = c->timing && (c->timing_seen[which]++ % c->timing) == 0;
            if (g && !c->time_iter) {
                HIP_TRY(hipGraphLaunch(g, c->stream));
            } else {
                ST_TRY(pair());
            }
            c->time_iter = false;
        }
        HIP_TRY(hipGetLastError());
        ST_TRY(read_states(c, which));
        bool all = true;
        for (int m = 0; m < B; ++m) all = all && c->host_state[m].done;
        if (all) break;
        batch = next_batch(c);
    }
    // per member: iterations and status (members that sat out report 0, 0)
    int most = 0, worst = 0;
    c->m_it.assign(B, 0);
    c->m_status.assign(B, 0);
    for (int m = 0; m < B; ++m) {
        const CgState& h = c->host_state[m];
        c->m_it[m] = h.it;
        c->m_status[m] = h.status;
        most = std::max(most, h.it);
        if (h.status == -4 || (h.status == 1 && worst == 0)) worst = h.status;
    }
    c->last_it[which] = most;
    *iters = most;
    *status = worst;
    return STOKES_OK;
}

template <class T>
GraphKey graph_key(int variant, const void* a, const void* b, const void* cc, const void* d, const void* e,
                   const void* f) {
    return {(uintptr_t)variant, (uintptr_t)sizeof(T), (uintptr_t)a, (uintptr_t)b, (uintptr_t)cc, (uintptr_t)d,
            (uintptr_t)e, (uintptr_t)f};
}

// Solve A x = b on the faces (b: an FP64 face vector, or nullptr for the
// uniform force), Jacobi-preconditioned.  One iteration: direction, stencil
// and update kernels.
template <class T>
stokes_status cg_A(stokes_ctx* c, InnerA<T> v, const double* b, double eps, int* iters, int* status) {
    const Sweep& s = inner_sweep(c, T());
    CgState* st = c->cg + 0;
    hipLaunchKernelGGL(k_cgA_init<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, b, c->force[0],
                       c->force[1], c->force[2], v.x, v.r, st, c->part, eps, c->max_inner);
    HIP_TRY(hipGetLastError());
    auto body = [c, s, st, v](int) -> stokes_status {
        bool open;
        ST_TRY(time_begin(c, kTimeADir, &open));
        hipLaunchKernelGGL(k_cgA_dir<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.r, v.d, st, c->part,
                           (const T*)nullptr);
        ST_TRY(time_end(c, open));
        ST_TRY(time_begin(c, kTimeAStencil, &open));
        hipLaunchKernelGGL(k_cgA_stencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.d, v.q, st,
                           c->part);
        ST_TRY(time_end(c, open));
        ST_TRY(time_begin(c, kTimeAUpdate, &open));
        hipLaunchKernelGGL(k_cgA_update<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.x, v.r, v.d, v.q,
                           st, c->part);
        ST_TRY(time_end(c, open));
        return STOKES_OK;
    };
    return run_inner(c, 0, graph_key<T>(0, v.x, v.r, v.d, v.q, nullptr, nullptr), body, iters, status);
}

// Solve Shat x = b on the cells (b: an FP64 cell vector, already projected),
// Jacobi-preconditioned.
template <class T>
stokes_status cg_S(stokes_ctx* c, InnerS<T> v, const double* b, double eps, int* iters, int* status) {
    const Sweep& s = inner_sweep(c, T());
    CgState* st = c->cg + 1;
    hipLaunchKernelGGL(k_cgS_init<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, v.invd, b, v.x, v.r, st, c->part,
                       eps, c->max_inner);
    HIP_TRY(hipGetLastError());
    auto body = [c, s, st, v](int) -> stokes_status {
        bool open;
        ST_TRY(time_begin(c, kTimeSDir, &open));
        hipLaunchKernelGGL(k_cgS_dir<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, v.invd, v.r, v.d, st, c->part,
                           (const T*)nullptr);
        ST_TRY(time_end(c, open));
        ST_TRY(time_begin(c, kTimeSStencil, &open));
        hipLaunchKernelGGL(k_cgS_stencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.d, v.q, st,
                           c->part);
        ST_TRY(time_end(c, open));
        ST_TRY(time_begin(c, kTimeSUpdate, &open));
        hipLaunchKernelGGL(k_cgS_update<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, v.invd, v.x, v.r, v.d, v.q,
                           st, c->part);
        ST_TRY(time_end(c, open));
        return STOKES_OK;
    };
    return run_inner(c, 1, graph_key<T>(1, v.x, v.r, v.d, v.q, v.invd, nullptr), body, iters, status);
}

// ---- multigrid preconditioners ---------------------------------------------
int flat_blocks(int n, int cap = 2048) { return std::max(1, std::min(cap, (n + kBlock - 1) / kBlock)); }
// one thread per item (kernels without a grid-stride loop)
unsigned exact_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }
using MgHier = stokes_ctx::MgHier;

// red-black Gauss-Seidel kernels: one workgroup per brick of kGsB^3 nodes of a
// plane.  A window reaches two nodes past its brick and is wrapped once, which
// holds for sides above kGsB; levels that are restricted further have an even
// side with more than 512 nodes, so at least 10.
constexpr int kGsMinSide = kGsB + 2;
unsigned gs_blocks(const MgGrid& g) {
    const int nbk = (g.n + kGsB - 1) / kGsB;
    return (unsigned)(g.nb * nbk * nbk * nbk);
}

// Levels: halve while the side is even and a level holds more than 512 nodes
// per plane; the coarsest level must fit one workgroup's LDS.
// Coarse levels with a side of at least this run the LDS-tiled kernels (over a
// sweep of about "mg_level_blocks" blocks); smaller ones are launch-latency
// bound and run the brick or one-thread-per-node kernels.
constexpr int kMgTiledMinSide = 64;

// Sides of the levels of a hierarchy with nb planes on an N^3 box (level 0
// first); a single entry when there is no hierarchy.
std::vector<int> mg_plan(int N, int nb) {
    std::vector<int> ns{N};
    int n = N;
    while (n % 2 == 0 && n / 2 >= 2 && n * n * n > 512) {
        n /= 2;
        ns.push_back(n);
    }
    if (ns.size() < 2 || (int64_t)nb * n * n * n > kMgCoarsestMax) ns.resize(1);
    return ns;
}

stokes_status build_mg(stokes_ctx* c, MgHier& h, int nb, int kind) {
    h.levels = 0;
    h.nb = nb;
    h.kind = kind;
    h.grid.clear();
    h.sweep.clear();
    for (int n : mg_plan(c->N, nb)) {
        h.grid.push_back({n, n * n, n * n * n, nb, c->bstride});
        h.sweep.push_back(member_sweep(c, make_sweep(n, c->mg_level_blocks)));
    }
    const int L = (int)h.grid.size() - 1;
    if (L < 1) return STOKES_OK;
    h.l64.assign(L + 1, {});
    for (int l = 1; l <= L; ++l) {
        auto& lv = h.l64[l];
        const size_t m = (size_t)nb * h.grid[l].n3;
        for (double** a : {&lv.D, &lv.Wx, &lv.Wy, &lv.Wz, &lv.b, &lv.x, &lv.y}) ST_TRY(dev_alloc(c, a, m));
        if (l == 1) ST_TRY(dev_alloc(c, &lv.w, m));
    }
    ST_TRY(dev_alloc(c, &h.z, (size_t)nb * c->n3));
    ST_TRY(dev_alloc(c, &h.r2, (size_t)nb * c->n3));
    ST_TRY(dev_alloc(c, &h.d2, (size_t)nb * c->n3));
    const int m1 = nb * h.grid[1].n3;
    hipLaunchKernelGGL(k_mg_coarsen_fine<double>, dim3((m1 + kBlock - 1) / kBlock, c->nbatch), dim3(kBlock), 0, c->stream,
                       h.grid[0], h.grid[1], kind, c->code, h.l64[1].D, h.l64[1].Wx, h.l64[1].Wy, h.l64[1].Wz);
    for (int l = 1; l < L; ++l) {
        const auto& f = h.l64[l];
        const auto& t = h.l64[l + 1];
        const int m = nb * h.grid[l + 1].n3;
        hipLaunchKernelGGL(k_mg_coarsen<double>, dim3((m + kBlock - 1) / kBlock, c->nbatch), dim3(kBlock), 0, c->stream,
                           h.grid[l], h.grid[l + 1], f.D, f.Wx, f.Wy, f.Wz, t.D, t.Wx, t.Wy, t.Wz);
    }
    // the FP32 copies the cycle reads (each level's Galerkin product formed in FP64 first)
    h.c32.assign(L + 1, {});
    for (int l = 1; l <= L; ++l) {
        auto& cc = h.c32[l];
        const int m = nb * h.grid[l].n3;
        for (float** a : {&cc.D, &cc.Wx, &cc.Wy, &cc.Wz}) ST_TRY(dev_alloc(c, a, (size_t)m));
        const auto& d = h.l64[l];
        const double* src[4] = {d.D, d.Wx, d.Wy, d.Wz};
        float* dst[4] = {cc.D, cc.Wx, cc.Wy, cc.Wz};
        for (int q = 0; q < 4; ++q)
            hipLaunchKernelGGL(k_narrow_flat, dim3(flat_blocks(m), c->nbatch), dim3(kBlock), 0, c->stream, m, src[q],
                               dst[q], c->bstride);
    }
    HIP_TRY(hipGetLastError());
    h.levels = L;
    return STOKES_OK;
}

// FP32 copy of a hierarchy for the mixed path
stokes_status build_mg32(stokes_ctx* c, MgHier& h) {
    const int L = h.levels;
    if (L < 1 || !h.l32.empty()) return STOKES_OK;
    h.l32.assign(L + 1, {});
    for (int l = 1; l <= L; ++l) {
        auto& lv = h.l32[l];
        const int m = h.nb * h.grid[l].n3;
        for (float** a : {&lv.b, &lv.x, &lv.y}) ST_TRY(dev_alloc(c, a, (size_t)m));
        if (l == 1) ST_TRY(dev_alloc(c, &lv.w, (size_t)m));
        lv.D = h.c32[l].D;
        lv.Wx = h.c32[l].Wx;
        lv.Wy = h.c32[l].Wy;
        lv.Wz = h.c32[l].Wz;
    }
    ST_TRY(dev_alloc(c, &h.z32, (size_t)h.nb * c->n3));
    ST_TRY(dev_alloc(c, &h.r2_32, (size_t)h.nb * c->n3));
    ST_TRY(dev_alloc(c, &h.d2_32, (size_t)h.nb * c->n3));
    HIP_TRY(hipGetLastError());
    return STOKES_OK;
}

template <class T>
struct MgView {
    T *D, *Wx, *Wy, *Wz, *b, *x, *y, *w;
};
MgView<double> mg_view(MgHier& h, int l, double) {
    auto& v = h.l64[l];
    return {v.D, v.Wx, v.Wy, v.Wz, v.b, v.x, v.y, v.w};
}
MgView<float> mg_view(MgHier& h, int l, float) {
    auto& v = h.l32[l];
    return {v.D, v.Wx, v.Wy, v.Wz, v.b, v.x, v.y, v.w};
}
double* mg_out(MgHier& h, double) { return h.z; }
float* mg_out(MgHier& h, float) { return h.z32; }
double* mg_r2(MgHier& h, double) { return h.r2; }
float* mg_r2(MgHier& h, float) { return h.r2_32; }
double* mg_d2(MgHier& h, double) { return h.d2; }
float* mg_d2(MgHier& h, float) { return h.d2_32; }

// The SIMPLE matrix's cycle visits level 1 twice where level 1 runs the tiled
// Jacobi kernels (a side of at least 64) and is not the coarsest, by default
// from a level-1 side of kMgTwoVisitMinSide: the second visit costs the
// latency-bound launches of the levels below 1 (about constant) and saves a
// third of the iterations on tight geometries, which pays where the level-0
// sweeps are long (measured: 256^3 tight spheres, FP64 solve 5.65 -> 4.74 s;
// 128^3 spheres, 1.01 -> 1.11 s).
// The auto mode also needs the estimate of prepare_two_visits below.
constexpr int kMgTwoVisitMinSide = 128;
bool mg_two_visits_allowed(const stokes_ctx* c, const MgHier& h) {
    return c->mg_visits != 1 && h.kind != kMgFineA && h.levels >= 2 && h.grid[1].n >= kMgTiledMinSide &&
           c->mg_coarse_gs != 2;
}
bool mg_two_visits(const stokes_ctx* c, const MgHier& h) {
    if (!mg_two_visits_allowed(c, h)) return false;
    return c->mg_visits == 2 || (h.grid[1].n >= kMgTwoVisitMinSide && c->mg_two_ok == 1);
}

// Scale of the SIMPLE matrix's coarse corrections into levels >= 2.
double mg_deep_scale(const stokes_ctx* c) {
    if (c->mg_scale_deep > 0.0) return c->mg_scale_deep;
    return c->mg_deep_auto > 0.0 ? c->mg_deep_auto : c->mg_scale;
}

// The coarse levels from..L of a cycle: the cycle on b_from (the right-hand
// side of level `from`), its result in y_from (the coarsest level's in its x);
// acc: added to y_from (a tiled level only).
template <class T>
stokes_status mg_coarse(stokes_ctx* c, MgHier& h, int from, const T* bfrom, bool acc, const CgState* st) {
    const int L = h.levels;
    const T omega = (T)c->mg_omega, scale0 = (T)(h.kind == kMgFineA ? c->mg_scale_A : c->mg_scale);
    const T scale_deep = h.kind == kMgFineA ? scale0 : (T)mg_deep_scale(c);
    std::vector<MgOp> ops(L + 1);
    for (int l = 1; l <= L; ++l) {
        const auto& cc = h.c32[l];
        ops[l] = {nullptr, 0, nullptr, cc.D, cc.Wx, cc.Wy, cc.Wz};
    }
    auto nodes = [&](int l) { return h.nb * h.grid[l].n3; };
    const bool kindA = h.kind == kMgFineA;
    // coarse level l (1 <= l < L) smooths by red-black Gauss-Seidel
    auto use_gs = [&](int l) {
        const int n = h.grid[l].n;
        return n >= kGsMinSide && (c->mg_coarse_gs == 2 || (c->mg_coarse_gs == 1 && n < kMgTiledMinSide));
    };
    // level l (1 <= l < L) going down: smooth on b_l from zero, restrict the residual into level l+1
    auto pre = [&](int l, const T* bl) {
        T* bn = mg_view(h, l + 1, T()).b;
        if (use_gs(l)) {
            hipLaunchKernelGGL(k_mgc_gs_restrict<T>, dim3(gs_blocks(h.grid[l]), c->nbatch), dim3(kGsThreads), 0, c->stream,
                               h.grid[l], h.grid[l + 1], ops[l], bl, bn, st);
        } else if (h.grid[l].n >= kMgTiledMinSide) {
            const Sweep& ls = h.sweep[l];
            if (kindA)
                hipLaunchKernelGGL((k_mgc_tiled<T, 3, kMgcPre>), grid_of(ls), dim3(kBlock), 0, c->stream, ls,
                                   h.grid[l + 1].n, ops[l], bl, (const T*)nullptr, T(0), omega, bn, st);
            else
                hipLaunchKernelGGL((k_mgc_tiled<T, 1, kMgcPre>), grid_of(ls), dim3(kBlock), 0, c->stream, ls,
                                   h.grid[l + 1].n, ops[l], bl, (const T*)nullptr, T(0), omega, bn, st);
        } else {
            hipLaunchKernelGGL(k_mgc_restrict<T>, dim3(exact_blocks(8 * (int64_t)nodes(l + 1)), c->nbatch), dim3(kBlock), 0,
                               c->stream, h.grid[l], h.grid[l + 1], ops[l], bl, bn, omega, st);
        }
    };
    // the result of level l is in its y (the coarsest level's in its x)
    auto coarse_x = [&](int l) -> const T* { return l == L ? mg_view(h, L, T()).x : mg_view(h, l, T()).y; };
    // level l going up: prolong the correction of level l+1 and postsmooth on b_l into y_l
    // (acc: added to y_l; tiled levels only)
    auto post = [&](int l, const T* bl, bool acc) {
        T* y = mg_view(h, l, T()).y;
        const T scale = l >= 2 ? scale_deep : scale0;
        if (use_gs(l)) {
            hipLaunchKernelGGL(k_mgc_gs_postsmooth<T>, dim3(gs_blocks(h.grid[l]), c->nbatch), dim3(kGsThreads), 0, c->stream,
                               h.grid[l], ops[l], bl, coarse_x(l + 1), h.grid[l + 1].n, scale, y, st);
        } else if (h.grid[l].n >= kMgTiledMinSide) {
            const Sweep& ls = h.sweep[l];
            if (kindA)
                hipLaunchKernelGGL((k_mgc_tiled<T, 3, kMgcPost>), grid_of(ls), dim3(kBlock), 0, c->stream, ls,
                                   h.grid[l + 1].n, ops[l], bl, coarse_x(l + 1), scale, omega, y, st);
            else if (acc)
                hipLaunchKernelGGL((k_mgc_tiled<T, 1, kMgcPostAcc>), grid_of(ls), dim3(kBlock), 0, c->stream, ls,
                                   h.grid[l + 1].n, ops[l], bl, coarse_x(l + 1), scale, omega, y, st);
            else
                hipLaunchKernelGGL((k_mgc_tiled<T, 1, kMgcPost>), grid_of(ls), dim3(kBlock), 0, c->stream, ls,
                                   h.grid[l + 1].n, ops[l], bl, coarse_x(l + 1), scale, omega, y, st);
        } else {
            hipLaunchKernelGGL(k_mgc_postsmooth<T>, dim3(exact_blocks(nodes(l)), c->nbatch), dim3(kBlock), 0, c->stream,
                               h.grid[l], ops[l], bl, coarse_x(l + 1), h.grid[l + 1].n, scale, omega, y, st);
        }
    };
    // levels from .. L: the cycle on b_from, result in y_from (acc: added to it)
    auto subcycle = [&](int from, const T* bfrom, bool acc) {
        for (int l = from; l < L; ++l) pre(l, l == from ? bfrom : mg_view(h, l, T()).b);
        auto v = mg_view(h, L, T());
        // coarsest: Jacobi sweeps in one workgroup, result in x
        hipLaunchKernelGGL(k_mg_coarsest<T>, dim3(1, c->nbatch), dim3(kMgCoarsestThreads), 0, c->stream, h.grid[L], ops[L],
                           (const T*)v.b, v.x, omega, c->mg_coarse_sweeps, st);
        for (int l = L - 1; l >= from; --l)
            post(l, l == from ? bfrom : mg_view(h, l, T()).b, acc && l == from);
    };
    subcycle(from, bfrom, acc);
    HIP_TRY(hipGetLastError());
    return STOKES_OK;
}

// w_1 = b_1 - A_1 y_1 on level 1 of a hierarchy (tiled level 1)
template <class T>
void mg_level1_residual(stokes_ctx* c, MgHier& h, const T* b1, const T* y1, T* w1, const CgState* st) {
    const auto& cc = h.c32[1];
    const MgOp op1 = {nullptr, 0, nullptr, cc.D, cc.Wx, cc.Wy, cc.Wz};
    const Sweep& ls = h.sweep[1];
    hipLaunchKernelGGL((k_mgc_tiled<T, 1, kMgcResid>), grid_of(ls), dim3(kBlock), 0, c->stream, ls, h.grid[2].n, op1,
                       b1, y1, T(0), (T)c->mg_omega, w1, st);
}

// z0 = V-cycle applied to the fine residual b0; the last fine sweep writes the
// partials of (b0, z0) into the RZ slot of the CG loop (grid = the CG sweeps').
template <class T>
stokes_status vcycle(stokes_ctx* c, MgHier& h, const T* b0, const T* invd0, T* z0, const CgState* st,
                     bool restricted = false) {
    const Sweep& s0 = inner_sweep(c, T());   // level 0: the inner solve's sweep
    const T omega = (T)c->mg_omega, scale = (T)(h.kind == kMgFineA ? c->mg_scale_A : c->mg_scale);
    const bool kindA = h.kind == kMgFineA;
    // descend: residual of the first Jacobi sweep, restricted (unless the
    // fused CG update already did)
    if (!restricted) {
        const MgGrid& cg = h.grid[1];
        T* bc = mg_view(h, 1, T()).b;
        bool open;
        ST_TRY(time_begin(c, kindA ? kTimeMgARestrict : kTimeMgSRestrict, &open));
        if (kindA)
            hipLaunchKernelGGL((k_mgf_tiled<T, kMgFineA, false>), grid_of(s0), dim3(kBlock), 0, c->stream,
                               s0, cg.n, c->code, invd0, b0, (const T*)nullptr, T(0), omega, bc, nullptr, 0, st);
        else
            hipLaunchKernelGGL((k_mgf_tiled<T, kMgFineShat, false>), grid_of(s0), dim3(kBlock), 0, c->stream,
                               s0, cg.n, c->code, invd0, b0, (const T*)nullptr, T(0), omega, bc, nullptr, 0, st);
        ST_TRY(time_end(c, open));
    }
    ST_TRY(mg_coarse<T>(c, h, 1, (const T*)mg_view(h, 1, T()).b, false, st));
    // Two visits of level 1 (the SIMPLE matrix; see mg_two_visits): the second
    // cycles on the residual the first leaves, w = b_1 - A_1 y_1, and adds its
    // result to y_1.  Linear and symmetric, so the inner CG stays standard.
    if (mg_two_visits(c, h)) {
        auto v1 = mg_view(h, 1, T());
        mg_level1_residual<T>(c, h, v1.b, v1.y, v1.w, st);
        ST_TRY(mg_coarse<T>(c, h, 1, (const T*)v1.w, true, st));
    }
    const T* xc1 = h.levels == 1 ? mg_view(h, 1, T()).x : mg_view(h, 1, T()).y;
    bool open;
    const bool pipe = !kindA && c->mg_pipe && sizeof(T) == 8;
    ST_TRY(time_begin(c, kindA ? kTimeMgASmooth : (pipe ? kTimeMgSSmoothPipe : kTimeMgSSmooth), &open));
    if (kindA)
        hipLaunchKernelGGL((k_mgf_tiled<T, kMgFineA, true>), grid_of(s0), dim3(kBlock), 0, c->stream, s0,
                           h.grid[1].n, c->code, invd0, b0, xc1, scale, omega, z0, c->part, kRZ, st);
    else if (pipe)
        // (1/D from the 16-bit codes: the same values as invd0, which is c->invdS here)
        hipLaunchKernelGGL(k_mgf_smooth_S_pipe<T>, grid_of(s0), dim3(kBlock), 0, c->stream, s0, h.grid[1].n,
                           c->code2, b0, xc1, scale, omega, z0, c->part, kRZ, st);
    else
        hipLaunchKernelGGL((k_mgf_tiled<T, kMgFineShat, true>), grid_of(s0), dim3(kBlock), 0, c->stream, s0,
                           h.grid[1].n, c->code, invd0, b0, xc1, scale, omega, z0, c->part, kRZ, st);
    ST_TRY(time_end(c, open));
    HIP_TRY(hipGetLastError());
    return STOKES_OK;
}

// Two visits of level 1 act on level 1 as 2 B_1 - B_1 A_1 B_1 (B_1: the cycle
// from level 1 down), whose eigenvalues relative to A_1 are 1 - (1 - mu)^2 for
// the eigenvalues mu of B_1 A_1: positive only while mu < 2.  The over-corrected
// coarse corrections push mu above 1, the more so the deeper the hierarchy below
// level 1 (CPU model, random-field packs: 1.40 with three levels below level 1,
// 1.73 with four).  So in the auto mode the largest mu is estimated once per
// context (again after a multigrid option changes) by power iteration on the
// device, and two visits are used only below kMgTwoVisitMaxLambda: a power
// iteration approaches the largest eigenvalue from below, so the bound keeps a
// margin under 2 (at 1.8 the top of the spectrum already maps to 0.36).  Plain
// contexts only (batched ones keep one visit).
constexpr double kMgTwoVisitMaxLambda = 1.8;
constexpr int kMgTwoVisitPowerIts = 20;
// Fallback scale of the corrections below level 1 when the estimate with the
// configured one is too large (measured on the 512^3 random field: 3.29 with
// 1.7, 2.60 with 1.5, 2.25 with 1.4, 1.64 with 1.3, and with 1.3 and two visits
// 21 % fewer inner iterations than one visit with 1.7; on the 256^3 tight pack
// 1.7 with two visits stays best, 5 707 against 6 106 inner iterations with 1.3).
constexpr double kMgDeepFallback = 1.3;

// Largest eigenvalue of B_1 A_1 with the current cycle, by power iteration
// on the device (dot products as per-block partials added on the host in
// block order).
stokes_status estimate_level1_lambda(stokes_ctx* c, double* mu_out) {
    MgHier& h = c->mgS;
    *mu_out = 0.0;
    auto v1 = mg_view(h, 1, 0.0);
    const int n1 = h.grid[1].n3;
    const int nbk = flat_blocks(n1, 1024);
    {
        // start: seeded uniform noise on the level's unknowns
        std::vector<double> D((size_t)n1), x((size_t)n1);
        HIP_TRY(hipMemcpyAsync(D.data(), v1.D, (size_t)n1 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        uint64_t seed = 0x9E3779B97F4A7C15ull;
        for (int i = 0; i < n1; ++i) {
            seed ^= seed << 13;
            seed ^= seed >> 7;
            seed ^= seed << 17;
            x[i] = D[i] > 0.0 ? (double)(seed >> 11) * 0x1.0p-53 - 0.5 : 0.0;
        }
        HIP_TRY(hipMemcpyAsync(v1.w, x.data(), (size_t)n1 * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemsetAsync(v1.x, 0, (size_t)n1 * sizeof(double), c->stream));   // zero right-hand side
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    double mu = 0.0;
    for (int it = 0; it < kMgTwoVisitPowerIts; ++it) {
        mg_level1_residual<double>(c, h, v1.x, v1.w, v1.b, nullptr);                 // b_1 = 0 - A_1 x
        ST_TRY(mg_coarse<double>(c, h, 1, (const double*)v1.b, false, nullptr));   // y_1 = B_1 b_1
        hipLaunchKernelGGL(k_dots3_flat, dim3(nbk), dim3(kBlock), 0, c->stream, n1, (const double*)v1.b,
                           (const double*)v1.y, (const double*)v1.w, c->dpart);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(c->host_part, c->dpart, (size_t)3 * nbk * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        // signs cancel: (A x, B A x) / (A x, x) from b_1 = -A x and y_1 = -B A x
        double num = 0.0, den = 0.0, yy = 0.0;
        for (int q = 0; q < nbk; ++q) {
            num += c->host_part[3 * q];
            den += c->host_part[3 * q + 1];
            yy += c->host_part[3 * q + 2];
        }
        den = -den;
        if (!(den > 0.0) || !(yy > 0.0) || !std::isfinite(num)) return STOKES_OK;   // nothing to estimate
        mu = num / den;
        hipLaunchKernelGGL(k_scale_flat, dim3(nbk), dim3(kBlock), 0, c->stream, n1, (const double*)v1.y,
                           -1.0 / std::sqrt(yy), v1.w);                              // next x = B A x / |B A x|
    }
    *mu_out = mu;
    return STOKES_OK;
}

stokes_status prepare_two_visits(stokes_ctx* c) {
    MgHier& h = c->mgS;
    if (c->mg_two_ok != 0) return STOKES_OK;
    c->mg_two_ok = -1;
    c->mg_deep_auto = 0.0;
    if (c->mg_visits != 0 || !c->use_mg || !mg_two_visits_allowed(c, h) || h.grid[1].n < kMgTwoVisitMinSide ||
        c->nbatch != 1)
        return STOKES_OK;
    double mu = 0.0;
    ST_TRY(estimate_level1_lambda(c, &mu));
    if (!(mu < kMgTwoVisitMaxLambda) && c->mg_scale_deep == 0.0 && c->mg_scale > kMgDeepFallback) {
        c->mg_deep_auto = kMgDeepFallback;
        double mu2 = 0.0;
        ST_TRY(estimate_level1_lambda(c, &mu2));
        if (mu2 > 0.0 && mu2 < kMgTwoVisitMaxLambda) mu = mu2;
        else c->mg_deep_auto = 0.0;
    }
    c->mg_lambda1 = mu;
    c->mg_two_ok = (mu > 0.0 && mu < kMgTwoVisitMaxLambda) ? 1 : -1;
    if (c->progress > 0) {
        std::fprintf(stderr, "[stokes] N=%d largest eigenvalue of B_1 A_1 ~ %.4f (corrections below level 1 scaled %.2f): "
                     "%s visit%s of level 1\n", c->N, mu, mg_deep_scale(c), c->mg_two_ok == 1 ? "two" : "one",
                     c->mg_two_ok == 1 ? "s" : "");
        std::fflush(stderr);
    }
    return STOKES_OK;
}

// Multigrid-preconditioned CG with the SIMPLE matrix; the stopping test stays
// on the Jacobi-scaled residual ||D^-1 r|| / ||D^-1 r_0||.  One iteration:
// direction, stencil, update, then the V-cycle that forms the next z.
template <class T>
stokes_status cg_S_mg(stokes_ctx* c, InnerS<T> v, const double* b, double eps, int* iters, int* status) {
    const Sweep& s = inner_sweep(c, T());
    CgState* st = c->cg + 1;
    T* z = mg_out(c->mgS, T());
    hipLaunchKernelGGL(k_cgS_init<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, v.invd, b, v.x, v.r, st, c->part,
                       eps, c->max_inner);
    HIP_TRY(hipGetLastError());
    ST_TRY(vcycle<T>(c, c->mgS, v.r, v.invd, z, nullptr));
    // the fused update's 2x2x2 sums pair planes within a block
    if ((s.lz & 1) || (s.bxlog != 5 && s.bxlog != 6)) return STOKES_E_LIMIT;
    T* r2 = mg_r2(c->mgS, T());
    T* d2 = mg_d2(c->mgS, T());
    T* bc = mg_view(c->mgS, 1, T()).b;
    const T omega = (T)c->mg_omega;
    const bool fuse = c->fuse_dir_S != 0;
    // the software-pipelined level-0 sweeps gain in FP64 only (FP32 at 256^3:
    // mixed solve 1.42 -> 1.43 s)
    const bool pipe = c->mg_pipe != 0 && sizeof(T) == 8;
    auto body = [c, s, st, v, z, r2, d2, bc, omega, fuse, pipe](int parity) -> stokes_status {
        T* rin = parity ? r2 : v.r;
        T* rout = parity ? v.r : r2;
        T* din = parity ? d2 : v.d;
        T* dout = parity ? v.d : d2;
        bool open;
        if (fuse) {
            ST_TRY(time_begin(c, pipe ? kTimeSDirStencilPipe : kTimeSDirStencil, &open));
            if (pipe)
                hipLaunchKernelGGL(k_cgS_dirstencil_pipe<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code2,
                                   (const T*)z, (const T*)din, dout, v.q, st, c->part);
            else
                hipLaunchKernelGGL(k_cgS_dirstencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code,
                                   (const T*)z, (const T*)din, dout, v.q, st, c->part);
            ST_TRY(time_end(c, open));
        } else {
            // direction in place (pointwise), then the stencil
            dout = v.d;
            ST_TRY(time_begin(c, kTimeSDir, &open));
            hipLaunchKernelGGL(k_cgS_dir<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, v.invd, rin, v.d, st, c->part,
                               (const T*)z);
            ST_TRY(time_end(c, open));
            ST_TRY(time_begin(c, kTimeSStencil, &open));
            hipLaunchKernelGGL(k_cgS_stencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.d,
                               v.q, st, c->part);
            ST_TRY(time_end(c, open));
        }
        ST_TRY(time_begin(c, pipe ? kTimeSUpdRestrictPipe : kTimeSUpdRestrict, &open));
        if (pipe)
            hipLaunchKernelGGL(k_mgf_update_restrict_S_pipe<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code2,
                               v.x, (const T*)rin, rout, (const T*)dout, (const T*)v.q, bc, omega, st, c->part);
        else
            hipLaunchKernelGGL((k_mgf_update_restrict<T, kMgFineShat>), grid_of(s), dim3(kBlock), 0, c->stream, s,
                               c->code, v.invd, v.x, (const T*)rin, rout, (const T*)dout, (const T*)v.q, bc, omega,
                               st, c->part);
        ST_TRY(time_end(c, open));
        return vcycle<T>(c, c->mgS, rout, v.invd, z, st, true);
    };
    return run_inner(c, 1, graph_key<T>(fuse ? 2 : 4, v.x, v.r, v.d, v.q, v.invd, z), body, iters, status);
}

// Multigrid-preconditioned CG with A (three planes); stopping test on the
// Jacobi-scaled residual as in the plain solve.
template <class T>
stokes_status cg_A_mg(stokes_ctx* c, InnerA<T> v, const double* b, double eps, int* iters, int* status) {
    const Sweep& s = inner_sweep(c, T());
    CgState* st = c->cg + 0;
    T* z = mg_out(c->mgA, T());
    hipLaunchKernelGGL(k_cgA_init<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, b, c->force[0],
                       c->force[1], c->force[2], v.x, v.r, st, c->part, eps, c->max_inner);
    HIP_TRY(hipGetLastError());
    ST_TRY(vcycle<T>(c, c->mgA, v.r, (const T*)nullptr, z, nullptr));
    // the fused update's 2x2x2 sums pair planes within a block
    if ((s.lz & 1) || (s.bxlog != 5 && s.bxlog != 6)) return STOKES_E_LIMIT;
    T* r2 = mg_r2(c->mgA, T());
    T* d2 = mg_d2(c->mgA, T());
    T* bc = mg_view(c->mgA, 1, T()).b;
    const T omega = (T)c->mg_omega;
    const bool fuse = c->fuse_dir_A != 0;
    auto body = [c, s, st, v, z, r2, d2, bc, omega, fuse](int parity) -> stokes_status {
        T* rin = parity ? r2 : v.r;
        T* rout = parity ? v.r : r2;
        T* din = parity ? d2 : v.d;
        T* dout = parity ? v.d : d2;
        bool open;
        if (fuse) {
            ST_TRY(time_begin(c, kTimeADirStencil, &open));
            hipLaunchKernelGGL(k_cgA_dirstencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code,
                               (const T*)z, (const T*)din, dout, v.q, st, c->part);
            ST_TRY(time_end(c, open));
        } else {
            // direction in place (pointwise), then the stencil
            dout = v.d;
            ST_TRY(time_begin(c, kTimeADir, &open));
            hipLaunchKernelGGL(k_cgA_dir<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, rin, v.d, st, c->part,
                               (const T*)z);
            ST_TRY(time_end(c, open));
            ST_TRY(time_begin(c, kTimeAStencil, &open));
            hipLaunchKernelGGL(k_cgA_stencil_tiled<T>, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, v.d,
                               v.q, st, c->part);
            ST_TRY(time_end(c, open));
        }
        ST_TRY(time_begin(c, kTimeAUpdRestrict, &open));
        hipLaunchKernelGGL((k_mgf_update_restrict<T, kMgFineA>), grid_of(s), dim3(kBlock), 0, c->stream, s, c->code,
                           (const T*)nullptr, v.x, (const T*)rin, rout, (const T*)dout, (const T*)v.q, bc, omega, st,
                           c->part);
        ST_TRY(time_end(c, open));
        return vcycle<T>(c, c->mgA, rout, (const T*)nullptr, z, st, true);
    };
    return run_inner(c, 0, graph_key<T>(fuse ? 3 : 5, v.x, v.r, v.d, v.q, nullptr, z), body, iters, status);
}

// precision-generic dispatch between the multigrid and Jacobi inner solves
template <class T>
stokes_status inner_A(stokes_ctx* c, InnerA<T> v, const double* b, double eps, int* iters, int* status) {
    if (c->use_mg_A && c->mgA.levels > 0) return cg_A_mg<T>(c, v, b, eps, iters, status);
    return cg_A<T>(c, v, b, eps, iters, status);
}
template <class T>
stokes_status inner_S(stokes_ctx* c, InnerS<T> v, const double* b, double eps, int* iters, int* status) {
    if (c->use_mg && c->mgS.levels > 0) return cg_S_mg<T>(c, v, b, eps, iters, status);
    return cg_S<T>(c, v, b, eps, iters, status);
}


stokes_status solve_S64(stokes_ctx* c, const double* b, double eps, int* iters, int* status) {
    return inner_S<double>(c, bufS64(c), b, eps, iters, status);
}
stokes_status solve_A64(stokes_ctx* c, const double* b, double eps, int* iters, int* status) {
    return inner_A<double>(c, bufA64(c), b, eps, iters, status);
}

// ---- outer-loop helpers ---------------------------------------------------------
// Remove each kept component's mean from the cell vector x.  part and mean are
// the partial sums (kMaxBlocks values for one component, kCompBlocks * K for
// several) and the K means; every entry read is written first in the call.
stokes_status project_with(stokes_ctx* c, double* x, double* part, double* mean) {
    const int K = c->ncomp_kept;
    if (K == 0) return STOKES_OK;
    if (K == 1 && !c->label) {
        hipLaunchKernelGGL(k_sum1, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, (const double*)x, part);
        hipLaunchKernelGGL(k_sub_mean1, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, x, c->bits, c->wpr,
                           (const double*)part, 1.0 / (double)c->nfluid);
        HIP_TRY(hipGetLastError());
        return STOKES_OK;
    }
    const int64_t chunk = ((c->n3 + kCompBlocks - 1) / kCompBlocks + 255) / 256 * 256;
    const int nb = (int)((c->n3 + chunk - 1) / chunk);
    const unsigned B = (unsigned)c->nbatch, act = c->sw.active;
    hipLaunchKernelGGL(k_comp_sum, dim3(nb, B), dim3(kBlock), (size_t)kWaves * K * sizeof(double), c->stream, x,
                       c->label, c->bits, c->N, c->wpr, c->n3, K, chunk, part, c->bstride, act);
    hipLaunchKernelGGL(k_comp_mean, dim3((K + kBlock - 1) / kBlock, B), dim3(kBlock), 0, c->stream, part, nb, K,
                       c->comp_count, mean, c->bstride, act);
    const int subblocks = (int)std::min<int64_t>(4096, (c->n3 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_comp_sub, dim3(subblocks, B), dim3(kBlock), 0, c->stream, x, c->label, c->bits, c->N, c->wpr,
                       c->n3, mean, c->bstride, act);
    HIP_TRY(hipGetLastError());
    return STOKES_OK;
}

stokes_status project(stokes_ctx* c, double* x) {
    const bool one = c->ncomp_kept == 1 && !c->label;
    return project_with(c, x, one ? c->proj_part : c->comp_part, c->comp_mean);
}

// per-block partials [3 * nblk] to the host, added there in block order
// Per member m: out[3 m + q] = its partials added in block order.
stokes_status host_totals(stokes_ctx* c, double* out) {
    const int nb = c->sw.nblk;
    const size_t row = (size_t)3 * nb * sizeof(double);
    if (c->nbatch == 1)
        HIP_TRY(hipMemcpyAsync(c->host_part, c->dpart, row, hipMemcpyDeviceToHost, c->stream));
    else
        HIP_TRY(hipMemcpy2DAsync(c->host_part, row, c->dpart, c->bstride, row, (size_t)c->nbatch,
                                 hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int m = 0; m < c->nbatch; ++m) {
        const double* hp = c->host_part + (size_t)3 * nb * m;
        double* o = out + 3 * m;
        o[0] = o[1] = o[2] = 0.0;
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < 3; ++q) o[q] += hp[3 * b + q];
    }
    return STOKES_OK;
}

stokes_status dots(stokes_ctx* c, const double* a0, const double* b0, const double* a1, const double* b1,
                   const double* a2, const double* b2, double out[3]) {
    hipLaunchKernelGGL(k_dots, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, a0, b0, a1, b1, a2, b2, c->dpart);
    HIP_TRY(hipGetLastError());
    return host_totals(c, out);
}

stokes_status face_sums(stokes_ctx* c, const double* u, double out[3]) {
    hipLaunchKernelGGL(k_face_sums, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, u, c->dpart);
    HIP_TRY(hipGetLastError());
    return host_totals(c, out);
}

// permeability (voxel units) along the force from face sums
double kvox_of(const stokes_ctx* c, const double sums[3], double mean[3]) {
    double f2 = 0.0, fu = 0.0;
    for (int a = 0; a < 3; ++a) {
        mean[a] = sums[a] / (double)c->n3;
        f2 += c->force[a] * c->force[a];
        fu += c->force[a] * mean[a];
    }
    return fu / f2;
}

// Extreme eigenvalues of the CG tridiagonal (Lanczos, Saad Sec. 6.7.3) by
// bisection on Sturm sequence counts.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b2, double x) {
    int cnt = 0;
    double qv = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        qv = a[i] - x - (i > 0 ? b2[i - 1] / qv : 0.0);
        if (qv == 0.0) qv = -1e-300;
        if (qv < 0.0) ++cnt;
    }
    return cnt;
}

void lanczos_extremes(const std::vector<double>& alpha, const std::vector<double>& beta, double* lo, double* hi) {
    const size_t k = alpha.size();
    *lo = *hi = std::nan("");
    if (k == 0) return;
    std::vector<double> a(k), b2(k > 0 ? k - 1 : 0);
    for (size_t j = 0; j < k; ++j) {
        a[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j > 0) b2[j - 1] = beta[j - 1] / (alpha[j - 1] * alpha[j - 1]);
    }
    double gl = 1e300, gh = -1e300;
    for (size_t j = 0; j < k; ++j) {
        double rad = (j > 0 ? std::sqrt(b2[j - 1]) : 0.0) + (j + 1 < k ? std::sqrt(b2[j]) : 0.0);
        gl = std::min(gl, a[j] - rad);
        gh = std::max(gh, a[j] + rad);
    }
    auto kth = [&](int idx) {  // idx-th smallest eigenvalue, 0-based
        double l = gl, h = gh;
        for (int it = 0; it < 200; ++it) {
            double m = 0.5 * (l + h);
            if (sturm_count(a, b2, m) > idx) h = m;
            else l = m;
            if (h - l <= 1e-14 * std::max(std::fabs(l), std::fabs(h))) break;
        }
        return 0.5 * (l + h);
    };
    *lo = kth(0);
    *hi = kth((int)k - 1);
}

}  // namespace

// ---- scratch of the no-allocation entry point ------------------------------------
// stokes_apply_device_noalloc keeps the masked copy of its input and the
// partial sums of the projection in this fixed array instead of the context's
// work vectors.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code the name stands for a host-side shadow, not a
// device address: host code only ever uses the address that
// hipGetSymbolAddress returns with the device current (scratch_address).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int64_t kNoAllocScratchWords = (int64_t)(kNoAllocScratchBytes / sizeof(double));
static __device__ __align__(256) double scratch[kNoAllocScratchWords];

namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device;
// resolved once per device and kept.
stokes_status scratch_address(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return STOKES_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return STOKES_E_DEVICE;
        g_scratch_addr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[device];
    return STOKES_OK;
}
}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* stokes_status_str(int s) {
    switch (s) {
    case STOKES_OK: return "ok";
    case STOKES_NOT_CONVERGED: return "not converged";
    case STOKES_E_ARG: return "invalid argument";
    case STOKES_E_NOMEM: return "out of memory";
    case STOKES_E_DEVICE: return "device error";
    case STOKES_E_BREAKDOWN: return "breakdown";
    case STOKES_E_STATE: return "invalid state";
    case STOKES_E_LIMIT: return "limit exceeded";
    default: return "unknown";
    }
}

// Set-up of a context with c->nbatch members (one: a plain context), the k-th
// from masks[k].  A batched context keeps every member's buffers at the same
// offsets of its part of one slab, so every buffer is allocated once, for
// member 0, and the other members' copies follow at multiples of bstride.
static stokes_status setup_impl(stokes_ctx* c, const uint8_t* const* masks) {
    const int B = c->nbatch;
    const int N = c->N;
    const int64_t n3 = c->n3;
    std::vector<Geometry> G(B);
    c->member.assign(B, {});
    int Kmax = 0;
    for (int m = 0; m < B; ++m) {
        preprocess(masks[m], N, c->force, (c->setup_flags & STOKES_KEEP_ALL_COMPONENTS) != 0, G[m]);
        if (G[m].ncomp_kept > kMaxCompLds) return STOKES_E_LIMIT;
        auto& mi = c->member[m];
        mi.nfluid_in = G[m].nfluid_in;
        mi.nfluid = G[m].nfluid;
        mi.nsurf = G[m].nsurf;
        mi.ncomp_all = G[m].ncomp_all;
        mi.ncomp_kept = G[m].ncomp_kept;
        Kmax = std::max(Kmax, G[m].ncomp_kept);
    }
    const Geometry& g = G[0];
    c->nfluid_in = g.nfluid_in;
    c->nfluid = g.nfluid;
    c->nsurf = g.nsurf;
    c->ncomp_all = g.ncomp_all;
    // batched: every member's projection covers Kmax components (a member with
    // fewer has empty ones), through the labels
    // (every context made by stokes_setup_batch does so, whatever its member
    // count, so that a member's arithmetic does not depend on its batch)
    const bool batched = B > 1 || c->batch_api;
    c->ncomp_kept = batched ? Kmax : g.ncomp_kept;

    // one sweep for every kernel of an inner solve (the fused update and
    // restriction re-adds the stencil's partials, so both need one block count)
    c->sw = member_sweep(c, make_sweep(N, c->sweep_blocks));
    c->sw32 = member_sweep(c, make_sweep32(N, c->sweep_blocks));
    if (c->sw.nblk > kMaxBlocks || c->sw32.nblk > kMaxBlocks) return STOKES_E_LIMIT;
    c->wpr = (N + 31) / 32;

    const int K = std::max(1, c->ncomp_kept);
    ST_TRY(dev_alloc(c, &c->bits, (size_t)N * N * c->wpr));
    ST_TRY(dev_alloc(c, &c->code, (size_t)n3));
    ST_TRY(dev_alloc(c, &c->code2, (size_t)n3));
    ST_TRY(dev_alloc(c, &c->comp_count, (size_t)K));
    ST_TRY(dev_alloc(c, &c->comp_part, (size_t)kCompBlocks * K));
    ST_TRY(dev_alloc(c, &c->proj_part, (size_t)kMaxBlocks));
    ST_TRY(dev_alloc(c, &c->comp_mean, (size_t)K));
    if (batched || g.ncomp_kept > 1) ST_TRY(dev_alloc(c, &c->label, (size_t)n3));
    for (double** f : {&c->fx, &c->fr, &c->fq, &c->u, &c->fd})
        ST_TRY(dev_alloc(c, f, (size_t)(3 * n3)));
    for (double** v : {&c->p, &c->r, &c->zs, &c->d, &c->q, &c->sr, &c->sq, &c->invdS, &c->sd})
        ST_TRY(dev_alloc(c, v, (size_t)n3));
    ST_TRY(dev_alloc(c, &c->cg, 2));
    ST_TRY(dev_alloc(c, &c->part, (size_t)kNumSlots * kMaxBlocks));
    ST_TRY(dev_alloc(c, &c->dpart, (size_t)3 * kMaxBlocks));
    if (hipHostMalloc((void**)&c->host_state, (size_t)B * sizeof(CgState)) != hipSuccess) return STOKES_E_NOMEM;
    if (hipHostMalloc((void**)&c->host_part, (size_t)B * 3 * kMaxBlocks * sizeof(double)) != hipSuccess)
        return STOKES_E_NOMEM;

    // per member: remaining-fluid bitmask, component sizes, labels
    std::vector<std::vector<uint32_t>> bits(B);
    std::vector<std::vector<double>> counts(B);
    for (int m = 0; m < B; ++m) {
        bits[m].assign((size_t)N * N * c->wpr, 0u);
        for (int64_t row = 0; row < (int64_t)N * N; ++row)
            for (int i = 0; i < N; ++i)
                if (G[m].fluid[row * N + i]) bits[m][row * c->wpr + (i >> 5)] |= 1u << (i & 31);
        // components a member does not have count 1 (their mean is 0; no voxel carries them)
        counts[m].assign(K, batched ? 1.0 : 0.0);
        for (int q = 0; q < G[m].ncomp_kept; ++q) counts[m][q] = (double)G[m].comp_size[q];
        const size_t o = (size_t)m * c->bstride;
        HIP_TRY(hipMemcpyAsync((char*)c->bits + o, bits[m].data(), bits[m].size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync((char*)c->comp_count + o, counts[m].data(), K * sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
        if (c->label) {
            if (G[m].label.empty()) return STOKES_E_LIMIT;
            HIP_TRY(hipMemcpyAsync((char*)c->label + o, G[m].label.data(), (size_t)n3 * sizeof(uint16_t),
                                   hipMemcpyHostToDevice, c->stream));
        }
    }
    hipLaunchKernelGGL(k_face_codes, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->bits, c->wpr, c->code);
    hipLaunchKernelGGL(k_inv_diag_Shat, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->code, c->invdS);
    hipLaunchKernelGGL(k_code2, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->code, c->code2);
    HIP_TRY(hipGetLastError());
    ST_TRY(build_mg(c, c->mgS, 1, kMgFineShat));
    ST_TRY(build_mg(c, c->mgA, 3, kMgFineA));
    HIP_TRY(hipStreamSynchronize(c->stream));  // the host vectors above go out of scope

    // active faces per direction (host count from the remaining fluid)
    for (int m = 0; m < B; ++m) {
        auto& nf = c->member[m].nface;
        const std::vector<uint8_t>& fl = G[m].fluid;
        nf[0] = nf[1] = nf[2] = 0;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    const int64_t X = i + (int64_t)N * (j + (int64_t)N * k);
                    if (!fl[X]) continue;
                    if (fl[((i + N - 1) % N) + (int64_t)N * (j + (int64_t)N * k)]) nf[0]++;
                    if (fl[i + (int64_t)N * (((j + N - 1) % N) + (int64_t)N * k)]) nf[1]++;
                    if (fl[i + (int64_t)N * (j + (int64_t)N * ((k + N - 1) % N))]) nf[2]++;
                }
    }
    for (int a = 0; a < 3; ++a) c->nface[a] = c->member[0].nface[a];
    return STOKES_OK;
}

static stokes_status check_inputs(const uint8_t* mask, int N, const double force[3], unsigned flags) {
    if (!mask || !force) return STOKES_E_ARG;
    if (N < 2 || N > kMaxN) return STOKES_E_ARG;
    if (flags & ~STOKES_KEEP_ALL_COMPONENTS) return STOKES_E_ARG;
    double f2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(force[a])) return STOKES_E_ARG;
        f2 += force[a] * force[a];
    }
    if (!(f2 > 0.0) || !std::isfinite(f2)) return STOKES_E_ARG;
    const int64_t n3 = (int64_t)N * N * N;
    for (int64_t x = 0; x < n3; ++x)
        if (mask[x] > 1) return STOKES_E_ARG;
    return STOKES_OK;
}

stokes_status stokes_preprocess(const uint8_t* mask, int N, const double force[3], unsigned flags, int64_t counts[6],
                                uint8_t* fluid, int32_t* label) {
    if (!counts) return STOKES_E_ARG;
    ST_TRY(check_inputs(mask, N, force, flags));
    try {
        Geometry g;
        preprocess(mask, N, force, (flags & STOKES_KEEP_ALL_COMPONENTS) != 0, g);
        counts[0] = g.nfluid_in;
        counts[1] = g.nfluid;
        counts[2] = g.nsurf;
        counts[3] = g.ncomp_all;
        counts[4] = g.ncomp_kept;
        counts[5] = 0;
        if (fluid) std::memcpy(fluid, g.fluid.data(), (size_t)g.n3);
        if (label) {
            if (g.label.empty() && g.ncomp_kept > 0) return STOKES_E_LIMIT;
            for (int64_t x = 0; x < g.n3; ++x)
                label[x] = g.ncomp_kept == 0 ? -1 : (g.label[x] == 0xFFFF ? -1 : (int32_t)g.label[x]);
        }
    } catch (const std::bad_alloc&) {
        return STOKES_E_NOMEM;
    }
    return STOKES_OK;
}

static stokes_status ensure_mixed_buffers(stokes_ctx* c);

static stokes_status setup_common(stokes_ctx** out, const uint8_t* const* masks, int B, int N,
                                  const double force[3], unsigned flags, hipStream_t stream,
                                  const stokes_allocator* alloc = nullptr, bool batch_api = false) {
    if (!out || !masks || B < 1 || B > kMaxBatch) return STOKES_E_ARG;
    for (int m = 0; m < B; ++m) ST_TRY(check_inputs(masks[m], N, force, flags));
    const int64_t n3 = (int64_t)N * N * N;

    stokes_ctx* c = new (std::nothrow) stokes_ctx();
    if (!c) return STOKES_E_NOMEM;
    c->N = N;
    c->n3 = n3;
    for (int a = 0; a < 3; ++a) c->force[a] = force[a];
    c->setup_flags = flags;
    c->stream = stream;
    c->nbatch = B;
    c->batch_api = batch_api;
    if (alloc) c->ext_alloc = *alloc;
    else c->async_alloc = stream != nullptr;
    stokes_status st = STOKES_OK;
    if (B > 1) {
        // one slab for all members: each member's part bounds a context's
        // buffers (FP32 vectors included; 256-byte alignment of each buffer)
        int64_t est = 0;
        st = stokes_estimate_bytes(N, flags, 1, &est);
        if (st == STOKES_OK) {
            c->bstride = (size_t)est;
            char* slab = nullptr;
            st = dev_alloc(c, &slab, c->bstride * (size_t)B);
            c->slab = slab;
        }
    }
    try {
        if (st == STOKES_OK) st = setup_impl(c, masks);
        // a batched context runs the mixed-precision solve: its FP32 vectors now
        if (st == STOKES_OK && batch_api) {
            st = ensure_mixed_buffers(c);
            c->precision = 1;
        }
    } catch (const std::bad_alloc&) {
        st = STOKES_E_NOMEM;
    }
    // the device this context runs on, and that device's copy of the
    // no-allocation scratch (resolved here, at set-up, with the device current)
    if (st >= 0 && hipGetDevice(&c->device) != hipSuccess) st = STOKES_E_DEVICE;
    if (st >= 0) st = scratch_address(c->device, &c->noalloc_scratch);
    if (st < 0) {
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return STOKES_OK;
}

stokes_status stokes_setup_ex(stokes_ctx** out, const uint8_t* mask, int N, const double force[3], unsigned flags) {
    return setup_common(out, &mask, 1, N, force, flags, nullptr);
}

stokes_status stokes_setup(stokes_ctx** out, const uint8_t* mask, int N, const double force[3]) {
    return setup_common(out, &mask, 1, N, force, 0u, nullptr);
}

stokes_status stokes_setup_on_stream(stokes_ctx** out, const uint8_t* mask, int N, const double force[3],
                                     unsigned flags, void* stream) {
    if (!stream) return STOKES_E_ARG;
    return setup_common(out, &mask, 1, N, force, flags, (hipStream_t)stream);
}

stokes_status stokes_setup_batch(stokes_ctx** out, const uint8_t* const* masks, int nmembers, int N,
                                 const double force[3], unsigned flags, void* stream) {
    if (!masks || nmembers < 1 || nmembers > kMaxBatch) return STOKES_E_ARG;
    for (int m = 0; m < nmembers; ++m)
        if (!masks[m]) return STOKES_E_ARG;
    return setup_common(out, masks, nmembers, N, force, flags, (hipStream_t)stream, nullptr, true);
}

stokes_status stokes_setup_with_allocator(stokes_ctx** out, const uint8_t* mask, int N, const double force[3],
                                          unsigned flags, void* stream, const stokes_allocator* alloc) {
    if (!alloc || !alloc->alloc || !alloc->free) return STOKES_E_ARG;
    return setup_common(out, &mask, 1, N, force, flags, (hipStream_t)stream, alloc);
}

// Mirrors the allocations of setup_impl, build_mg, ensure_mixed_buffers and
// build_mg32, with the component arrays at their limit and the label array
// present, so the result bounds what a context holds.
stokes_status stokes_estimate_bytes(int N, unsigned flags, int precision, int64_t* bytes) {
    if (!bytes || N < 2 || N > kMaxN || (flags & ~STOKES_KEEP_ALL_COMPONENTS) || (precision != 0 && precision != 1))
        return STOKES_E_ARG;
    const int64_t n3 = (int64_t)N * N * N, wpr = (N + 31) / 32;
    auto blk = [](int64_t count, int64_t size) { return std::max<int64_t>(count, 1) * size; };
    const int64_t K = kMaxCompLds;
    int64_t t = blk((int64_t)N * N * wpr, 4) + blk(n3, 1) + blk(n3, 2) + blk(K, 8) + blk((int64_t)kCompBlocks * K, 8) +
                blk(K, 8) + blk(n3, 2);
    t += 5 * blk(3 * n3, 8) + 9 * blk(n3, 8);
    t += blk(2, sizeof(CgState)) + blk((int64_t)kNumSlots * kMaxBlocks, 8) + blk(3 * (int64_t)kMaxBlocks, 8) +
         blk(kMaxBlocks, 8);
    for (int nb : {1, 3}) {
        const std::vector<int> ns = mg_plan(N, nb);
        if (ns.size() < 2) continue;
        for (int prec = 0; prec <= precision; ++prec) {
            const int64_t w = prec == 0 ? 8 : 4;
            for (size_t l = 1; l < ns.size(); ++l) {
                const int64_t m = nb * (int64_t)ns[l] * ns[l] * ns[l];
                // FP64: operator (4), vectors b, x, y (and w on level 1), FP32 operator (4);
                // FP32: vectors only
                t += prec == 0 ? (l == 1 ? 8 : 7) * blk(m, 8) + 4 * blk(m, 4) : (l == 1 ? 4 : 3) * blk(m, 4);
            }
            t += 3 * blk(nb * n3, w);   // cycle output, second residual and direction on level 0
        }
    }
    if (precision == 1) t += 4 * blk(3 * n3, 4) + 5 * blk(n3, 4);
    // 256-byte alignment of every buffer inside a batched context's member
    // part (fewer than 256 buffers), rounded to whole 4 KiB pages: a member's
    // part of a batched context is exactly this many bytes
    t += 256 * 256;
    *bytes = (t + 4095) / 4096 * 4096;
    return STOKES_OK;
}

stokes_status stokes_set_stream(stokes_ctx* c, void* stream) {
    if (!c) return STOKES_E_ARG;
    c->stream = (hipStream_t)stream;
    return STOKES_OK;
}

// FP32 vectors of the mixed-precision path, allocated on first use.
static stokes_status ensure_mixed_buffers(stokes_ctx* c) {
    if (c->fx32) return STOKES_OK;
    const int64_t n3 = c->n3;
    for (float** f : {&c->fx32, &c->fr32, &c->fd32, &c->fq32}) ST_TRY(dev_alloc(c, f, (size_t)(3 * n3)));
    for (float** v : {&c->zs32, &c->sr32, &c->sd32, &c->sq32, &c->invdS32}) ST_TRY(dev_alloc(c, v, (size_t)n3));
    for (float* f : {c->fx32, c->fr32, c->fd32, c->fq32})
        HIP_TRY(hipMemsetAsync(f, 0, (size_t)(3 * n3) * sizeof(float), c->stream));
    for (float* v : {c->zs32, c->sr32, c->sd32, c->sq32})
        HIP_TRY(hipMemsetAsync(v, 0, (size_t)n3 * sizeof(float), c->stream));
    hipLaunchKernelGGL(k_narrow_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->invdS, c->invdS32);
    HIP_TRY(hipGetLastError());
    ST_TRY(build_mg32(c, c->mgS));
    ST_TRY(build_mg32(c, c->mgA));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STOKES_OK;
}

stokes_status stokes_set_option(stokes_ctx* c, const char* key, double v) {
    if (!c || !key || !std::isfinite(v)) return STOKES_E_ARG;
    const std::string k(key);
    // captured iterations bake in launch shapes and multigrid parameters
    drop_graphs(c);
    if (k.compare(0, 2, "mg") == 0) c->mg_two_ok = 0;   // the two-visit estimate depends on the cycle
    if (k == "eps_A") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->eps_A = v; }
    else if (k == "eps_S") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->eps_S = v; }
    else if (k == "max_outer") { if (v < 1 || v > 1e7) return STOKES_E_ARG; c->max_outer = (int)v; }
    else if (k == "max_inner") { if (v < 1 || v > 1e8) return STOKES_E_ARG; c->max_inner = (int)v; }
    else if (k == "stop_prec") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->stop_prec = (int)v; }
    else if (k == "check_every") { if (v < 0 || v > 4096) return STOKES_E_ARG; c->check_every = (int)v; }
    else if (k == "kernel_timing") {
        if (v < 0 || v > 1e6 || v != std::floor(v)) return STOKES_E_ARG;
        c->timing = (int)v;
    }
    else if (k == "true_velocity") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->true_velocity = (int)v; }
    else if (k == "precision") {
        if (v != 0.0 && v != 1.0) return STOKES_E_ARG;
        if (c->nbatch > 1 && v != 1.0) return STOKES_E_ARG;   // batched contexts solve in mixed precision
        if (v == 1.0) ST_TRY(ensure_mixed_buffers(c));
        c->precision = (int)v;
    }
    else if (k == "eps_A32") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->eps_A32 = v; }
    else if (k == "eps_S32") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->eps_S32 = v; }
    else if (k == "cycle_rtol") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->cycle_rtol = v; }
    else if (k == "eps_refine") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->eps_refine = v; }
    else if (k == "zero_rhs_factor") { if (!(v >= 0.0 && v <= 1e12)) return STOKES_E_ARG; c->zero_rhs_factor = v; }
    else if (k == "mg") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->use_mg = (int)v; }
    else if (k == "mg_A") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->use_mg_A = (int)v; }
    else if (k == "mg_omega") { if (!(v > 0.0 && v < 1.0)) return STOKES_E_ARG; c->mg_omega = v; }
    else if (k == "mg_scale_deep") { if (!(v >= 0.0 && v <= 2.0)) return STOKES_E_ARG; c->mg_scale_deep = v; }
    else if (k == "mg_scale") { if (!(v > 0.0 && v <= 2.0)) return STOKES_E_ARG; c->mg_scale = v; }
    else if (k == "mg_scale_A") { if (!(v > 0.0 && v <= 2.0)) return STOKES_E_ARG; c->mg_scale_A = v; }
    else if (k == "mg_coarse_sweeps") { if (v < 1 || v > 1000) return STOKES_E_ARG; c->mg_coarse_sweeps = (int)v; }
    else if (k == "mg_level_blocks") {
        if (v < 8 || v > kMaxBlocks) return STOKES_E_ARG;
        c->mg_level_blocks = (int)v;
        for (MgHier* h : {&c->mgS, &c->mgA})
            for (size_t l = 0; l < h->sweep.size(); ++l)
                h->sweep[l] = member_sweep(c, make_sweep(h->grid[l].n, c->mg_level_blocks));
    }
    else if (k == "mg_coarse_gs") { if (v != 0.0 && v != 1.0 && v != 2.0) return STOKES_E_ARG; c->mg_coarse_gs = (int)v; }
    else if (k == "sweep_blocks") {
        if (v < 8 || v > kMaxBlocks) return STOKES_E_ARG;
        const Sweep sw = make_sweep(c->N, (int)v);
        const Sweep sw32 = make_sweep32(c->N, (int)v);
        if (sw.nblk > kMaxBlocks || sw32.nblk > kMaxBlocks) return STOKES_E_ARG;
        c->sweep_blocks = (int)v;
        c->sw = member_sweep(c, sw);
        c->sw32 = member_sweep(c, sw32);
    }
    else if (k == "progress") { if (v < 0 || v > 1e7 || v != std::floor(v)) return STOKES_E_ARG; c->progress = (int)v; }
    else if (k == "fuse_dir_A") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->fuse_dir_A = (int)v; }
    else if (k == "fuse_dir_S") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->fuse_dir_S = (int)v; }
    else if (k == "mg_visits") { if (v != 0.0 && v != 1.0 && v != 2.0) return STOKES_E_ARG; c->mg_visits = (int)v; }
    else if (k == "mg_pipe") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->mg_pipe = (int)v; }
    else if (k == "graphs") { if (v != 0.0 && v != 1.0) return STOKES_E_ARG; c->use_graphs = (int)v; }
    else return STOKES_E_ARG;
    return STOKES_OK;
}

static stokes_status solve_mixed(stokes_ctx* c, stokes_precond precond, double tol);

// Level below which the right-hand side g = B u0, u0 = A^{-1} f, is taken to be
// zero.  S = B A^{-1} B^T has no eigenvalue above 1 (Sec. 4.2.2, eq.
// lambda_cg_rate), so ||B A^{-1/2}|| <= 1: an inner-solve residual r_A perturbs
// g by at most ||A^{-1/2} r_A||, and an exact g obeys
// ||g||^2 <= g^T S^+ g <= f^T A^{-1} f = f . u0 (the energy of the exact flow,
// f . u = f^T A^{-1} f - g^T S^+ g, is not negative).  With u0 accurate to the relative
// inner tolerance eps, a g below zero_rhs_factor * eps * sqrt(f . u0) cannot
// be told from the inner solve's error (straight channels along the force,
// whose exact g is 0); the pressure is then zero and u = u0.
static stokes_status rhs_floor(stokes_ctx* c, double eps, double* floor_out) {
    double sums[3];
    ST_TRY(face_sums(c, c->u, sums));
    double fu = 0.0;
    for (int a = 0; a < 3; ++a) fu += c->force[a] * sums[a];
    *floor_out = fu > 0.0 ? c->zero_rhs_factor * eps * std::sqrt(fu) : 0.0;
    return STOKES_OK;
}

// one line on stderr every `progress` outer iterations (option "progress")
static void report_progress(stokes_ctx* c, int k, double rel, double k_hat) {
    if (c->progress <= 0 || k % c->progress != 0) return;
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - c->t_solve0).count();
    std::fprintf(stderr, "[stokes] N=%d outer %d rel_res %.3e k_hat %.10e  %.1f s\n", c->N, k, rel, k_hat, t);
    std::fflush(stderr);
}

static stokes_status solve_impl(stokes_ctx* c, stokes_precond precond, double tol, const double* g_host = nullptr) {
    stokes_report& R = c->rep;
    const Sweep& s = c->sw;
    const int64_t n3 = c->n3;
    R = stokes_report{};
    R.n_components = c->ncomp_all;
    R.n_components_kept = c->ncomp_kept;
    R.porosity = (double)c->nfluid_in / (double)n3;
    R.porosity_effective = (double)c->nfluid / (double)n3;
    R.stv_ratio = c->nfluid_in ? (double)c->nsurf / (double)c->nfluid_in : 0.0;
    R.cond_est = R.ritz_min = R.ritz_max = std::nan("");
    c->hist.clear();
    c->have_solution = false;
    const double N2 = (double)c->N * (double)c->N;

    HIP_TRY(hipMemsetAsync(c->p, 0, (size_t)n3 * sizeof(double), c->stream));
    if (c->nfluid == 0) {
        HIP_TRY(hipMemsetAsync(c->u, 0, (size_t)(3 * n3) * sizeof(double), c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        R.flags |= STOKES_FLAG_NO_FLOW;
        R.status = STOKES_OK;
        c->have_solution = true;
        return STOKES_OK;
    }
    if (c->precision == 1) return solve_mixed(c, precond, tol);

    int itA = 0, itS = 0, stA = 0, stS = 0;
    int64_t totA = 0, totS = 0;
    int status = STOKES_OK;
    auto note_inner = [&](int st) {
        if (st == -4) status = STOKES_E_BREAKDOWN;
        else if (st == 1) R.flags |= STOKES_FLAG_INNER_MAXIT;
    };

    double g_floor = 0.0;
    if (g_host) {
        // a given right-hand side: p0 = 0, u0 = 0, r0 = g on the fluid cells
        // (only an exactly zero g skips the loop)
        HIP_TRY(hipMemsetAsync(c->u, 0, (size_t)(3 * n3) * sizeof(double), c->stream));
        HIP_TRY(hipMemcpyAsync(c->r, g_host, (size_t)n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_mask_cells, grid_of(s), dim3(kBlock), 0, c->stream, s, c->bits, c->wpr, c->r);
        HIP_TRY(hipGetLastError());
    } else {
        // u0 = A^{-1} f
        ST_TRY(solve_A64(c, nullptr, c->eps_A, &itA, &stA));
        totA += itA;
        note_inner(stA);
        std::swap(c->u, c->fx);
        ST_TRY(rhs_floor(c, c->eps_A, &g_floor));
        // r0 = g - S 0 = B u0
        hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, c->u, c->r);
        HIP_TRY(hipGetLastError());
    }
    ST_TRY(project(c, c->r));
    double* z = c->r;
    if (precond == STOKES_SIMPLE) {
        ST_TRY(solve_S64(c, c->r, c->eps_S, &itS, &stS));
        totS += itS;
        note_inner(stS);
        ST_TRY(project(c, c->zs));
        z = c->zs;
    }
    double dd[3];
    ST_TRY(dots(c, c->r, z, c->r, c->r, z, z, dd));
    double rz = dd[0];
    const double r0 = std::sqrt(dd[1]), z0 = std::sqrt(dd[2]);
    R.r0_norm = r0;
    HIP_TRY(hipMemcpyAsync(c->d, z, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));

    std::vector<double> alphas, betas;
    int k = 0;
    double rel = 0.0, relz = 0.0;
    if (!(r0 > g_floor)) {
        R.flags |= STOKES_FLAG_ZERO_RHS;
    } else {
        while (status >= 0) {
            if (k >= c->max_outer) {
                status = STOKES_NOT_CONVERGED;
                break;
            }
            const int64_t a0 = totA, s0 = totS;
            // q = S d = B A^{-1} B^T d
            hipLaunchKernelGGL(k_apply_BT, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, c->d, c->fr);
            HIP_TRY(hipGetLastError());
            ST_TRY(solve_A64(c, c->fr, c->eps_A, &itA, &stA));
            totA += itA;
            note_inner(stA);
            hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, c->fx, c->q);
            HIP_TRY(hipGetLastError());
            double dq3[3];
            ST_TRY(dots(c, c->d, c->q, nullptr, nullptr, nullptr, nullptr, dq3));
            const double dq = dq3[0];
            if (!(dq > 0.0) || !std::isfinite(dq)) {
                status = STOKES_E_BREAKDOWN;
                break;
            }
            const double alpha = rz / dq;
            hipLaunchKernelGGL(k_outer_update, grid_of(s), dim3(kBlock), 0, c->stream, s, c->p, c->r, c->d, c->q,
                               ms1(alpha));
            hipLaunchKernelGGL(k_axpy_faces, grid_of(s), dim3(kBlock), 0, c->stream, s, c->u, c->fx, ms1(-alpha));
            HIP_TRY(hipGetLastError());
            ST_TRY(project(c, c->r));
            if (precond == STOKES_SIMPLE) {
                ST_TRY(solve_S64(c, c->r, c->eps_S, &itS, &stS));
                totS += itS;
                note_inner(stS);
                ST_TRY(project(c, c->zs));
            }
            ST_TRY(dots(c, c->r, z, c->r, c->r, z, z, dd));
            ++k;
            rel = std::sqrt(dd[1]) / r0;
            relz = std::sqrt(dd[2]) / z0;
            if (!std::isfinite(rel) || !std::isfinite(relz)) {
                status = STOKES_E_BREAKDOWN;
                break;
            }
            const bool stop = c->stop_prec ? (relz < tol) : (rel < tol);
            double beta = 0.0;
            if (!stop) {
                beta = dd[0] / rz;
                rz = dd[0];
                hipLaunchKernelGGL(k_dir_cells, grid_of(s), dim3(kBlock), 0, c->stream, s, c->d, z, ms1(beta));
                HIP_TRY(hipGetLastError());
            }
            alphas.push_back(alpha);
            if (!stop) betas.push_back(beta);
            double sums[3], mean[3];
            ST_TRY(face_sums(c, c->u, sums));
            const double kk = kvox_of(c, sums, mean) / N2;
            c->hist.insert(c->hist.end(), {rel, relz, kk, (double)(totA - a0), (double)(totS - s0), alpha, beta, 0.0});
            report_progress(c, k, rel, kk);
            if (stop) break;
        }
    }
    ST_TRY(project(c, c->p));

    // optional true velocity u = A^{-1}(f - B^T p) (eq. velocity_schur)
    if (c->true_velocity && status >= 0) {
        hipLaunchKernelGGL(k_force_minus_BT, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, c->p, c->force[0],
                           c->force[1], c->force[2], c->fr);
        HIP_TRY(hipGetLastError());
        ST_TRY(solve_A64(c, c->fr, c->eps_A, &itA, &stA));
        totA += itA;
        note_inner(stA);
        std::swap(c->u, c->fx);
    }

    double sums[3], mean[3];
    ST_TRY(face_sums(c, c->u, sums));
    R.k_vox = kvox_of(c, sums, mean);
    R.k_hat = R.k_vox / N2;
    for (int a = 0; a < 3; ++a) R.mean_u[a] = mean[a];
    hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, c->u, c->q);
    HIP_TRY(hipGetLastError());
    double dv[3];
    ST_TRY(dots(c, c->q, c->q, nullptr, nullptr, nullptr, nullptr, dv));
    R.div_norm = std::sqrt(dv[0]);
    R.outer_iters = k;
    R.inner_A_iters = (int)totA;
    R.inner_S_iters = (int)totS;
    R.rel_res = rel;
    R.rel_res_prec = relz;
    if (!alphas.empty()) {
        betas.resize(alphas.size() - 1 < betas.size() ? alphas.size() - 1 : betas.size());
        lanczos_extremes(alphas, betas, &R.ritz_min, &R.ritz_max);
        R.cond_est = R.ritz_max / R.ritz_min;
    }
    R.status = status;
    ST_TRY(collect_timing(c));
    c->have_solution = status >= 0;
    return (stokes_status)status;
}

// ---------------------------------------------------------------------------
// Mixed precision: FP32 inner solves, FP64 outer recurrences.
//
// Defect correction around a flexible outer CG.  Each cycle starts from the
// true residual r = g - S p = B u, u = A^{-1}(f - B^T p) held in FP64 and
// refined to eps_refine (FP32 CG sweeps on FP64 residuals); inside a cycle the
// outer CG (flexible beta = (z_k+1, r_k+1 - r_k) / (z_k, r_k), Notay's FCG,
// which tolerates the inexact FP32 preconditioner and S) reduces the recursive
// residual by cycle_rtol, updating p and the recursive velocity; the cycle ends
// with the refinement of u and a fresh true residual.  The solve stops when the
// true residual meets tol.
// ---------------------------------------------------------------------------
// Members that the outer-loop kernels (and the first kernel of each inner
// solve) work on; the others sit the step out.
static void set_active(stokes_ctx* c, unsigned mask) {
    c->sw.active = mask;
    c->sw32.active = mask;
}

static bool has(unsigned mask, int m) { return (mask >> m) & 1u; }

// zero `bytes` of a per-member buffer in every member
static stokes_status zero_members(stokes_ctx* c, void* p, size_t bytes) {
    if (c->nbatch == 1) HIP_TRY(hipMemsetAsync(p, 0, bytes, c->stream));
    else HIP_TRY(hipMemset2DAsync(p, c->bstride, 0, bytes, (size_t)c->nbatch, c->stream));
    return STOKES_OK;
}

// Per-member state of the mixed-precision solve.
struct MixedMember {
    int k = 0, cycle = 0;
    double r0 = 0.0, z0 = 0.0, rz = 0.0, target = 0.0, rel = 0.0, relz = 0.0, g_floor = 0.0;
    int status = STOKES_OK;
    int inner_status = 0;
    unsigned flags = 0;
    int64_t totA = 0, totS = 0;
    std::vector<double> alphas, betas;   // first cycle only: a restart starts a new Krylov space
};

// u <- A^{-1}(f - B^T p) to eps_refine, starting from the current u, for the
// members in `mask` (each refines until its own residual meets the tolerance).
static stokes_status refine_velocity(stokes_ctx* c, unsigned mask, std::vector<MixedMember>& M) {
    const int B = c->nbatch;
    set_active(c, mask);
    hipLaunchKernelGGL(k_force_minus_BT, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->code, c->p,
                       c->force[0], c->force[1], c->force[2], c->fr);
    HIP_TRY(hipGetLastError());
    std::vector<double> t(3 * (size_t)B);
    MemberScalars one{};
    for (int m = 0; m < B; ++m) one.v[m] = 1.0;
    unsigned todo = mask;
    for (int round = 0; todo; ++round) {
        set_active(c, todo);
        hipLaunchKernelGGL(k_residual_A, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->code, c->fr, c->u,
                           c->fq, c->dpart);
        HIP_TRY(hipGetLastError());
        ST_TRY(host_totals(c, t.data()));
        unsigned next = 0;
        for (int m = 0; m < B; ++m) {
            if (!has(todo, m)) continue;
            const double rel = t[3 * m + 1] > 0.0 ? std::sqrt(t[3 * m] / t[3 * m + 1]) : 0.0;
            if (!std::isfinite(rel)) {
                M[m].status = STOKES_E_BREAKDOWN;
                continue;
            }
            if (!(rel < c->eps_refine || round >= c->max_refine)) next |= 1u << m;
        }
        todo = next;
        if (!todo) break;
        set_active(c, todo);
        int it = 0, st = 0;
        ST_TRY(inner_A<float>(c, bufA32(c), c->fq, c->eps_A32, &it, &st));
        for (int m = 0; m < B; ++m) {
            if (!has(todo, m)) continue;
            M[m].totA += c->m_it[m];
            if (c->m_status[m] == -4) M[m].inner_status = -4;
        }
        set_active(c, todo);
        hipLaunchKernelGGL(k_axpy_faces_f32, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->u, c->fx32, one);
        HIP_TRY(hipGetLastError());
    }
    return STOKES_OK;
}

// z <- SIMPLE^+ r in FP32 (widened and projected), or z = r for Uzawa, for the
// members in `mask`
static stokes_status mixed_precond(stokes_ctx* c, stokes_precond precond, unsigned mask, std::vector<MixedMember>& M) {
    set_active(c, mask);
    if (precond == STOKES_UZAWA) {
        hipLaunchKernelGGL(k_copy_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->zs,
                           (const double*)c->r);
        HIP_TRY(hipGetLastError());
        return STOKES_OK;
    }
    int it = 0, st = 0;
    ST_TRY(inner_S<float>(c, bufS32(c), c->r, c->eps_S32, &it, &st));
    for (int m = 0; m < c->nbatch; ++m) {
        if (!has(mask, m)) continue;
        M[m].totS += c->m_it[m];
        if (c->m_status[m] == -4) M[m].inner_status = -4;
    }
    set_active(c, mask);
    hipLaunchKernelGGL(k_widen_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->zs32, c->zs);
    HIP_TRY(hipGetLastError());
    return project(c, c->zs);
}

// Defect correction around a flexible outer CG, for every member of the
// context at once (one member: a plain context).  Each cycle starts from the
// true residual r = g - S p = B u, u = A^{-1}(f - B^T p) held in FP64 and
// refined to eps_refine (FP32 CG sweeps on FP64 residuals); inside a cycle the
// outer CG (flexible beta = (z_k+1, r_k+1 - r_k) / (z_k, r_k), Notay's FCG,
// which tolerates the inexact FP32 preconditioner and S) reduces the recursive
// residual by cycle_rtol, updating p and the recursive velocity; the cycle ends
// with the refinement of u and a fresh true residual.  A member stops when its
// true residual meets tol.  The members run in lockstep: every step is one
// launch per kernel for all members still in that step; a member that has
// left a loop sits out its remaining steps, so its arithmetic is exactly
// that of a solve of its own.
static stokes_status solve_mixed(stokes_ctx* c, stokes_precond precond, double tol) {
    const int B = c->nbatch;
    const int64_t n3 = c->n3;
    const double N2 = (double)c->N * (double)c->N;
    ST_TRY(ensure_mixed_buffers(c));
    double* z = c->zs;        // FP64 preconditioned residual
    double* r_old = c->sr;    // FP64 previous residual (flexible beta)
    std::vector<MixedMember> M(B);
    c->mhist.assign(B, {});
    unsigned live = 0;        // members with conducting fluid
    for (int m = 0; m < B; ++m) {
        if (c->member[m].nfluid > 0) live |= 1u << m;
        else M[m].flags |= STOKES_FLAG_NO_FLOW;
    }
    ST_TRY(zero_members(c, c->p, (size_t)n3 * sizeof(double)));
    ST_TRY(zero_members(c, c->u, (size_t)(3 * n3) * sizeof(double)));
    std::vector<double> dd(3 * (size_t)B), zz(3 * (size_t)B), sums(3 * (size_t)B);
    auto drop = [&](unsigned& mask) {   // members that failed or hit a cap leave `mask`
        for (int m = 0; m < B; ++m)
            if (has(mask, m) && (M[m].status < 0 || M[m].status == STOKES_NOT_CONVERGED)) mask &= ~(1u << m);
    };
    unsigned going = live;
    if (going) ST_TRY(refine_velocity(c, going, M));
    drop(going);
    if (going) {
        // g counts as zero below zero_rhs_factor * eps_refine * sqrt(f . u0)
        set_active(c, going);
        ST_TRY(face_sums(c, c->u, sums.data()));
        for (int m = 0; m < B; ++m) {
            double fu = 0.0;
            for (int a = 0; a < 3; ++a) fu += c->force[a] * sums[3 * m + a];
            M[m].g_floor = fu > 0.0 ? c->zero_rhs_factor * c->eps_refine * std::sqrt(fu) : 0.0;
        }
        hipLaunchKernelGGL(k_apply_B, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->u, c->r);
        HIP_TRY(hipGetLastError());
        ST_TRY(project(c, c->r));
        ST_TRY(dots(c, c->r, c->r, nullptr, nullptr, nullptr, nullptr, dd.data()));
        for (int m = 0; m < B; ++m) {
            if (!has(going, m)) continue;
            M[m].r0 = std::sqrt(dd[3 * m]);
            if (!(M[m].r0 > M[m].g_floor)) {
                M[m].flags |= STOKES_FLAG_ZERO_RHS;
                going &= ~(1u << m);
            }
        }
    }
    std::vector<double> alpha(B, 0.0);
    std::vector<int64_t> a0(B), s0(B);
    while (going) {
        // one defect-correction cycle on the current true residual
        ST_TRY(mixed_precond(c, precond, going, M));
        set_active(c, going);
        ST_TRY(dots(c, c->r, z, c->r, c->r, z, z, dd.data()));
        for (int m = 0; m < B; ++m) {
            if (!has(going, m)) continue;
            MixedMember& q = M[m];
            q.rz = dd[3 * m];
            const double rs = std::sqrt(dd[3 * m + 1]);
            if (q.z0 == 0.0) q.z0 = std::sqrt(dd[3 * m + 2]);
            q.target = std::max(tol * q.r0, c->cycle_rtol * rs);
        }
        hipLaunchKernelGGL(k_copy_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->d, (const double*)z);
        HIP_TRY(hipGetLastError());
        unsigned inner = going;
        while (inner) {
            for (int m = 0; m < B; ++m)
                if (has(inner, m) && M[m].k >= c->max_outer) M[m].status = STOKES_NOT_CONVERGED;
            drop(inner);
            if (!inner) break;
            for (int m = 0; m < B; ++m) {
                a0[m] = M[m].totA;
                s0[m] = M[m].totS;
            }
            set_active(c, inner);
            hipLaunchKernelGGL(k_apply_BT, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->code, c->d, c->fr);
            HIP_TRY(hipGetLastError());
            int it = 0, st = 0;
            ST_TRY(inner_A<float>(c, bufA32(c), c->fr, c->eps_A32, &it, &st));
            for (int m = 0; m < B; ++m) {
                if (!has(inner, m)) continue;
                M[m].totA += c->m_it[m];
                if (c->m_status[m] == -4) M[m].inner_status = -4;
            }
            set_active(c, inner);
            hipLaunchKernelGGL(k_apply_B_f32, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->fx32, c->q);
            HIP_TRY(hipGetLastError());
            ST_TRY(dots(c, c->d, c->q, nullptr, nullptr, nullptr, nullptr, dd.data()));
            MemberScalars am{}, nam{};
            for (int m = 0; m < B; ++m) {
                if (!has(inner, m)) continue;
                const double dq = dd[3 * m];
                if (!(dq > 0.0) || !std::isfinite(dq)) {
                    M[m].status = STOKES_E_BREAKDOWN;
                    continue;
                }
                alpha[m] = M[m].rz / dq;
                am.v[m] = alpha[m];
                nam.v[m] = -alpha[m];
            }
            drop(inner);
            if (!inner) break;
            set_active(c, inner);
            hipLaunchKernelGGL(k_copy_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, r_old,
                               (const double*)c->r);
            hipLaunchKernelGGL(k_outer_update, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->p, c->r, c->d,
                               c->q, am);
            hipLaunchKernelGGL(k_axpy_faces_f32, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->u, c->fx32,
                               nam);
            HIP_TRY(hipGetLastError());
            ST_TRY(project(c, c->r));
            ST_TRY(mixed_precond(c, precond, inner, M));
            set_active(c, inner);
            ST_TRY(dots(c, z, c->r, z, r_old, c->r, c->r, dd.data()));
            ST_TRY(dots(c, z, z, nullptr, nullptr, nullptr, nullptr, zz.data()));
            unsigned cont = 0, noted = 0;
            MemberScalars bm{};
            for (int m = 0; m < B; ++m) {
                if (!has(inner, m)) continue;
                MixedMember& q = M[m];
                ++q.k;
                const double rn = std::sqrt(dd[3 * m + 2]);
                q.rel = rn / q.r0;
                q.relz = std::sqrt(zz[3 * m]) / q.z0;
                if (!std::isfinite(q.rel)) {
                    q.status = STOKES_E_BREAKDOWN;
                    continue;
                }
                noted |= 1u << m;
                const bool stop = rn <= q.target;
                double beta = 0.0;
                if (!stop) {
                    beta = (dd[3 * m] - dd[3 * m + 1]) / q.rz;   // flexible (Notay) beta
                    q.rz = dd[3 * m];
                    bm.v[m] = beta;
                    cont |= 1u << m;
                }
                if (q.cycle == 0) {
                    q.alphas.push_back(alpha[m]);
                    if (!stop) q.betas.push_back(beta);
                }
                c->mhist[m].insert(c->mhist[m].end(), {q.rel, q.relz, 0.0, (double)(q.totA - a0[m]),
                                                       (double)(q.totS - s0[m]), alpha[m], beta, 0.0});
            }
            if (cont) {
                set_active(c, cont);
                hipLaunchKernelGGL(k_dir_cells, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->d, z, bm);
                HIP_TRY(hipGetLastError());
            }
            if (noted) {
                // permeability of the recursive velocity, per iteration
                set_active(c, noted);
                ST_TRY(face_sums(c, c->u, sums.data()));
                for (int m = 0; m < B; ++m) {
                    if (!has(noted, m)) continue;
                    double mean[3];
                    const double kk = kvox_of(c, &sums[3 * m], mean) / N2;
                    c->mhist[m][c->mhist[m].size() - 6] = kk;
                    if (B == 1) report_progress(c, M[m].k, M[m].rel, kk);
                }
            }
            inner = cont;
            drop(going);
        }
        drop(going);
        if (!going) break;
        // the true residual of the new pressure
        ST_TRY(refine_velocity(c, going, M));
        drop(going);
        if (!going) break;
        set_active(c, going);
        hipLaunchKernelGGL(k_apply_B, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->u, c->r);
        HIP_TRY(hipGetLastError());
        ST_TRY(project(c, c->r));
        ST_TRY(dots(c, c->r, c->r, nullptr, nullptr, nullptr, nullptr, dd.data()));
        for (int m = 0; m < B; ++m) {
            if (!has(going, m)) continue;
            MixedMember& q = M[m];
            q.rel = std::sqrt(dd[3 * m]) / q.r0;
            auto& h = c->mhist[m];
            if (!h.empty()) h[h.size() - 8] = q.rel;   // the cycle's last entry: true residual
            ++q.cycle;
            if (q.rel < tol) going &= ~(1u << m);
        }
    }
    // results of every member with conducting fluid
    std::vector<double> div(3 * (size_t)B, 0.0);
    if (live) {
        set_active(c, live);
        ST_TRY(project(c, c->p));
        ST_TRY(face_sums(c, c->u, sums.data()));
        hipLaunchKernelGGL(k_apply_B, grid_of(c->sw), dim3(kBlock), 0, c->stream, c->sw, c->u, c->q);
        HIP_TRY(hipGetLastError());
        ST_TRY(dots(c, c->q, c->q, nullptr, nullptr, nullptr, nullptr, div.data()));
    }
    set_active(c, all_members_of(B));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mrep.assign(B, stokes_report{});
    int worst = STOKES_OK;
    for (int m = 0; m < B; ++m) {
        MixedMember& q = M[m];
        stokes_report& R = c->mrep[m];
        const auto& g = c->member[m];
        R.n_components = g.ncomp_all;
        R.n_components_kept = g.ncomp_kept;
        R.porosity = (double)g.nfluid_in / (double)n3;
        R.porosity_effective = (double)g.nfluid / (double)n3;
        R.stv_ratio = g.nfluid_in ? (double)g.nsurf / (double)g.nfluid_in : 0.0;
        R.cond_est = R.ritz_min = R.ritz_max = std::nan("");
        R.flags = q.flags;
        if (q.status >= 0 && q.inner_status == -4) q.status = STOKES_E_BREAKDOWN;
        if (has(live, m)) {
            double mean[3];
            R.k_vox = kvox_of(c, &sums[3 * m], mean);
            R.k_hat = R.k_vox / N2;
            for (int a = 0; a < 3; ++a) R.mean_u[a] = mean[a];
            R.div_norm = std::sqrt(div[3 * m]);
        }
        R.r0_norm = q.r0;
        R.outer_iters = q.k;
        R.inner_A_iters = (int)q.totA;
        R.inner_S_iters = (int)q.totS;
        R.rel_res = q.rel;
        R.rel_res_prec = q.relz;
        if (!q.alphas.empty()) {
            q.betas.resize(q.alphas.size() - 1 < q.betas.size() ? q.alphas.size() - 1 : q.betas.size());
            lanczos_extremes(q.alphas, q.betas, &R.ritz_min, &R.ritz_max);
            R.cond_est = R.ritz_max / R.ritz_min;
        }
        R.status = q.status;
        if (q.status < 0) worst = std::min(worst, q.status);
        else if (q.status > 0 && worst == STOKES_OK) worst = q.status;
    }
    c->rep = c->mrep[0];
    c->hist = c->mhist[0];
    ST_TRY(collect_timing(c));
    c->have_solution = B > 1 || worst >= 0;
    return (stokes_status)worst;
}

stokes_status stokes_solve(stokes_ctx* c, stokes_precond precond, double tol, stokes_report* report) {
    if (!c) return STOKES_E_ARG;
    if (precond != STOKES_UZAWA && precond != STOKES_SIMPLE) return STOKES_E_ARG;
    if (!(tol > 0.0) || !std::isfinite(tol)) return STOKES_E_ARG;
    if (precond == STOKES_SIMPLE) ST_TRY(prepare_two_visits(c));   // the SIMPLE preconditioner's cycle only
    const auto t0 = std::chrono::steady_clock::now();
    c->t_solve0 = t0;
    stokes_status st;
    try {
        // a batched context solves all of its members at once (mixed precision)
        st = c->batch_api ? solve_mixed(c, precond, tol) : solve_impl(c, precond, tol);
    } catch (const std::bad_alloc&) {
        st = STOKES_E_NOMEM;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->rep.seconds = secs;
    for (auto& r : c->mrep) r.seconds = secs;
    if (precond == STOKES_SIMPLE && c->use_mg && mg_two_visits(c, c->mgS)) {
        c->rep.flags |= STOKES_FLAG_MG_TWO_VISITS;
        for (auto& r : c->mrep) r.flags |= STOKES_FLAG_MG_TWO_VISITS;
    }
    if (report) *report = c->rep;
    return st;
}

stokes_status stokes_solve_rhs(stokes_ctx* c, stokes_precond precond, double tol, const double* g,
                               stokes_report* report) {
    if (!c || !g) return STOKES_E_ARG;
    if (precond != STOKES_UZAWA && precond != STOKES_SIMPLE) return STOKES_E_ARG;
    if (!(tol > 0.0) || !std::isfinite(tol)) return STOKES_E_ARG;
    if (c->batch_api || c->precision != 0) return STOKES_E_STATE;
    if (precond == STOKES_SIMPLE) ST_TRY(prepare_two_visits(c));
    const auto t0 = std::chrono::steady_clock::now();
    c->t_solve0 = t0;
    stokes_status st;
    try {
        st = solve_impl(c, precond, tol, g);
    } catch (const std::bad_alloc&) {
        st = STOKES_E_NOMEM;
    }
    c->rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (precond == STOKES_SIMPLE && c->use_mg && mg_two_visits(c, c->mgS)) c->rep.flags |= STOKES_FLAG_MG_TWO_VISITS;
    if (report) *report = c->rep;
    return st;
}

stokes_status stokes_batch_result(stokes_ctx* c, int member, stokes_report* report, double* p, double* u) {
    if (!c || member < 0 || member >= c->nbatch) return STOKES_E_ARG;
    if (!c->have_solution || (int)c->mrep.size() != c->nbatch) return STOKES_E_STATE;
    if (report) *report = c->mrep[member];
    const size_t o = (size_t)member * c->bstride;
    if (p)
        HIP_TRY(hipMemcpyAsync(p, (const char*)c->p + o, (size_t)c->n3 * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    if (u)
        HIP_TRY(hipMemcpyAsync(u, (const char*)c->u + o, (size_t)(3 * c->n3) * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STOKES_OK;
}

stokes_status stokes_permeability(stokes_ctx* c, double* k_hat) {
    if (!c || !k_hat) return STOKES_E_ARG;
    if (!c->have_solution) return STOKES_E_STATE;
    *k_hat = c->rep.k_hat;
    return STOKES_OK;
}

stokes_status stokes_get_report(stokes_ctx* c, stokes_report* report) {
    if (!c || !report) return STOKES_E_ARG;
    if (!c->have_solution) return STOKES_E_STATE;
    *report = c->rep;
    return STOKES_OK;
}

stokes_status stokes_history(stokes_ctx* c, double* out, int cap, int* n_out) {
    if (!c || !n_out || cap < 0 || (cap > 0 && !out)) return STOKES_E_ARG;
    const int n = (int)(c->hist.size() / 8);
    *n_out = n;
    const int m = std::min(n, cap);
    if (m > 0) std::memcpy(out, c->hist.data(), (size_t)m * 8 * sizeof(double));
    return STOKES_OK;
}

stokes_status stokes_get_fields(stokes_ctx* c, double* p, double* u) {
    if (!c) return STOKES_E_ARG;
    if (!c->have_solution) return STOKES_E_STATE;
    if (p) HIP_TRY(hipMemcpyAsync(p, c->p, (size_t)c->n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (u) HIP_TRY(hipMemcpyAsync(u, c->u, (size_t)(3 * c->n3) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STOKES_OK;
}

// Operators on device fields.  The input is first copied into context
// scratch (inner-solve work vectors; the solution p, u is not touched) and
// masked, so entries that are not unknowns are ignored.
static stokes_status apply_impl(stokes_ctx* c, int op, const double* in, double* out, hipMemcpyKind kin,
                                hipMemcpyKind kout) {
    const Sweep& s = c->sw;
    const int64_t n3 = c->n3;
    const bool face_in = op == STOKES_OP_A || op == STOKES_OP_B || op == STOKES_OP_MG_A;
    const bool face_out = op == STOKES_OP_A || op == STOKES_OP_BT || op == STOKES_OP_DIAG_A || op == STOKES_OP_MG_A;
    const bool no_in = op == STOKES_OP_DIAG_A || op == STOKES_OP_DIAG_SHAT;
    if (op == STOKES_OP_MG_SHAT) ST_TRY(prepare_two_visits(c));
    double* src = face_in ? c->fd : c->sd;
    double* dst = face_out ? c->fq : c->sq;
    if (!no_in) {
        if (!in) return STOKES_E_ARG;
        HIP_TRY(hipMemcpyAsync(src, in, (size_t)((face_in ? 3 : 1) * n3) * sizeof(double), kin, c->stream));
        if (face_in) hipLaunchKernelGGL(k_mask_faces, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src);
        else hipLaunchKernelGGL(k_mask_cells, grid_of(s), dim3(kBlock), 0, c->stream, s, c->bits, c->wpr, src);
    }
    switch (op) {
    case STOKES_OP_A: hipLaunchKernelGGL(k_apply_A, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, dst); break;
    case STOKES_OP_B: hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, src, dst); break;
    case STOKES_OP_BT: hipLaunchKernelGGL(k_apply_BT, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, dst); break;
    case STOKES_OP_SHAT: hipLaunchKernelGGL(k_apply_Shat, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, dst); break;
    case STOKES_OP_DIAG_A: hipLaunchKernelGGL(k_diag_A, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, dst); break;
    case STOKES_OP_DIAG_SHAT: hipLaunchKernelGGL(k_diag_Shat, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, dst); break;
    case STOKES_OP_PROJECT:
        HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        ST_TRY(project(c, dst));
        break;
    case STOKES_OP_S: {
        hipLaunchKernelGGL(k_apply_BT, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, c->fr);
        int it = 0, st = 0;
        ST_TRY(solve_A64(c, c->fr, c->eps_A, &it, &st));
        if (st == -4) return STOKES_E_BREAKDOWN;
        hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, c->fx, dst);
        break;
    }
    case STOKES_OP_MG_SHAT:
        if (c->mgS.levels < 1) return STOKES_E_LIMIT;
        ST_TRY(vcycle<double>(c, c->mgS, src, c->invdS, dst, nullptr));
        break;
    case STOKES_OP_MG_A:
        if (c->mgA.levels < 1) return STOKES_E_LIMIT;
        ST_TRY(vcycle<double>(c, c->mgA, src, (const double*)nullptr, dst, nullptr));
        break;
    default: return STOKES_E_ARG;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, dst, (size_t)((face_out ? 3 : 1) * n3) * sizeof(double), kout, c->stream));
    return STOKES_OK;
}

stokes_status stokes_apply(stokes_ctx* c, int op, const double* in, double* out) {
    if (!c || !out || op < 0 || op > STOKES_OP_MG_A) return STOKES_E_ARG;
    if (c->nbatch > 1) return STOKES_E_STATE;
    ST_TRY(apply_impl(c, op, in, out, hipMemcpyHostToDevice, hipMemcpyDeviceToHost));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STOKES_OK;
}

stokes_status stokes_apply_device(stokes_ctx* c, int op, const double* in, double* out) {
    if (!c || !out || op < 0 || op > STOKES_OP_MG_A) return STOKES_E_ARG;
    if (c->nbatch > 1) return STOKES_E_STATE;
    return apply_impl(c, op, in, out, hipMemcpyDeviceToDevice, hipMemcpyDeviceToDevice);
}

// The variant of stokes_apply_device that allocates nothing: the same kernels,
// with the masked input copy and the projection's partial sums in `scratch`
// (this device's copy, resolved at set-up) and the result written straight to
// `out`.  Layout in scratch (doubles): [partials, rounded up to 256 bytes]
// [input copy].  Only device copies and kernel launches on the context's
// stream: no allocation, no memset, no synchronisation.
stokes_status stokes_apply_device_noalloc(stokes_ctx* c, int op, const double* in, double* out) {
    if (!c || !out) return STOKES_E_ARG;
    if (c->nbatch > 1) return STOKES_E_STATE;
    if (op != STOKES_OP_A && op != STOKES_OP_B && op != STOKES_OP_BT && op != STOKES_OP_SHAT &&
        op != STOKES_OP_DIAG_A && op != STOKES_OP_DIAG_SHAT && op != STOKES_OP_PROJECT)
        return STOKES_E_ARG;
    const bool no_in = op == STOKES_OP_DIAG_A || op == STOKES_OP_DIAG_SHAT;
    const bool face_in = op == STOKES_OP_A || op == STOKES_OP_B;
    if (!no_in && !in) return STOKES_E_ARG;
    double* base = c->noalloc_scratch;
    if (!base) return STOKES_E_DEVICE;
    const Sweep& s = c->sw;
    const int64_t n3 = c->n3;
    const int K = c->ncomp_kept;
    const bool one = K == 1 && !c->label;
    int64_t part_words = 0, mean_off = 0;
    if (op == STOKES_OP_PROJECT && K > 0) {
        part_words = one ? (int64_t)kMaxBlocks : (int64_t)kCompBlocks * K;
        mean_off = part_words;
        part_words += one ? 0 : K;
    }
    part_words = (part_words + 31) / 32 * 32;
    const int64_t in_words = (no_in || op == STOKES_OP_PROJECT) ? 0 : (face_in ? 3 : 1) * n3;
    if (part_words + in_words > kNoAllocScratchWords) return STOKES_E_LIMIT;
    if (op == STOKES_OP_PROJECT) {
        // in place on out: copy, mask, remove the component means
        if (out != in)
            HIP_TRY(hipMemcpyAsync(out, in, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_mask_cells, grid_of(s), dim3(kBlock), 0, c->stream, s, c->bits, c->wpr, out);
        HIP_TRY(hipGetLastError());
        return project_with(c, out, base, base + mean_off);
    }
    double* src = base + part_words;
    if (!no_in) {
        HIP_TRY(hipMemcpyAsync(src, in, (size_t)in_words * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if (face_in) hipLaunchKernelGGL(k_mask_faces, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src);
        else hipLaunchKernelGGL(k_mask_cells, grid_of(s), dim3(kBlock), 0, c->stream, s, c->bits, c->wpr, src);
    }
    switch (op) {
    case STOKES_OP_A: hipLaunchKernelGGL(k_apply_A, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, out); break;
    case STOKES_OP_B: hipLaunchKernelGGL(k_apply_B, grid_of(s), dim3(kBlock), 0, c->stream, s, src, out); break;
    case STOKES_OP_BT: hipLaunchKernelGGL(k_apply_BT, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, out); break;
    case STOKES_OP_SHAT: hipLaunchKernelGGL(k_apply_Shat, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, src, out); break;
    case STOKES_OP_DIAG_A: hipLaunchKernelGGL(k_diag_A, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, out); break;
    default: hipLaunchKernelGGL(k_diag_Shat, grid_of(s), dim3(kBlock), 0, c->stream, s, c->code, out); break;
    }
    HIP_TRY(hipGetLastError());
    return STOKES_OK;
}

stokes_status stokes_info(stokes_ctx* c, int64_t info[12]) {
    if (!c || !info) return STOKES_E_ARG;
    info[0] = c->N;
    info[1] = c->nfluid_in;
    info[2] = c->nfluid;
    info[3] = c->nsurf;
    info[4] = c->ncomp_all;
    info[5] = c->ncomp_kept;
    info[6] = c->nface[0];
    info[7] = c->nface[1];
    info[8] = c->nface[2];
    info[9] = c->device_bytes;
    info[10] = c->mgS.levels;
    info[11] = c->mgA.levels;
    return STOKES_OK;
}

stokes_status stokes_kernel_timing(stokes_ctx* c, int kernel, double* ms_total, int64_t* launches,
                                   double* bytes_per_launch) {
    if (!c || !ms_total || !launches || !bytes_per_launch || kernel < 0 || kernel >= kTimeKinds) return STOKES_E_ARG;
    ST_TRY(collect_timing(c));
    *ms_total = c->timing_ms[kernel];
    *launches = c->timing_launches[kernel];
    *bytes_per_launch = kBytesPerCell[kernel] * (double)c->n3;
    c->timing_ms[kernel] = 0.0;
    c->timing_launches[kernel] = 0;
    return STOKES_OK;
}

void stokes_destroy(stokes_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    release(c);
    delete c;
}

}  // extern "C"
