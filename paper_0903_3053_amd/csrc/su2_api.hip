// su2_api.hip -- the C ABI of libsu2.so (declared in include/su2.h): one
// global lattice context, device-resident state, graph-replayed sweeps.
//
// Program model (Sec. 2.1): all data stay in GPU memory, every kernel is
// launched by the host and does one complete operation, and results cross to
// the host only when asked for.  A sweep is eight pass launches plus a one-lane
// kernel that advances the device-resident sweep index, so the same captured
// hipGraph replays any number of sweeps with no host round trip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "su2.h"
#include "su2_kernels.hpp"
#include "su2_learned.hpp"

using namespace su2;

namespace su2 {

// Polyakov loop at every spatial site xs = x0 + L0 (x1 + L1 x2): (1/2)Tr of the
// ordered product of U_3(xs, t), t = 0 .. L3-1 (FP32 products), stored in FP64.
__global__ __launch_bounds__(kBlock) void k_polyakov_field(const float4 *__restrict__ L, Geo g,
                                                           uint32_t vs, double *__restrict__ field)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= vs) return;
    const uint32_t x0 = i % g.L[0];
    const uint32_t r = i / g.L[0];
    const uint32_t x1 = r % g.L[1];
    const uint32_t x2 = r / g.L[1];
    float4 P = make_float4(1.f, 0.f, 0.f, 0.f);
    for (uint32_t t = 0; t < g.L[3]; ++t) {
        const uint32_t p = (x0 + x1 + x2 + t) & 1u;
        const uint32_t h = (x0 >> 1) + x1 * g.st[1] + x2 * g.st[2] + t * g.st[3];
        P = qmul(P, L[arr(g, 3, p) + h]);
    }
    field[i] = (double)P.x;
}

// partial[r * gridDim.x + b]: workgroup b's sum over its sites xs of
// L(xs) (L(xs + r e0) + L(xs + r e1) + L(xs + r e2)), r = blockIdx.y
__global__ __launch_bounds__(kBlock) void k_polyakov_corr(const double *__restrict__ field, Geo g,
                                                          uint32_t vs, double *__restrict__ partial)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t rr = blockIdx.y;
    double acc = 0.0;
    if (i < vs) {
        const uint32_t x0 = i % g.L[0];
        const uint32_t q = i / g.L[0];
        const uint32_t x1 = q % g.L[1];
        const uint32_t x2 = q / g.L[1];
        const uint32_t y0 = (x0 + rr) % g.L[0], y1 = (x1 + rr) % g.L[1], y2 = (x2 + rr) % g.L[2];
        const double n = field[y0 + g.L[0] * (x1 + g.L[1] * x2)] + field[x0 + g.L[0] * (y1 + g.L[1] * x2)] +
                         field[x0 + g.L[0] * (x1 + g.L[1] * y2)];
        acc = field[i] * n;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partial[(size_t)rr * gridDim.x + blockIdx.x] = s;
}

// out[r] = (sum of the nb partials of r, in order) / (3 vs); one workgroup per r
__global__ __launch_bounds__(kBlock) void k_polyakov_corr_reduce(const double *__restrict__ partial,
                                                                 uint32_t nb, uint32_t vs,
                                                                 double *__restrict__ out)
{
    double a = 0.0;
    for (uint32_t j = threadIdx.x; j < nb; j += kBlock) a += partial[(size_t)blockIdx.x * nb + j];
    const double s = block_sum(a);
    if (threadIdx.x == 0) out[blockIdx.x] = s / (3.0 * (double)vs);
}

// The correlator's three launches: the Polyakov field (vs doubles) into
// `field`, the per-workgroup products into `partial` (nb * (rmax + 1)
// doubles, nb = ceil(vs / 256)), their fixed-order sums into out[0..rmax].
// Every element of field and partial is written before it is read.
hipError_t launch_polyakov_correlator(const float4 *links, const Geo &g, uint32_t rmax, double *field,
                                      double *partial, double *out, hipStream_t st)
{
    const uint32_t vs = g.L[0] * g.L[1] * g.L[2];
    const uint32_t nb = (vs + kBlock - 1) / kBlock, nr = rmax + 1;
    hipLaunchKernelGGL(k_polyakov_field, dim3(nb), dim3(kBlock), 0, st, links, g, vs, field);
    hipLaunchKernelGGL(k_polyakov_corr, dim3(nb, nr), dim3(kBlock), 0, st, field, g, vs, partial);
    hipLaunchKernelGGL(k_polyakov_corr_reduce, dim3(nr), dim3(kBlock), 0, st, partial, nb, vs, out);
    return hipGetLastError();
}

// Scratch of su2_polyakov_correlator_noalloc: the field and the partials of
// one correlator, in device memory that exists as long as the process does
// (each GPU the library runs on holds its own copy).  Host code uses it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocDoubles = size_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

}  // namespace su2

namespace {

constexpr int kGraphSweeps = (int)kSweepSlots;  // sweeps per replay of the large graph

struct Context {
    bool ready = false;
    Geo g{};
    Key key{};
    double beta = 0.0;
    uint64_t V = 0;
    float4 *links = nullptr;
    bool owns_links = false;
    uint32_t *d_sweep = nullptr;        // device-resident sweep index: kSweepSlots words, index + j
    uint64_t sweep = 0;                 // host mirror
    unsigned long long *d_counters = nullptr;  // per-wave (attempts, failures)
    uint32_t n_waves = 0;
    double2 *d_partials = nullptr;      // per-workgroup partial sums of a measurement
    double2 *d_meas = nullptr;          // plaquette partials written by a measured sweep
    size_t n_meas = 0;                  // ... room for that many
    double2 *d_scratch = nullptr;       // first-level reduction results
    double *d_out = nullptr;            // 3 doubles for scalar results
    bool meas_fresh = false;            // d_meas holds the plaquette of the current links
    hipStream_t stream = nullptr;
    // graphS[m][k]: k = 1..kGraphSweeps sweeps and one sweep-index tick; with
    // m = 1 the last of them also measures the plaquette (built on first use)
    hipGraphExec_t graphS[2][kGraphSweeps + 1] = {};
    hipGraphExec_t graphOR[kGraphSweeps + 1] = {};  // graphOR[k]: k overrelaxation sweeps
    // graphMH[e]: kGraphSweeps / e measurements e sweeps apart, each reduced
    // into the next entry of d_hist (built on first use)
    hipGraphExec_t graphMH[kGraphSweeps + 1] = {};
    double *d_hist = nullptr;           // plaquette history of su2_sweep_measure (3 doubles each)
    size_t hist_cap = 0;                // ... entries it has room for
    uint32_t *d_cursor = nullptr;       // next history entry graphMH writes
    PassPlan plan;                      // launch plan of k_pass (tile order, LDS reservation)
    uint32_t *d_order = nullptr;        // device tile-order table of the plan
    int32_t order_kind = 0;
    int32_t proposal = 0;               // 0 heat-bath, 1 learned independence-Metropolis
    float creutz_below = 0.0f;          // heat-bath: Creutz's draw for alpha below this
    float *d_table = nullptr;           // this lattice's copy of the knot table
    unsigned long long *d_imh_stats = nullptr;  // per wave: (proposals, accepts)
};

Context ctx;
char last_error[512] = "no error";

// Device address of the scratch array on each device, looked up once per
// device (at the first lattice initialised there) with that device current.
constexpr int kMaxDevices = 64;
double *scratch_dev[kMaxDevices] = {};
int ctx_device = -1;  // device current when the lattice was initialised

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(last_error, sizeof last_error, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(SU2_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

void release_graphs()
{
    for (auto &row : ctx.graphS)
        for (hipGraphExec_t &gr : row) {
            if (gr) hipGraphExecDestroy(gr);
            gr = nullptr;
        }
    for (hipGraphExec_t &gr : ctx.graphOR) {
        if (gr) hipGraphExecDestroy(gr);
        gr = nullptr;
    }
    for (hipGraphExec_t &gr : ctx.graphMH) {
        if (gr) hipGraphExecDestroy(gr);
        gr = nullptr;
    }
}

void release_all()
{
    if (ctx.stream || ctx.links) hipStreamSynchronize(ctx.stream);
    release_graphs();
    if (ctx.owns_links && ctx.links) hipFree(ctx.links);
    if (ctx.d_sweep) hipFree(ctx.d_sweep);
    if (ctx.d_counters) hipFree(ctx.d_counters);
    if (ctx.d_partials) hipFree(ctx.d_partials);
    if (ctx.d_meas) hipFree(ctx.d_meas);
    if (ctx.d_scratch) hipFree(ctx.d_scratch);
    if (ctx.d_order) hipFree(ctx.d_order);
    if (ctx.d_table) hipFree(ctx.d_table);
    if (ctx.d_imh_stats) hipFree(ctx.d_imh_stats);
    if (ctx.d_out) hipFree(ctx.d_out);
    if (ctx.d_hist) hipFree(ctx.d_hist);
    if (ctx.d_cursor) hipFree(ctx.d_cursor);
    hipStream_t keep = ctx.stream;
    ctx = Context{};
    ctx.stream = keep;
}

int check_dims(const int32_t dims[4], uint64_t *V)
{
    if (!dims) return fail(SU2_EINVAL, "dims is NULL");
    uint64_t v = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || (dims[d] & 1))
            return fail(SU2_EINVAL, "dims[%d] = %d: every extent must be even and >= 2", d,
                        dims[d]);
        v *= (uint64_t)dims[d];
        if (v >= (1ull << 32)) return fail(SU2_EINVAL, "lattice volume must be below 2^32");
    }
    *V = v;
    return SU2_OK;
}

Geo make_geo(const int32_t dims[4], uint64_t V)
{
    Geo g{};
    for (int d = 0; d < 4; ++d) g.L[d] = (uint32_t)dims[d];
    g.H0 = g.L[0] / 2;
    g.half = (uint32_t)(V / 2);
    g.st[0] = 1;
    g.st[1] = g.H0;
    g.st[2] = g.H0 * g.L[1];
    g.st[3] = g.H0 * g.L[1] * g.L[2];
    for (int d = 0; d < 4; ++d) g.wrap[d] = (g.L[d] - 1) * g.st[d];
    g.dH0 = make_fastdiv(g.H0);
    g.dL1 = make_fastdiv(g.L[1]);
    g.dL2 = make_fastdiv(g.L[2]);
    g.dL0 = make_fastdiv(g.L[0]);
    return g;
}

// A graph of nsweeps sweeps and one sweep-index tick.  measure_last: the last
// sweep also sums the plaquette (its partials stay in d_meas).  measure_every
// = e > 0: sweeps e, 2e, ... do, and each is followed by the reduction of its
// partials into the next entry of d_hist (at d_cursor).
int build_graph(int nsweeps, bool measure_last, hipGraphExec_t *out, int measure_every = 0)
{
    ReduceLaunch rl;
    if (measure_every > 0 &&
        !measure_reduce_launch(ctx.d_meas, meas_partials(ctx.g, ctx.plan), ctx.g, ctx.d_hist,
                               ctx.d_cursor, rl))
        return fail(SU2_EDEVICE, "a measured sweep's partials need a two-level reduction");
    hipGraph_t graph;
    HIP_TRY(hipGraphCreate(&graph, 0));
    hipGraphNode_t prev = nullptr;
    int rc = SU2_OK;
    auto add = [&](const void *func, dim3 grid, dim3 block, uint32_t lds, void **args) {
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(func);
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.sharedMemBytes = lds;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) {
            rc = fail(SU2_EDEVICE, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
            return false;
        }
        prev = node;
        return true;
    };
    for (int s = 0; s < nsweeps && rc == SU2_OK; ++s) {
        const bool hist = measure_every > 0 && (s + 1) % measure_every == 0;
        const bool measure = hist || (measure_last && s == nsweeps - 1);
        // eight passes (Sec. 2.4: odd sites for every direction, then even
        // sites), or four fused pairs of them
        // sweep s of the graph reads sweep-index word s (= index + s)
        std::vector<PassLaunch> pls = sweep_launches(ctx.links, ctx.g, ctx.key, (float)ctx.beta,
                                                     ctx.d_sweep + s, ctx.d_counters,
                                                     measure ? ctx.d_meas : nullptr, ctx.plan);
        for (PassLaunch &pl : pls) {
            pl.bind();
            if (!add(pl.func, pl.grid, pl.block, pl.lds, pl.args)) break;
        }
        if (hist && rc == SU2_OK) {
            rl.bind();
            add(rl.func, dim3(1), dim3(kBlock), 0, rl.args);
        }
    }
    // one tick after the graph's sweeps advances every sweep-index word by them
    uint32_t *sp = ctx.d_sweep;
    uint32_t nadv = (uint32_t)nsweeps;
    if (rc == SU2_OK) {
        void *targs[2] = { &sp, &nadv };
        add(tick_func(), dim3(1), dim3(kWave), 0, targs);
    }
    if (rc == SU2_OK) {
        hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(SU2_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    hipGraphDestroy(graph);
    return rc;
}

// nsweeps overrelaxation sweeps (the eight passes each in the heat-bath
// sweep's order) as a graph; no sweep-index tick (they draw no random numbers).
int build_or_graph(int nsweeps, hipGraphExec_t *out)
{
    hipGraph_t graph;
    HIP_TRY(hipGraphCreate(&graph, 0));
    hipGraphNode_t prev = nullptr;
    int rc = SU2_OK;
    for (int s = 0; s < nsweeps && rc == SU2_OK; ++s)
        for (int p = 1; p >= 0 && rc == SU2_OK; --p)
            for (uint32_t mu = 0; mu < 4 && rc == SU2_OK; ++mu) {
                PassLaunch pl = or_launch(ctx.links, ctx.g, (uint32_t)p, mu, ctx.plan);
                // as in the heat-bath sweep: odd passes walk the tile order backwards
                if (ctx.plan.alternate && !ctx.plan.fused && (mu & 1u)) {
                    pl.order = ctx.plan.order + pass_blocks(ctx.g);
                    pl.bind();
                }
                hipKernelNodeParams kp{};
                kp.func = const_cast<void *>(pl.func);
                kp.gridDim = pl.grid;
                kp.blockDim = pl.block;
                kp.sharedMemBytes = pl.lds;
                kp.kernelParams = pl.args;
                kp.extra = nullptr;
                hipGraphNode_t node;
                hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                                     &kp);
                if (e != hipSuccess)
                    rc = fail(SU2_EDEVICE, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
                else
                    prev = node;
            }
    if (rc == SU2_OK) {
        hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(SU2_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    hipGraphDestroy(graph);
    return rc;
}

// Install a k_pass launch plan: tile order kind (0 = identity) and LDS bytes
// reserved per workgroup.  Graphs are rebuilt on next use.
int set_plan(int32_t kind, uint32_t lds)
{
    std::vector<uint32_t> order;
    PairGeo pg01, pg23;
    const bool fused = kind == kFusedPairs;
    if (fused ? !make_pair_geo(ctx.g, ctx.n_waves, pg01, pg23) : !make_order(ctx.g, kind, order))
        return fail(SU2_EINVAL, "tile order %d does not fit this lattice", kind);
    if (lds > 65536u) return fail(SU2_EINVAL, "LDS reservation must be <= 65536 bytes");
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    if (ctx.d_order) {
        hipFree(ctx.d_order);
        ctx.d_order = nullptr;
    }
    if (kind > 0 && !fused) {
        if (hipMalloc(&ctx.d_order, order.size() * sizeof(uint32_t)) != hipSuccess) {
            hipGetLastError();
            return fail(SU2_ENOMEM, "cannot allocate the tile order");
        }
        HIP_TRY(hipMemcpy(ctx.d_order, order.data(), order.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    }
    ctx.plan.order = ctx.d_order;
    ctx.plan.alternate = kind >= kAlternate;
    ctx.plan.lds_bytes = lds;
    ctx.plan.fused = fused;
    ctx.plan.pg01 = pg01;
    ctx.plan.pg23 = pg23;
    ctx.order_kind = kind;
    ctx.meas_fresh = false;  // partials of a measured sweep are laid out per plan
    release_graphs();
    return SU2_OK;
}

// Device sweep-index words index + j, j < kSweepSlots (the copy is complete
// when the call returns).
hipError_t write_sweep_index(uint32_t index)
{
    uint32_t w[kSweepSlots];
    for (uint32_t j = 0; j < kSweepSlots; ++j) w[j] = index + j;
    hipError_t e = hipMemcpyAsync(ctx.d_sweep, w, sizeof w, hipMemcpyHostToDevice, ctx.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
    return e;
}

int require_ready()
{
    if (!ctx.ready) return fail(SU2_ESTATE, "no lattice: call su2_init first");
    return SU2_OK;
}

// n sweeps; with measured, the last one also leaves the plaquette partials of
// its result in d_meas (the even passes mu >= 1 accumulate them)
int run_sweeps(int32_t n, bool measured = false)
{
    if (n <= 0) return SU2_OK;
    auto graph = [](int m, int32_t k, hipGraphExec_t **out) {
        hipGraphExec_t &gr = ctx.graphS[m][k];
        int rc = gr ? SU2_OK : build_graph(k, m == 1, &gr);
        *out = &gr;
        return rc;
    };
    // whole graphs of kGraphSweeps plain sweeps, then one graph for the rest
    // (its last sweep measured when asked): one launch and one tick per graph
    int32_t left = n;
    hipGraphExec_t *gr = nullptr;
    while (left > kGraphSweeps || (left == kGraphSweeps && !measured)) {
        int rc = graph(0, kGraphSweeps, &gr);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(*gr, ctx.stream));
        left -= kGraphSweeps;
    }
    if (left > 0) {
        int rc = graph(measured ? 1 : 0, left, &gr);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(*gr, ctx.stream));
    }
    ctx.sweep += (uint64_t)n;
    ctx.meas_fresh = measured;
    return SU2_OK;
}

// (P, P_s, P_t) of the current links into device out[0..2]: from the partials
// of the last measured sweep when they are current, else by k_plaquette
hipError_t enqueue_plaquette(double *out)
{
    if (ctx.meas_fresh)
        return launch_measure_reduce(ctx.d_meas, meas_partials(ctx.g, ctx.plan), ctx.g,
                                     ctx.d_scratch, out, ctx.stream);
    return launch_plaquette(ctx.links, ctx.g, ctx.d_partials, ctx.d_scratch, out, ctx.stream);
}

}  // namespace

extern "C" {

int su2_init_ex(const int32_t dims[4], double beta, uint64_t seed, int32_t start, void *dev_links,
                size_t bytes)
{
    uint64_t V;
    int rc = check_dims(dims, &V);
    if (rc) return rc;
    if (!std::isfinite(beta) || beta < 0.0) return fail(SU2_EINVAL, "beta must be finite and >= 0");
    if (start != SU2_COLD && start != SU2_HOT) return fail(SU2_EINVAL, "start must be 0 or 1");
    const size_t link_bytes = (size_t)V * 4 * sizeof(float4);
    if (dev_links) {
        if (bytes < link_bytes)
            return fail(SU2_EINVAL, "device buffer holds %zu bytes, %zu needed", bytes, link_bytes);
        if ((uintptr_t)dev_links % 16)
            return fail(SU2_EINVAL, "device buffer must be 16-byte aligned");
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SU2_EDEVICE, "device %d: at most %d devices", dev, kMaxDevices);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(su2::scratch));
        if (e != hipSuccess || !p)
            return fail(SU2_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        scratch_dev[dev] = static_cast<double *>(p);
    }
    release_all();
    ctx.g = make_geo(dims, V);
    ctx.V = V;
    ctx.beta = beta;
    ctx.key = Key{ (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    ctx.n_waves = counter_waves(ctx.g);
    const uint32_t nb = std::max(plaquette_blocks(ctx.g), polyakov_blocks(ctx.g));
    // room for the plaquette partials of either sweep form
    size_t n_meas = (size_t)3 * pass_blocks(ctx.g);
    PairGeo pg01, pg23;
    if (make_pair_geo(ctx.g, ctx.n_waves, pg01, pg23))
        n_meas = std::max(n_meas, (size_t)pg01.n_wg + pg23.n_wg);
    ctx.n_meas = n_meas;
    if (dev_links) {
        ctx.links = static_cast<float4 *>(dev_links);
        ctx.owns_links = false;
    } else {
        if (hipMalloc(&ctx.links, link_bytes) != hipSuccess) {
            hipGetLastError();
            ctx.links = nullptr;
            release_all();
            return fail(SU2_ENOMEM, "cannot allocate %zu bytes of links", link_bytes);
        }
        ctx.owns_links = true;
    }
    if (hipMalloc(&ctx.d_sweep, kSweepSlots * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&ctx.d_counters, (size_t)ctx.n_waves * 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx.d_partials, (size_t)nb * sizeof(double2)) != hipSuccess ||
        hipMalloc(&ctx.d_meas, n_meas * sizeof(double2)) != hipSuccess ||
        hipMalloc(&ctx.d_scratch, (size_t)reduce_scratch() * sizeof(double2)) != hipSuccess ||
        hipMalloc(&ctx.d_out, 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx.d_cursor, sizeof(uint32_t)) != hipSuccess) {
        hipGetLastError();
        release_all();
        return fail(SU2_ENOMEM, "cannot allocate work buffers");
    }
    HIP_TRY(write_sweep_index(0));
    HIP_TRY(hipMemsetAsync(ctx.d_counters, 0, (size_t)ctx.n_waves * 2 * sizeof(unsigned long long),
                           ctx.stream));
    HIP_TRY(launch_init(ctx.links, ctx.g, ctx.key, start == SU2_HOT, ctx.stream));
    ctx.sweep = 0;
    ctx.meas_fresh = false;
    ctx.ready = true;
    ctx_device = dev;
    return SU2_OK;
}

int su2_init(const int32_t dims[4], double beta, uint64_t seed, int32_t start)
{
    return su2_init_ex(dims, beta, seed, start, nullptr, 0);
}

int su2_sweep(int32_t n)
{
    int rc = require_ready();
    if (rc) return rc;
    if (n < 0) return fail(SU2_EINVAL, "n must be >= 0");
    if (ctx.sweep + (uint64_t)n > 0xffffffffull)
        return fail(SU2_EINVAL, "sweep index would pass 2^32 - 1");
    return run_sweeps(n);
}

int su2_sweep_measured(int32_t n)
{
    int rc = require_ready();
    if (rc) return rc;
    if (n < 1) return fail(SU2_EINVAL, "n must be >= 1");
    if (ctx.sweep + (uint64_t)n > 0xffffffffull)
        return fail(SU2_EINVAL, "sweep index would pass 2^32 - 1");
    return run_sweeps(n, true);
}

int su2_pass(int32_t parity, int32_t mu)
{
    int rc = require_ready();
    if (rc) return rc;
    if (parity < 0 || parity > 1 || mu < 0 || mu > 3)
        return fail(SU2_EINVAL, "parity must be 0/1 and mu 0..3");
    PassLaunch pl = pass_launch(ctx.links, ctx.g, ctx.key, (float)ctx.beta, (uint32_t)parity,
                                (uint32_t)mu, ctx.d_sweep, ctx.d_counters, nullptr, ctx.plan);
    HIP_TRY(launch(pl, ctx.stream));
    ctx.meas_fresh = false;
    return SU2_OK;
}

int su2_overrelax(int32_t n)
{
    int rc = require_ready();
    if (rc) return rc;
    if (n < 0) return fail(SU2_EINVAL, "n must be >= 0");
    if (n == 0) return SU2_OK;
    // graphs of kGraphSweeps sweeps, then one graph for the rest
    for (int32_t left = n; left > 0;) {
        const int32_t k = std::min<int32_t>(left, kGraphSweeps);
        if (!ctx.graphOR[k]) {
            rc = build_or_graph(k, &ctx.graphOR[k]);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(ctx.graphOR[k], ctx.stream));
        left -= k;
    }
    ctx.meas_fresh = false;
    return SU2_OK;
}

int su2_overrelax_pass(int32_t parity, int32_t mu)
{
    int rc = require_ready();
    if (rc) return rc;
    if (parity < 0 || parity > 1 || mu < 0 || mu > 3)
        return fail(SU2_EINVAL, "parity must be 0/1 and mu 0..3");
    PassLaunch pl = or_launch(ctx.links, ctx.g, (uint32_t)parity, (uint32_t)mu, ctx.plan);
    HIP_TRY(launch(pl, ctx.stream));
    ctx.meas_fresh = false;
    return SU2_OK;
}

int su2_plaquette_st(double out[3])
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    HIP_TRY(enqueue_plaquette(ctx.d_out));
    HIP_TRY(hipMemcpyAsync(out, ctx.d_out, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    return SU2_OK;
}

double su2_plaquette(void)
{
    double o[3];
    if (su2_plaquette_st(o) != SU2_OK) return NAN;
    return o[0];
}

int su2_polyakov(double *out)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    double o[3];
    HIP_TRY(launch_polyakov(ctx.links, ctx.g, ctx.d_partials, ctx.d_scratch, ctx.d_out, ctx.stream));
    HIP_TRY(hipMemcpyAsync(o, ctx.d_out, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    *out = o[0];
    return SU2_OK;
}

int su2_polyakov_correlator(int32_t rmax, double *out)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    const uint32_t lmin = std::min({ ctx.g.L[0], ctx.g.L[1], ctx.g.L[2] });
    if (rmax < 0 || (uint32_t)rmax > lmin / 2)
        return fail(SU2_EINVAL, "rmax must be in 0 .. min(L0, L1, L2) / 2 = %u", lmin / 2);
    const uint32_t vs = ctx.g.L[0] * ctx.g.L[1] * ctx.g.L[2];
    const uint32_t nb = (vs + kBlock - 1) / kBlock, nr = (uint32_t)rmax + 1;
    double *d_field = nullptr, *d_part = nullptr, *d_res = nullptr;
    if (hipMalloc(&d_field, (size_t)vs * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_part, (size_t)nb * nr * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_res, nr * sizeof(double)) != hipSuccess) {
        hipGetLastError();
        if (d_field) hipFree(d_field);
        if (d_part) hipFree(d_part);
        return fail(SU2_ENOMEM, "cannot allocate the Polyakov correlator buffers");
    }
    hipError_t e = launch_polyakov_correlator(ctx.links, ctx.g, (uint32_t)rmax, d_field, d_part, d_res, ctx.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_res, nr * sizeof(double), hipMemcpyDeviceToHost, ctx.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
    hipFree(d_field);
    hipFree(d_part);
    hipFree(d_res);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_polyakov_correlator: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_polyakov_correlator_noalloc(int32_t rmax, double *dev_out)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!dev_out || (uintptr_t)dev_out % 8) return fail(SU2_EINVAL, "dev_out must be 8-byte aligned device memory");
    const uint32_t lmin = std::min({ ctx.g.L[0], ctx.g.L[1], ctx.g.L[2] });
    if (rmax < 0 || (uint32_t)rmax > lmin / 2)
        return fail(SU2_EINVAL, "rmax must be in 0 .. min(L0, L1, L2) / 2 = %u", lmin / 2);
    const size_t vs = (size_t)ctx.g.L[0] * ctx.g.L[1] * ctx.g.L[2];
    const size_t nb = (vs + kBlock - 1) / kBlock, nr = (size_t)rmax + 1;
    const size_t need = vs + nb * nr;
    if (need > kNoAllocDoubles)
        return fail(SU2_EINVAL, "the correlator needs %zu doubles of scratch (L0 L1 L2 + ceil(L0 L1 L2 / 256) "
                    "(rmax + 1)); the no-allocation scratch holds %zu", need, kNoAllocDoubles);
    double *sp = ctx_device >= 0 ? scratch_dev[ctx_device] : nullptr;
    if (!sp) return fail(SU2_ESTATE, "no scratch address for this device");
    hipError_t e = launch_polyakov_correlator(ctx.links, ctx.g, (uint32_t)rmax, sp, sp + vs, dev_out, ctx.stream);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_polyakov_correlator_noalloc: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_measure_device(double *dev_out)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!dev_out || (uintptr_t)dev_out % 8) return fail(SU2_EINVAL, "dev_out must be 8-byte aligned device memory");
    HIP_TRY(enqueue_plaquette(dev_out));
    HIP_TRY(launch_polyakov(ctx.links, ctx.g, ctx.d_partials, ctx.d_scratch, dev_out + 3, ctx.stream));
    return SU2_OK;
}

int su2_sweep_measure(int32_t n, int32_t every, double *host_hist)
{
    int rc = require_ready();
    if (rc) return rc;
    if (every < 1 || n < 0 || n % every) return fail(SU2_EINVAL, "need every >= 1 and n % every == 0");
    if (!host_hist && n > 0) return fail(SU2_EINVAL, "host_hist is NULL");
    if (ctx.sweep + (uint64_t)n > 0xffffffffull)
        return fail(SU2_EINVAL, "sweep index would pass 2^32 - 1");
    const int32_t m = n / every;
    if (m == 0) return SU2_OK;
    // the history stays on the device until the end, in a buffer the context
    // keeps (the graph below writes it in place, so it bakes in its address)
    if (ctx.hist_cap < (size_t)m) {
        HIP_TRY(hipStreamSynchronize(ctx.stream));
        for (hipGraphExec_t &gr : ctx.graphMH) {
            if (gr) hipGraphExecDestroy(gr);
            gr = nullptr;
        }
        if (ctx.d_hist) hipFree(ctx.d_hist);
        ctx.d_hist = nullptr;
        ctx.hist_cap = 0;
        const size_t cap = std::max<size_t>((size_t)m, 1024);
        if (hipMalloc(&ctx.d_hist, cap * 3 * sizeof(double)) != hipSuccess) {
            hipGetLastError();
            ctx.d_hist = nullptr;
            return fail(SU2_ENOMEM, "cannot allocate the measurement history");
        }
        ctx.hist_cap = cap;
    }
    int32_t i = 0;
    // measurements at most kGraphSweeps sweeps apart: graphs of k = 16 / every
    // of them (k * every sweeps), each measured sweep followed by the
    // one-workgroup reduction of its partials into the next history entry (the
    // same kernel and order as enqueue_plaquette)
    const int32_t k = every <= kGraphSweeps ? kGraphSweeps / every : 0;
    if (k > 0 && m >= k && meas_partials(ctx.g, ctx.plan) <= kReduceOneLevel) {
        hipGraphExec_t &gr = ctx.graphMH[every];
        if (!gr) {
            rc = build_graph(k * every, false, &gr, every);
            if (rc) return rc;
        }
        HIP_TRY(hipMemsetAsync(ctx.d_cursor, 0, sizeof(uint32_t), ctx.stream));
        for (; i + k <= m; i += k) HIP_TRY(hipGraphLaunch(gr, ctx.stream));
        ctx.sweep += (uint64_t)i * (uint64_t)every;
        ctx.meas_fresh = true;
    }
    for (; i < m && rc == SU2_OK; ++i) {
        rc = run_sweeps(every, true);
        if (rc == SU2_OK) {
            hipError_t e = enqueue_plaquette(ctx.d_hist + 3 * (size_t)i);
            if (e != hipSuccess) rc = fail(SU2_EDEVICE, "plaquette launch: %s", hipGetErrorString(e));
        }
    }
    if (rc == SU2_OK) {
        hipError_t e = hipMemcpyAsync(host_hist, ctx.d_hist, (size_t)m * 3 * sizeof(double),
                                      hipMemcpyDeviceToHost, ctx.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
        if (e != hipSuccess) rc = fail(SU2_EDEVICE, "history copy: %s", hipGetErrorString(e));
    }
    hipStreamSynchronize(ctx.stream);
    return rc;
}

int su2_links(float *host_out, size_t n_floats)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!host_out) return fail(SU2_EINVAL, "host_out is NULL");
    if (n_floats != (size_t)ctx.V * 16)
        return fail(SU2_EINVAL, "n_floats = %zu, expected 16*V = %zu", n_floats, (size_t)ctx.V * 16);
    float4 *stage = nullptr;
    if (hipMalloc(&stage, n_floats * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        return fail(SU2_ENOMEM, "cannot allocate the staging buffer");
    }
    hipError_t e = launch_pack(ctx.links, ctx.g, stage, ctx.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_out, stage, n_floats * sizeof(float), hipMemcpyDeviceToHost, ctx.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
    hipStreamSynchronize(ctx.stream);
    hipFree(stage);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_links: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_set_links(const float *host_in, size_t n_floats, uint64_t sweep_index)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!host_in) return fail(SU2_EINVAL, "host_in is NULL");
    if (n_floats != (size_t)ctx.V * 16)
        return fail(SU2_EINVAL, "n_floats = %zu, expected 16*V = %zu", n_floats, (size_t)ctx.V * 16);
    if (sweep_index > 0xffffffffull) return fail(SU2_EINVAL, "sweep index must be below 2^32");
    float4 *stage = nullptr;
    if (hipMalloc(&stage, n_floats * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        return fail(SU2_ENOMEM, "cannot allocate the staging buffer");
    }
    const uint32_t s32 = (uint32_t)sweep_index;
    hipError_t e = hipMemcpyAsync(stage, host_in, n_floats * sizeof(float), hipMemcpyHostToDevice,
                                  ctx.stream);
    if (e == hipSuccess) e = launch_unpack(ctx.links, ctx.g, stage, ctx.stream);
    ctx.meas_fresh = false;
    if (e == hipSuccess) e = write_sweep_index(s32);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
    hipStreamSynchronize(ctx.stream);
    hipFree(stage);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_set_links: %s", hipGetErrorString(e));
    ctx.sweep = sweep_index;
    return SU2_OK;
}

int su2_sweep_index(uint64_t *out)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = ctx.sweep;
    return SU2_OK;
}

// Sum of the per-wave counter pairs in dev (n_waves pairs) into out[0..1].
static int sum_wave_counters(const unsigned long long *dev, uint64_t out[2])
{
    out[0] = out[1] = 0;
    if (!dev) return SU2_OK;
    std::vector<unsigned long long> h((size_t)ctx.n_waves * 2);
    HIP_TRY(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           ctx.stream));
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    for (uint32_t w = 0; w < ctx.n_waves; ++w) {
        out[0] += h[2 * w];
        out[1] += h[2 * w + 1];
    }
    return SU2_OK;
}

int su2_counters(uint64_t out[4])
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    rc = sum_wave_counters(ctx.d_counters, out);
    if (rc) return rc;
    return sum_wave_counters(ctx.d_imh_stats, out + 2);
}

int su2_bind(void *dev_links, size_t bytes)
{
    int rc = require_ready();
    if (rc) return rc;
    const size_t link_bytes = (size_t)ctx.V * 4 * sizeof(float4);
    if (!dev_links) return fail(SU2_EINVAL, "dev_links is NULL");
    if (bytes < link_bytes)
        return fail(SU2_EINVAL, "device buffer holds %zu bytes, %zu needed", bytes, link_bytes);
    if ((uintptr_t)dev_links % 16) return fail(SU2_EINVAL, "device buffer must be 16-byte aligned");
    if (dev_links == (void *)ctx.links) return SU2_OK;
    const uintptr_t a = (uintptr_t)dev_links, b = (uintptr_t)ctx.links;
    if (a < b + link_bytes && b < a + link_bytes)
        return fail(SU2_EINVAL, "device buffer overlaps the current links");
    HIP_TRY(hipMemcpyAsync(dev_links, ctx.links, link_bytes, hipMemcpyDeviceToDevice, ctx.stream));
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    if (ctx.owns_links) hipFree(ctx.links);
    ctx.links = static_cast<float4 *>(dev_links);
    ctx.owns_links = false;
    release_graphs();  // the captured launches point at the old buffer
    return SU2_OK;
}

int su2_set_stream(void *hip_stream)
{
    if (ctx.ready || ctx.stream) HIP_TRY(hipStreamSynchronize(ctx.stream));
    ctx.stream = static_cast<hipStream_t>(hip_stream);
    return SU2_OK;
}

int su2_philox(uint64_t seed, const uint32_t *ctr, size_t n, uint32_t *out)
{
    if (n == 0) return SU2_OK;
    if (!ctr || !out) return fail(SU2_EINVAL, "NULL buffer");
    if (n > (1u << 28)) return fail(SU2_EINVAL, "at most 2^28 blocks per call");
    uint4 *d = nullptr;
    if (hipMalloc(&d, 2 * n * sizeof(uint4)) != hipSuccess) {
        hipGetLastError();
        return fail(SU2_ENOMEM, "cannot allocate %zu blocks", n);
    }
    const Key key{ (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    hipError_t e = hipMemcpyAsync(d, ctr, n * sizeof(uint4), hipMemcpyHostToDevice, ctx.stream);
    if (e == hipSuccess) e = launch_philox(d, (uint32_t)n, key, d + n, ctx.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d + n, n * sizeof(uint4), hipMemcpyDeviceToHost, ctx.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
    hipStreamSynchronize(ctx.stream);
    hipFree(d);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_philox: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_set_plan(int32_t order_kind, int32_t lds_bytes)
{
    int rc = require_ready();
    if (rc) return rc;
    if (order_kind < 0 || lds_bytes < 0) return fail(SU2_EINVAL, "negative plan parameter");
    return set_plan(order_kind, (uint32_t)lds_bytes);
}

int su2_tune(int32_t reps, int32_t out[2])
{
    int rc = require_ready();
    if (rc) return rc;
    if (reps < 1) return fail(SU2_EINVAL, "reps must be >= 1");
    const size_t link_bytes = (size_t)ctx.V * 4 * sizeof(float4);
    const size_t ctr_bytes = (size_t)ctx.n_waves * 2 * sizeof(unsigned long long);
    const size_t part_bytes = ctx.n_meas * sizeof(double2);
    float4 *tl = nullptr;
    unsigned long long *tc = nullptr;
    double2 *tp = nullptr;
    if (hipMalloc(&tl, link_bytes) != hipSuccess || hipMalloc(&tc, ctr_bytes) != hipSuccess ||
        hipMalloc(&tp, part_bytes) != hipSuccess) {
        hipGetLastError();
        if (tl) hipFree(tl);
        if (tc) hipFree(tc);
        return fail(SU2_ENOMEM, "cannot allocate the tuning copy of the links");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(tl, ctx.links, link_bytes, hipMemcpyDeviceToDevice, ctx.stream);
    if (e == hipSuccess) e = hipMemsetAsync(tc, 0, ctr_bytes, ctx.stream);
    // candidates: tile order x LDS reservation.  Each is timed on `reps` full
    // measured sweeps (as su2_sweep_measured runs them) of a copy of the links,
    // in three rounds over all candidates; the median of its rounds ranks it,
    // so slow drifts of the clock or of the cache state do not pick the plan.
    const int32_t kinds[] = { 0, 4, 8, 16, 108, 208, kAlternate, kAlternate + 8, kAlternate + 104,
                              kAlternate + 108, kAlternate + 116, kAlternate + 204, kAlternate + 208,
                              kFusedPairs };
    const uint32_t ldss[] = { 0u, 16384u, 24576u, 32768u, 40960u };
    constexpr int kRounds = 3;
    std::vector<int32_t> cand_kind;
    std::vector<uint32_t> cand_lds;
    for (int32_t kind : kinds) {
        std::vector<uint32_t> order;
        PairGeo pg01, pg23;
        if (kind == kFusedPairs ? !make_pair_geo(ctx.g, ctx.n_waves, pg01, pg23)
                                : !make_order(ctx.g, kind, order))
            continue;
        for (uint32_t lds : ldss) {
            cand_kind.push_back(kind);
            cand_lds.push_back(lds);
        }
    }
    std::vector<float> ms_all(cand_kind.size() * kRounds, 1e30f);
    // the learned proposal's counters go to the scratch counters meanwhile
    unsigned long long *imh_stats = ctx.plan.imh.stats;
    if (ctx.plan.learned) ctx.plan.imh.stats = tc;
    for (int round = 0; round < kRounds && e == hipSuccess && !rc; ++round) {
        for (size_t c = 0; c < cand_kind.size() && e == hipSuccess; ++c) {
            if (c == 0 || cand_kind[c] != cand_kind[c - 1]) {
                rc = set_plan(cand_kind[c], 0);
                if (rc) break;
            }
            ctx.plan.lds_bytes = cand_lds[c];
            for (int warm = 0; warm < 2 && e == hipSuccess; ++warm) {
                if (warm == 1) e = hipEventRecord(e0, ctx.stream);
                for (int32_t r = 0; r < (warm ? reps : 1) && e == hipSuccess; ++r) {
                    std::vector<PassLaunch> pls = sweep_launches(tl, ctx.g, ctx.key, (float)ctx.beta,
                                                                 ctx.d_sweep, tc, tp, ctx.plan);
                    for (size_t i = 0; i < pls.size() && e == hipSuccess; ++i) e = launch(pls[i], ctx.stream);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, ctx.stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) ms_all[c * kRounds + round] = ms;
        }
    }
    hipStreamSynchronize(ctx.stream);
    ctx.plan.imh.stats = imh_stats;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(tl);
    hipFree(tc);
    hipFree(tp);
    if (e != hipSuccess) return fail(SU2_EDEVICE, "su2_tune: %s", hipGetErrorString(e));
    if (rc) return rc;
    float best = 1e30f;
    int32_t best_kind = 0;
    uint32_t best_lds = 0;
    for (size_t c = 0; c < cand_kind.size(); ++c) {
        float *m = &ms_all[c * kRounds];
        std::sort(m, m + kRounds);
        if (m[kRounds / 2] < best) {
            best = m[kRounds / 2];
            best_kind = cand_kind[c];
            best_lds = cand_lds[c];
        }
    }
    rc = set_plan(best_kind, best_lds);
    if (rc) return rc;
    if (out) {
        out[0] = best_kind;
        out[1] = (int32_t)best_lds;
    }
    return SU2_OK;
}

int su2_set_proposal(int32_t kind, const uint16_t *bf16_weights, size_t n_weights)
{
    int rc = require_ready();
    if (rc) return rc;
    if (kind != 0 && kind != 1) return fail(SU2_EINVAL, "proposal kind must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    if (kind == 1 && bf16_weights) {
        // the network takes these weights (its FP32 master becomes their exact
        // values) and is tabulated at the current table size
        if (n_weights != (size_t)kLearnedParams)
            return fail(SU2_EINVAL, "expected %d BF16 weights, got %zu", kLearnedParams, n_weights);
        std::vector<float> w(n_weights);
        for (size_t i = 0; i < n_weights; ++i) {
            const uint32_t bits = (uint32_t)bf16_weights[i] << 16;
            std::memcpy(&w[i], &bits, sizeof bits);
        }
        const float *knots0 = nullptr;
        uint32_t G = 0;
        float amax0 = 0.f;
        const int32_t points = su2_learned_table(&knots0, &G, &amax0) ? (int32_t)G : (int32_t)kImhLdsRows;
        if (su2_mlp_set_params(w.data(), n_weights) != SU2_OK || su2_mlp_tabulate(points) != SU2_OK)
            return fail(SU2_EDEVICE, "loading the proposal weights: %s", su2_mlp_last_error());
    }
    if (kind == 0) {
        // the proposal counters count since the last su2_set_proposal(1, ...)
        if (ctx.d_imh_stats)
            HIP_TRY(hipMemset(ctx.d_imh_stats, 0, (size_t)ctx.n_waves * 2 * sizeof(unsigned long long)));
        ctx.proposal = 0;
        ctx.plan.learned = false;
        ctx.plan.imh = ImhTable{};
        ctx.plan.imh.creutz_below = ctx.creutz_below;
        ctx.plan.imh_lds_bytes = 0;
        release_graphs();
        return SU2_OK;
    }
    const float *knots = nullptr;
    uint32_t G = 0;
    float amax = 0.f;
    if (!su2_learned_table(&knots, &G, &amax))
        return fail(SU2_ESTATE, "no knot table: train or load the network and call su2_mlp_tabulate");
    if (ctx.d_table) hipFree(ctx.d_table);
    ctx.d_table = nullptr;
    const size_t stats_bytes = (size_t)ctx.n_waves * 2 * sizeof(unsigned long long);
    if (!ctx.d_imh_stats && hipMalloc(&ctx.d_imh_stats, stats_bytes) != hipSuccess) {
        hipGetLastError();
        ctx.d_imh_stats = nullptr;
        return fail(SU2_ENOMEM, "cannot allocate proposal counters");
    }
    // padded so that the pass kernels' fixed-size LDS copy stays inside it
    const uint32_t n_vec4 = std::max((G * 33u + 3u) / 4u, kImhLdsVec4);
    if (hipMalloc(&ctx.d_table, (size_t)n_vec4 * 4 * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        ctx.d_table = nullptr;
        return fail(SU2_ENOMEM, "cannot allocate the knot table");
    }
    HIP_TRY(hipMemset(ctx.d_table, 0, (size_t)n_vec4 * 4 * sizeof(float)));
    HIP_TRY(hipMemcpy(ctx.d_table, knots, (size_t)G * 33 * sizeof(float), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemset(ctx.d_imh_stats, 0, stats_bytes));
    ImhTable t;
    t.knots = ctx.d_table;
    t.G = G;
    t.alpha_max = amax;
    t.inv_step = (float)((double)(G - 1) / (double)amax);
    t.stats = ctx.d_imh_stats;
    ctx.proposal = 1;
    ctx.plan.learned = true;
    ctx.plan.imh = t;  // the Creutz switch is off under the learned proposal
    ctx.plan.imh_lds_bytes = kImhLdsBytes;
    release_graphs();
    return SU2_OK;
}

int su2_set_wide_offsets(int32_t on)
{
    int rc = require_ready();
    if (rc) return rc;
    if (on != 0 && on != 1) return fail(SU2_EINVAL, "on must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    ctx.plan.wide = on == 1;
    release_graphs();
    return SU2_OK;
}

int su2_set_creutz(double alpha_below)
{
    int rc = require_ready();
    if (rc) return rc;
    if (!(alpha_below >= 0.0 && alpha_below <= 4.0))
        return fail(SU2_EINVAL, "the Creutz switch must lie in [0, 4]");
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    ctx.creutz_below = (float)alpha_below;
    if (!ctx.plan.learned) ctx.plan.imh.creutz_below = ctx.creutz_below;
    release_graphs();
    return SU2_OK;
}

int su2_imh_counters(uint64_t out[2])
{
    int rc = require_ready();
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    return sum_wave_counters(ctx.d_imh_stats, out);
}

int su2_synchronize(void)
{
    HIP_TRY(hipStreamSynchronize(ctx.stream));
    return SU2_OK;
}

const char *su2_last_error(void) { return last_error; }

void su2_finalize(void) { release_all(); }

}  // extern "C"
