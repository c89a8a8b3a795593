// su2_kernels.hpp -- host-side launchers of the lattice kernels.
#pragma once

#include <vector>

#include "su2_pair.hpp"
#include "su2_pass.hpp"

namespace su2 {

// How k_pass is launched: tile order table (device, nullptr = identity) and
// LDS bytes reserved per workgroup (caps resident workgroups per CU; 0 = none).
// Neither changes any result: every update is a pure function of the links it
// reads and of its Philox counter.
struct PassPlan {
    const uint32_t *order = nullptr;
    uint32_t lds_bytes = 0;
    bool alternate = false;         // odd passes use the table's second half (the order backwards)
    bool fused = false;             // a sweep as four k_pair launches (U_0,U_1 and U_2,U_3 per parity)
    PairGeo pg01, pg23;             // their workgroup sets (valid when fused)
    bool learned = false;           // learned proposal (imh) or heat-bath only
    ImhTable imh;                   // the learned proposal's table, passed by value
    uint32_t imh_lds_bytes = 0;     // LDS the learned-proposal pass stages its table in
    bool wide = false;              // 64-bit element offsets even where 32-bit ones suffice
};

// Arguments of one k_pass or k_pair launch, kept together so a graph node can
// point at them.
struct PassLaunch {
    const void *func;
    dim3 grid, block;
    float4 *links;
    Geo g;
    Key key;
    float beta;
    uint32_t p;
    const uint32_t *sweep_ptr;
    unsigned long long *counters;
    double2 *meas_out;
    const uint32_t *order;
    ImhTable imh;
    uint32_t lds;
    bool pair = false;
    bool or_pass = false;  // k_or: (links, g, p, order)
    PairGeo pg;
    void *args[10];
    // point args at this object's own fields (call after every copy)
    void bind()
    {
        if (or_pass) {
            args[0] = &links;
            args[1] = &g;
            args[2] = &p;
            args[3] = &order;
            return;
        }
        if (pair) {
            void *a[10] = { &links, &g, &pg, &key, &beta, &p, &sweep_ptr, &counters, &meas_out, &imh };
            for (int i = 0; i < 10; ++i) args[i] = a[i];
            return;
        }
        args[0] = &links;
        args[1] = &g;
        args[2] = &key;
        args[3] = &beta;
        args[4] = &p;
        args[5] = &sweep_ptr;
        args[6] = &counters;
        args[7] = &meas_out;
        args[8] = &order;
        args[9] = &imh;
    }
};

bool use_off32(const Geo &g);
uint32_t pass_blocks(const Geo &g);
// meas_out != nullptr: the even passes mu >= 1 add their plaquette partials
// (one double2 per workgroup) to meas_out + (mu - 1) * pass_blocks(g)
PassLaunch pass_launch(float4 *links, const Geo &g, Key key, float beta, uint32_t p, uint32_t mu,
                       const uint32_t *sweep_ptr, unsigned long long *counters,
                       double2 *meas_out, const PassPlan &plan);
bool make_order(const Geo &g, int kind, std::vector<uint32_t> &order);
// Tile order kind of the fused-pair sweep (k_pair with XCD-chunked workgroups).
constexpr int kFusedPairs = 300;
// kAlternate + K: order K for the even passes of a sweep, the same backwards for
// the odd ones (the table holds both)
constexpr int kAlternate = 1000;
// The workgroup sets of the two k_pair launches of a parity; false if the
// lattice does not fit them (L0 > 256).
bool make_pair_geo(const Geo &g, uint32_t counter_slots, PairGeo &pg01, PairGeo &pg23);
// The launches of one sweep in order (odd parity, then even): eight k_pass,
// or four k_pair when plan.fused.  meas_out != nullptr: the even-parity
// launches leave their plaquette partials in meas_out (meas_partials of them).
std::vector<PassLaunch> sweep_launches(float4 *links, const Geo &g, Key key, float beta,
                                       const uint32_t *sweep_ptr, unsigned long long *counters,
                                       double2 *meas_out, const PassPlan &plan);
uint32_t meas_partials(const Geo &g, const PassPlan &plan);
// One overrelaxation pass (parity p, direction mu) with the plan's tile order
// and LDS reservation (the identity order under the fused-pair plan).
PassLaunch or_launch(float4 *links, const Geo &g, uint32_t p, uint32_t mu, const PassPlan &plan);
hipError_t launch(PassLaunch &pl, hipStream_t st);
hipError_t launch_init(float4 *links, const Geo &g, Key key, int hot, hipStream_t st);
// The device sweep index: kSweepSlots words, word j = index + j (see k_tick).
constexpr uint32_t kSweepSlots = 16;
hipError_t launch_tick(uint32_t *sweep_ptr, uint32_t n, hipStream_t st);
const void *tick_func();

uint32_t plaquette_blocks(const Geo &g);
uint32_t polyakov_blocks(const Geo &g);
uint32_t counter_waves(const Geo &g);
uint32_t reduce_scratch();
hipError_t launch_plaquette(const float4 *links, const Geo &g, double2 *partials,
                            double2 *scratch, double *out, hipStream_t st);
hipError_t launch_measure_reduce(const double2 *meas_partials, uint32_t n, const Geo &g,
                                 double2 *scratch, double *out, hipStream_t st);
// Partials that one workgroup reduces directly (one kernel instead of two).
constexpr uint32_t kReduceOneLevel = 4096;
// The reduction of a measured sweep's partials as a graph kernel node: the
// plaquette triple goes to hist + 3 * (*cursor), and the cursor advances by
// one.  The same kernel and order as launch_measure_reduce, so the values are
// bit-identical.  false when n > kReduceOneLevel (two levels needed).
struct ReduceLaunch {
    const void *func = nullptr;
    const double2 *partials = nullptr;
    uint32_t n = 0;
    double sa = 0.0, sb = 0.0;
    int mode = 0;
    double *out = nullptr;
    uint32_t *cursor = nullptr;
    void *args[7];
    void bind()
    {
        void *a[7] = { &partials, &n, &sa, &sb, &mode, &out, &cursor };
        for (int i = 0; i < 7; ++i) args[i] = a[i];
    }
};
bool measure_reduce_launch(const double2 *meas_partials, uint32_t n, const Geo &g, double *hist,
                           uint32_t *cursor, ReduceLaunch &rl);
hipError_t launch_polyakov(const float4 *links, const Geo &g, double2 *partials,
                           double2 *scratch, double *out, hipStream_t st);
hipError_t launch_pack(const float4 *links, const Geo &g, float4 *stage, hipStream_t st);
hipError_t launch_unpack(float4 *links, const Geo &g, const float4 *stage, hipStream_t st);
hipError_t launch_philox(const uint4 *ctr, uint32_t n, Key key, uint4 *out, hipStream_t st);

}  // namespace su2
