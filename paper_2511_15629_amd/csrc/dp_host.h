// Host-side helpers shared by the single-solve and batched translation units.
#pragma once
#include "dp_internal.h"
#include "dpgpu.h"

namespace dpgpu {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate_problem(const dp_problem *pb);
dpk::SweepShape pick_shape(const dp_problem *pb);

// The balanced sweep's plan for a problem (cached per shape of the problem).
struct FlatPlan {
    bool ok = false;
    dpk::FlatShape sh = {0, 0, 0};
    dpk::FlatArgs f = {};
    size_t lds = 0;
    double cost = 1e300;
};
FlatPlan plan_flat(const dp_problem *pb);
// The single solve's sweep: the balanced kernel when its plan fits (and no per-row-tile
// shape is forced), else the per-row-tile kernel.
struct SweepChoice {
    bool ok = false, flat = false;
    dpk::SweepShape sh = {0, 0, 0, 0};
    FlatPlan fp;
};
SweepChoice choose_sweep(const dp_problem *pb);

struct SolveLayout {
    int Spad;                 // row stride of the value planes and the W plane
    int npk;                  // stages of P_t held repacked for the expectation
    size_t vA, vB, W, off, flag, Pp, rho, total;
};
SolveLayout solve_layout(const dp_problem *pb);
// The same layout with the ring of repacked P_t shrunk until the total fits cap bytes (if it
// can); results do not depend on the ring's size.
SolveLayout solve_layout(const dp_problem *pb, size_t cap);

struct StageOutputs {
    float *vall;         // [(t_hi - t_lo + 2)][K][S] absolute values, slice t - t_lo (nullable)
    float *v1;           // [K][S] absolute values of stage t_lo (nullable)
    int16_t *pol;        // [(t_hi - t_lo + 1)][K][S] (nullable)
    float *ckpt_v;       // checkpoint slots (nullable)
    double *ckpt_off;
    int ckpt_every;
};

// ws holds solve_layout(pb, ws_cap); timing = false keeps the measurement hook's events out.
int run_stages(const dp_problem *pb, int t_lo, int t_hi, const float *lam, const float *P,
               const float *v_src, const double *off_src, const StageOutputs &out, void *ws,
               hipStream_t stream, size_t ws_cap = SIZE_MAX, bool timing = true);

}  // namespace dpgpu
