// Host-side helpers shared by the single-solve and batched translation units.
#pragma once
#include "dp_internal.h"
#include "dpgpu.h"

namespace dpgpu {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate_problem(const dp_problem *pb);
dpk::SweepShape pick_shape(const dp_problem *pb);

struct SolveLayout {
    int Spad;                 // row stride of the value planes
    int npk;                  // stages whose row sums of P_t are held
    size_t vA, vB, off, flag, rho, total;
};
SolveLayout solve_layout(const dp_problem *pb);
// The same layout with the ring of row sums shrunk until the total fits cap bytes (if it
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
