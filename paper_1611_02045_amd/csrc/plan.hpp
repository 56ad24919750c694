// Host-side plan object behind the opaque gpe_plan_t of the C ABI.
#pragma once

#include "internal.hpp"

struct gpe_plan {
    gpe_problem_t prob;
    int dtype = GPE_F64;
    int device = 0;
    gpe::Geo g;
    gpe::Twiddles tw;
    gpe::Reduce red;
    gpe::DevBuf tmp;               // scratch field(s) for multi-pass operators
    gpe::DevBuf solver;            // solver fields of the plan's precision (FP64 phase when mixed)
    gpe::DevBuf solver32;          // FP32 solver fields of a mixed-precision solve
    gpe::DevBuf scal;              // per-instance solver scalars
    gpe::DevBuf hist;              // per-iteration history rows
    int64_t hist_rows = 0;
    bool f64() const { return dtype == GPE_F64; }
    void release() {
        for (int a = 0; a < 3; ++a) {
            tw.t64[a].release();
            tw.t32[a].release();
        }
        red.parts.release();
        red.counters.release();
        red.scalars.release();
        tmp.release();
        solver.release();
        solver32.release();
        scal.release();
        hist.release();
    }
};
