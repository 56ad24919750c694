// Internal host interfaces of libgpe (not part of the C ABI).
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "../../include/gpe.h"
#include "common.hpp"

namespace gpe {

// Serialises a graph capture with the calls that synchronise the device or use the legacy default
// stream (allocation, frees, table uploads, counter resets): HIP refuses them while another host
// thread captures.  Held for the whole capture, and around each such call.
std::mutex& capture_mutex();

// Device buffer owned by a plan; grows on demand (never during graph capture).
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need) {
        if (need <= bytes) return hipSuccess;
        std::lock_guard<std::mutex> lock(capture_mutex());
        if (ptr) {
            hipError_t e = hipFree(ptr);
            if (e != hipSuccess) return e;
            ptr = nullptr;
            bytes = 0;
        }
        hipError_t e = hipMalloc(&ptr, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release() {
        if (ptr) {
            std::lock_guard<std::mutex> lock(capture_mutex());
            (void)hipFree(ptr);
        }
        ptr = nullptr;
        bytes = 0;
    }
};

// Twiddle tables exp(-2 pi i e / M), e < M, for each axis, in both precisions.
struct Twiddles {
    DevBuf t64[3], t32[3];
    const void* get(int axis, bool f64) const { return f64 ? t64[axis].ptr : t32[axis].ptr; }
};

hipError_t build_twiddles(const Geo& g, Twiddles& tw);
Geo make_geo(const gpe_problem_t& p);

// Reduction scratch: partial sums (doubles) and per-instance ticket counters (zeroed once).
struct Reduce {
    DevBuf parts;      // doubles
    DevBuf counters;   // unsigned ints, one per instance per counter slot
    DevBuf scalars;    // small device scalars (alpha, energy parts, ...)
    int counter_slots = 0;
};

hipError_t reduce_init(Reduce& r, int instances, int slots, size_t part_doubles);

// ---------------------------------------------------------------------------------------------
// Operator launchers (ops.hip).  `f64` selects the precision of the fields (complex128/float64
// vs complex64/float32).  Fields of B instances are stored back to back.  `tmp` is a workspace
// of at least B*N complex values.
// ---------------------------------------------------------------------------------------------
hipError_t op_apply(const Geo& g, bool f64, int B, const Twiddles& tw, const void* f, const void* V,
                    void* out, void* tmp, double beta, double omega, bool nonlinear, hipStream_t s);

// Whole-plane kernel of the H apply (plane.hip): whether the grid's xy-plane fits one workgroup's
// LDS in this dtype on the current device, whether op_apply takes it for a launch of B instances
// (the process-wide kind set by gpe_set_apply_kernel: 0 automatic, 1 passes, 2 plane where it
// fits), and the launch itself (out = H f in 2-D, its xy-part with the pointwise term in 3-D).
void set_apply_kind(int kind);
int apply_kind();
bool plane_fits(const Geo& g, bool f64);
bool plane_preferred(const Geo& g, bool f64, int B);
hipError_t op_apply_plane(const Geo& g, bool f64, int B, const Twiddles& tw, const void* f, const void* V, void* out,
                          double beta, double omega, bool nonlinear, hipStream_t s);

// out = -L_z f (dim >= 2), tmp: one field of workspace.
hipError_t op_rotation(const Geo& g, bool f64, const Twiddles& tw, const void* f, void* out, void* tmp, hipStream_t s);
// Interpolation of one field on the grid g onto the grid with twice the points per axis (out:
// 2^dim N points).  tmp: at least 2N (2-D) or 4N (3-D) complex values; unused in 1-D.
hipError_t op_prolong(const Geo& g, bool f64, const Twiddles& tw, const void* in, void* out, void* tmp, hipStream_t s);

// Tile measurement of the directional passes over B fields of the grid g (f, out: B*N complex
// scratch values each); records the fastest lines per workgroup per axis (tiles, us: per axis).
hipError_t op_autotune(const Geo& g, bool f64, int B, const Twiddles& tw, void* f, void* out, hipStream_t s,
                       int tiles[3], double us[3]);

// Energy parts of one field: dst (device, 4 doubles) <- {kinetic, potential, interaction, rotation}.
hipError_t op_energy(const Geo& g, bool f64, const Twiddles& tw, const void* phi, const void* V,
                     double beta, double omega, Reduce& red, double* dst, hipStream_t s);

// Preconditioner application with the shift read from device memory (*alpha_dev).
hipError_t op_precond(const Geo& g, bool f64, const Twiddles& tw, int kind, const void* phi,
                      const void* V, const double* alpha_dev, double beta, const void* r, void* out,
                      void* tmp, hipStream_t s);

// Minimum over the grid of alpha + V + beta |phi|^2 into *dst (device).
hipError_t op_min_diag(const Geo& g, bool f64, const void* phi, const void* V, const double* alpha_dev,
                       double beta, Reduce& red, double* dst, hipStream_t s);

// lambda~ = kinetic + potential + 2 interaction from energy parts (device to device).
hipError_t op_lambda_tilde(const double* parts, double* dst, hipStream_t s);

// Energy gradient pieces: grad_phi = 2 h^d H phi (in place scaling of Hphi), grad_V = h^d |phi|^2.
hipError_t op_scale_complex(const Geo& g, bool f64, void* x, double s, int64_t count, hipStream_t st);
hipError_t op_density(const Geo& g, bool f64, const void* phi, void* out, double scale, hipStream_t s);

// Thread-local error message.
void set_error(const std::string& msg);

// Validates a problem against the supported grids (sets the error message).
int validate_problem(const gpe_problem_t* p);

// Combine statuses: any error (most negative) wins, else NOT_CONVERGED over OK.
inline int worse_status(int a, int b) {
    if (a < 0 || b < 0) return a < b ? a : b;
    return a > b ? a : b;
}

}  // namespace gpe
