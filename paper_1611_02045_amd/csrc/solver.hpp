// Declarations shared by the solver driver (solve.hip) and the C ABI (api_solve.hip).
#pragma once

#include <vector>

#include "pcg.hpp"

namespace gpe {

struct PhaseArgs {
    Geo g;
    int B;
    const Twiddles* tw;
    Scal* S;               // device, B entries
    Reduce* red;
    size_t region_doubles;
    int precond;
    int check_every;
    int refresh_every;
    bool use_graph = false;  // replay chunks of check_every iterations as a captured graph
    bool final_f_r_is_rp;
};

template <typename T>
hipError_t run_phase(PhaseArgs& pa, IterFields<T> f, std::vector<Scal>& host_S, hipStream_t s);

template <typename T>
hipError_t profile_phase(PhaseArgs& pa, IterFields<T> f, std::vector<Scal>& host_S, int iters, KernelTimer& timer,
                         hipStream_t s);

template <typename T>
hipError_t verify_field(const Geo& g, const Twiddles& tw, const void* phi, const void* V, void* hphi, void* tmp,
                        double beta, double omega, Reduce& red, double out[3], hipStream_t s);

template <typename T>
IterFields<T> carve_fields(DevBuf& buf, int64_t BN, hipError_t* err);

hipError_t convert_complex(bool to64, const void* in, void* out, int64_t n, hipStream_t s);
hipError_t convert_real(bool to64, const void* in, void* out, int64_t n, hipStream_t s);
hipError_t copy_bytes(const void* in, void* out, size_t bytes, hipStream_t s);

Scal make_scal(const gpe_problem_t& p, const Geo& g, const gpe_pcg_opts_t& o);
int validate_opts(const gpe_pcg_opts_t* o);
int status_of(int st);

// Size of one partial-sum region for B instances of grid g.
inline size_t region_doubles_for(const Geo& g, int B) {
    int64_t nb = 1;
    for (int a = 0; a < g.dim; ++a) {
        nb = std::max<int64_t>(nb, lines_per_field(g, a));  // upper bound on blocks per pass
    }
    nb = std::max<int64_t>(nb, 512);
    return (size_t)B * (size_t)nb * 16;
}

}  // namespace gpe
