// Whole-plane H apply: one workgroup holds an xy-plane of n_x x n_y points in LDS and applies both
// directional parts of the operator to it in a single pass (Section 3: the discrete operator acts as
// 1-D transforms along x at fixed y and along y at fixed x), so a 2-D field is written once (H phi)
// and its inputs (phi, V) are taken from HBM once: 5sN bytes against the 11sN of an x pass followed
// by a y pass.  In 3-D the kernel covers the xy-part of every plane and a z pass adds the third
// direction.
//
// Per plane:
//   y phase   columns of phi come from global memory into registers, 8 points per thread; each is
//             transformed along y with the column's own LDS slots as the exchange buffer,
//             multiplied by sigma_y = mu^2/2 - omega x mu (x of the column), transformed back and
//             left in its slots.  128-point columns of a workgroup with 8 threads per column take 16
//             points per thread instead: all columns in one round, a radix-16 stage in registers and
//             one exchange per transform (fft128_col16).
//   x phase   each row's y-part is taken from the plane into registers and the row's slots become
//             the exchange buffer of its x transform (sigma_x = xi^2/2 + omega y xi); phi's row is
//             read a second time (a cache hit: the workgroup read it moments before) for the
//             transform and the pointwise term (V + beta|phi|^2) phi, and the row of H phi is
//             written (x-fastest, coalesced).
// The transforms, multipliers and the order of the additions (y-part + (x-part + pointwise part))
// are those of the directional passes, so both paths agree to rounding (the compiler may contract
// products into FMAs differently in the two kernels).
//
// LDS: the plane with padded rows (n_x + n_x/8 + 1 points: the row transforms' exchange layout,
// and an odd stride between rows) plus the two twiddle tables: 128^2 complex64 takes 147 KiB,
// 64 x 128 complex128 146 KiB, so one workgroup runs per CU.  A thread takes 8 points of a line per
// round; workgroups have at most 1024 (complex64) or 512 (complex128) threads and larger planes
// take several rounds.
#include <algorithm>
#include <array>
#include <atomic>

#include "internal.hpp"
#include "launch.hpp"

namespace gpe {

template <typename T, int LGX, int LGY>
struct PlaneCfg;
// whether the y phase takes 128-point columns 16 points per thread, all columns in one round
template <class P, int LGY>
constexpr bool kCol16 = LGY == 7 && P::NX * 8 == P::W;

template <typename T, int LGX, int LGY>
struct PlaneCfg {
    static constexpr int NX = 1 << LGX, NY = 1 << LGY, NP = NX * NY;
    static constexpr int WMAX = sizeof(T) == 4 ? 1024 : 512;  // threads: registers per lane vs waves
    static constexpr int R = NP / 8 > WMAX ? NP / (8 * WMAX) : 1;  // rows (and columns) per thread
    static constexpr int W = NP / (8 * R);       // threads of the workgroup
    static constexpr int TX = NX / 8, TY = NY / 8;  // threads per row, per column
    static constexpr int CX = W / TX;            // rows per round of the x phase (NY / R)
    static constexpr int CY = W / TY;            // columns per round of the y phase (NX / R)
    static constexpr int RS = NX + NX / 8 + 1;   // LDS row stride in points
    static constexpr size_t LDS = sizeof(C2<T>) * ((size_t)NY * RS + NX + NY);
    // supported: 32..256 points per axis, at most 16384 points (8192 for complex128)
    static constexpr bool OK = LGX >= 5 && LGX <= 8 && LGY >= 5 && LGY <= 8 && NP <= (sizeof(T) == 4 ? 16384 : 8192);
};

// 16-point DFT in place, y_k = sum_s v_s e^{DIR 2 pi i s k / 16}, as 4 x 4: DFTs over a of v[4a + b],
// the twiddles e^{DIR 2 pi i b c / 16}, DFTs over b.  Output y_{c + 4d} is left in v[d + 4c].
template <typename T, int DIR>
__device__ __forceinline__ void dft16_t(C2<T> (&v)[16]) {
    const T c1 = (T)0.923879532511286756128183189396788933;  // cos(pi/8)
    const T s1 = (T)0.382683432365089771728459984030398866;  // sin(pi/8)
    const T h = (T)0.707106781186547524400844362104849039;   // cos(pi/4)
    const T d = (T)DIR;
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4<T, DIR>(v[b], v[4 + b], v[8 + b], v[12 + b]);  // v[b + 4c] = z_bc
    v[5] = mul(v[5], mk(c1, d * s1));     // b = 1, c = 1: e^{DIR i pi/8}
    v[9] = mul(v[9], mk(h, d * h));       // b = 1, c = 2: e^{DIR i pi/4}
    v[13] = mul(v[13], mk(s1, d * c1));   // b = 1, c = 3: e^{DIR 3 i pi/8}
    v[6] = mul(v[6], mk(h, d * h));       // b = 2, c = 1
    v[10] = rot90<T, DIR>(v[10]);         // b = 2, c = 2: e^{DIR i pi/2}
    v[14] = mul(v[14], mk(-h, d * h));    // b = 2, c = 3: e^{DIR 3 i pi/4}
    v[7] = mul(v[7], mk(s1, d * c1));     // b = 3, c = 1
    v[11] = mul(v[11], mk(-h, d * h));    // b = 3, c = 2
    v[15] = mul(v[15], mk(-c1, -d * s1)); // b = 3, c = 3: e^{DIR 9 i pi/8}
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4<T, DIR>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}

// A 128-point column held as 16 points per thread: thread t of the column's 8 keeps positions
// t + 8s (s = 0..15).  A radix-16 stage in registers (butterfly t: positions t + 8s), one exchange
// through the column's LDS slots (point i at buf[i * CS]), then a radix-8 stage (Ns = 16) whose two
// butterflies per thread, t and t + 8, read exactly the thread's own positions again and leave
// X[t + 8s] in v[s]: one exchange per transform.  tw: the 128-entry table e^{-2 pi i e / 128}.
template <typename T, int DIR, int CS>
__device__ __forceinline__ void fft128_col16(C2<T> (&v)[16], C2<T>* buf, const C2<T>* tw, int t) {
    dft16_t<T, DIR>(v);
#pragma unroll
    for (int k = 0; k < 16; ++k) buf[(16 * t + k) * CS] = v[(k >> 2) + 4 * (k & 3)];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = buf[(t + 8 * s) * CS];
    __syncthreads();
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int j = t + 8 * half;  // butterfly: positions j + 16 r, twiddles e^{DIR 2 pi i j r / 128}
        C2<T> e[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) e[r] = v[2 * r + half];
        C2<T> w1 = tw[j], w2 = tw[2 * j], w4 = tw[4 * j];
        if (DIR > 0) {
            w1.y = -w1.y;
            w2.y = -w2.y;
            w4.y = -w4.y;
        }
        const C2<T> w3 = mul(w1, w2);
        e[1] = mul(e[1], w1);
        e[2] = mul(e[2], w2);
        e[3] = mul(e[3], w3);
        e[4] = mul(e[4], w4);
        e[5] = mul(e[5], mul(w1, w4));
        e[6] = mul(e[6], mul(w2, w4));
        e[7] = mul(e[7], mul(w3, w4));
        dft8<T, DIR>(e);
#pragma unroll
        for (int r = 0; r < 8; ++r) v[2 * r + half] = e[r];
    }
}

template <typename T, int LGX, int LGY>
__global__ __launch_bounds__((PlaneCfg<T, LGX, LGY>::W)) void plane_apply_kernel(
    Geo g, int planes, const C2<T>* __restrict__ twx_g, const C2<T>* __restrict__ twy_g, const C2<T>* __restrict__ f,
    const T* __restrict__ V, C2<T>* __restrict__ out, double beta, double omega, int nonlinear) {
    using P = PlaneCfg<T, LGX, LGY>;
    extern __shared__ double4 smem_raw[];
    C2<T>* plane = reinterpret_cast<C2<T>*>(smem_raw);
    C2<T>* twx = plane + (size_t)P::NY * P::RS;
    C2<T>* twy = twx + P::NX;
    const int tid = threadIdx.x;
    const int bi = blockIdx.x / planes;  // instance within the launch
    const int z = blockIdx.x - bi * planes;
    const int b = g.imap ? g.imap[bi] : g.b0 + bi;
    const C2<T>* fp = f + (int64_t)b * g.N + (int64_t)z * P::NP;  // the plane's first point
    C2<T>* op = out + (int64_t)b * g.N + (int64_t)z * P::NP;
    const T* vp = V ? V + (int64_t)z * P::NP : nullptr;             // V is shared by the instances
    const bool rot = g.dim >= 2 && omega != 0.0;
    const double kin = 1.0;

    // y phase.  Columns come straight from global memory (a wave reads one row segment of 64
    // adjacent columns), the first round's in one round trip with the twiddle tables.
    C2<T> v[8];
    if constexpr (kCol16<P, LGY>) {
        // 128-point columns, all at once: 16 points per thread, one exchange per transform
        const int col = tid % P::NX, t = tid / P::NX;
        C2<T> u[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) u[s] = fp[(int64_t)(t + 8 * s) * P::NX + col];
        for (int i = tid; i < P::NX; i += P::W) twx[i] = twx_g[i];
        for (int i = tid; i < P::NY; i += P::W) twy[i] = twy_g[i];
        __syncthreads();
        C2<T>* cbuf = plane + lpad(col);
        fft128_col16<T, -1, P::RS>(u, cbuf, twy, t);
        const double rc = rot ? -omega * coord_of(col, g.L[0], g.h[0]) : 0.0;
        const double inv = 1.0 / P::NY;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const double mu = freq_of(t + 8 * s, P::NY, g.dk[1]);
            u[s] = scl(u[s], (T)((0.5 * kin * mu * mu + rc * mu) * inv));
        }
        fft128_col16<T, +1, P::RS>(u, cbuf, twy, t);
#pragma unroll
        for (int s = 0; s < 16; ++s) cbuf[(t + 8 * s) * P::RS] = u[s];
    } else {
    // thread ty of column cy (+ ry * CY)
    const int cy = tid % P::CY, ty = tid / P::CY;
    auto load_col = [&](int col) {
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = fp[(int64_t)(ty + s * P::TY) * P::NX + col];
    };
    load_col(cy);
    for (int i = tid; i < P::NX; i += P::W) twx[i] = twx_g[i];
    for (int i = tid; i < P::NY; i += P::W) twy[i] = twy_g[i];
    __syncthreads();
#pragma unroll
    for (int ry = 0; ry < P::R; ++ry) {
        const int col = ry * P::CY + cy;
        if (ry > 0) load_col(col);
        C2<T>* cbuf = plane + lpad(col);  // the column's slots: exchange buffer, then its y-part
        fft_line_ct<T, -1, LGY, false, false, P::RS>(v, cbuf, twy, ty);
        const double rc = rot ? -omega * coord_of(col, g.L[0], g.h[0]) : 0.0;
        const double inv = 1.0 / P::NY;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double mu = freq_of(ty + s * P::TY, P::NY, g.dk[1]);
            v[s] = scl(v[s], (T)((0.5 * kin * mu * mu + rc * mu) * inv));
        }
        fft_line_ct<T, +1, LGY, false, false, P::RS>(v, cbuf, twy, ty);
        // the transform's last exchange ended with a barrier: the slots are free
#pragma unroll
        for (int s = 0; s < 8; ++s) cbuf[(ty + s * P::TY) * P::RS] = v[s];
    }
    }
    __syncthreads();  // the y-part is complete in the plane

    // x phase: thread tx of row rx (+ rr * CX).  The row's y-part is taken into registers, then the
    // row's slots serve as the exchange buffer of its x transform; phi is read again (the plane
    // was just read: a cache hit), and H phi = y-part + (x-part + (V + beta|phi|^2) phi).
    const int tx = tid & (P::TX - 1), rx = tid / P::TX;
#pragma unroll
    for (int rr = 0; rr < P::R; ++rr) {
        const int row = rr * P::CX + rx;
        C2<T>* buf = plane + (size_t)row * P::RS;
        C2<T> ay[8], f0[8];
        T vv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int x = tx + s * P::TX;
            f0[s] = fp[(int64_t)row * P::NX + x];
            vv[s] = vp ? vp[(int64_t)row * P::NX + x] : (T)0;
            ay[s] = buf[lpad(x)];
        }
        wave_lds_sync();  // (each row lies in one wave) its y-part is read before the slots are reused
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = f0[s];
        fft_line_ct<T, -1, LGX, true>(v, buf, twx, tx);
        const double rc = rot ? omega * coord_of(row, g.L[1], g.h[1]) : 0.0;
        const double inv = 1.0 / P::NX;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double xi = freq_of(tx + s * P::TX, P::NX, g.dk[0]);
            v[s] = scl(v[s], (T)((0.5 * kin * xi * xi + rc * xi) * inv));
        }
        fft_line_ct<T, +1, LGX, true>(v, buf, twx, tx);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            C2<T> o = v[s];
            if (vp) {
                T w = vv[s];
                if (nonlinear) w += (T)beta * abs2(f0[s]);
                o = add(o, scl(f0[s], w));
            }
            op[(int64_t)row * P::NX + tx + s * P::TX] = add(ay[s], o);
        }
    }
}

namespace {

template <typename T>
using PlaneKernel = void (*)(Geo, int, const C2<T>*, const C2<T>*, const C2<T>*, const T*, C2<T>*, double, double, int);

struct PlaneEntry {
    const void* kern;  // nullptr: unsupported shape
    size_t lds;
    int threads;
};

template <typename T, int LGX, int LGY>
constexpr PlaneEntry plane_entry() {
    using P = PlaneCfg<T, LGX, LGY>;
    if constexpr (P::OK)
        return PlaneEntry{(const void*)&plane_apply_kernel<T, LGX, LGY>, P::LDS, P::W};
    else
        return PlaneEntry{nullptr, 0, 0};
}

template <typename T, int LGX>
constexpr std::array<PlaneEntry, 4> plane_row() {
    return {plane_entry<T, LGX, 5>(), plane_entry<T, LGX, 6>(), plane_entry<T, LGX, 7>(), plane_entry<T, LGX, 8>()};
}

template <typename T>
PlaneEntry plane_lookup(int lgx, int lgy) {
    static const std::array<std::array<PlaneEntry, 4>, 4> table = {plane_row<T, 5>(), plane_row<T, 6>(),
                                                                   plane_row<T, 7>(), plane_row<T, 8>()};
    if (lgx < 5 || lgx > 8 || lgy < 5 || lgy > 8) return PlaneEntry{nullptr, 0, 0};
    return table[lgx - 5][lgy - 5];
}

// LDS a workgroup may allocate on the current device (queried once per device).
size_t device_lds_per_block() {
    static std::atomic<long long> cached[16] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 64 * 1024;
    long long n = cached[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        n = v;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return (size_t)n;
}

std::atomic<int> g_apply_kind{0};  // GPE_APPLY_AUTO

PlaneEntry plane_entry_for(const Geo& g, bool f64) {
    if (g.dim < 2 || g.f5[0] || g.f5[1]) return PlaneEntry{nullptr, 0, 0};
    const PlaneEntry e = f64 ? plane_lookup<double>(g.lg[0], g.lg[1]) : plane_lookup<float>(g.lg[0], g.lg[1]);
    if (!e.kern || e.lds > device_lds_per_block()) return PlaneEntry{nullptr, 0, 0};
    return e;
}

}  // namespace

void set_apply_kind(int kind) { g_apply_kind.store(kind, std::memory_order_relaxed); }
int apply_kind() { return g_apply_kind.load(std::memory_order_relaxed); }

bool plane_fits(const Geo& g, bool f64) { return plane_entry_for(g, f64).kern != nullptr; }

// The automatic choice, from timings of both kernels over batch sizes (MI355X, 256 CUs): planes of
// up to 4096 points (several workgroups per CU) beat the passes at every batch size, 1.2-2.9x
// (64^2 complex64: 8.3 against 11.0 us for one field, 77 against 140 us for 4096); larger planes
// hold a CU each and lose while a launch leaves CUs idle (128^2 complex64: 20.4 against 11.7 us
// for one field), then win once every CU has one (1.2-1.5x at 256 planes).
bool plane_preferred(const Geo& g, bool f64, int B) {
    const int kind = apply_kind();
    if (kind == 1) return false;                 // GPE_APPLY_PASSES
    if (!plane_fits(g, f64)) return false;
    if (kind == 2) return true;                  // GPE_APPLY_PLANE
    const int64_t planes = (int64_t)(g.bl > 0 ? g.bl : B) * g.n[2];
    return (int64_t)g.n[0] * g.n[1] <= 4096 || planes >= device_cus();
}

// out = (xy-part of H) f over B instances (2-D: all of H f).  Requires plane_fits(g, f64).
hipError_t op_apply_plane(const Geo& g, bool f64, int B, const Twiddles& tw, const void* f, const void* V, void* out,
                          double beta, double omega, bool nonlinear, hipStream_t s) {
    const PlaneEntry e = plane_entry_for(g, f64);
    if (!e.kern) return hipErrorInvalidConfiguration;
    const int planes = g.n[2];
    const int64_t blocks = (int64_t)(g.bl > 0 ? g.bl : B) * planes;
    if (blocks <= 0 || blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    static std::once_flag attr_once[2];
    std::call_once(attr_once[f64 ? 1 : 0], [&] {
        // raise the dynamic-LDS cap of every shape once; a runtime that does not need it may refuse
        for (int lx = 5; lx <= 8; ++lx)
            for (int ly = 5; ly <= 8; ++ly) {
                const PlaneEntry q = f64 ? plane_lookup<double>(lx, ly) : plane_lookup<float>(lx, ly);
                if (q.kern && hipFuncSetAttribute(q.kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)q.lds) !=
                                  hipSuccess)
                    (void)hipGetLastError();
            }
    });
    if (f64) {
        auto k = (PlaneKernel<double>)e.kern;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(e.threads), e.lds, s, g, planes,
                           (const C2<double>*)tw.get(0, true), (const C2<double>*)tw.get(1, true), (const C2<double>*)f,
                           (const double*)V, (C2<double>*)out, beta, omega, nonlinear ? 1 : 0);
    } else {
        auto k = (PlaneKernel<float>)e.kern;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(e.threads), e.lds, s, g, planes,
                           (const C2<float>*)tw.get(0, false), (const C2<float>*)tw.get(1, false), (const C2<float>*)f,
                           (const float*)V, (C2<float>*)out, beta, omega, nonlinear ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace gpe
