// LDS-staged Stockham FFT of one line held across TPL = M/8 threads (8 points per thread).
//
// A line of M = 2^lg complex points (8 <= M <= 1024), or M = 5 * 2^lg (40 <= M <= 640), is owned
// by TPL threads; thread t keeps the eight points x[t + s*TPL], s = 0..7, in registers.  The
// transform is a sequence of Stockham autosort stages: one radix-2 or radix-4 stage when lg is
// not a multiple of 3, then radix-8 stages, and for M = 5 * 2^lg a last radix-5 stage worked in
// LDS (its 2^lg butterflies are spread over the TPL threads).  Every stage reads its inputs from the positions t + s*TPL, so the first stage can
// take its operands straight from a coalesced global load, and the last stage leaves
// X[t + s*TPL] (natural frequency order) in the same registers.  Consequently a spectral
// multiplier can be applied in registers and an inverse transform can follow with no LDS round
// trip in between, and the inverse returns each thread the very positions it loaded -- so
// pointwise epilogues see the original input in registers.  Between stages the data goes
// through a padded LDS line buffer (one write, barrier, one read, barrier; the barriers are
// wave-level when each line lies within one wave).
//
// The forward transform is unnormalised, sum_j x_j e^{-2 pi i jk/M}; the inverse uses e^{+...}
// and is also unnormalised (callers fold 1/M into their multiplier), matching the expansions
// of Section 3 of the paper.  Twiddles come from an LDS table tw[e] = exp(-2 pi i e/M) built
// from FP64 host values (three per radix-8 stage; the other four are products of two of them).
#pragma once

#include "common.hpp"

namespace gpe {

// Padded LDS index: one spare slot per 8 points spreads the stride-Ns Stockham writes over banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }
// Padded length (in points) of one LDS line of a workgroup holding C lines.  x passes keep each
// line in consecutive lanes, and an odd length starts neighbouring lines in different banks.
// Strided passes interleave their lines lane by lane (lane = line + C t); with U = 16 (8-byte
// points) or 8 (16-byte points) points per LDS cycle, a length of U/C mod U points puts the U
// lanes served together on distinct banks in every exchange.
__host__ __device__ constexpr int line_stride(int M, int point_bytes = 8, int axis = 0, int C = 1) {
    const int U = point_bytes == 8 ? 16 : 8;
    const int pad = C >= U ? 1 : U / C;
    return axis == 0 ? M + (M >> 3) + 1 : ((M + (M >> 3) + U - 1) & ~(U - 1)) + pad;
}

// a * (DIR * i)
template <typename T, int DIR>
__host__ __device__ __forceinline__ C2<T> rot90(C2<T> a) {
    return DIR < 0 ? mk(a.y, -a.x) : mk(-a.y, a.x);
}

template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft2(C2<T>& x0, C2<T>& x1) {
    C2<T> a = add(x0, x1), b = sub(x0, x1);
    x0 = a;
    x1 = b;
}

// In-place 4-point DFT: (x0,x1,x2,x3) <- (X0,X1,X2,X3), X_k = sum_r x_r e^{DIR 2 pi i rk/4}.
template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft4(C2<T>& x0, C2<T>& x1, C2<T>& x2, C2<T>& x3) {
    C2<T> c0 = add(x0, x2), c2 = sub(x0, x2), c1 = add(x1, x3), c3 = rot90<T, DIR>(sub(x1, x3));
    x0 = add(c0, c1);
    x1 = add(c2, c3);
    x2 = sub(c0, c1);
    x3 = sub(c2, c3);
}

// In-place 8-point DFT on v[0..7] (natural order in and out): two radix-2 layers of 4 and the
// twiddles e^{DIR 2 pi i r/8} in between, then two 4-point DFTs (even and odd outputs).
template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft8(C2<T> (&v)[8]) {
    const T c = (T)0.707106781186547524400844362104849039;
    C2<T> a0 = add(v[0], v[4]), b0 = sub(v[0], v[4]);
    C2<T> a1 = add(v[1], v[5]), b1 = sub(v[1], v[5]);
    C2<T> a2 = add(v[2], v[6]), b2 = sub(v[2], v[6]);
    C2<T> a3 = add(v[3], v[7]), b3 = sub(v[3], v[7]);
    if (DIR < 0) {
        b1 = mk(c * (b1.x + b1.y), c * (b1.y - b1.x));    // * e^{-i pi/4}
        b2 = mk(b2.y, -b2.x);                            // * -i
        b3 = mk(c * (b3.y - b3.x), -c * (b3.x + b3.y));  // * e^{-3 i pi/4}
    } else {
        b1 = mk(c * (b1.x - b1.y), c * (b1.x + b1.y));   // * e^{+i pi/4}
        b2 = mk(-b2.y, b2.x);                            // * +i
        b3 = mk(-c * (b3.x + b3.y), c * (b3.x - b3.y));  // * e^{+3 i pi/4}
    }
    dft4<T, DIR>(a0, a1, a2, a3);
    dft4<T, DIR>(b0, b1, b2, b3);
    v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
    v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

// In-place 5-point DFT: X_k = sum_r x_r e^{DIR 2 pi i rk/5}.  With c_m = cos(2 pi m/5),
// s_m = sin(2 pi m/5): X_1,4 = x0 + c1 (x1 + x4) + c2 (x2 + x3) +- DIR i (s1 (x1 - x4) + s2 (x2 - x3))
// and X_2,3 = x0 + c2 (x1 + x4) + c1 (x2 + x3) +- DIR i (s2 (x1 - x4) - s1 (x2 - x3)).
template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft5(C2<T>& x0, C2<T>& x1, C2<T>& x2, C2<T>& x3, C2<T>& x4) {
    const T c1 = (T)0.309016994374947424102293417182819059;   // cos(2 pi/5)
    const T c2 = (T)-0.809016994374947424102293417182819059;  // cos(4 pi/5)
    const T s1 = (T)0.951056516295153572116439333379382143;   // sin(2 pi/5)
    const T s2 = (T)0.587785252292473129168705954639072769;   // sin(4 pi/5)
    const C2<T> a1 = add(x1, x4), b1 = sub(x1, x4), a2 = add(x2, x3), b2 = sub(x2, x3);
    const C2<T> t1 = mk(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const C2<T> t2 = mk(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    const C2<T> u1 = rot90<T, DIR>(mk(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const C2<T> u2 = rot90<T, DIR>(mk(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    x0 = add(x0, add(a1, a2));
    x1 = add(t1, u1);
    x4 = sub(t1, u1);
    x2 = add(t2, u2);
    x3 = sub(t2, u2);
}

// Order this wave's LDS accesses (a wave's LDS operations execute in issue order; the fences keep
// the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Read back v[s] = buf[t + s*TPL] after a stage's scattered write, synchronised on both sides:
// across the workgroup, or only within the wave when every line lies inside one wave (`wave`).
// For TPL a multiple of 8, lpad(t + s*TPL) = lpad(t) + s*lpad(TPL): one base and one stride.
template <typename T>
__device__ __forceinline__ void exchange_read(C2<T> (&v)[8], const C2<T>* buf, int t, int TPL, bool wave) {
    if (wave) wave_lds_sync(); else __syncthreads();
    if ((TPL & 7) == 0) {
        const C2<T>* p = buf + lpad(t);
        const int st = lpad(TPL);
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = p[s * st];
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = buf[lpad(t + s * TPL)];
    }
    if (wave) wave_lds_sync(); else __syncthreads();
}

// Full line transform (see file comment).  All threads of the block must call it with the same
// lg, M (2^lg or 5 * 2^lg) and `wave`; `buf` is this thread's line region in LDS (one padded line)
// and `tw` the table of M entries.  wave: each line is held by threads of a single wave (lines of
// at most 512 points laid along consecutive lanes), so the exchanges need no workgroup barrier.
template <typename T, int DIR>
__device__ __forceinline__ void fft_line(C2<T> (&v)[8], C2<T>* buf, const C2<T>* tw, int t, int lg, int M,
                                         bool wave = false) {
    const bool f5 = M != (1 << lg);
    const int TPL = M >> 3;
    const int rem = lg % 3;
    const int n8 = lg / 3;
    int lgNs = 0;
    if (rem == 1) {
        // radix-2 stage at Ns = 1: butterflies j = t + q*TPL on (v[q], v[q+4]); out[2j + r]
#pragma unroll
        for (int q = 0; q < 4; ++q) dft2<T, DIR>(v[q], v[q + 4]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = t + q * TPL;
            buf[lpad(2 * j)] = v[q];
            buf[lpad(2 * j + 1)] = v[q + 4];
        }
        exchange_read(v, buf, t, TPL, wave);
        lgNs = 1;
    } else if (rem == 2) {
        // radix-4 stage at Ns = 1: butterflies j = t on v[0,2,4,6] and j = t + TPL on v[1,3,5,7]
        dft4<T, DIR>(v[0], v[2], v[4], v[6]);
        dft4<T, DIR>(v[1], v[3], v[5], v[7]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            buf[lpad(4 * t + r)] = v[2 * r];
            buf[lpad(4 * (t + TPL) + r)] = v[2 * r + 1];
        }
        exchange_read(v, buf, t, TPL, wave);
        lgNs = 2;
    }
    for (int k = 0; k < n8; ++k) {
        // radix-8 stage at Ns = 2^lgNs: butterfly j = t on v[r] (positions t + r*TPL)
        if (lgNs > 0) {
            // w_r = tw[r * step]: w1, w2, w4 from the table, the other four as products of two
            const int jm = t & ((1 << lgNs) - 1);
            const int step = jm * (TPL >> lgNs);  // jm * M / (8 Ns)
            C2<T> w1 = tw[step], w2 = tw[2 * step], w4 = tw[4 * step];
            if (DIR > 0) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w4.y = -w4.y;
            }
            const C2<T> w3 = mul(w1, w2);
            v[1] = mul(v[1], w1);
            v[2] = mul(v[2], w2);
            v[3] = mul(v[3], w3);
            v[4] = mul(v[4], w4);
            v[5] = mul(v[5], mul(w1, w4));
            v[6] = mul(v[6], mul(w2, w4));
            v[7] = mul(v[7], mul(w3, w4));
        }
        dft8<T, DIR>(v);
        if (k + 1 < n8 || f5) {
            const int Ns = 1 << lgNs;
            const int base = ((t >> lgNs) << (lgNs + 3)) + (t & (Ns - 1));
            if (Ns == 1 || Ns >= 8) {
                // base + r*Ns never crosses a multiple of 8 for Ns = 1 (base = 8t) and keeps
                // base's offset within its group of 8 for Ns >= 8: lpad is affine in r
                C2<T>* p = buf + lpad(base);
                const int st = Ns == 1 ? 1 : lpad(Ns);
#pragma unroll
                for (int r = 0; r < 8; ++r) p[r * st] = v[r];
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r) buf[lpad(base + r * Ns)] = v[r];
            }
            if (k + 1 < n8) exchange_read(v, buf, t, TPL, wave);
        }
        lgNs += 3;
    }
    if (f5) {
        // radix-5 stage at Ns = P = 2^lg = M/5: butterfly j < P takes the points j + r P, twiddles
        // them by e^{-+2 pi i jr/M} and writes its outputs back to the same places (natural order)
        const int P = 1 << lg;
        if (wave) wave_lds_sync(); else __syncthreads();
        for (int j = t; j < P; j += TPL) {
            C2<T> x[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) x[r] = buf[lpad(j + r * P)];
#pragma unroll
            for (int r = 1; r < 5; ++r) {
                C2<T> w = tw[j * r];
                if (DIR > 0) w.y = -w.y;
                x[r] = mul(x[r], w);
            }
            dft5<T, DIR>(x[0], x[1], x[2], x[3], x[4]);
#pragma unroll
            for (int r = 0; r < 5; ++r) buf[lpad(j + r * P)] = x[r];
        }
        exchange_read(v, buf, t, TPL, wave);
    }
}

// fft_line for a compile-time size 2^LG (F5: 5 * 2^LG): the same stages, with every stride, offset
// and stage count a constant (LDS addresses become immediate offsets).  WAVE: lines lie within one
// wave.  CS > 0: point i of the line's LDS region sits at buf[i * CS] instead of the padded
// buf[lpad(i)] (a column of a plane held in LDS, whose neighbouring columns go to neighbouring
// lanes, so the stride needs no padding).
template <typename T, int DIR, int LG, bool WAVE, bool F5 = false, int CS = 0>
__device__ __forceinline__ void fft_line_ct(C2<T> (&v)[8], C2<T>* buf, const C2<T>* tw, int t) {
    static_assert(LG >= 3 && LG <= 10, "lines of 8 to 1024 points");
    static_assert(!F5 || (LG <= 7 && !WAVE), "lines of 5 * 2^LG points: at most 640, across waves");
    static_assert(CS == 0 || !F5, "strided regions for lines of 2^LG points only");
    constexpr int TPL = F5 ? 5 << (LG - 3) : 1 << (LG - 3);
    constexpr int REM = LG % 3;
    constexpr int N8 = LG / 3;
    auto ix = [](int i) {
        if constexpr (CS > 0) return i * CS; else return lpad(i);
    };
    auto sync = [] {
        if constexpr (WAVE) wave_lds_sync(); else __syncthreads();
    };
    auto read_back = [&] {
        sync();
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = buf[ix(t + s * TPL)];
        sync();
    };
    if constexpr (REM == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) dft2<T, DIR>(v[q], v[q + 4]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = t + q * TPL;
            buf[ix(2 * j)] = v[q];
            buf[ix(2 * j + 1)] = v[q + 4];
        }
        read_back();
    } else if constexpr (REM == 2) {
        dft4<T, DIR>(v[0], v[2], v[4], v[6]);
        dft4<T, DIR>(v[1], v[3], v[5], v[7]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            buf[ix(4 * t + r)] = v[2 * r];
            buf[ix(4 * (t + TPL) + r)] = v[2 * r + 1];
        }
        read_back();
    }
#pragma unroll
    for (int k = 0; k < N8; ++k) {
        const int lgNs = REM + 3 * k;
        const int Ns = 1 << lgNs;
        if (lgNs > 0) {
            const int jm = t & (Ns - 1);
            const int step = jm * (TPL >> lgNs);  // jm * M / (8 Ns)
            C2<T> w1 = tw[step], w2 = tw[2 * step], w4 = tw[4 * step];
            if (DIR > 0) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w4.y = -w4.y;
            }
            const C2<T> w3 = mul(w1, w2);
            v[1] = mul(v[1], w1);
            v[2] = mul(v[2], w2);
            v[3] = mul(v[3], w3);
            v[4] = mul(v[4], w4);
            v[5] = mul(v[5], mul(w1, w4));
            v[6] = mul(v[6], mul(w2, w4));
            v[7] = mul(v[7], mul(w3, w4));
        }
        dft8<T, DIR>(v);
        if (k + 1 < N8 || F5) {
            const int base = ((t >> lgNs) << (lgNs + 3)) + (t & (Ns - 1));
#pragma unroll
            for (int r = 0; r < 8; ++r) buf[ix(base + r * Ns)] = v[r];
            if (k + 1 < N8) read_back();
        }
    }
    if constexpr (F5) {
        // radix-5 stage at Ns = P = 2^LG (see fft_line): butterflies j = t + q TPL < P
        constexpr int P = 1 << LG;
        sync();
#pragma unroll
        for (int q = 0; q < (P + TPL - 1) / TPL; ++q) {
            const int j = t + q * TPL;
            if (j < P) {
                C2<T> x[5];
#pragma unroll
                for (int r = 0; r < 5; ++r) x[r] = buf[ix(j + r * P)];
#pragma unroll
                for (int r = 1; r < 5; ++r) {
                    C2<T> w = tw[j * r];
                    if (DIR > 0) w.y = -w.y;
                    x[r] = mul(x[r], w);
                }
                dft5<T, DIR>(x[0], x[1], x[2], x[3], x[4]);
#pragma unroll
                for (int r = 0; r < 5; ++r) buf[ix(j + r * P)] = x[r];
            }
        }
        read_back();
    }
}

// Copy the twiddle table of an M-point transform from global memory into LDS and barrier.
template <typename T>
__device__ __forceinline__ void load_twiddles(C2<T>* tw_lds, const C2<T>* tw_glob, int M) {
    for (int i = threadIdx.x; i < M; i += blockDim.x) tw_lds[i] = tw_glob[i];
    __syncthreads();
}

}  // namespace gpe
