// HIP kernels for gfx950 (wave64).  See svq_dev.hpp for the descriptor
// tables and kernels.hpp for the host launch interface.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "kernels.hpp"
#include "svq_dev.hpp"

namespace svq {

template <typename R> struct V2T;
template <> struct V2T<float> { using type = float2; };
template <> struct V2T<double> { using type = double2; };

// Insert a zero bit at each of the (ascending) positions pos[0..k-1].
template <typename TI>
__device__ __forceinline__ uint64_t spread(uint64_t b, const TI *pos, int k) {
    for (int j = 0; j < k; ++j) {
        const int p = pos[j];
        const uint64_t lo = b & ((1ULL << p) - 1);
        b = ((b >> p) << (p + 1)) | lo;
    }
    return b;
}

// ---------------------------------------------------------------------------
// register-tile gate kernels
// ---------------------------------------------------------------------------

template <typename R, int NR> struct Regs {
    R re[NR], im[NR];
};

template <int NWB>
__device__ __forceinline__ uint32_t thread_tile_index(const PhaseDesc &P, uint32_t lane,
                                                      uint32_t wave) {
    uint32_t tt = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) tt |= ((lane >> b) & 1u) << P.lane[b];
#pragma unroll
    for (int b = 0; b < NWB; ++b) tt |= ((wave >> b) & 1u) << P.wave[b];
    return tt;
}

template <int RB>
__device__ __forceinline__ uint32_t reg_offset(const PhaseDesc &P, int j) {
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < RB; ++b)
        if ((j >> b) & 1) r |= 1u << P.reg[b];
    return r;
}

// Physical element offset of tile-local index t inside its tile.  Tile bits
// are chunk-local and a chunk holds at most 2^32 elements, so 32 bits hold it.
template <int K>
__device__ __forceinline__ uint32_t tile_to_phys(uint32_t t, const int8_t *tphys) {
    uint32_t p = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((t >> j) & 1) p |= 1u << tphys[j];
    return p;
}

// ---- gate ops on compile-time register bits -------------------------------

// In-place rotation of (x, y) by the angle whose shear parameters are
// (t, s): x' = cos(a) x - sin(a) y, y' = sin(a) x + cos(a) y.
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
__device__ __forceinline__ void shear_rot(R &x, R &y, R t, R s) {
    x = fma_r(-t, y, x);
    y = fma_r(s, x, y);
    x = fma_r(-t, y, x);
}

// Register moves pinned by inline asm.  put_reg writes `val` into the
// register that already holds `dst`; swap_reg exchanges two registers in
// place.  The permuting and dense ops end with these, so every op leaves each
// amplitude in the register that held it before.  Otherwise the op loop's
// single back edge merges handlers whose results sit in different registers,
// and register allocation then copies every amplitude after every op.
__device__ __forceinline__ void put_reg(float &dst, float val) {
    asm("v_mov_b32 %0, %1" : "+v"(dst) : "v"(val));
}
__device__ __forceinline__ void put_reg(double &dst, double val) {
    asm("v_mov_b64 %0, %1" : "+v"(dst) : "v"(val));
}
__device__ __forceinline__ void swap_reg(float &a, float &b) {
    asm("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap_reg(double &a, double &b) {
    const double t = a;
    put_reg(a, b);
    put_reg(b, t);
}

template <int B, typename R, int NR, typename OP>
__device__ __forceinline__ void op_diag1(Regs<R, NR> &v, const OP &o) {
    const R t0 = (R)o.sh[0], s0 = (R)o.sh[1], t1 = (R)o.sh[2], s1 = (R)o.sh[3];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if ((j >> B) & 1) shear_rot(v.re[j], v.im[j], t1, s1);
        else shear_rot(v.re[j], v.im[j], t0, s0);
    }
    if (o.flip & 1) {
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (!((j >> B) & 1)) { v.re[j] = -v.re[j]; v.im[j] = -v.im[j]; }
    }
    if (o.flip & 2) {
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if ((j >> B) & 1) { v.re[j] = -v.re[j]; v.im[j] = -v.im[j]; }
    }
}

template <int B0, int B1, typename R, int NR, typename OP>
__device__ __forceinline__ void op_cphase(Regs<R, NR> &v, const OP &o) {
    const R t = (R)o.sh[0], sn = (R)o.sh[1];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (!((j >> B0) & 1) || !((j >> B1) & 1)) continue;
        shear_rot(v.re[j], v.im[j], t, sn);
    }
    if (o.flip & 1) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (!((j >> B0) & 1) || !((j >> B1) & 1)) continue;
            v.re[j] = -v.re[j];
            v.im[j] = -v.im[j];
        }
    }
}

template <int B, typename R, int NR>
__device__ __forceinline__ void op_mix1(Regs<R, NR> &v, const OpDesc &o) {
    const R a_r = (R)o.m[0], a_i = (R)o.m[1], b_r = (R)o.m[2], b_i = (R)o.m[3];
    const R c_r = (R)o.m[4], c_i = (R)o.m[5], d_r = (R)o.m[6], d_i = (R)o.m[7];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const R x0r = v.re[j], x0i = v.im[j], x1r = v.re[j1], x1i = v.im[j1];
        const R y0r = a_r * x0r - a_i * x0i + b_r * x1r - b_i * x1i;
        const R y0i = a_r * x0i + a_i * x0r + b_r * x1i + b_i * x1r;
        const R y1r = c_r * x0r - c_i * x0i + d_r * x1r - d_i * x1i;
        const R y1i = c_r * x0i + c_i * x0r + d_r * x1i + d_i * x1r;
        put_reg(v.re[j], y0r);
        put_reg(v.im[j], y0i);
        put_reg(v.re[j1], y1r);
        put_reg(v.im[j1], y1i);
    }
}

template <int B, typename R, int NR, typename OP>
__device__ __forceinline__ void op_roty(Regs<R, NR> &v, const OP &o) {
    const R t = (R)o.sh[0], sn = (R)o.sh[1];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        shear_rot(v.re[j], v.re[j1], t, sn);
        shear_rot(v.im[j], v.im[j1], t, sn);
    }
    if (o.flip & 1) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            v.re[j] = -v.re[j];
            v.im[j] = -v.im[j];
        }
    }
}

template <int B, typename R, int NR, typename OP>
__device__ __forceinline__ void op_xswap(Regs<R, NR> &v, const OP &) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        swap_reg(v.re[j], v.re[j1]);
        swap_reg(v.im[j], v.im[j1]);
    }
}

template <int B0, int B1, typename R, int NR, typename OP>
__device__ __forceinline__ void op_cnot(Regs<R, NR> &v, const OP &) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (!((j >> B0) & 1) || ((j >> B1) & 1)) continue;
        const int j1 = j | (1 << B1);
        swap_reg(v.re[j], v.re[j1]);
        swap_reg(v.im[j], v.im[j1]);
    }
}

template <int B0, int B1, typename R, int NR, typename OP>
__device__ __forceinline__ void op_givens(Regs<R, NR> &v, const OP &o) {
    const R t = (R)o.sh[0], sn = (R)o.sh[1];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int ju = j | (1 << B0);   // b0 = 1, b1 = 0
        const int jw = j | (1 << B1);   // b0 = 0, b1 = 1
        shear_rot(v.re[ju], v.re[jw], t, sn);
        shear_rot(v.im[ju], v.im[jw], t, sn);
    }
    if (o.flip & 1) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j & ((1 << B0) | (1 << B1))) continue;
            const int ju = j | (1 << B0), jw = j | (1 << B1);
            v.re[ju] = -v.re[ju];
            v.im[ju] = -v.im[ju];
            v.re[jw] = -v.re[jw];
            v.im[jw] = -v.im[jw];
        }
    }
}

template <int B0, int B1, typename R, int NR>
__device__ __forceinline__ void op_mix2(Regs<R, NR> &v, const OpDesc &o) {
    R mr[16], mi[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        mr[e] = (R)o.m[2 * e];
        mi[e] = (R)o.m[2 * e + 1];
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        int jl[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) jl[l] = j | ((l & 1) ? (1 << B0) : 0) | ((l & 2) ? (1 << B1) : 0);
        R xr[4], xi[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            xr[l] = v.re[jl[l]];
            xi[l] = v.im[jl[l]];
        }
        R yr[4], yi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            R sr = 0, si = 0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                sr += mr[r * 4 + cc] * xr[cc] - mi[r * 4 + cc] * xi[cc];
                si += mr[r * 4 + cc] * xi[cc] + mi[r * 4 + cc] * xr[cc];
            }
            yr[r] = sr;
            yi[r] = si;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            put_reg(v.re[jl[r]], yr[r]);
            put_reg(v.im[jl[r]], yi[r]);
        }
    }
}

// Dispatch on register-bit positions with explicit cases so that every
// variant is inlined and the register arrays never leave VGPRs.
#define SVQ_C1(FN, I)                                        \
    case I:                                                  \
        if constexpr (I < RB) FN<I, R, NR>(v, o);            \
        break;
#define SVQ_C2(FN, I, J)                                                      \
    case I * 8 + J:                                                           \
        if constexpr (I < RB && J < RB && I != J) FN<I, J, R, NR>(v, o);      \
        break;
#define SVQ_ALL1(FN) SVQ_C1(FN, 0) SVQ_C1(FN, 1) SVQ_C1(FN, 2) SVQ_C1(FN, 3) SVQ_C1(FN, 4)
#define SVQ_ROW(FN, I) SVQ_C2(FN, I, 0) SVQ_C2(FN, I, 1) SVQ_C2(FN, I, 2) SVQ_C2(FN, I, 3) SVQ_C2(FN, I, 4)
#define SVQ_ALL2(FN) SVQ_ROW(FN, 0) SVQ_ROW(FN, 1) SVQ_ROW(FN, 2) SVQ_ROW(FN, 3) SVQ_ROW(FN, 4)

// The code and shear parameters of an op: the first 64 bytes of its
// descriptor, read with one scalar load before the dispatch (otherwise the
// parameters are fetched inside the handler, a second load that waits on the
// first).
struct OpHead {
    int32_t type, b0, b1, flip;
    double sh[4];
};

#define SVQ_H1(FN, I)                                        \
    case I:                                                  \
        if constexpr (I < RB) FN<I, R, NR>(v, h);            \
        break;
#define SVQ_H2(FN, I, J)                                                      \
    case (I < RB && J < RB) ? I * RB + J : 64 + I * 8 + J:                    \
        if constexpr (I < RB && J < RB && I != J) FN<I, J, R, NR>(v, h);      \
        break;
#define SVQ_HALL1(FN) SVQ_H1(FN, 0) SVQ_H1(FN, 1) SVQ_H1(FN, 2) SVQ_H1(FN, 3) SVQ_H1(FN, 4)
#define SVQ_HROW(FN, I) SVQ_H2(FN, I, 0) SVQ_H2(FN, I, 1) SVQ_H2(FN, I, 2) SVQ_H2(FN, I, 3) SVQ_H2(FN, I, 4)
#define SVQ_HALL2(FN) SVQ_HROW(FN, 0) SVQ_HROW(FN, 1) SVQ_HROW(FN, 2) SVQ_HROW(FN, 3) SVQ_HROW(FN, 4)

template <typename R, int NR, int RB>
__device__ __forceinline__ void apply_op(Regs<R, NR> &v, const OpDesc &o) {
    static_assert(RB <= 5, "dispatch covers at most 5 register bits");
    OpHead h;
    h.type = o.type;
    h.b0 = o.b0;
    h.b1 = o.b1;
    h.flip = o.flip;
#pragma unroll
    for (int i = 0; i < 4; ++i) h.sh[i] = o.sh[i];
    asm volatile("" ::"s"(h.type), "s"(h.b0), "s"(h.b1), "s"(h.flip), "s"(h.sh[0]), "s"(h.sh[1]),
                 "s"(h.sh[2]), "s"(h.sh[3]));
    const int b2 = h.b0 * RB + h.b1;   // the dense key of SVQ_H2
    const int b2o = h.b0 * 8 + h.b1;   // the key of SVQ_C2 (dense ops)
    // the two kinds of a fabric circuit first, then the rest
    if (h.type == OP_GIVENS) {
        switch (b2) { SVQ_HALL2(op_givens) }
        return;
    }
    if (h.type == OP_CPHASE) {
        switch (b2) { SVQ_HALL2(op_cphase) }
        return;
    }
    switch (h.type) {
    case OP_DIAG1: switch (h.b0) { SVQ_HALL1(op_diag1) } break;
    case OP_MIX1: switch (h.b0) { SVQ_ALL1(op_mix1) } break;
    case OP_ROTY: switch (h.b0) { SVQ_HALL1(op_roty) } break;
    case OP_XSWAP: switch (h.b0) { SVQ_HALL1(op_xswap) } break;
    case OP_CNOT: switch (b2) { SVQ_HALL2(op_cnot) } break;
    default: switch (b2o) { SVQ_ALL2(op_mix2) } break;
    }
}

// ---- adjoint: 2 Im <lambda|K|psi> over this thread's amplitudes ------------
// Products are formed in the state's precision and summed in FP64.  The
// generator entries of DIAG1/MIX1 carry the angle's scale (chain rule); the
// hard-coded CPHASE and GIVENS generators take it from k[0].

template <int B0, int B1, typename R, int NR>
__device__ __forceinline__ double gen_value(const Regs<R, NR> &x, const Regs<R, NR> &l,
                                            const OpDesc &o) {
    double acc = 0.0;
    if (o.gtype == GEN_DIAG1) {
        const R k0 = (R)o.k[0], k1 = (R)o.k[1];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const R kk = ((j >> B0) & 1) ? k1 : k0;
            acc += (double)(kk * (l.re[j] * x.im[j] - l.im[j] * x.re[j]));   // Im(conj(l) x)
        }
    } else if (o.gtype == GEN_CPHASE) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (!((j >> B0) & 1) || !((j >> B1) & 1)) continue;
            acc -= (double)(l.re[j] * x.im[j] - l.im[j] * x.re[j]);
        }
        acc *= o.k[0];
    } else if (o.gtype == GEN_MIX1) {
        const R k00r = (R)o.k[0], k00i = (R)o.k[1], k01r = (R)o.k[2], k01i = (R)o.k[3];
        const R k10r = (R)o.k[4], k10i = (R)o.k[5], k11r = (R)o.k[6], k11i = (R)o.k[7];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j & (1 << B0)) continue;
            const int j1 = j | (1 << B0);
            const R y0r = k00r * x.re[j] - k00i * x.im[j] + k01r * x.re[j1] - k01i * x.im[j1];
            const R y0i = k00r * x.im[j] + k00i * x.re[j] + k01r * x.im[j1] + k01i * x.re[j1];
            const R y1r = k10r * x.re[j] - k10i * x.im[j] + k11r * x.re[j1] - k11i * x.im[j1];
            const R y1i = k10r * x.im[j] + k10i * x.re[j] + k11r * x.im[j1] + k11i * x.re[j1];
            acc += (double)(l.re[j] * y0i - l.im[j] * y0r) + (double)(l.re[j1] * y1i - l.im[j1] * y1r);
        }
    } else {   // GEN_GIVENS: Im<l|K|x> = (Re(conj(l_w) x_u) - Re(conj(l_u) x_w)) / 2
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j & ((1 << B0) | (1 << B1))) continue;
            const int ju = j | (1 << B0), jw = j | (1 << B1);
            acc += (double)(l.re[jw] * x.re[ju] + l.im[jw] * x.im[ju])
                 - (double)(l.re[ju] * x.re[jw] + l.im[ju] * x.im[jw]);
        }
        acc *= 0.5 * o.k[0];
    }
    return 2.0 * acc;
}

#define SVQ_G1(I)                                                          \
    case I:                                                                \
        if constexpr (I < RB) g = gen_value<I, 0, R, NR>(x, l, o);         \
        break;
#define SVQ_G2(I, J)                                                                   \
    case I * 8 + J:                                                                    \
        if constexpr (I < RB && J < RB && I != J) g = gen_value<I, J, R, NR>(x, l, o); \
        break;
#define SVQ_GROW(I) SVQ_G2(I, 0) SVQ_G2(I, 1) SVQ_G2(I, 2) SVQ_G2(I, 3) SVQ_G2(I, 4)

template <typename R, int NR, int RB>
__device__ __forceinline__ double op_gradient(const Regs<R, NR> &x, const Regs<R, NR> &l,
                                              const OpDesc &o) {
    double g = 0.0;
    if (o.gtype == GEN_DIAG1 || o.gtype == GEN_MIX1) {
        switch (o.b0) { SVQ_G1(0) SVQ_G1(1) SVQ_G1(2) SVQ_G1(3) SVQ_G1(4) }
    } else {
        switch (o.b0 * 8 + o.b1) { SVQ_GROW(0) SVQ_GROW(1) SVQ_GROW(2) SVQ_GROW(3) SVQ_GROW(4) }
    }
    return g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---- the pass ---------------------------------------------------------------

// The maps register index j -> physical offset and j -> LDS slot are linear
// over GF(2) (sums of disjoint bits; the pass's slot map is an XOR map), so
// they are built from RB basis values instead of bit by bit.
template <int RB, int K>
struct RegMap {
    uint32_t ph[RB];    // physical offset of register bit b
    uint32_t sl[RB];    // LDS slot contribution of register bit b
    template <typename TI>
    __device__ __forceinline__ void init(const PhaseDesc &P, const TI *tphys) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            ph[b] = 1u << tphys[P.reg[b]];
            sl[b] = (uint32_t)P.rsl[b];
        }
    }
    __device__ __forceinline__ uint32_t phys(int j) const {
        uint32_t p = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if ((j >> b) & 1) p += ph[b];
        return p;
    }
    __device__ __forceinline__ uint32_t slot(int j) const {
        uint32_t p = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if ((j >> b) & 1) p ^= sl[b];
        return p;
    }
};

// Physical offset and LDS slot of the thread's own (lane, wave) bits.
template <int NWB, int K, typename TI>
__device__ __forceinline__ void thread_maps(const PhaseDesc &P, const TI *tphys, uint32_t lane,
                                            uint32_t wave, uint32_t &tp, uint32_t &tslot) {
    uint32_t t = 0, p = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint32_t bit = (lane >> b) & 1u;
        t ^= bit ? (uint32_t)P.lsl[b] : 0u;
        p |= bit << tphys[P.lane[b]];
    }
#pragma unroll
    for (int b = 0; b < NWB; ++b) {
        const uint32_t bit = (wave >> b) & 1u;
        t ^= bit ? (uint32_t)P.wsl[b] : 0u;
        p |= bit << tphys[P.wave[b]];
    }
    tp = p;
    tslot = t;
}

// Tile loads and stores.  With OFF32 the in-tile byte offset fits 32 bits
// (the tile's highest physical bit times the element size stays below 2^32),
// so every access is a uniform base plus one 32-bit VGPR offset.
template <typename V, typename R, int NR, int RB, int K, bool OFF32 = false>
__device__ __forceinline__ void load_regs(Regs<R, NR> &v, const V *__restrict__ src, uint32_t tp,
                                          const RegMap<RB, K> &m) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        V e;
        if constexpr (OFF32 && sizeof(V) == 16) {
            // 16-byte amplitudes stream with non-temporal accesses (measured
            // faster for complex128; for 8-byte amplitudes the non-temporal
            // stores are several times slower, so complex64 keeps the plain
            // ones)
            const uint32_t off = (tp + m.phys(j)) * (uint32_t)sizeof(V);
            typedef R r2_t __attribute__((ext_vector_type(2)));
            const r2_t t2 = __builtin_nontemporal_load((const r2_t *)((const char *)src + off));
            e.x = t2.x;
            e.y = t2.y;
        } else if constexpr (OFF32) {
            const uint32_t off = (tp + m.phys(j)) * (uint32_t)sizeof(V);
            e = *(const V *)((const char *)src + off);
        } else {
            e = src[tp + m.phys(j)];
        }
        v.re[j] = e.x;
        v.im[j] = e.y;
    }
}

template <typename V, typename R, int NR, int RB, int K, bool OFF32 = false>
__device__ __forceinline__ void store_regs(const Regs<R, NR> &v, V *__restrict__ dst, uint32_t tp,
                                           const RegMap<RB, K> &m) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        V e;
        e.x = v.re[j];
        e.y = v.im[j];
        if constexpr (OFF32 && sizeof(V) == 16) {
            const uint32_t off = (tp + m.phys(j)) * (uint32_t)sizeof(V);
            typedef R r2_t __attribute__((ext_vector_type(2)));
            r2_t t2;
            t2.x = e.x;
            t2.y = e.y;
            __builtin_nontemporal_store(t2, (r2_t *)((char *)dst + off));
        } else if constexpr (OFF32) {
            const uint32_t off = (tp + m.phys(j)) * (uint32_t)sizeof(V);
            *(V *)((char *)dst + off) = e;
        } else {
            dst[tp + m.phys(j)] = e;
        }
    }
}

// Gradient values of one adjoint pass are collected per wave in LDS and
// summed over the block's waves in a fixed order, GCAP ops at a time.
constexpr int kGradCap = 32;

// One gate pass (forward), or one reverse adjoint pass when ADJ: psi and
// lam both get U^dagger of every op in reverse order, and each parametric op
// first records 2 Im <lam|K|psi>.  Its i-th parametric op (in the order the
// pass visits them) writes the block's FP64 sum to gpart[i * ntiles + tile].
// One block per tile: load with the first phase's mapping, run the phases (an
// LDS transpose between consecutive ones), store with the last phase's
// mapping.
template <typename R, int K, int RB, bool ADJ, bool OFF32>
__global__ __launch_bounds__(1 << (K - RB)) void k_gate_pass(
    typename V2T<R>::type *__restrict__ psi, typename V2T<R>::type *__restrict__ lam,
    const PassArgs a, const PhaseDesc *__restrict__ phases, const OpDesc *__restrict__ ops,
    double *__restrict__ gpart, uint32_t ntiles) {
    using V = typename V2T<R>::type;
    constexpr int NR = 1 << RB;
    constexpr int NT = 1 << (K - RB);
    constexpr int NW = NT / 64;
    constexpr int NWB = K - RB - 6;
    __shared__ V lds[1 << K];
    __shared__ double gacc[ADJ ? kGradCap * NW : 1];
    if (blockIdx.x >= ntiles) return;
    // Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD
    // b mod 8); give each XCD one contiguous eighth of the tiles.  Every tile
    // of a gate pass does the same work, so no XCD ends up with more.
    uint32_t tile = blockIdx.x;
    if ((ntiles & 7u) == 0) tile = (blockIdx.x & 7u) * (ntiles >> 3) + (blockIdx.x >> 3);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const int np = a.nphase;
    const PhaseDesc &P0 = phases[a.phase0 + (ADJ ? np - 1 : 0)];   // load mapping
    const PhaseDesc &PL = phases[a.phase0 + (ADJ ? 0 : np - 1)];   // store mapping
    // The pass reads its tile with positions tphys and writes it with
    // tphys_out (a permutation of the same positions); the reverse pass runs
    // it backwards.
    const int32_t *tp_in = ADJ ? a.tphys_out : a.tphys;
    const int32_t *tp_out = ADJ ? a.tphys : a.tphys_out;
    const uint64_t base = spread(tile, a.tphys, K);
    Regs<R, NR> v, w;
    uint32_t sw;
    RegMap<RB, K> mc;
    {
        uint32_t tp0;
        thread_maps<NWB, K>(P0, tp_in, lane, wave, tp0, sw);
        mc.init(P0, tp_in);
        load_regs<V, R, NR, RB, K, OFF32>(v, psi + base, tp0, mc);
        if constexpr (ADJ) load_regs<V, R, NR, RB, K, OFF32>(w, lam + base, tp0, mc);
    }
    // adjoint: ng values pending in gacc, nflushed already written
    int ng = 0, nflushed = 0;
    auto flush = [&]() {
        __syncthreads();
        if ((int)threadIdx.x < ng) {
            double sum = 0.0;
#pragma unroll
            for (int wv = 0; wv < NW; ++wv) sum += gacc[threadIdx.x * NW + wv];
            gpart[(size_t)(nflushed + threadIdx.x) * ntiles + tile] = sum;
        }
        nflushed += ng;
        ng = 0;
        __syncthreads();
    };
    for (int s = 0; s < np; ++s) {
        const PhaseDesc &Pc = phases[a.phase0 + (ADJ ? np - 1 - s : s)];
        if (s > 0) {
            // transpose through LDS: write with the old mapping, read with the
            // new.  The reverse pass moves psi and then lam through the same
            // tile buffer (half the LDS of two buffers: more blocks per CU).
            const uint32_t swo = sw;
            const RegMap<RB, K> mo = mc;
            uint32_t tpx;
            thread_maps<NWB, K>(Pc, a.tphys, lane, wave, tpx, sw);
            mc.init(Pc, a.tphys);
            auto transpose = [&](Regs<R, NR> &r) {
                __syncthreads();
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    V e;
                    e.x = r.re[j];
                    e.y = r.im[j];
                    lds[swo ^ mo.slot(j)] = e;
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const V e = lds[sw ^ mc.slot(j)];
                    r.re[j] = e.x;
                    r.im[j] = e.y;
                }
            };
            transpose(v);
            if constexpr (ADJ) transpose(w);
        }
        const int nop = Pc.nop;
        const int op0 = Pc.op0;
        for (int q = 0; q < nop; ++q) {
            const OpDesc &o = ops[op0 + (ADJ ? nop - 1 - q : q)];
            if constexpr (ADJ) {
                if (o.gtype != GEN_NONE) {
                    const double gv = wave_sum(op_gradient<R, NR, RB>(v, w, o));
                    if (lane == 0) gacc[ng * NW + wave] = gv;
                    if (++ng == kGradCap) flush();
                }
                apply_op<R, NR, RB>(w, o);
            }
            apply_op<R, NR, RB>(v, o);
        }
    }
    uint32_t tpL, tsL;
    thread_maps<NWB, K>(PL, tp_out, lane, wave, tpL, tsL);
    (void)tsL;
    RegMap<RB, K> mL;
    mL.init(PL, tp_out);
    store_regs<V, R, NR, RB, K, OFF32>(v, psi + base, tpL, mL);
    if constexpr (ADJ) {
        store_regs<V, R, NR, RB, K, OFF32>(w, lam + base, tpL, mL);
        if (ng) flush();
    }
}

// ---------------------------------------------------------------------------
// qubit reordering: in-place involution on physical bit positions
// ---------------------------------------------------------------------------

// Swap the bit pairs pairs[0..np) of x (at most MAXP pairs; the loop bound
// is a compile-time constant so the kernel-argument array stays in SGPRs).
template <int MAXP>
__device__ __forceinline__ uint64_t apply_pairs(uint64_t x, const int8_t *pairs, int np) {
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
        if (i < np) {
            const int a = pairs[2 * i], b = pairs[2 * i + 1];
            const uint64_t d = ((x >> a) ^ (x >> b)) & 1ULL;
            x ^= (d << a) | (d << b);
        }
    }
    return x;
}

// No exchanged bit below 6: rows of 64 consecutive elements map to rows, so
// a wave swaps row r with row pi(r) (once, from the smaller side) with fully
// coalesced loads and stores.  Each wave owns U consecutive rows, so that 2U
// loads are in flight before the first store; one launch covers every row.
// 16-byte amplitudes stream with non-temporal accesses (reorder passes and
// tile staging, as in the complex128 gate pass); 8-byte ones use plain
// accesses (their non-temporal stores are several times slower).
template <typename V>
__device__ __forceinline__ V ld_amp(const V *p) {
    if constexpr (sizeof(V) == 16) {
        typedef double d2_t __attribute__((ext_vector_type(2)));
        const d2_t t = __builtin_nontemporal_load((const d2_t *)p);
        V v;
        v.x = t.x;
        v.y = t.y;
        return v;
    } else {
        return *p;
    }
}
template <typename V>
__device__ __forceinline__ void st_amp(V *p, const V &v) {
    if constexpr (sizeof(V) == 16) {
        typedef double d2_t __attribute__((ext_vector_type(2)));
        d2_t t;
        t.x = v.x;
        t.y = v.y;
        __builtin_nontemporal_store(t, (d2_t *)p);
    } else {
        *p = v;
    }
}

template <typename V, int U>
__global__ __launch_bounds__(256) void k_qr_rows(V *__restrict__ psi, const QrArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    // Let h be the highest exchanged row bit and l its partner.  A row with
    // bits (h, l) = (1, 0) is the larger side of its pair, so rows are
    // enumerated as those with h = 0 (the first half), then those with
    // h = l = 1 (a quarter): three quarters of the rows, no wave idle on the
    // (1, 0) quarter.
    // Row indices have n - 6 <= 28 bits, so all index work is 32-bit.
    const uint32_t nrows = (uint32_t)a.nrows;
    const uint32_t nhalf = nrows >> 1, nenum = nhalf + (nrows >> 2);
    const int h = a.hbit, l = a.lbit;
    const uint32_t r0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * U;
    V x[U], y[U];
    uint64_t ra[U], rb[U];
    bool act[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t i = r0 + u;
        uint32_t r;
        if (i < nhalf) {
            r = ((i >> h) << (h + 1)) | (i & ((1u << h) - 1u));
        } else {
            const uint32_t j = i - nhalf;
            const uint32_t t = ((j >> l) << (l + 1)) | (1u << l) | (j & ((1u << l) - 1u));
            r = ((t >> h) << (h + 1)) | (1u << h) | (t & ((1u << h) - 1u));
        }
        // the partner row: every exchanged pair is of physical bits >= 6
        uint32_t pr = r;
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if (q < a.nouter) {
                const int pa = a.outer[2 * q] - 6, pb = a.outer[2 * q + 1] - 6;
                const uint32_t d = ((pr >> pa) ^ (pr >> pb)) & 1u;
                pr ^= (0u - d) & ((1u << pa) | (1u << pb));
            }
        }
        act[u] = i < nenum && r < pr;
        ra[u] = ((uint64_t)r << 6) | lane;
        rb[u] = ((uint64_t)pr << 6) | lane;
        if (act[u]) {
            x[u] = ld_amp(psi + ra[u]);
            y[u] = ld_amp(psi + rb[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (act[u]) {
            st_amp(psi + ra[u], y[u]);
            st_amp(psi + rb[u], x[u]);
        }
    }
}

// General case: a tile T of TB bits holds the low bits, their partners and
// further unpaired bits; pi maps tile b to tile pi(b) and permutes inside the
// tile.  One block per tile; the block of the smaller tile of a pair (b, pi(b))
// swaps the two through LDS so that loads and stores both walk the low bits
// contiguously, the other block exits at once.
template <typename V, int TB>
__global__ __launch_bounds__(256) void k_qr_tiles(V *__restrict__ psi, const QrArgs a) {
    constexpr int TS = 1 << TB;
    constexpr int E = TS / 256;
    __shared__ V l0[TS], l1[TS];
    // With outer pairs, tiles are enumerated like the rows of k_qr_rows: the
    // highest outer bit h = 0 (first half), then h = l = 1 (a quarter).
    uint64_t tile = blockIdx.x;
    if (a.nouter) {
        const uint64_t nhalf = a.ntiles >> 1;
        if (tile >= nhalf + (a.ntiles >> 2)) return;
        const int h = a.hbit, l = a.lbit;
        if (tile < nhalf) {
            tile = ((tile >> h) << (h + 1)) | (tile & ((1ULL << h) - 1));
        } else {
            const uint64_t j = tile - nhalf;
            const uint64_t t = ((j >> l) << (l + 1)) | (1ULL << l) | (j & ((1ULL << l) - 1));
            tile = ((t >> h) << (h + 1)) | (1ULL << h) | (t & ((1ULL << h) - 1));
        }
    } else if (tile >= a.ntiles) {
        return;
    }
    const uint64_t b = spread(tile, a.tphys, TB);
    const uint64_t pb = apply_pairs<32>(b, a.outer, a.nouter);
    if (pb < b) return;
    if (pb == b && a.ninner == 0) return;
    uint64_t off[E];
    uint32_t perm[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t t = threadIdx.x + 256u * e;
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < TB; ++j)
            if ((t >> j) & 1) o |= 1ULL << a.tphys[j];
        off[e] = o;
        perm[e] = (uint32_t)apply_pairs<16>(t, a.inner, a.ninner);
    }
    V x[E], y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        x[e] = ld_amp(psi + b + off[e]);
        if (pb != b) y[e] = ld_amp(psi + pb + off[e]);
    }
    // LDS slot of tile element i: the element bits above one bank row
    // (256 bytes) are folded into the bits below it.  An in-tile transposition
    // sends neighbouring lanes to elements 2^j apart, which would otherwise
    // hit the same banks.
    constexpr int SH = sizeof(V) == 8 ? 5 : 4;
    auto slot = [](uint32_t i) { return i ^ ((i >> SH) & ((1u << SH) - 1u)); };
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = slot(perm[e]);
        l0[q] = x[e];
        if (pb != b) l1[q] = y[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t t = threadIdx.x + 256u * e;
        const uint32_t q = slot(t);
        st_amp(psi + pb + off[e], l0[q]);
        if (pb != b) st_amp(psi + b + off[e], l1[q]);
    }
}

// ---------------------------------------------------------------------------
// Pauli expectation pass
// ---------------------------------------------------------------------------

// In-place Walsh-Hadamard transform: out[s] = sum_j (-1)^{popcount(j&s)} in[j].
template <typename R, int N>
__device__ __forceinline__ void wht(R *x) {
#pragma unroll
    for (int h = 1; h < N; h <<= 1)
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (!(j & h)) {
                const R a = x[j], b = x[j | h];
                x[j] = a + b;
                x[j | h] = a - b;
            }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    return s;
}

// Stage one tile into LDS: every thread issues all of its loads before the
// first LDS write.  Thread bits are the tile's low bits (coalesced); the
// offsets of the high part are uniform.  16-byte amplitudes are read with
// non-temporal loads.
template <typename V, int K, int TPB, typename TI>
__device__ __forceinline__ void stage_tile(V *lds, const V *__restrict__ src, const TI *tphys) {
    constexpr int NT = 1 << TPB;
    constexpr int E = 1 << (K - TPB);
    const uint32_t tid = threadIdx.x;
    uint32_t tp = 0;
#pragma unroll
    for (int b = 0; b < TPB; ++b) tp |= ((tid >> b) & 1u) << tphys[b];
    V x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uint32_t hp = 0;
#pragma unroll
        for (int b = 0; b < K - TPB; ++b)
            if ((e >> b) & 1) hp |= 1u << tphys[TPB + b];
        x[e] = ld_amp(src + tp + hp);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) lds[tid + NT * e] = x[e];
}

// v with its sign flipped when bit 0 of par is set (an XOR of the sign bit).
__device__ __forceinline__ float neg_if_odd(float v, uint32_t par) {
    return __uint_as_float(__float_as_uint(v) ^ (par << 31));
}
__device__ __forceinline__ double neg_if_odd(double v, uint32_t par) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)((uint64_t)par << 63));
}

template <typename R, int K>
__global__ __launch_bounds__(1 << evc_tpb(K, sizeof(R) == 8)) void k_evc_pass(
    const typename V2T<R>::type *__restrict__ psi, const EvcPassArgs a,
    const EvcGroup *__restrict__ groups, const EvcTerm *__restrict__ terms,
    double *__restrict__ partials) {
    using V = typename V2T<R>::type;
    constexpr int TPB = evc_tpb(K, sizeof(R) == 8);
    constexpr int NT = 1 << TPB;
    constexpr int TS = 1 << K;
    constexpr int Q = K - 1 - TPB;
    constexpr int NQ = 1 << Q;
    static_assert(K <= kEvcWiShift && Q + 1 <= 32 - kEvcWiShift, "EvcTerm::ztw fields overlap");
    __shared__ V lds[TS];
    __shared__ double red[NT / 64];
    const uint64_t base = spread(blockIdx.x, a.tphys, K);
    const uint32_t blk = blockIdx.x;
    stage_tile<V, K, TPB, int8_t>(lds, psi + base, a.tphys);
    __syncthreads();
    double acc = 0.0;
    const char *lb = (const char *)lds;
    // A pass's groups hold consecutive term ranges, so each group's first
    // term follows from the previous group's count.
    int tcur = a.ngroups > 0 ? groups[a.group0].t0 : 0;
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const EvcGroup &G = groups[a.group0 + gi];
        // every descriptor field and the group's first four terms first
        // (scalar loads share the LDS counter: a scalar load between LDS
        // reads would drain them)
        const uint32_t xl = G.xl;
        const int hb = G.hbit;
        const int need = G.need;
        const int nt = G.nt;
        int wb[Q > 0 ? Q : 1];
#pragma unroll
        for (int b = 0; b < Q; ++b) wb[b] = G.wbits[b];
        EvcTerm T0[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) T0[u] = terms[tcur + u];
        // pin the term loads here, so that one wait covers them and the
        // descriptor (left alone, the compiler sinks them to their use)
#pragma unroll
        for (int u = 0; u < 4; ++u) asm volatile("" ::"s"(T0[u].coef), "s"(T0[u].ztw), "s"(T0[u].zb));
        asm volatile("" ::"s"(nt));
        // The thread-index bits are the lowest TPB tile bits other than the
        // half-space bit hb (the group layout the planner builds), so the
        // thread's tile index is threadIdx.x with a zero inserted at hb.
        const uint32_t tid = threadIdx.x;
        const uint32_t tt = tid + (tid & ~((1u << hb) - 1u));
        uint32_t tt8 = tt * (uint32_t)sizeof(V);
        // keep the byte offset opaque: otherwise (tt8 | wo8) is rewritten as
        // (tt | wo) * 8, one extra shift per LDS address
        asm volatile("" : "+v"(tt8));
        R w[2 * NQ];   // [0, NQ): real / sum array, [NQ, 2NQ): imaginary / difference
        R *re = w, *im = w + NQ;
        V x[NQ], y[NQ];
        if (xl) {
            const uint32_t xl8 = xl * (uint32_t)sizeof(V);
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) {
                uint32_t wo = 0;
#pragma unroll
                for (int b = 0; b < Q; ++b)
                    if ((jj >> b) & 1) wo |= 1u << wb[b];
                const uint32_t j8 = tt8 | (wo * (uint32_t)sizeof(V));
                x[jj] = *(const V *)(lb + j8);
                y[jj] = *(const V *)(lb + (j8 ^ xl8));
            }
            // w = conj(psi_{j^x}) psi_j; the imaginary part only when a term
            // of the group reads it (an odd number of Y)
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) re[jj] = y[jj].x * x[jj].x + y[jj].y * x[jj].y;
            if (need & 2) {
#pragma unroll
                for (int jj = 0; jj < NQ; ++jj) im[jj] = y[jj].x * x[jj].y - y[jj].y * x[jj].x;
            }
        } else {
            const uint32_t hm8 = (1u << hb) * (uint32_t)sizeof(V);
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) {
                uint32_t wo = 0;
#pragma unroll
                for (int b = 0; b < Q; ++b)
                    if ((jj >> b) & 1) wo |= 1u << wb[b];
                const uint32_t j8 = tt8 | (wo * (uint32_t)sizeof(V));
                x[jj] = *(const V *)(lb + j8);
                y[jj] = *(const V *)(lb + (j8 | hm8));
            }
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) {
                const R n0 = x[jj].x * x[jj].x + x[jj].y * x[jj].y;
                const R n1 = y[jj].x * y[jj].x + y[jj].y * y[jj].y;
                re[jj] = n0 + n1;
                im[jj] = n0 - n1;
            }
        }
        if (need & 1) wht<R, NQ>(re);
        if (need & 2) wht<R, NQ>(im);
        // tt < 2^kEvcWiShift, so the Walsh index in the high bits of ztw
        // drops out of tt & ztw.
        auto term = [&](const EvcTerm &T) {
            const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(T.ztw >> kEvcWiShift));
            const uint32_t par = __builtin_popcount(tt & T.ztw) + __builtin_popcount(blk & T.zb);
            acc += T.coef * (double)neg_if_odd(w[wi], par);
        };
        if (nt >= 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) term(T0[u]);
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u)
                if (u < nt) term(T0[u]);
        }
        // the rest four at a time (one 64-byte scalar load), then one wait
        const int t1 = tcur + nt;
        int ti = tcur + 4;
        for (; ti + 4 <= t1; ti += 4) {
            EvcTerm T[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) T[u] = terms[ti + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) term(T[u]);
        }
        for (; ti < t1; ++ti) term(terms[ti]);
        tcur = t1;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[a.part0 + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// H|psi> pass
// ---------------------------------------------------------------------------

// One H|psi> group's terms, accumulated into the per-thread spectra fr/fi
// (index: the term's cube z bits; sign: the parity of the thread's and the
// tile's z bits).  T0 holds the group's first four terms, loaded with its
// descriptor; the rest are read four at a time.  sthr < 2^kHpsiZwShift, so
// the cube bits in the high part of ztw drop out of sthr & ztw.
template <typename R, int NQ>
__device__ __forceinline__ void hpsi_terms(const HpsiTerm *__restrict__ terms, const HpsiTerm *T0,
                                           int t0, int nt, uint32_t sthr, uint32_t tile, R *fr, R *fi) {
    auto term = [&](const HpsiTerm &T) {
        const uint32_t zw =
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(T.ztw >> kHpsiZwShift)) & (NQ - 1);
        const uint32_t par = __builtin_popcount(sthr & T.ztw) + __builtin_popcount(tile & T.zb);
        R ar, ai;
        if constexpr (sizeof(R) == 4) {
            ar = T.are_f;
            ai = T.aim_f;
        } else {
            ar = T.are;
            ai = T.aim;
        }
        fr[zw] += neg_if_odd(ar, par);
        fi[zw] += neg_if_odd(ai, par);
    };
    if (nt >= 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) term(T0[u]);
    } else {
#pragma unroll
        for (int u = 0; u < 3; ++u)
            if (u < nt) term(T0[u]);
    }
    const int t1 = t0 + nt;
    int ti = t0 + 4;
    for (; ti + 4 <= t1; ti += 4) {
        HpsiTerm T[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) T[u] = terms[ti + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) term(T[u]);
    }
    for (; ti < t1; ++ti) term(terms[ti]);
}

// The first four terms of a group (the term table ends in four zero terms,
// so these loads stay inside it), pinned next to the descriptor loads so
// that one wait covers both.
template <typename R>
__device__ __forceinline__ void hpsi_first_terms(const HpsiTerm *__restrict__ terms, int t0,
                                                 HpsiTerm *T0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) T0[u] = terms[t0 + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if constexpr (sizeof(R) == 4)
            asm volatile("" ::"s"(T0[u].are_f), "s"(T0[u].aim_f), "s"(T0[u].ztw), "s"(T0[u].zb));
        else
            asm volatile("" ::"s"(T0[u].are), "s"(T0[u].aim), "s"(T0[u].ztw), "s"(T0[u].zb));
    }
}

template <typename R, int K>
__global__ __launch_bounds__(1 << hpsi_tpb(K)) void k_hpsi_pass(
    const typename V2T<R>::type *__restrict__ psi, typename V2T<R>::type *__restrict__ lam,
    const HpsiPassArgs a, const HpsiGroup *__restrict__ groups, const HpsiTerm *__restrict__ terms) {
    using V = typename V2T<R>::type;
    constexpr int TPB = hpsi_tpb(K);
    constexpr int NT = 1 << TPB;
    constexpr int TS = 1 << K;
    constexpr int QH = K - TPB;
    constexpr int NQ = 1 << QH;
    __shared__ V lds[TS];
    const uint64_t base = spread(blockIdx.x, a.tphys, K);
    stage_tile<V, K, TPB, int8_t>(lds, psi + base, a.tphys);
    __syncthreads();
    double lr[NQ], li[NQ];
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) lr[jj] = li[jj] = 0.0;
    const uint32_t tid = threadIdx.x;
    // a pass's groups hold consecutive term ranges
    int tcur = a.ngroups > 0 ? groups[a.group0].t0 : 0;
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const HpsiGroup &G = groups[a.group0 + gi];
        const uint32_t xt = G.xt;
        const int nt = G.nt;
        HpsiTerm T0[4];
        hpsi_first_terms<R>(terms, tcur, T0);
        asm volatile("" ::"s"(xt), "s"(nt));
        const uint32_t sthr = tid ^ xt;
        R fr[NQ], fi[NQ];
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj) fr[jj] = fi[jj] = (R)0;
        hpsi_terms<R, NQ>(terms, T0, tcur, nt, sthr, blockIdx.x, fr, fi);
        tcur += nt;
        wht<R, NQ>(fr);
        wht<R, NQ>(fi);
        // The planner folded (-1)^(zw . xw) into each term's coefficient, so
        // the transform's output jj is the spectrum at the source's cube
        // index jj ^ xw (an XOR shift): the spectra are indexed at compile
        // time and only the LDS address depends on xw.  Reads in batches of
        // up to eight, all issued before their products.
        const uint32_t xw = (uint32_t)__builtin_amdgcn_readfirstlane((int)G.xw);
        constexpr int PB = NQ < 8 ? NQ : 8;   // reads per batch
#pragma unroll
        for (int j0 = 0; j0 < NQ; j0 += PB) {
            V p[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) p[u] = lds[sthr | ((((uint32_t)(j0 + u)) ^ xw) & (NQ - 1)) << TPB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int jj = j0 + u;
                lr[jj] += (double)(fr[jj] * p[u].x - fi[jj] * p[u].y);
                li[jj] += (double)(fr[jj] * p[u].y + fi[jj] * p[u].x);
            }
        }
    }
    uint32_t tpo = 0;
#pragma unroll
    for (int b = 0; b < TPB; ++b) tpo |= ((tid >> b) & 1u) << a.tphys[b];
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) {
        uint32_t hp = 0;
#pragma unroll
        for (int b = 0; b < QH; ++b)
            if ((jj >> b) & 1) hp |= 1u << a.tphys[TPB + b];
        const uint64_t off = tpo + hp;
        V o;
        if (a.accumulate) {
            const V prev = lam[base + off];
            o.x = (R)((double)prev.x + lr[jj]);
            o.y = (R)((double)prev.y + li[jj]);
        } else {
            o.x = (R)lr[jj];
            o.y = (R)li[jj];
        }
        lam[base + off] = o;
    }
}

// ---------------------------------------------------------------------------
// wide Pauli strings (flip masks that fit no tile): direct evaluation
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(256) void k_evc_direct(const typename V2T<R>::type *__restrict__ psi,
                                                     uint64_t N, const WideTerm *__restrict__ wt,
                                                     int nw, double *__restrict__ partials) {
    __shared__ double red[4];
    double acc = 0.0;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < N;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const auto x = psi[j];
        for (int t = 0; t < nw; ++t) {
            const auto p = psi[j ^ wt[t].x];
            // conj(psi_{j^x}) psi_j i^{nY} (-1)^{popcount(j & z)}
            const double wr = (double)p.x * x.x + (double)p.y * x.y;
            const double wi = (double)p.x * x.y - (double)p.y * x.x;
            const double sg = (__builtin_popcountll(j & wt[t].z) & 1) ? -1.0 : 1.0;
            // real part of i^{nY} w
            double v;
            switch (wt[t].ny & 3) {
            case 0: v = wr; break;
            case 1: v = -wi; break;
            case 2: v = -wr; break;
            default: v = wi; break;
            }
            acc += wt[t].coef * sg * v;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename R>
__global__ __launch_bounds__(256) void k_hpsi_direct(const typename V2T<R>::type *__restrict__ psi,
                                                      typename V2T<R>::type *__restrict__ lam,
                                                      uint64_t N, const WideTerm *__restrict__ wt,
                                                      int nw, int accumulate) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < nw; ++t) {
            const uint64_t s = i ^ wt[t].x;
            const auto p = psi[s];
            const double sg = (__builtin_popcountll(s & wt[t].z) & 1) ? -wt[t].coef : wt[t].coef;
            double pr = p.x, pi = p.y, qr, qi;
            switch (wt[t].ny & 3) {
            case 0: qr = pr; qi = pi; break;
            case 1: qr = -pi; qi = pr; break;
            case 2: qr = -pr; qi = -pi; break;
            default: qr = pi; qi = -pr; break;
            }
            ar += sg * qr;
            ai += sg * qi;
        }
        auto o = lam[i];
        if (accumulate) {
            o.x = (R)((double)o.x + ar);
            o.y = (R)((double)o.y + ai);
        } else {
            o.x = (R)ar;
            o.y = (R)ai;
        }
        lam[i] = o;
    }
}

// ---------------------------------------------------------------------------
// reductions and small helpers
// ---------------------------------------------------------------------------

// Two-level deterministic reduction of the per-block partials into chunk
// sums.  Level 1: block (c, s) sums, for every pass p in order, the s-th of
// kReduceSplit equal slices of chunk c's blocks in that pass
// (partials[pass_off[p] + c * per_chunk + j]); level 2: chunk_out[c] = sum over
// s of the level-1 values, in order of s.
constexpr int kReduceSplit = 64;

__global__ __launch_bounds__(256) void k_reduce_chunks_a(const double *__restrict__ partials,
                                                          const int *__restrict__ pass_off,
                                                          const int *__restrict__ pass_nblk, int npass,
                                                          int nchunk, double *__restrict__ tmp) {
    __shared__ double red[4];
    const int c = blockIdx.x / kReduceSplit, sl = blockIdx.x % kReduceSplit;
    double acc = 0.0;
    for (int p = 0; p < npass; ++p) {
        const int per_chunk = pass_nblk[p] / nchunk;
        const int j0 = (int)(((long long)per_chunk * sl) / kReduceSplit);
        const int j1 = (int)(((long long)per_chunk * (sl + 1)) / kReduceSplit);
        const double *src = partials + pass_off[p] + (size_t)c * per_chunk;
        for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) acc += src[j];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) tmp[blockIdx.x] = s;
}

__global__ void k_reduce_chunks_b(const double *__restrict__ tmp, int nchunk,
                                  double *__restrict__ chunk_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunk) return;
    double s = 0.0;
    for (int i = 0; i < kReduceSplit; ++i) s += tmp[c * kReduceSplit + i];
    chunk_out[c] = s;
}

// out[0] = extra[0..nextra) + sum_c chunk[c], sequentially.
__global__ void k_finish_energy(const double *__restrict__ chunk, int nchunk,
                                const double *__restrict__ extra, int nextra, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += chunk[c];
        for (int e = 0; e < nextra; ++e) s += extra[e];
        out[0] = s;
    }
}

__global__ __launch_bounds__(256) void k_sum(const double *__restrict__ in, int n, double *out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += in[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[0] = s;
}

// Re <a|b> block partials.
template <typename R>
__global__ __launch_bounds__(256) void k_dot_re(const typename V2T<R>::type *__restrict__ a,
                                                 const typename V2T<R>::type *__restrict__ b,
                                                 uint64_t N, double *__restrict__ partials) {
    __shared__ double red[4];
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto x = a[i];
        const auto y = b[i];
        acc += (double)x.x * y.x + (double)x.y * y.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// grad[p] = sum over gates of p (CSR) of sum over their nper partials.
__global__ __launch_bounds__(256) void k_grad_reduce(const double *__restrict__ gpart, int nper,
                                                      const int *__restrict__ pptr,
                                                      const int *__restrict__ pgate,
                                                      double *__restrict__ grad) {
    __shared__ double red[4];
    const int p = blockIdx.x;
    double acc = 0.0;
    for (int e = pptr[p]; e < pptr[p + 1]; ++e) {
        const double *src = gpart + (size_t)pgate[e] * nper;
        for (int j = threadIdx.x; j < nper; j += blockDim.x) acc += src[j];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) grad[p] = s;
}

// Sum of one adjoint pass's block partials over the tiles (fixed order):
// gop[gates[i]] = sum_t gpart[i * ntiles + t].
__global__ __launch_bounds__(256) void k_grad_tiles(const double *__restrict__ gpart,
                                                     uint32_t ntiles, const int *__restrict__ gates,
                                                     double *__restrict__ gop) {
    __shared__ double red[4];
    const double *src = gpart + (size_t)blockIdx.x * ntiles;
    double acc = 0.0;
    for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) acc += src[t];
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) gop[gates[blockIdx.x]] = sum;
}

template <typename V>
__global__ __launch_bounds__(256) void k_fill_basis(V *__restrict__ psi, uint64_t N, uint64_t idx) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        V e;
        e.x = (i == idx) ? 1 : 0;
        e.y = 0;
        psi[i] = e;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static int grid_for(uint64_t N) {
    uint64_t b = (N + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

static int g_num_cu = 0;

static int num_cu() {
    if (g_num_cu == 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            g_num_cu <= 0)
            g_num_cu = 256;
    }
    return g_num_cu;
}

template <typename R, int KK, int RB, bool ADJ>
static hipError_t launch_gate_kr(void *psi, void *lam, const PassArgs &a, const PhaseDesc *ph,
                                 const OpDesc *ops, double *gpart, hipStream_t s) {
    using V = typename V2T<R>::type;
    constexpr int NT = 1 << (KK - RB);
    if constexpr (sizeof(R) * 2 * (ADJ ? 2 : 1) * (1 << KK) > 160 * 1024) {
        return hipErrorInvalidValue;
    } else {
        const uint32_t ntiles = (uint32_t)a.nblocks;
        // in-tile byte offsets stay below 2^(top tile bit + 1) * sizeof(V)
        const bool off32 = ((uint64_t)sizeof(V) << (a.tphys[KK - 1] + 1)) <= (1ull << 32);
        if (off32)
            hipLaunchKernelGGL((k_gate_pass<R, KK, RB, ADJ, true>), dim3(ntiles), dim3(NT), 0, s,
                               (V *)psi, (V *)lam, a, ph, ops, gpart, ntiles);
        else
            hipLaunchKernelGGL((k_gate_pass<R, KK, RB, ADJ, false>), dim3(ntiles), dim3(NT), 0, s,
                               (V *)psi, (V *)lam, a, ph, ops, gpart, ntiles);
        return hipGetLastError();
    }
}

// The plan fixes the register bits: a forward pass runs either its own width
// or (inside sv_grad, on the adjoint's plan) the adjoint's.
template <typename R, int KK, bool ADJ>
static hipError_t launch_gate_k(int rb, void *psi, void *lam, const PassArgs &a,
                                const PhaseDesc *ph, const OpDesc *ops, double *gpart,
                                hipStream_t s) {
    constexpr int RB_OWN = gate_rb(KK, sizeof(R) == 8, ADJ);
    constexpr int RB_ADJ = gate_rb(KK, sizeof(R) == 8, true);
    if (rb == RB_OWN) return launch_gate_kr<R, KK, RB_OWN, ADJ>(psi, lam, a, ph, ops, gpart, s);
    if constexpr (RB_ADJ != RB_OWN) {
        if (rb == RB_ADJ) return launch_gate_kr<R, KK, RB_ADJ, ADJ>(psi, lam, a, ph, ops, gpart, s);
    }
    return hipErrorInvalidValue;
}

template <typename R>
static hipError_t launch_gate_t(int k, int rb, bool adj, void *psi, void *lam, const PassArgs &a,
                                const PhaseDesc *ph, const OpDesc *ops, double *gpart, hipStream_t s) {
#define SVQ_GATE_CASE(KK)                                                                   \
    case KK:                                                                                \
        return adj ? launch_gate_k<R, KK, true>(rb, psi, lam, a, ph, ops, gpart, s)         \
                   : launch_gate_k<R, KK, false>(rb, psi, lam, a, ph, ops, gpart, s);
    switch (k) {
        SVQ_GATE_CASE(8)
        SVQ_GATE_CASE(9)
        SVQ_GATE_CASE(10)
        SVQ_GATE_CASE(11)
        SVQ_GATE_CASE(12)
        SVQ_GATE_CASE(13)
    default:
        return hipErrorInvalidValue;
    }
#undef SVQ_GATE_CASE
}

hipError_t launch_gate_pass(bool dbl, int k, int rb, bool adj, void *psi, void *lam,
                            const PassArgs &a, const PhaseDesc *ph, const OpDesc *ops,
                            double *gpart, int nbt, hipStream_t s) {
    (void)nbt;
    return dbl ? launch_gate_t<double>(k, rb, adj, psi, lam, a, ph, ops, gpart, s)
               : launch_gate_t<float>(k, rb, adj, psi, lam, a, ph, ops, gpart, s);
}

hipError_t launch_qr(bool dbl, void *psi, const QrArgs &a, hipStream_t s) {
    if (a.rows_path) {
        constexpr int U = 4;
        const uint64_t nb = ((a.nrows >> 1) + (a.nrows >> 2) + 4 * U - 1) / (4 * U);
        if (nb > 0x7fffffffULL) return hipErrorInvalidValue;
        if (dbl) hipLaunchKernelGGL((k_qr_rows<double2, U>), dim3((uint32_t)nb), dim3(256), 0, s, (double2 *)psi, a);
        else hipLaunchKernelGGL((k_qr_rows<float2, U>), dim3((uint32_t)nb), dim3(256), 0, s, (float2 *)psi, a);
        return hipGetLastError();
    }
    if (a.ntiles > 0x7fffffffULL) return hipErrorInvalidValue;
    const uint32_t g2 = (uint32_t)(a.nouter ? (a.ntiles >> 1) + (a.ntiles >> 2) : a.ntiles);
#define SVQ_QR_TB(TBV)                                                                                    \
    case TBV:                                                                                             \
        if (dbl) hipLaunchKernelGGL((k_qr_tiles<double2, TBV>), dim3(g2), dim3(256), 0, s, (double2 *)psi, a); \
        else hipLaunchKernelGGL((k_qr_tiles<float2, TBV>), dim3(g2), dim3(256), 0, s, (float2 *)psi, a);       \
        break;
    switch (a.tbits) {
        SVQ_QR_TB(8)
        SVQ_QR_TB(9)
        SVQ_QR_TB(10)
    default:
        return hipErrorInvalidValue;
    }
#undef SVQ_QR_TB
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_evc_t(int k, const void *psi, const EvcPassArgs &a, const EvcGroup *g,
                               const EvcTerm *t, double *part, hipStream_t s) {
    using V = typename V2T<R>::type;
    const V *p = (const V *)psi;
    constexpr bool D = sizeof(R) == 8;
#define SVQ_EVC_CASE(KK)                                                                          \
    case KK:                                                                                      \
        if constexpr (sizeof(V) * (1 << KK) <= 128 * 1024)                                        \
            hipLaunchKernelGGL((k_evc_pass<R, KK>), dim3(a.nblocks), dim3(1 << evc_tpb(KK, D)),   \
                               0, s, p, a, g, t, part);                                           \
        else                                                                                      \
            return hipErrorInvalidValue;                                                          \
        break;
    switch (k) {
        SVQ_EVC_CASE(8)
        SVQ_EVC_CASE(9)
        SVQ_EVC_CASE(10)
        SVQ_EVC_CASE(11)
        SVQ_EVC_CASE(12)
        SVQ_EVC_CASE(13)
        SVQ_EVC_CASE(14)
    default:
        return hipErrorInvalidValue;
    }
#undef SVQ_EVC_CASE
    return hipGetLastError();
}

hipError_t launch_evc_pass(bool dbl, int k, const void *psi, const EvcPassArgs &a,
                           const EvcGroup *g, const EvcTerm *t, double *part, hipStream_t s) {
    return dbl ? launch_evc_t<double>(k, psi, a, g, t, part, s)
               : launch_evc_t<float>(k, psi, a, g, t, part, s);
}

template <typename R>
static hipError_t launch_hpsi_t(int k, int nblocks, const void *psi, void *lam,
                                const HpsiPassArgs &a, const HpsiGroup *g, const HpsiTerm *t,
                                hipStream_t s) {
    using V = typename V2T<R>::type;
    const V *p = (const V *)psi;
    V *l = (V *)lam;
#define SVQ_HPSI_CASE(KK)                                                                      \
    case KK:                                                                                   \
        hipLaunchKernelGGL((k_hpsi_pass<R, KK>), dim3(nblocks), dim3(1 << hpsi_tpb(KK)), 0, s, \
                           p, l, a, g, t);                                                     \
        break;
    switch (k) {
        SVQ_HPSI_CASE(8)
        SVQ_HPSI_CASE(9)
        SVQ_HPSI_CASE(10)
        SVQ_HPSI_CASE(11)
        SVQ_HPSI_CASE(12)
        SVQ_HPSI_CASE(13)
    default:
        return hipErrorInvalidValue;
    }
#undef SVQ_HPSI_CASE
    return hipGetLastError();
}

hipError_t launch_hpsi_pass(bool dbl, int k, int nblocks, const void *psi, void *lam,
                            const HpsiPassArgs &a, const HpsiGroup *g, const HpsiTerm *t,
                            hipStream_t s) {
    return dbl ? launch_hpsi_t<double>(k, nblocks, psi, lam, a, g, t, s)
               : launch_hpsi_t<float>(k, nblocks, psi, lam, a, g, t, s);
}

int direct_grid(uint64_t N) { return grid_for(N) > 1024 ? 1024 : grid_for(N); }

hipError_t launch_evc_direct(bool dbl, const void *psi, uint64_t N, const WideTerm *wt, int nw,
                             double *part, hipStream_t s) {
    const int g = direct_grid(N);
    if (dbl) hipLaunchKernelGGL(k_evc_direct<double>, dim3(g), dim3(256), 0, s, (const double2 *)psi, N, wt, nw, part);
    else hipLaunchKernelGGL(k_evc_direct<float>, dim3(g), dim3(256), 0, s, (const float2 *)psi, N, wt, nw, part);
    return hipGetLastError();
}

hipError_t launch_hpsi_direct(bool dbl, const void *psi, void *lam, uint64_t N, const WideTerm *wt,
                              int nw, int accumulate, hipStream_t s) {
    const int g = grid_for(N);
    if (dbl) hipLaunchKernelGGL(k_hpsi_direct<double>, dim3(g), dim3(256), 0, s, (const double2 *)psi, (double2 *)lam, N, wt, nw, accumulate);
    else hipLaunchKernelGGL(k_hpsi_direct<float>, dim3(g), dim3(256), 0, s, (const float2 *)psi, (float2 *)lam, N, wt, nw, accumulate);
    return hipGetLastError();
}

int reduce_scratch(int nchunk) { return nchunk * kReduceSplit; }

hipError_t launch_reduce_chunks(const double *partials, const int *pass_off, const int *pass_nblk,
                                int npass, int nchunk, double *tmp, double *chunk_out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_chunks_a, dim3(nchunk * kReduceSplit), dim3(256), 0, s, partials,
                       pass_off, pass_nblk, npass, nchunk, tmp);
    hipLaunchKernelGGL(k_reduce_chunks_b, dim3((nchunk + 63) / 64), dim3(64), 0, s, tmp, nchunk,
                       chunk_out);
    return hipGetLastError();
}

hipError_t launch_finish_energy(const double *chunk, int nchunk, const double *extra, int nextra,
                                double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(64), 0, s, chunk, nchunk, extra, nextra, out);
    return hipGetLastError();
}

hipError_t launch_sum(const double *in, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

int dot_grid(uint64_t N) { return direct_grid(N); }

hipError_t launch_dot_re(bool dbl, const void *a, const void *b, uint64_t N, double *partials,
                         hipStream_t s) {
    const int g = dot_grid(N);
    if (dbl) hipLaunchKernelGGL(k_dot_re<double>, dim3(g), dim3(256), 0, s, (const double2 *)a, (const double2 *)b, N, partials);
    else hipLaunchKernelGGL(k_dot_re<float>, dim3(g), dim3(256), 0, s, (const float2 *)a, (const float2 *)b, N, partials);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double *gpart, int nper, const int *pptr, const int *pgate,
                              int nparam, double *grad, hipStream_t s) {
    if (nparam == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_reduce, dim3(nparam), dim3(256), 0, s, gpart, nper, pptr, pgate, grad);
    return hipGetLastError();
}

// Plain streaming copy (16-byte accesses): the reference for achievable
// bandwidth and for calibrating the HBM traffic counters.
// One 16-byte element per thread over a grid that covers the whole range
// (the fastest of the plain copy shapes measured: grid-stride loops and
// several elements per thread came out slower).
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                              uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    const uint64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const uint64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffffULL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)grid), dim3(256), 0, s, (const float4 *)src, (float4 *)dst, n);
    return hipGetLastError();
}

// grad[p] = sum over e in [ptr[p], ptr[p+1]) of coef[e] * evals[e] (fixed order).
__global__ __launch_bounds__(64) void k_shift_combine(const double *__restrict__ evals,
                                                       const double *__restrict__ coef,
                                                       const int *__restrict__ ptr, int nparam,
                                                       double *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nparam) return;
    double acc = 0.0;
    for (int e = ptr[p]; e < ptr[p + 1]; ++e) acc += coef[e] * evals[e];
    grad[p] = acc;
}

hipError_t launch_shift_combine(const double *evals, const double *coef, const int *ptr, int nparam,
                                double *grad, hipStream_t s) {
    if (nparam == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shift_combine, dim3((nparam + 63) / 64), dim3(64), 0, s, evals, coef, ptr,
                       nparam, grad);
    return hipGetLastError();
}

hipError_t launch_grad_tiles(const double *gpart, uint32_t ntiles, int nslots, const int *gates,
                             double *gop, hipStream_t s) {
    if (nslots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_tiles, dim3(nslots), dim3(256), 0, s, gpart, ntiles, gates, gop);
    return hipGetLastError();
}

hipError_t launch_fill_basis(bool dbl, void *psi, uint64_t N, uint64_t idx, hipStream_t s) {
    const int g = grid_for(N);
    if (dbl) hipLaunchKernelGGL(k_fill_basis<double2>, dim3(g), dim3(256), 0, s, (double2 *)psi, N, idx);
    else hipLaunchKernelGGL(k_fill_basis<float2>, dim3(g), dim3(256), 0, s, (float2 *)psi, N, idx);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// batched persistent launch (complex64, 2^10-amplitude tiles, one wave/block)
// ---------------------------------------------------------------------------

namespace batch {

constexpr int K = kBatchK;
constexpr int RB = gate_rb(K);          // 4
constexpr int NR = 1 << RB;             // 16 amplitudes per lane
constexpr int HTPB = hpsi_tpb(K);       // 6
constexpr int HQ = K - HTPB;            // 4
constexpr int HNQ = 1 << HQ;
static_assert((1 << (K - RB)) == 64, "one wave per tile");
static_assert((1 << HTPB) == 64, "one wave per tile");

__device__ __forceinline__ double wave_sum_d(double v) { return wave_sum(v); }

// One gate-pass tile of a batched instance: 2^KT amplitudes on 2^(KT-RB)
// threads (one wave for KT = 10, four for KT = 12), as k_gate_pass does it.
// The reverse pass adds each parametric op's block sum into the op's
// (gate, chunk) slot; with several waves the per-wave sums are collected in
// gacc (gsl holds the slot's gate) and summed in a fixed order.
template <bool ADJ, int KT>
__device__ __forceinline__ void gate_item(const BatchArgs &a, const BatchInst &N, const BatchPass &bp,
                                          uint32_t tile, float2 *lds, double *gacc, int *gsl, int chunk,
                                          bool first) {
    using R = float;
    using V = float2;
    constexpr int RBT = gate_rb(KT);
    constexpr int NRT = 1 << RBT;
    constexpr int NW = 1 << (KT - RBT - 6);
    constexpr int NWB = KT - RBT - 6;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    V *psi = a.arena + N.psi_off;
    V *lam = a.arena + N.lam_off;
    const OpDesc *ops = ADJ ? a.ops_inv : a.ops_fwd;
    const int np = bp.nphase;
    const PhaseDesc &P0 = a.phases[bp.phase0 + (ADJ ? np - 1 : 0)];
    const PhaseDesc &PL = a.phases[bp.phase0 + (ADJ ? 0 : np - 1)];
    const uint64_t base = spread(tile, bp.tphys, KT);
    // instances have at most 26 qubits: in-tile byte offsets fit 32 bits
    Regs<R, NRT> v, w;
    uint32_t sw;
    RegMap<RBT, KT> mc;
    {
        uint32_t tp0;
        thread_maps<NWB, KT>(P0, bp.tphys, lane, wave, tp0, sw);
        mc.init(P0, bp.tphys);
        load_regs<V, R, NRT, RBT, KT, true>(v, psi + base, tp0, mc);
        if constexpr (ADJ) load_regs<V, R, NRT, RBT, KT, true>(w, lam + base, tp0, mc);
    }
    int ng = 0;
    auto flush = [&]() {
        __syncthreads();
        if ((int)threadIdx.x < ng) {
            double sum = 0.0;
#pragma unroll
            for (int wv = 0; wv < NW; ++wv) sum += gacc[threadIdx.x * NW + wv];
            double *slot = a.gpart + N.gpart_off + (size_t)gsl[threadIdx.x] * N.nchunks + chunk;
            *slot = first ? sum : *slot + sum;   // this block owns the slot
        }
        ng = 0;
        __syncthreads();
    };
    for (int s = 0; s < np; ++s) {
        const PhaseDesc &Pc = a.phases[bp.phase0 + (ADJ ? np - 1 - s : s)];
        if (s > 0) {
            // psi, then lam (reverse items), through the one tile buffer
            const uint32_t swo = sw;
            const RegMap<RBT, KT> mo = mc;
            uint32_t tpx;
            thread_maps<NWB, KT>(Pc, bp.tphys, lane, wave, tpx, sw);
            mc.init(Pc, bp.tphys);
            auto transpose = [&](Regs<R, NRT> &r, bool after_read) {
                if (NW == 1 && !after_read) __builtin_amdgcn_wave_barrier();
                else __syncthreads();
#pragma unroll
                for (int j = 0; j < NRT; ++j) lds[swo ^ mo.slot(j)] = make_float2(r.re[j], r.im[j]);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < NRT; ++j) {
                    const V e = lds[sw ^ mc.slot(j)];
                    r.re[j] = e.x;
                    r.im[j] = e.y;
                }
            };
            transpose(v, false);
            if constexpr (ADJ) transpose(w, true);
            if constexpr (NW == 1) __syncthreads();
        }
        const int nop = Pc.nop;
        const int op0 = Pc.op0;
        for (int q = 0; q < nop; ++q) {
            const OpDesc &o = ops[op0 + (ADJ ? nop - 1 - q : q)];
            if constexpr (ADJ) {
                if (o.gtype != GEN_NONE) {
                    const double gv = wave_sum(op_gradient<R, NRT, RBT>(v, w, o));
                    if constexpr (NW == 1) {
                        if (lane == 0) {
                            double *slot = a.gpart + N.gpart_off + (size_t)o.gslot * N.nchunks + chunk;
                            *slot = first ? gv : *slot + gv;   // this block owns the slot
                        }
                    } else {
                        if (lane == 0) gacc[ng * NW + wave] = gv;
                        if (threadIdx.x == 0) gsl[ng] = o.gslot;
                        if (++ng == kGradCap) flush();
                    }
                }
                apply_op<R, NRT, RBT>(w, o);
            }
            apply_op<R, NRT, RBT>(v, o);
        }
    }
    uint32_t tpL, tsL;
    thread_maps<NWB, KT>(PL, bp.tphys, lane, wave, tpL, tsL);
    (void)tsL;
    RegMap<RBT, KT> mL;
    mL.init(PL, bp.tphys);
    store_regs<V, R, NRT, RBT, KT, true>(v, psi + base, tpL, mL);
    if constexpr (ADJ) {
        store_regs<V, R, NRT, RBT, KT, true>(w, lam + base, tpL, mL);
        if constexpr (NW > 1) {
            if (ng) flush();
        }
    }
}

// One H|psi> tile of a batched instance: 2^KH amplitudes on 2^(KH-4)
// threads (one wave for KH = 10, four for KH = 12).
template <int KH>
__device__ __forceinline__ void hpsi_item(const BatchArgs &a, const BatchInst &N, const BatchHPass &hp,
                                          int accumulate, uint32_t tile, float2 *lds) {
    using R = float;
    using V = float2;
    constexpr int HTPB = hpsi_tpb(KH);
    constexpr int HQ = KH - HTPB;
    constexpr int HNQ = 1 << HQ;
    static_assert(HQ == 4, "16 accumulators per thread");
    const float2 *psi = a.arena + N.psi_off;
    float2 *lam = a.arena + N.lam_off;
    const uint64_t base = spread(tile, hp.tphys, KH);
    stage_tile<V, KH, HTPB, int32_t>(lds, psi + base, hp.tphys);
    __syncthreads();
    double lr[HNQ], li[HNQ];
#pragma unroll
    for (int jj = 0; jj < HNQ; ++jj) lr[jj] = li[jj] = 0.0;
    const uint32_t tid = threadIdx.x;
    int tcur = hp.ngroups > 0 ? a.hgroups[hp.group0].t0 : 0;
    for (int gi = 0; gi < hp.ngroups; ++gi) {
        const HpsiGroup &G = a.hgroups[hp.group0 + gi];
        const uint32_t xt = G.xt;
        const int nt = G.nt;
        HpsiTerm T0[4];
        hpsi_first_terms<R>(a.hterms, tcur, T0);
        asm volatile("" ::"s"(xt), "s"(nt));
        const uint32_t sthr = tid ^ xt;
        R fr[HNQ], fi[HNQ];
#pragma unroll
        for (int jj = 0; jj < HNQ; ++jj) fr[jj] = fi[jj] = (R)0;
        hpsi_terms<R, HNQ>(a.hterms, T0, tcur, nt, sthr, tile, fr, fi);
        tcur += nt;
        wht<R, HNQ>(fr);
        wht<R, HNQ>(fi);
        // The planner folded (-1)^(zw . xw) into each term's coefficient, so
        // the transform's output jj is the spectrum at the source's cube
        // index jj ^ xw (an XOR shift): the spectra are indexed at compile
        // time and only the LDS address depends on xw.  Reads in batches of
        // up to eight, all issued before their products.
        const uint32_t xw = (uint32_t)__builtin_amdgcn_readfirstlane((int)G.xw);
        constexpr int PB = HNQ < 8 ? HNQ : 8;   // reads per batch
#pragma unroll
        for (int j0 = 0; j0 < HNQ; j0 += PB) {
            V p[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) p[u] = lds[sthr | ((((uint32_t)(j0 + u)) ^ xw) & (HNQ - 1)) << HTPB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int jj = j0 + u;
                lr[jj] += (double)(fr[jj] * p[u].x - fi[jj] * p[u].y);
                li[jj] += (double)(fr[jj] * p[u].y + fi[jj] * p[u].x);
            }
        }
    }
    uint32_t tpo = 0;
#pragma unroll
    for (int b = 0; b < HTPB; ++b) tpo |= ((tid >> b) & 1u) << hp.tphys[b];
#pragma unroll
    for (int jj = 0; jj < HNQ; ++jj) {
        uint32_t hb = 0;
#pragma unroll
        for (int b = 0; b < HQ; ++b)
            if ((jj >> b) & 1) hb |= 1u << hp.tphys[HTPB + b];
        const uint64_t off = base + tpo + hb;
        V o;
        if (accumulate) {
            const V prev = lam[off];
            o.x = (R)((double)prev.x + lr[jj]);
            o.y = (R)((double)prev.y + li[jj]);
        } else {
            o.x = (R)lr[jj];
            o.y = (R)li[jj];
        }
        lam[off] = o;
    }
    __syncthreads();
}

// Contiguous tile t of an instance: element t * 2^K + j * 64 + lane.
__device__ __forceinline__ void init_item(const BatchArgs &a, const BatchInst &N, uint32_t tile) {
    const uint32_t lane = threadIdx.x & 63u;
    float2 *psi = a.arena + N.psi_off;
    const uint64_t idx0 = ((uint64_t)N.psi0_hi << 32) | N.psi0_lo;
#pragma unroll
    for (int j = 0; j < (1 << K) / 64; ++j) {
        const uint64_t e = ((uint64_t)tile << K) + (uint64_t)j * 64 + lane;
        psi[e] = make_float2(e == idx0 ? 1.f : 0.f, 0.f);
    }
}

__device__ __forceinline__ double dot_tile(const BatchArgs &a, const BatchInst &N, uint32_t tile) {
    const uint32_t lane = threadIdx.x & 63u;
    const float2 *psi = a.arena + N.psi_off;
    const float2 *lam = a.arena + N.lam_off;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < (1 << K) / 64; ++j) {
        const uint64_t e = ((uint64_t)tile << K) + (uint64_t)j * 64 + lane;
        const float2 x = psi[e], y = lam[e];
        acc += (double)x.x * y.x + (double)x.y * y.y;
    }
    return acc;
}

// Final sums of one instance, slots [s0, s0 + ns): slot p < ntheta is
// dE/dtheta_p (its gates' chunk partials), slot ntheta the energy (the
// chunk partials of <psi|H psi>).  Several blocks share an instance's slots.
__device__ __forceinline__ void final_item(const BatchArgs &a, const BatchInst &N, int inst, int s0,
                                           int ns) {
    const uint32_t lane = threadIdx.x & 63u;
    for (int p = s0; p < s0 + ns; ++p) {
        double g = 0.0;
        if (p == N.ntheta) {
            for (int t = lane; t < N.nchunks; t += 64) g += a.epart[N.epart_off + t];
            g = wave_sum(g);
            if (lane == 0) a.energies[inst] = g;
            continue;
        }
        const int e0 = a.pptr[N.pptr_off + p], e1 = a.pptr[N.pptr_off + p + 1];
        for (int q = e0; q < e1; ++q) {
            const double *src = a.gpart + N.gpart_off + (size_t)a.pgate[q] * N.nchunks;
            for (int t = lane; t < N.nchunks; t += 64) g += src[t];
        }
        g = wave_sum(g);
        if (lane == 0) a.grads[N.grad_off + p] = g;
    }
}

// Completion time of an instance: the latest of its final blocks.
__device__ __forceinline__ void stamp_done(const BatchArgs &a, int inst) {
    __hip_atomic_fetch_max(a.t_done + inst, (uint64_t)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace batch

// Persistent work-queue kernel.  Items are stored stage-major (all first
// stages of every instance, then all second stages, ...), so every item a
// block waits for was dequeued earlier by a running block; every wait is
// bounded by spin_limit sleeps, after which the error flag is set and all
// blocks drain.
__global__ __launch_bounds__(64) void k_batch(const BatchArgs a) {
    __shared__ float2 lds[1 << kBatchK];
    const uint32_t lane = threadIdx.x & 63u;
    if (blockIdx.x == 0 && lane == 0) *a.t_start = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        int it = 0;
        if (lane == 0) it = __hip_atomic_fetch_add(a.head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        it = __shfl(it, 0, 64);
        if (it >= a.nitems) break;
        int err = 0;
        if (lane == 0) err = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__shfl(err, 0, 64)) break;
        const BatchItem I = a.items[it];
        const BatchInst &N = a.insts[I.inst];
        const int sidx = N.stage0 + I.stage;
        const BatchStage S = a.stages[sidx];
        if (I.stage > 0) {
            const int need = a.stages[sidx - 1].ntiles;
            int ok = 1;
            if (lane == 0) {
                // spin with relaxed loads (an acquire per iteration would
                // invalidate this XCD's L2 under the working waves), then
                // acquire once
                int spins = 0;
                while (__hip_atomic_load(a.done + sidx - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > a.spin_limit) {
                        __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
            if (!__shfl(ok, 0, 64)) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        double dacc = 0.0;
        for (int k = 0; k < I.ntile; ++k) {
            const uint32_t tile = (uint32_t)(I.tile0 + k);
            switch (S.type) {
            case IT_INIT: batch::init_item(a, N, tile); break;
            case IT_FWD: batch::gate_item<false, kBatchK>(a, N, a.passes[S.desc], tile, lds, nullptr, nullptr, I.chunk, k == 0); break;
            case IT_HPSI: batch::hpsi_item<kBatchK>(a, N, a.hpasses[S.desc], S.accumulate, tile, lds); break;
            case IT_DOT: dacc += batch::dot_tile(a, N, tile); break;
            case IT_ADJ: batch::gate_item<true, kBatchK>(a, N, a.passes[S.desc], tile, lds, nullptr, nullptr, I.chunk, k == 0); break;
            default: batch::final_item(a, N, I.inst, I.tile0, I.ntile); k = I.ntile; break;
            }
        }
        if (S.type == IT_DOT) {
            dacc = wave_sum(dacc);
            if (lane == 0) a.epart[N.epart_off + I.chunk] = dacc;
        }
        if (lane == 0) {
            __hip_atomic_fetch_add(a.done + sidx, I.ntile, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (S.type == IT_FINAL) batch::stamp_done(a, I.inst);
        }
    }
}

// Level-synchronous batch: one launch per (stage level, item type) over the
// items of that level, block b running item item0 + b to the end.  Stream
// order between the launches carries every dependency, so no block waits,
// and each item type gets a kernel of its own (registers and LDS sized for
// that type alone rather than for the largest of all types).  The 2^12
// reverse and H|psi> items are held to four blocks per CU (128 VGPRs, no
// spills; their LDS allows four and five): left alone they take 163 and
// 149 VGPRs, three blocks.  The forward item would spill at 128.
template <int TYPE>
__global__ __launch_bounds__((TYPE == IT_FWD_W || TYPE == IT_ADJ_W || TYPE == IT_HPSI_W) ? 256 : 64,
                             (TYPE == IT_ADJ_W || TYPE == IT_HPSI_W) ? 4 : 1) void
k_batch_stage(const BatchArgs a, int item0) {
    constexpr int NLDS = (TYPE == IT_ADJ_W || TYPE == IT_FWD_W || TYPE == IT_HPSI_W) ? (1 << kBatchKWide)
                       : (TYPE == IT_ADJ || TYPE == IT_FWD || TYPE == IT_HPSI) ? (1 << kBatchK) : 1;
    constexpr int NGW = TYPE == IT_ADJ_W ? kGradCap * 4 : 1;
    __shared__ float2 lds[NLDS];
    __shared__ double gacc[NGW];
    __shared__ int gsl[TYPE == IT_ADJ_W ? kGradCap : 1];
    const uint32_t lane = threadIdx.x & 63u;
    const BatchItem I = a.items[item0 + (int)blockIdx.x];
    const BatchInst &N = a.insts[I.inst];
    const BatchStage S = a.stages[N.stage0 + I.stage];
    double dacc = 0.0;
    for (int k = 0; k < I.ntile; ++k) {
        const uint32_t tile = (uint32_t)(I.tile0 + k);
        if constexpr (TYPE == IT_INIT) batch::init_item(a, N, tile);
        else if constexpr (TYPE == IT_FWD) batch::gate_item<false, kBatchK>(a, N, a.passes[S.desc], tile, lds, gacc, gsl, I.chunk, k == 0);
        else if constexpr (TYPE == IT_FWD_W) batch::gate_item<false, kBatchKWide>(a, N, a.passes[S.desc], tile, lds, gacc, gsl, I.chunk, k == 0);
        else if constexpr (TYPE == IT_ADJ_W) batch::gate_item<true, kBatchKWide>(a, N, a.passes[S.desc], tile, lds, gacc, gsl, I.chunk, k == 0);
        else if constexpr (TYPE == IT_HPSI) batch::hpsi_item<kBatchK>(a, N, a.hpasses[S.desc], S.accumulate, tile, lds);
        else if constexpr (TYPE == IT_HPSI_W) batch::hpsi_item<kBatchKWide>(a, N, a.hpasses[S.desc], S.accumulate, tile, lds);
        else if constexpr (TYPE == IT_DOT) dacc += batch::dot_tile(a, N, tile);
        else if constexpr (TYPE == IT_ADJ) batch::gate_item<true, kBatchK>(a, N, a.passes[S.desc], tile, lds, gacc, gsl, I.chunk, k == 0);
    }
    if constexpr (TYPE == IT_DOT) {
        dacc = wave_sum(dacc);
        if (lane == 0) a.epart[N.epart_off + I.chunk] = dacc;
    }
    if constexpr (TYPE == IT_FINAL) {
        batch::final_item(a, N, I.inst, I.tile0, I.ntile);
        if (lane == 0) batch::stamp_done(a, I.inst);
    }
}

// ---------------------------------------------------------------------------
// batched instances held in one workgroup's LDS
// ---------------------------------------------------------------------------

namespace lds_batch {

// Index of pair/quad p with zeros inserted at the gate's qubits.
__device__ __forceinline__ uint32_t insert0(uint32_t p, int q) {
    const uint32_t lo = p & ((1u << q) - 1u);
    return ((p >> q) << (q + 1)) | lo;
}

__device__ __forceinline__ double block_sum_all(double v, double *red) {
    v = wave_sum(v);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBatchLdsThreads / 64; ++w) s += red[w];
    return s;
}

// One op over the LDS state(s): 1-qubit ops on pairs (register bit 0 on the
// qubit), 2-qubit ops on quads (register bits 0/1 on the first/second
// qubit).  With ADJ the op's gradient term 2 Im <lambda|K|psi> is returned
// (this thread's part) before U^dagger is applied to both.
template <bool ADJ, int NRT, int RBT>
__device__ __forceinline__ double op_on_lds(float2 *psi, float2 *lam, const OpDesc &o, uint32_t S) {
    const int q0 = o.spare, q1 = o.pad;
    double g = 0.0;
    const uint32_t nitems = S >> RBT;
    for (uint32_t p = threadIdx.x; p < nitems; p += kBatchLdsThreads) {
        uint32_t base;
        if constexpr (RBT == 1) {
            base = insert0(p, q0);
        } else {
            const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
            base = insert0(insert0(p, lo), hi);
        }
        uint32_t idx[NRT];
#pragma unroll
        for (int j = 0; j < NRT; ++j) {
            idx[j] = base;
            if (j & 1) idx[j] |= 1u << q0;
            if constexpr (RBT == 2) {
                if (j & 2) idx[j] |= 1u << q1;
            }
        }
        Regs<float, NRT> v, w;
#pragma unroll
        for (int j = 0; j < NRT; ++j) {
            const float2 e = psi[idx[j]];
            v.re[j] = e.x;
            v.im[j] = e.y;
            if constexpr (ADJ) {
                const float2 f = lam[idx[j]];
                w.re[j] = f.x;
                w.im[j] = f.y;
            }
        }
        if constexpr (ADJ) {
            if (o.gtype != GEN_NONE) g += op_gradient<float, NRT, RBT>(v, w, o);
            apply_op<float, NRT, RBT>(w, o);
        }
        apply_op<float, NRT, RBT>(v, o);
#pragma unroll
        for (int j = 0; j < NRT; ++j) {
            psi[idx[j]] = make_float2(v.re[j], v.im[j]);
            if constexpr (ADJ) lam[idx[j]] = make_float2(w.re[j], w.im[j]);
        }
    }
    return g;
}

}  // namespace lds_batch

// One block per instance: psi0, the gates in order, lambda = H psi (FP64 per
// element), E, then the reverse sweep with each parametric gate's gradient
// term summed over the block in a fixed order, and the per-parameter sums.
// psi and lambda stay in LDS throughout.
__global__ __launch_bounds__(kBatchLdsThreads) void k_batch_lds(const BatchArgs a) {
    extern __shared__ float2 smem[];
    __shared__ double red[kBatchLdsThreads / 64];
    const BatchLdsInst L = a.linst[blockIdx.x];
    const uint32_t S = 1u << L.n;
    float2 *psi = smem, *lam = smem + S;
    const WideTerm *terms = (const WideTerm *)a.lterms;
    const uint64_t idx0 = ((uint64_t)L.psi0_hi << 32) | L.psi0_lo;
    for (uint32_t e = threadIdx.x; e < S; e += kBatchLdsThreads)
        psi[e] = make_float2(e == idx0 ? 1.f : 0.f, 0.f);
    __syncthreads();
    for (int gi = 0; gi < L.m; ++gi) {
        const OpDesc &o = a.lops_fwd[L.op0 + gi];
        if (o.pad < 0) (void)lds_batch::op_on_lds<false, 2, 1>(psi, nullptr, o, S);
        else (void)lds_batch::op_on_lds<false, 4, 2>(psi, nullptr, o, S);
        __syncthreads();
    }
    // lambda = H psi and E = Re <psi|lambda>
    double eacc = 0.0;
    for (uint32_t e = threadIdx.x; e < S; e += kBatchLdsThreads) {
        double ar = 0.0, ai = 0.0;
        for (int t = L.t0; t < L.t0 + L.nt; ++t) {
            const WideTerm &T = terms[t];
            const uint32_t src = e ^ (uint32_t)T.x;
            const float2 p = psi[src];
            const double sg = (__builtin_popcount(src & (uint32_t)T.z) & 1) ? -T.coef : T.coef;
            double qr, qi;
            switch (T.ny & 3) {
            case 0: qr = p.x; qi = p.y; break;
            case 1: qr = -p.y; qi = p.x; break;
            case 2: qr = -p.x; qi = -p.y; break;
            default: qr = p.y; qi = -p.x; break;
            }
            ar += sg * qr;
            ai += sg * qi;
        }
        const float2 me = psi[e];
        eacc += (double)me.x * ar + (double)me.y * ai;
        lam[e] = make_float2((float)ar, (float)ai);
    }
    const double E = lds_batch::block_sum_all(eacc, red);
    if (threadIdx.x == 0) a.energies[L.inst] = E;
    __syncthreads();
    for (int gi = L.m - 1; gi >= 0; --gi) {
        const OpDesc &o = a.lops_inv[L.op0 + gi];
        double gp;
        if (o.pad < 0) gp = lds_batch::op_on_lds<true, 2, 1>(psi, lam, o, S);
        else gp = lds_batch::op_on_lds<true, 4, 2>(psi, lam, o, S);
        if (o.gtype != GEN_NONE) {
            const double gsum = lds_batch::block_sum_all(gp, red);
            if (threadIdx.x == 0) a.gvals[L.gv_off + gi] = gsum;
        }
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    for (int p = threadIdx.x; p < L.ntheta; p += kBatchLdsThreads) {
        double g = 0.0;
        for (int q = a.pptr[L.pptr_off + p]; q < a.pptr[L.pptr_off + p + 1]; ++q)
            g += a.gvals[L.gv_off + a.pgate[q]];
        a.grads[L.grad_off + p] = g;
    }
    if (threadIdx.x == 0)
        __hip_atomic_fetch_max(a.t_done + L.inst, (uint64_t)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_batch(const BatchArgs &a, int32_t *counters, int ncounters, hipStream_t s,
                        int *grid_out) {
    // counters = [done..., head, error] in one array; a fill kernel (not a
    // memset) resets them so the sequence can live in a captured graph
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, s, counters, ncounters, 0);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, 64, 0) != hipSuccess || per_cu <= 0)
        per_cu = 4;
    const int grid = per_cu * num_cu();
    if (grid_out) *grid_out = grid;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t prepare_batch_lds(int max_n) {
    const size_t bytes = sizeof(float2) * ((size_t)2 << max_n);
    return hipFuncSetAttribute((const void *)k_batch_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_batch_lds(const BatchArgs &a, int ninst, int max_n, hipStream_t s) {
    if (ninst <= 0) return hipSuccess;
    const size_t bytes = sizeof(float2) * ((size_t)2 << max_n);
    hipLaunchKernelGGL(k_batch_lds, dim3(ninst), dim3(kBatchLdsThreads), bytes, s, a);
    return hipGetLastError();
}

__global__ void k_stamp(uint64_t *t) { *t = __builtin_amdgcn_s_memrealtime(); }

hipError_t launch_stamp(uint64_t *t, hipStream_t s) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_batch_stage(const BatchArgs &a, int type, int item0, int nitem, hipStream_t s) {
    if (nitem <= 0) return hipSuccess;
    switch (type) {
    case IT_INIT: hipLaunchKernelGGL(k_batch_stage<IT_INIT>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_FWD: hipLaunchKernelGGL(k_batch_stage<IT_FWD>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_HPSI: hipLaunchKernelGGL(k_batch_stage<IT_HPSI>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_DOT: hipLaunchKernelGGL(k_batch_stage<IT_DOT>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_ADJ: hipLaunchKernelGGL(k_batch_stage<IT_ADJ>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_FINAL: hipLaunchKernelGGL(k_batch_stage<IT_FINAL>, dim3(nitem), dim3(64), 0, s, a, item0); break;
    case IT_FWD_W: hipLaunchKernelGGL(k_batch_stage<IT_FWD_W>, dim3(nitem), dim3(256), 0, s, a, item0); break;
    case IT_ADJ_W: hipLaunchKernelGGL(k_batch_stage<IT_ADJ_W>, dim3(nitem), dim3(256), 0, s, a, item0); break;
    case IT_HPSI_W: hipLaunchKernelGGL(k_batch_stage<IT_HPSI_W>, dim3(nitem), dim3(256), 0, s, a, item0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace svq
