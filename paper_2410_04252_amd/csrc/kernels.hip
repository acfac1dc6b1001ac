// HIP kernels for gfx950 (wave64).  See svq_dev.hpp for the descriptor
// tables and kernels.hpp for the host launch interface.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "svq_dev.hpp"

namespace svq {

template <typename R> struct V2T;
template <> struct V2T<float> { using type = float2; };
template <> struct V2T<double> { using type = double2; };

// Insert a zero bit at each of the (ascending) positions pos[0..k-1].
__device__ __forceinline__ uint64_t spread(uint64_t b, const int8_t *pos, int k) {
    for (int j = 0; j < k; ++j) {
        const int p = pos[j];
        const uint64_t lo = b & ((1ULL << p) - 1);
        b = ((b >> p) << (p + 1)) | lo;
    }
    return b;
}

// LDS slot of tile-local index t: the six low bits are XORed with the folded
// higher bits so that a wave whose lanes walk any six tile bits with distinct
// residues mod 6 hits 64 distinct 8-byte slots modulo 64.
__device__ __forceinline__ uint32_t swz(uint32_t t) {
    return t ^ (((t >> 6) ^ (t >> 12)) & 63u);
}

// ---------------------------------------------------------------------------
// register-tile gate kernels
// ---------------------------------------------------------------------------

template <typename R, int NR> struct Regs {
    R re[NR], im[NR];
};

struct PhaseIdx {
    uint32_t tt;   // tile-local index bits contributed by lane and wave
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

template <int K>
__device__ __forceinline__ uint64_t tile_to_phys(uint32_t t, const int8_t *tphys) {
    uint64_t p = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((t >> j) & 1) p |= 1ULL << tphys[j];
    return p;
}

template <typename R, int NR, int RB>
__device__ __forceinline__ void op_diag(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                        const OpDesc &o) {
    const R d0r = (R)o.m[0], d0i = (R)o.m[1], d1r = (R)o.m[2], d1i = (R)o.m[3];
    const int pb = o.pbit;
    const uint32_t cm = o.cmask;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const uint32_t t = tt | reg_offset<RB>(P, j);
        const bool b = (t >> pb) & 1u;
        const bool c = (t & cm) == cm;
        R dr = b ? d1r : d0r, di = b ? d1i : d0i;
        dr = c ? dr : (R)1;
        di = c ? di : (R)0;
        const R xr = v.re[j], xi = v.im[j];
        v.re[j] = xr * dr - xi * di;
        v.im[j] = xr * di + xi * dr;
    }
}

template <int B, typename R, int NR, int RB>
__device__ __forceinline__ void op_mix1(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                        const OpDesc &o) {
    const R a_r = (R)o.m[0], a_i = (R)o.m[1], b_r = (R)o.m[2], b_i = (R)o.m[3];
    const R c_r = (R)o.m[4], c_i = (R)o.m[5], d_r = (R)o.m[6], d_i = (R)o.m[7];
    const uint32_t cm = o.cmask;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const uint32_t t = tt | reg_offset<RB>(P, j);
        const bool c = (t & cm) == cm;
        const R x0r = v.re[j], x0i = v.im[j], x1r = v.re[j1], x1i = v.im[j1];
        const R y0r = a_r * x0r - a_i * x0i + b_r * x1r - b_i * x1i;
        const R y0i = a_r * x0i + a_i * x0r + b_r * x1i + b_i * x1r;
        const R y1r = c_r * x0r - c_i * x0i + d_r * x1r - d_i * x1i;
        const R y1i = c_r * x0i + c_i * x0r + d_r * x1i + d_i * x1r;
        v.re[j] = c ? y0r : x0r;
        v.im[j] = c ? y0i : x0i;
        v.re[j1] = c ? y1r : x1r;
        v.im[j1] = c ? y1i : x1i;
    }
}

template <int B, typename R, int NR, int RB>
__device__ __forceinline__ void op_xswap(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                         const OpDesc &o) {
    const uint32_t cm = o.cmask;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const uint32_t t = tt | reg_offset<RB>(P, j);
        const bool c = (t & cm) == cm;
        const R x0r = v.re[j], x0i = v.im[j], x1r = v.re[j1], x1i = v.im[j1];
        v.re[j] = c ? x1r : x0r;
        v.im[j] = c ? x1i : x0i;
        v.re[j1] = c ? x0r : x1r;
        v.im[j1] = c ? x0i : x1i;
    }
}

template <int B0, int B1, typename R, int NR, int RB>
__device__ __forceinline__ void op_givens(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                          const OpDesc &o) {
    const R cs = (R)o.m[0], sn = (R)o.m[1];
    const uint32_t cm = o.cmask;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int ju = j | (1 << B0);   // b0 = 1, b1 = 0
        const int jw = j | (1 << B1);   // b0 = 0, b1 = 1
        const uint32_t t = tt | reg_offset<RB>(P, j);
        const bool c = (t & cm) == cm;
        const R ur = v.re[ju], ui = v.im[ju], wr = v.re[jw], wi = v.im[jw];
        const R nur = cs * ur - sn * wr, nui = cs * ui - sn * wi;
        const R nwr = sn * ur + cs * wr, nwi = sn * ui + cs * wi;
        v.re[ju] = c ? nur : ur;
        v.im[ju] = c ? nui : ui;
        v.re[jw] = c ? nwr : wr;
        v.im[jw] = c ? nwi : wi;
    }
}

template <int B0, int B1, typename R, int NR, int RB>
__device__ __forceinline__ void op_mix2(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                        const OpDesc &o) {
    R mr[16], mi[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        mr[e] = (R)o.m[2 * e];
        mi[e] = (R)o.m[2 * e + 1];
    }
    const uint32_t cm = o.cmask;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        int jl[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) jl[l] = j | ((l & 1) ? (1 << B0) : 0) | ((l & 2) ? (1 << B1) : 0);
        const uint32_t t = tt | reg_offset<RB>(P, j);
        const bool c = (t & cm) == cm;
        R xr[4], xi[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            xr[l] = v.re[jl[l]];
            xi[l] = v.im[jl[l]];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            R sr = 0, si = 0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                sr += mr[r * 4 + cc] * xr[cc] - mi[r * 4 + cc] * xi[cc];
                si += mr[r * 4 + cc] * xi[cc] + mi[r * 4 + cc] * xr[cc];
            }
            v.re[jl[r]] = c ? sr : xr[r];
            v.im[jl[r]] = c ? si : xi[r];
        }
    }
}

// Dispatch on register-bit positions with explicit cases so that every
// variant is inlined and the register arrays never leave VGPRs.
#define SVQ_C1(FN, I)                                                   \
    case I:                                                             \
        if constexpr (I < RB) FN<I, R, NR, RB>(v, tt, P, o);            \
        break;
#define SVQ_C2(FN, I, J)                                                \
    case I * 8 + J:                                                     \
        if constexpr (I < RB && J < RB && I != J) FN<I, J, R, NR, RB>(v, tt, P, o); \
        break;
#define SVQ_ALL1(FN) SVQ_C1(FN, 0) SVQ_C1(FN, 1) SVQ_C1(FN, 2) SVQ_C1(FN, 3) SVQ_C1(FN, 4)
#define SVQ_ROW(FN, I) SVQ_C2(FN, I, 0) SVQ_C2(FN, I, 1) SVQ_C2(FN, I, 2) SVQ_C2(FN, I, 3) SVQ_C2(FN, I, 4)
#define SVQ_ALL2(FN) SVQ_ROW(FN, 0) SVQ_ROW(FN, 1) SVQ_ROW(FN, 2) SVQ_ROW(FN, 3) SVQ_ROW(FN, 4)

template <typename R, int NR, int RB>
__device__ __forceinline__ void apply_op(Regs<R, NR> &v, uint32_t tt, const PhaseDesc &P,
                                         const OpDesc &o) {
    static_assert(RB <= 5, "dispatch covers at most 5 register bits");
    switch (o.type) {
    case OP_DIAG:
        op_diag<R, NR, RB>(v, tt, P, o);
        break;
    case OP_MIX1:
        switch (o.b0) { SVQ_ALL1(op_mix1) }
        break;
    case OP_XSWAP:
        switch (o.b0) { SVQ_ALL1(op_xswap) }
        break;
    case OP_GIVENS:
        switch (o.b0 * 8 + o.b1) { SVQ_ALL2(op_givens) }
        break;
    default:
        switch (o.b0 * 8 + o.b1) { SVQ_ALL2(op_mix2) }
        break;
    }
}

// 2 Im <lambda|K|psi> over this thread's amplitudes, for the generator of o.
template <int B0, int B1, typename R, int NR, int RB>
__device__ __forceinline__ double gen_value(const Regs<R, NR> &x, const Regs<R, NR> &l,
                                           uint32_t tt, const PhaseDesc &P, const OpDesc &o) {
    R acc = 0;
    if (o.gtype == GEN_DIAG) {
        const R k0 = (R)o.k[0], k1 = (R)o.k[1];
        const uint32_t cm = o.cmask;
        const int pb = o.pbit;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const uint32_t t = tt | reg_offset<RB>(P, j);
            const bool c = (t & cm) == cm;
            const R kk = ((t >> pb) & 1u) ? k1 : k0;
            // Im(conj(l) x) = l.re x.im - l.im x.re
            const R im = l.re[j] * x.im[j] - l.im[j] * x.re[j];
            acc += c ? kk * im : (R)0;
        }
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
            acc += l.re[j] * y0i - l.im[j] * y0r + l.re[j1] * y1i - l.im[j1] * y1r;
        }
    } else {   // GEN_GIVENS: Im<l|K|x> = (Re(conj(l_w) x_u) - Re(conj(l_u) x_w)) / 2
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j & ((1 << B0) | (1 << B1))) continue;
            const int ju = j | (1 << B0), jw = j | (1 << B1);
            acc += (R)0.5 * (l.re[jw] * x.re[ju] + l.im[jw] * x.im[ju]
                             - l.re[ju] * x.re[jw] - l.im[ju] * x.im[jw]);
        }
    }
    return 2.0 * (double)acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

#define SVQ_G1(I)                                                               \
    case I:                                                                     \
        if constexpr (I < RB) g = gen_value<I, 0, R, NR, RB>(x, l, tt, P, o);   \
        break;
#define SVQ_G2(I, J)                                                            \
    case I * 8 + J:                                                             \
        if constexpr (I < RB && J < RB && I != J) g = gen_value<I, J, R, NR, RB>(x, l, tt, P, o); \
        break;
#define SVQ_GROW(I) SVQ_G2(I, 0) SVQ_G2(I, 1) SVQ_G2(I, 2) SVQ_G2(I, 3) SVQ_G2(I, 4)

template <typename R, int NR, int RB>
__device__ __forceinline__ double op_gradient(const Regs<R, NR> &x, const Regs<R, NR> &l,
                                              uint32_t tt, const PhaseDesc &P, const OpDesc &o) {
    double g = 0.0;
    if (o.gtype == GEN_DIAG) {
        g = gen_value<0, 0, R, NR, RB>(x, l, tt, P, o);
    } else if (o.gtype == GEN_MIX1) {
        switch (o.b0) { SVQ_G1(0) SVQ_G1(1) SVQ_G1(2) SVQ_G1(3) SVQ_G1(4) }
    } else {
        switch (o.b0 * 8 + o.b1) { SVQ_GROW(0) SVQ_GROW(1) SVQ_GROW(2) SVQ_GROW(3) SVQ_GROW(4) }
    }
    return g;
}

template <typename V, typename R, int NR>
__device__ __forceinline__ void to_lds(V *lds, const Regs<R, NR> &v, uint32_t tt,
                                       const uint32_t *roff) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        V e;
        e.x = v.re[j];
        e.y = v.im[j];
        lds[swz(tt | roff[j])] = e;
    }
}

template <typename V, typename R, int NR>
__device__ __forceinline__ void from_lds(const V *lds, Regs<R, NR> &v, uint32_t tt,
                                         const uint32_t *roff) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const V e = lds[swz(tt | roff[j])];
        v.re[j] = e.x;
        v.im[j] = e.y;
    }
}

// One gate pass (forward), or one reverse adjoint pass when ADJ: psi and
// lam both get U^dagger of every op in reverse order, and each parametric
// op first records 2 Im <lam|K|psi> per wave into gpart.
template <typename R, int K, int RB, bool ADJ>
__global__ __launch_bounds__(1 << (K - RB)) void k_gate_pass(
    typename V2T<R>::type *__restrict__ psi, typename V2T<R>::type *__restrict__ lam,
    const PassArgs a, const PhaseDesc *__restrict__ phases, const OpDesc *__restrict__ ops,
    double *__restrict__ gpart, int nblocks_total) {
    using V = typename V2T<R>::type;
    constexpr int NR = 1 << RB;
    constexpr int NT = 1 << (K - RB);
    constexpr int NWB = K - RB - 6;
    __shared__ V lds[(ADJ ? 2 : 1) << K];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint64_t base = spread(blockIdx.x, a.tphys, K);

    const int np = a.nphase;
    const int p_first = ADJ ? np - 1 : 0;
    const PhaseDesc *Pp = phases + a.phase0 + p_first;
    uint32_t tt = thread_tile_index<NWB>(*Pp, lane, wave);
    uint32_t roff[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) roff[j] = reg_offset<RB>(*Pp, j);

    Regs<R, NR> v, w;
    {
        const uint64_t tp = tile_to_phys<K>(tt, a.tphys);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const uint64_t addr = base + tp + tile_to_phys<K>(roff[j], a.tphys);
            const V e = psi[addr];
            v.re[j] = e.x;
            v.im[j] = e.y;
            if constexpr (ADJ) {
                const V f = lam[addr];
                w.re[j] = f.x;
                w.im[j] = f.y;
            }
        }
    }
    for (int s = 0; s < np; ++s) {
        const int p = ADJ ? np - 1 - s : s;
        if (s > 0) {
            if (s > 1) __syncthreads();
            to_lds<V, R, NR>(lds, v, tt, roff);
            if constexpr (ADJ) to_lds<V, R, NR>(lds + (1 << K), w, tt, roff);
            __syncthreads();
            Pp = phases + a.phase0 + p;
            tt = thread_tile_index<NWB>(*Pp, lane, wave);
#pragma unroll
            for (int j = 0; j < NR; ++j) roff[j] = reg_offset<RB>(*Pp, j);
            from_lds<V, R, NR>(lds, v, tt, roff);
            if constexpr (ADJ) from_lds<V, R, NR>(lds + (1 << K), w, tt, roff);
        }
        const int nop = Pp->nop;
        const int op0 = Pp->op0;
        for (int q = 0; q < nop; ++q) {
            const int oi = op0 + (ADJ ? nop - 1 - q : q);
            const OpDesc &o = ops[oi];
            const PhaseDesc &P = *Pp;
            if constexpr (ADJ) {
                if (o.gtype != GEN_NONE) {
                    const double gv = wave_sum(op_gradient<R, NR, RB>(v, w, tt, P, o));
                    if (lane == 0)
                        gpart[((size_t)o.gslot * nblocks_total + a.gslot_base + blockIdx.x) * (NT / 64) +
                              wave] = gv;
                }
                apply_op<R, NR, RB>(w, tt, P, o);
            }
            apply_op<R, NR, RB>(v, tt, P, o);
        }
    }
    {
        const uint64_t tp = tile_to_phys<K>(tt, a.tphys);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const uint64_t addr = base + tp + tile_to_phys<K>(roff[j], a.tphys);
            V e;
            e.x = v.re[j];
            e.y = v.im[j];
            psi[addr] = e;
            if constexpr (ADJ) {
                V f;
                f.x = w.re[j];
                f.y = w.im[j];
                lam[addr] = f;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// qubit reordering: in-place involution on physical bit positions
// ---------------------------------------------------------------------------

// Tile T = the low bits, their partners, and further unpaired bits; the
// permutation maps tile b to tile pi(b) and permutes inside the tile.  A
// block swaps the pair (b, pi(b)) once, through LDS so that both the loads
// and the stores walk the low bits contiguously.
template <typename V>
__global__ __launch_bounds__(256) void k_qr(V *__restrict__ psi, const QrArgs a) {
    extern __shared__ unsigned char smem[];
    V *l0 = reinterpret_cast<V *>(smem);
    V *l1 = l0 + (1 << a.tbits);
    const int TS = 1 << a.tbits;
    for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const uint64_t b = spread(tile, a.tphys, a.tbits);
        uint64_t pb = b;
        for (int i = 0; i < a.nouter; ++i) {
            const int x = a.outer[2 * i], y = a.outer[2 * i + 1];
            const uint64_t d = ((pb >> x) ^ (pb >> y)) & 1ULL;
            pb ^= (d << x) | (d << y);
        }
        if (pb < b) continue;
        if (pb == b && a.ninner == 0) continue;
        for (int t = threadIdx.x; t < TS; t += blockDim.x) {
            uint64_t off = 0;
            for (int j = 0; j < a.tbits; ++j)
                if ((t >> j) & 1) off |= 1ULL << a.tphys[j];
            uint32_t u = (uint32_t)t;
            for (int i = 0; i < a.ninner; ++i) {
                const int x = a.inner[2 * i], y = a.inner[2 * i + 1];
                const uint32_t d = ((u >> x) ^ (u >> y)) & 1u;
                u ^= (d << x) | (d << y);
            }
            l0[u] = psi[b + off];
            if (pb != b) l1[u] = psi[pb + off];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < TS; t += blockDim.x) {
            uint64_t off = 0;
            for (int j = 0; j < a.tbits; ++j)
                if ((t >> j) & 1) off |= 1ULL << a.tphys[j];
            psi[pb + off] = l0[t];
            if (pb != b) psi[b + off] = l1[t];
        }
        __syncthreads();
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

template <typename R, int K>
__global__ __launch_bounds__(1 << evc_tpb(K)) void k_evc_pass(
    const typename V2T<R>::type *__restrict__ psi, const EvcPassArgs a,
    const EvcGroup *__restrict__ groups, const EvcTerm *__restrict__ terms,
    double *__restrict__ partials) {
    using V = typename V2T<R>::type;
    constexpr int TPB = evc_tpb(K);
    constexpr int NT = 1 << TPB;
    constexpr int TS = 1 << K;
    constexpr int Q = K - 1 - TPB;
    constexpr int NQ = 1 << Q;
    __shared__ V lds[TS];
    __shared__ double red[NT / 64];
    const uint64_t base = spread(blockIdx.x, a.tphys, K);
    for (int t = threadIdx.x; t < TS; t += NT) {
        uint64_t off = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((t >> j) & 1) off |= 1ULL << a.tphys[j];
        lds[t] = psi[base + off];
    }
    __syncthreads();
    double acc = 0.0;
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const EvcGroup &G = groups[a.group0 + gi];
        uint32_t tt = 0;
#pragma unroll
        for (int b = 0; b < TPB; ++b) tt |= ((threadIdx.x >> b) & 1u) << G.tbits[b];
        R w[2 * NQ];   // [0, NQ): real / sum array, [NQ, 2NQ): imaginary / difference
        R *re = w, *im = w + NQ;
        const uint32_t xl = G.xl;
        const int hb = G.hbit;
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj) {
            uint32_t j = tt;
#pragma unroll
            for (int b = 0; b < Q; ++b)
                if ((jj >> b) & 1) j |= 1u << G.wbits[b];
            const V x = lds[j];
            if (xl) {
                const V p = lds[j ^ xl];
                // w = conj(psi_{j^x}) psi_j
                re[jj] = p.x * x.x + p.y * x.y;
                im[jj] = p.x * x.y - p.y * x.x;
            } else {
                const V y = lds[j | (1u << hb)];
                const R n0 = x.x * x.x + x.y * x.y, n1 = y.x * y.x + y.y * y.y;
                re[jj] = n0 + n1;
                im[jj] = n0 - n1;
            }
        }
        if (G.need & 1) wht<R, NQ>(re);
        if (G.need & 2) wht<R, NQ>(im);
        const int t1 = G.t0 + G.nt;
        for (int ti = G.t0; ti < t1; ++ti) {
            const EvcTerm &T = terms[ti];
            const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane(
                (int)((T.zw & (NQ - 1)) | (T.use_im ? NQ : 0)));
            const R val = w[wi];
            const uint32_t par = (__builtin_popcount(tt & T.zt) + __builtin_popcountll(base & T.zg)) & 1u;
            acc += T.coef * (double)(par ? -val : val);
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[a.part0 + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// H|psi> pass
// ---------------------------------------------------------------------------

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
    for (int t = threadIdx.x; t < TS; t += NT) {
        uint64_t off = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((t >> j) & 1) off |= 1ULL << a.tphys[j];
        lds[t] = psi[base + off];
    }
    __syncthreads();
    double lr[NQ], li[NQ];
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) lr[jj] = li[jj] = 0.0;
    const uint32_t tid = threadIdx.x;
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const HpsiGroup &G = groups[a.group0 + gi];
        const uint32_t sthr = tid ^ G.xt;
        R fr[NQ], fi[NQ];
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj) fr[jj] = fi[jj] = (R)0;
        const int t1 = G.t0 + G.nt;
        for (int ti = G.t0; ti < t1; ++ti) {
            const HpsiTerm &T = terms[ti];
            const uint32_t zw = (uint32_t)__builtin_amdgcn_readfirstlane((int)T.zw) & (NQ - 1);
            const uint32_t par = (__builtin_popcount(sthr & T.zt) + __builtin_popcountll(base & T.zg)) & 1u;
            const R ar = (R)T.are, ai = (R)T.aim;
            fr[zw] += par ? -ar : ar;
            fi[zw] += par ? -ai : ai;
        }
        wht<R, NQ>(fr);
        wht<R, NQ>(fi);
        const uint32_t xw = (uint32_t)__builtin_amdgcn_readfirstlane((int)G.xw);
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj) {
            const uint32_t sc = (jj ^ xw) & (NQ - 1);
            const R f_r = fr[sc], f_i = fi[sc];
            const V p = lds[sthr | (sc << TPB)];
            lr[jj] += (double)(f_r * p.x - f_i * p.y);
            li[jj] += (double)(f_r * p.y + f_i * p.x);
        }
    }
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) {
        const uint32_t t = tid | ((uint32_t)jj << TPB);
        uint64_t off = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((t >> j) & 1) off |= 1ULL << a.tphys[j];
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

// chunk_out[c] = sum over passes p and within-chunk blocks j of
// partials[p * per_pass + c * per_chunk + j], in that order.
__global__ __launch_bounds__(256) void k_reduce_chunks(const double *__restrict__ partials,
                                                        const int *__restrict__ pass_off,
                                                        const int *__restrict__ pass_nblk, int npass,
                                                        int nchunk, double *__restrict__ chunk_out) {
    __shared__ double red[4];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int p = 0; p < npass; ++p) {
        const int per_chunk = pass_nblk[p] / nchunk;
        const double *src = partials + pass_off[p] + (size_t)c * per_chunk;
        for (int j = threadIdx.x; j < per_chunk; j += blockDim.x) acc += src[j];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) chunk_out[c] = s;
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

template <typename R>
static hipError_t launch_gate_t(int k, bool adj, void *psi, void *lam, const PassArgs &a,
                                const PhaseDesc *ph, const OpDesc *ops, double *gpart, int nbt,
                                int nblocks, hipStream_t s) {
    using V = typename V2T<R>::type;
    V *p = (V *)psi, *l = (V *)lam;
#define SVQ_GATE_CASE(KK)                                                                      \
    case KK:                                                                                   \
        if (adj) {                                                                             \
            if constexpr (sizeof(R) * 2 * 2 * (1 << KK) <= 160 * 1024)                         \
                hipLaunchKernelGGL((k_gate_pass<R, KK, gate_rb(KK), true>), dim3(nblocks),     \
                                   dim3(1 << (KK - gate_rb(KK))), 0, s, p, l, a, ph, ops,     \
                                   gpart, nbt);                                                \
            else                                                                               \
                return hipErrorInvalidValue;                                                   \
        } else {                                                                               \
            hipLaunchKernelGGL((k_gate_pass<R, KK, gate_rb(KK), false>), dim3(nblocks),        \
                               dim3(1 << (KK - gate_rb(KK))), 0, s, p, l, a, ph, ops, gpart,   \
                               nbt);                                                           \
        }                                                                                      \
        break;
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
    return hipGetLastError();
}

hipError_t launch_gate_pass(bool dbl, int k, bool adj, void *psi, void *lam, const PassArgs &a,
                            const PhaseDesc *ph, const OpDesc *ops, double *gpart, int nbt,
                            hipStream_t s) {
    const int nblocks = a.nblocks;
    return dbl ? launch_gate_t<double>(k, adj, psi, lam, a, ph, ops, gpart, nbt, nblocks, s)
               : launch_gate_t<float>(k, adj, psi, lam, a, ph, ops, gpart, nbt, nblocks, s);
}

hipError_t launch_qr(bool dbl, void *psi, const QrArgs &a, hipStream_t s) {
    const size_t esz = dbl ? 16 : 8;
    const size_t smem = 2 * ((size_t)1 << a.tbits) * esz;
    uint64_t grid = a.ntiles < 4096 ? a.ntiles : 4096;
    if (grid == 0) return hipSuccess;
    if (dbl) hipLaunchKernelGGL(k_qr<double2>, dim3((unsigned)grid), dim3(256), smem, s, (double2 *)psi, a);
    else hipLaunchKernelGGL(k_qr<float2>, dim3((unsigned)grid), dim3(256), smem, s, (float2 *)psi, a);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_evc_t(int k, const void *psi, const EvcPassArgs &a, const EvcGroup *g,
                               const EvcTerm *t, double *part, hipStream_t s) {
    using V = typename V2T<R>::type;
    const V *p = (const V *)psi;
#define SVQ_EVC_CASE(KK)                                                                       \
    case KK:                                                                                   \
        hipLaunchKernelGGL((k_evc_pass<R, KK>), dim3(a.nblocks), dim3(1 << evc_tpb(KK)), 0, s, \
                           p, a, g, t, part);                                                  \
        break;
    switch (k) {
        SVQ_EVC_CASE(8)
        SVQ_EVC_CASE(9)
        SVQ_EVC_CASE(10)
        SVQ_EVC_CASE(11)
        SVQ_EVC_CASE(12)
        SVQ_EVC_CASE(13)
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

hipError_t launch_reduce_chunks(const double *partials, const int *pass_off, const int *pass_nblk,
                                int npass, int nchunk, double *chunk_out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nchunk), dim3(256), 0, s, partials, pass_off, pass_nblk,
                       npass, nchunk, chunk_out);
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

hipError_t launch_fill_basis(bool dbl, void *psi, uint64_t N, uint64_t idx, hipStream_t s) {
    const int g = grid_for(N);
    if (dbl) hipLaunchKernelGGL(k_fill_basis<double2>, dim3(g), dim3(256), 0, s, (double2 *)psi, N, idx);
    else hipLaunchKernelGGL(k_fill_basis<float2>, dim3(g), dim3(256), 0, s, (float2 *)psi, N, idx);
    return hipGetLastError();
}

}  // namespace svq
