// Host launch interface of the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "svq_dev.hpp"

namespace svq {

// In-place relayout by disjoint transpositions of physical bits.
struct QrArgs {
    int32_t tbits;          // tile bits (tile path)
    int32_t nouter;         // transpositions outside the tile (rows path: all of them)
    int32_t ninner;         // transpositions inside the tile (tile-local bits)
    int32_t rows_path;      // 1: no exchanged bit below 6, swap rows of 64 elements
    int32_t hbit, lbit;     // rows path: row bits of the highest exchanged bit and its partner
    uint64_t ntiles;        // 2^(n - tbits)
    uint64_t nrows;         // 2^(n - 6)
    int8_t tphys[16];       // physical bit of tile-local bit j (ascending)
    int8_t outer[64];       // pairs (a, b) of physical bits
    int8_t inner[32];       // pairs (a, b) of tile-local bits
};

struct WideTerm {
    uint64_t x, z;          // physical masks
    double coef;
    int32_t ny;             // popcount(x & z)
    int32_t pad;
};

// rb: the register bits the plan was built for (CircuitPlan::rb).
hipError_t launch_gate_pass(bool dbl, int k, int rb, bool adj, void *psi, void *lam, const PassArgs &a,
                            const PhaseDesc *ph, const OpDesc *ops, double *gpart, int nbt,
                            hipStream_t s);
hipError_t launch_qr(bool dbl, void *psi, const QrArgs &a, hipStream_t s);
hipError_t launch_evc_pass(bool dbl, int k, const void *psi, const EvcPassArgs &a,
                           const EvcGroup *g, const EvcTerm *t, double *part, hipStream_t s);
hipError_t launch_hpsi_pass(bool dbl, int k, int nblocks, const void *psi, void *lam,
                            const HpsiPassArgs &a, const HpsiGroup *g, const HpsiTerm *t,
                            hipStream_t s);
int direct_grid(uint64_t N);
hipError_t launch_evc_direct(bool dbl, const void *psi, uint64_t N, const WideTerm *wt, int nw,
                             double *part, hipStream_t s);
hipError_t launch_hpsi_direct(bool dbl, const void *psi, void *lam, uint64_t N, const WideTerm *wt,
                              int nw, int accumulate, hipStream_t s);
// Deterministic chunk sums of the per-block EVC partials; tmp holds
// reduce_scratch(nchunk) doubles.
int reduce_scratch(int nchunk);
hipError_t launch_reduce_chunks(const double *partials, const int *pass_off, const int *pass_nblk,
                                int npass, int nchunk, double *tmp, double *chunk_out, hipStream_t s);
hipError_t launch_finish_energy(const double *chunk, int nchunk, const double *extra, int nextra,
                                double *out, hipStream_t s);
hipError_t launch_sum(const double *in, int n, double *out, hipStream_t s);
int dot_grid(uint64_t N);
hipError_t launch_dot_re(bool dbl, const void *a, const void *b, uint64_t N, double *partials,
                         hipStream_t s);
hipError_t launch_grad_reduce(const double *gpart, int nper, const int *pptr, const int *pgate,
                              int nparam, double *grad, hipStream_t s);
// gop[gates[i]] = sum over tiles of gpart[i * ntiles + t], i < nslots (the
// block partials of one adjoint pass).
hipError_t launch_grad_tiles(const double *gpart, uint32_t ntiles, int nslots, const int *gates,
                             double *gop, hipStream_t s);
// grad[p] = sum_{e in [ptr[p], ptr[p+1])} coef[e] * evals[e]: the
// parameter-shift combination of shifted energies.
hipError_t launch_shift_combine(const double *evals, const double *coef, const int *ptr, int nparam,
                                double *grad, hipStream_t s);
// dst[0, bytes) = src[0, bytes), bytes a multiple of 16.
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_basis(bool dbl, void *psi, uint64_t N, uint64_t idx, hipStream_t s);
// Reset counters (fill kernel) and launch the persistent batch kernel.
hipError_t launch_batch(const BatchArgs &a, int32_t *counters, int ncounters, hipStream_t s,
                        int *grid_out);
// One block per LDS-resident instance (a.linst[0, ninst)), 2 x 2^max_n
// complex64 of dynamic LDS; prepare_batch_lds(max_n) first (outside any
// stream capture) raises the kernel's dynamic LDS limit.
hipError_t prepare_batch_lds(int max_n);
hipError_t launch_batch_lds(const BatchArgs &a, int ninst, int max_n, hipStream_t s);
// *t = the realtime clock (one thread; the batch graph's start time).
hipError_t launch_stamp(uint64_t *t, hipStream_t s);
// p[0, n) = v with a fill kernel (no memset node in a captured graph).
hipError_t launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s);
// One level-synchronous launch: items [item0, item0 + nitem), all of one type.
hipError_t launch_batch_stage(const BatchArgs &a, int type, int item0, int nitem, hipStream_t s);

}  // namespace svq
