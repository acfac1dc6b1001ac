/*
 * CPU oracle for the state-vector hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct complex128 code.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library: gate matrices, Pauli action and reductions are written out here
 * from their definitions.
 *
 * Index convention (paper, Section "Preliminaries", eq. sv): qubit q is bit q
 * of the amplitude index, qubit 0 the least significant bit.  A gate on
 * qubits q[0..d-1] uses the local index l = sum_j bit_{q[j]}(i) * 2^j, so q[0]
 * is the low bit of the gate matrix's row/column index.
 *
 * Functions:
 *   orc_apply_gate      one gate, U|psi>         (eq. update_sv_gate)
 *   orc_apply_circuit   U_{m-1}...U_0|psi>       (eq. update_sv_gate, in the given order)
 *   orc_apply_generator K|psi> for a parametric gate's generator (U = exp(-i t K))
 *   orc_pauli_apply     P|psi>                   (eq. pauli_form, eq. pauli_matrix)
 *   orc_expectation     sum_t a_t <psi|P_t|psi>  (eq. evc) and per-chunk sums E_j
 *                       (eq. local_evc, eq. aggregation)
 *   orc_hpsi            H|psi>                   (eq. hamiltonian)
 *   orc_adjoint_grad    dE/dtheta by the adjoint recursion over U_j^dagger
 *
 * All loops are OpenMP-parallel over independent output elements only, so
 * results do not depend on the thread count except through the final sums,
 * which are summed in a fixed order per thread block (schedule(static)).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Gate kind codes of the oracle's own loader (oracle/__init__.py). */
enum {
    OK_H = 0, OK_X, OK_Y, OK_Z, OK_S, OK_T, OK_RX, OK_RY, OK_RZ,
    OK_CNOT, OK_CZ, OK_CPHASE, OK_GIVENS, OK_SWAP, OK_U1, OK_U2
};

static int kind_arity(int kind) {
    switch (kind) {
    case OK_CNOT: case OK_CZ: case OK_CPHASE: case OK_GIVENS: case OK_SWAP: case OK_U2:
        return 2;
    default:
        return 1;
    }
}

/* Dense matrix of a gate, row-major M[r*dim + c]; returns dim (2 or 4).
 * umat (U1/U2 only): row-major complex entries as (re, im) pairs. */
static int gate_matrix(int kind, double th, const double *umat, cplx *M) {
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    const double r2 = 1.0 / sqrt(2.0);
    int d = kind_arity(kind) == 2 ? 4 : 2;
    for (int i = 0; i < d * d; ++i) M[i] = 0.0;
    switch (kind) {
    case OK_H:  M[0] = r2; M[1] = r2; M[2] = r2; M[3] = -r2; break;
    case OK_X:  M[1] = 1.0; M[2] = 1.0; break;
    case OK_Y:  M[1] = -I; M[2] = I; break;                 /* [[0,-i],[i,0]] */
    case OK_Z:  M[0] = 1.0; M[3] = -1.0; break;
    case OK_S:  M[0] = 1.0; M[3] = I; break;
    case OK_T:  M[0] = 1.0; M[3] = cexp(I * M_PI / 4.0); break;
    case OK_RX: M[0] = c; M[1] = -I * s; M[2] = -I * s; M[3] = c; break;
    case OK_RY: M[0] = c; M[1] = -s; M[2] = s; M[3] = c; break;
    case OK_RZ: M[0] = cexp(-0.5 * I * th); M[3] = cexp(0.5 * I * th); break;
    case OK_U1:
        for (int i = 0; i < 4; ++i) M[i] = umat[2 * i] + I * umat[2 * i + 1];
        break;
    case OK_CNOT:   /* q[0] control, q[1] target: |c=1,t=0> (l=1) <-> |c=1,t=1> (l=3) */
        M[0 * 4 + 0] = 1.0; M[2 * 4 + 2] = 1.0; M[1 * 4 + 3] = 1.0; M[3 * 4 + 1] = 1.0; break;
    case OK_CZ:
        M[0] = 1.0; M[5] = 1.0; M[10] = 1.0; M[15] = -1.0; break;
    case OK_CPHASE: /* diag(1, 1, 1, e^{i th}) */
        M[0] = 1.0; M[5] = 1.0; M[10] = 1.0; M[15] = cexp(I * th); break;
    case OK_GIVENS: /* real rotation in span{|a=1,b=0> (l=1), |a=0,b=1> (l=2)} */
        M[0] = 1.0; M[15] = 1.0;
        M[1 * 4 + 1] = c; M[1 * 4 + 2] = -s;
        M[2 * 4 + 1] = s; M[2 * 4 + 2] = c;
        break;
    case OK_SWAP:
        M[0] = 1.0; M[15] = 1.0; M[1 * 4 + 2] = 1.0; M[2 * 4 + 1] = 1.0; break;
    case OK_U2:
        for (int i = 0; i < 16; ++i) M[i] = umat[2 * i] + I * umat[2 * i + 1];
        break;
    default:
        return 0;
    }
    return d;
}

/* Generator K of a parametric gate, U(t) = exp(-i t K); returns dim, 0 if the
 * gate has no parameter.  RX/RY/RZ: sigma/2.  CPHASE: -|11><11|.
 * GIVENS: (X_a Y_b - Y_a X_b)/4, i.e. K|l=1> = (i/2)|l=2>, K|l=2> = -(i/2)|l=1>. */
static int gen_matrix(int kind, cplx *K) {
    int d = kind_arity(kind) == 2 ? 4 : 2;
    for (int i = 0; i < d * d; ++i) K[i] = 0.0;
    switch (kind) {
    case OK_RX: K[1] = 0.5; K[2] = 0.5; return 2;
    case OK_RY: K[1] = -0.5 * I; K[2] = 0.5 * I; return 2;
    case OK_RZ: K[0] = 0.5; K[3] = -0.5; return 2;
    case OK_CPHASE: K[15] = -1.0; return 4;
    case OK_GIVENS: K[2 * 4 + 1] = 0.5 * I; K[1 * 4 + 2] = -0.5 * I; return 4;
    default: return 0;
    }
}

/* Insert a zero bit at each sorted position in pos[0..d-1] into b. */
static inline uint64_t spread_base(uint64_t b, const int *sorted_pos, int d) {
    for (int j = 0; j < d; ++j) {
        uint64_t lo = b & ((1ULL << sorted_pos[j]) - 1);
        b = ((b >> sorted_pos[j]) << (sorted_pos[j] + 1)) | lo;
    }
    return b;
}

/* out[i] = (M applied on qubits q[0..d-1]) psi, in place (out may equal psi). */
static void apply_dense(cplx *psi, int n, const int *q, int nq, const cplx *M) {
    int sp[2] = {q[0], nq > 1 ? q[1] : 0};
    if (nq == 2 && sp[0] > sp[1]) { int t = sp[0]; sp[0] = sp[1]; sp[1] = t; }
    const int dim = 1 << nq;
    uint64_t off[4];
    for (int l = 0; l < dim; ++l) {
        off[l] = 0;
        for (int j = 0; j < nq; ++j)
            if ((l >> j) & 1) off[l] |= 1ULL << q[j];
    }
    const int64_t nb = (int64_t)1 << (n - nq);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        uint64_t base = spread_base((uint64_t)b, sp, nq);
        cplx in[4], out[4];
        for (int l = 0; l < dim; ++l) in[l] = psi[base | off[l]];
        for (int r = 0; r < dim; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < dim; ++c) acc += M[r * dim + c] * in[c];
            out[r] = acc;
        }
        for (int l = 0; l < dim; ++l) psi[base | off[l]] = out[l];
    }
}

/* Returns 0 on success, -1 on a bad gate. */
int orc_apply_gate(double *psi_ri, int n, int kind, const int *q, double theta,
                   const double *umat, int dagger) {
    cplx M[16];
    int d = gate_matrix(kind, theta, umat, M);
    if (d == 0) return -1;
    int nq = d == 4 ? 2 : 1;
    if (dagger) {
        cplx T[16];
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) T[r * d + c] = conj(M[c * d + r]);
        memcpy(M, T, sizeof(cplx) * d * d);
    }
    apply_dense((cplx *)psi_ri, n, q, nq, M);
    return 0;
}

/* gates: kinds[m], qs[m*2], angles[m] (already theta[param] or the fixed
 * angle), umats[m*32] (may be NULL when no U1/U2 gate is present). */
int orc_apply_circuit(double *psi_ri, int n, int m, const int *kinds, const int *qs,
                      const double *angles, const double *umats) {
    for (int i = 0; i < m; ++i) {
        int rc = orc_apply_gate(psi_ri, n, kinds[i], qs + 2 * i, angles[i],
                                umats ? umats + 32 * i : NULL, 0);
        if (rc) return rc;
    }
    return 0;
}

int orc_apply_generator(double *psi_ri, int n, int kind, const int *q) {
    cplx K[16];
    int d = gen_matrix(kind, K);
    if (d == 0) return -1;
    apply_dense((cplx *)psi_ri, n, q, d == 4 ? 2 : 1, K);
    return 0;
}

static inline int popc64(uint64_t v) { return __builtin_popcountll(v); }

/* i^k for integer k */
static inline cplx ipow(int k) {
    switch (k & 3) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
    }
}

/* out = P psi with P|j> = i^{nY} (-1)^{popcount(j & z)} |j xor x>
 * (derived from eq. pauli_matrix: X|b> = |1-b>, Y|b> = i(-1)^b|1-b>,
 * Z|b> = (-1)^b|b>; Y sits where both x and z have the bit). */
void orc_pauli_apply(double *out_ri, const double *psi_ri, int n, uint64_t x, uint64_t z) {
    const cplx *psi = (const cplx *)psi_ri;
    cplx *out = (cplx *)out_ri;
    const cplx ph = ipow(popc64(x & z));
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        uint64_t j = (uint64_t)i ^ x;          /* source index: P|j> lands on |i> */
        double sg = (popc64(j & z) & 1) ? -1.0 : 1.0;
        out[i] = ph * sg * psi[j];
    }
}

/* E = sum_t a_t <psi|P_t|psi> computed literally as
 * sum_t a_t sum_i conj(psi_i) (P_t psi)_i.  Also, when chunk_out != NULL,
 * the per-chunk sums E_c = sum_t a_t sum_{i in chunk c} conj(psi_i)(P_t psi)_i
 * where chunk(i) = phys(i) >> (n - g) and phys() deposits logical bit q at
 * physical position pos[q] (pos == NULL: identity).  Returns Re E; *im_out
 * gets Im E. */
double orc_expectation(const double *psi_ri, int n, int nt, const uint64_t *xs,
                       const uint64_t *zs, const double *coef, int g, const int *pos,
                       double *chunk_out, double *im_out) {
    const cplx *psi = (const cplx *)psi_ri;
    const int64_t N = (int64_t)1 << n;
    const int nchunk = 1 << g;
    double *cre = (double *)calloc((size_t)nchunk, sizeof(double));
    double tot_re = 0.0, tot_im = 0.0;
    for (int t = 0; t < nt; ++t) {
        const uint64_t x = xs[t], z = zs[t];
        const cplx ph = ipow(popc64(x & z));
        double sre = 0.0, sim = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : sre, sim)
        for (int64_t i = 0; i < N; ++i) {
            uint64_t j = (uint64_t)i ^ x;
            double sg = (popc64(j & z) & 1) ? -1.0 : 1.0;
            cplx v = conj(psi[i]) * ph * sg * psi[j];
            sre += creal(v);
            sim += cimag(v);
        }
        tot_re += coef[t] * sre;
        tot_im += coef[t] * sim;
        if (chunk_out) {
            for (int c = 0; c < nchunk; ++c) {
                double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
                for (int64_t i = 0; i < N; ++i) {
                    uint64_t ph_i = 0;
                    for (int q = 0; q < n; ++q)
                        if (((uint64_t)i >> q) & 1) ph_i |= 1ULL << (pos ? pos[q] : q);
                    if ((int)(ph_i >> (n - g)) != c) continue;
                    uint64_t j = (uint64_t)i ^ x;
                    double sg = (popc64(j & z) & 1) ? -1.0 : 1.0;
                    acc += creal(conj(psi[i]) * ph * sg * psi[j]);
                }
                cre[c] += coef[t] * acc;
            }
        }
    }
    if (chunk_out) memcpy(chunk_out, cre, sizeof(double) * (size_t)nchunk);
    free(cre);
    if (im_out) *im_out = tot_im;
    return tot_re;
}

/* out = H psi = sum_t a_t P_t psi */
void orc_hpsi(double *out_ri, const double *psi_ri, int n, int nt, const uint64_t *xs,
              const uint64_t *zs, const double *coef) {
    const cplx *psi = (const cplx *)psi_ri;
    cplx *out = (cplx *)out_ri;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        cplx acc = 0.0;
        for (int t = 0; t < nt; ++t) {
            uint64_t j = (uint64_t)i ^ xs[t];
            double sg = (popc64(j & zs[t]) & 1) ? -1.0 : 1.0;
            acc += coef[t] * ipow(popc64(xs[t] & zs[t])) * sg * psi[j];
        }
        out[i] = acc;
    }
}

static cplx inner(const cplx *a, const cplx *b, int64_t N) {
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (int64_t i = 0; i < N; ++i) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

/* Adjoint-method gradient of E(theta) = <psi0|U^dag H U|psi0>.
 * psi_ri holds psi0 on entry and U psi0 on exit.  angles[i] is gate i's
 * angle, umats[i*32..] its U1/U2 matrix (NULL when no gate is dense),
 * gate_param[i] the theta index the angle depends on (-1: fixed) and
 * gate_scale[i] = d(angle_i)/d(theta[gate_param[i]]).  grad[n_theta] is
 * overwritten, *energy_out receives E.  Returns 0, or -1 on a bad gate.
 *
 * With psi_j = U_j ... U_0 psi0 and lambda_j = U_{j+1}^dag ... U_{m-1}^dag H psi_{m-1}:
 * dE/da_j = 2 Re <lambda_j| dU_j/da |psi_{j-1}> = 2 Im <lambda_j| K_j |psi_j>
 * because dU/da = -i K U for U = exp(-i a K); the chain rule multiplies by
 * gate_scale[j].  Walk j = m-1 .. 0, evaluating the term, then
 * psi <- U_j^dag psi, lambda <- U_j^dag lambda. */
int orc_adjoint_grad(double *psi_ri, int n, int m, const int *kinds, const int *qs,
                     const double *angles, const double *umats, const int *gate_param,
                     const double *gate_scale, int n_theta, int nt, const uint64_t *xs,
                     const uint64_t *zs, const double *coef, double *grad, double *energy_out) {
    const int64_t N = (int64_t)1 << n;
    cplx *psi = (cplx *)psi_ri;
    int rc = orc_apply_circuit(psi_ri, n, m, kinds, qs, angles, umats);
    if (rc) return rc;
    cplx *lam = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *keep = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!lam || !tmp || !keep) {
        free(lam); free(tmp); free(keep);
        return -2;
    }
    orc_hpsi((double *)lam, psi_ri, n, nt, xs, zs, coef);
    *energy_out = creal(inner(psi, lam, N));
    /* keep U psi0 for the caller */
    memcpy(keep, psi, sizeof(cplx) * (size_t)N);
    for (int t = 0; t < n_theta; ++t) grad[t] = 0.0;
    for (int i = m - 1; i >= 0 && rc == 0; --i) {
        const double *um = umats ? umats + 32 * i : NULL;
        if (gate_param[i] >= 0) {
            memcpy(tmp, psi, sizeof(cplx) * (size_t)N);
            rc = orc_apply_generator((double *)tmp, n, kinds[i], qs + 2 * i);
            if (rc) break;
            cplx v = inner(lam, tmp, N);
            grad[gate_param[i]] += gate_scale[i] * 2.0 * cimag(v);
        }
        rc = orc_apply_gate(psi_ri, n, kinds[i], qs + 2 * i, angles[i], um, 1);
        if (rc == 0) rc = orc_apply_gate((double *)lam, n, kinds[i], qs + 2 * i, angles[i], um, 1);
    }
    memcpy(psi, keep, sizeof(cplx) * (size_t)N);
    free(keep);
    free(tmp);
    free(lam);
    return rc;
}

/* OpenMP threads used by the parallel loops above. */
int orc_threads(void) { return omp_get_max_threads(); }
