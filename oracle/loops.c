/*
 * Tier-1 oracle in plain C loops (TEST INFRASTRUCTURE ONLY: called by the
 * tests, the golden-value script under tests/golden/ and the CPU baseline of
 * the benchmark; never by the product library).
 *
 * What it computes is the textbook action of the paper's two simulators
 * (Sec. II): a state-vector simulator, psi <- U psi for each gate, and a
 * density-matrix simulator, rho <- sum_m K_m rho K_m^dagger for each gate
 * (one Kraus operator, U) and each noise channel of Sec. III, followed by the
 * observables of Sec. III (Pauli expectation values, Tr(rho P), purity,
 * trace).  The matrices themselves come from the Python side of the oracle
 * (oracle/gates.py); this file only applies them.
 *
 * Conventions: qubit q is bit q of the basis index; a k-qubit operator on
 * (q_0, .., q_{k-1}) has row/column index u = sum_j bit(q_j) 2^j; the density
 * matrix is row-major, rho[r * 2^n + c].  Complex numbers are C99 double
 * _Complex (interleaved re, im: the numpy complex128 layout); complex results
 * are written to out[0] (real part) and out[1] (imaginary part).
 *
 * Every loop is written from the definition, with no blocking or fusion:
 * a k-qubit operator acts on the group of 2^k indices that agree outside its
 * qubits.  The group is enumerated by scanning every index and keeping those
 * whose bits on the operator's qubits are all zero.  Loops over independent
 * groups are shared among OpenMP threads; every group is computed by one
 * thread in a fixed order, so updated states do not depend on the thread
 * count.  Sums (expectation values, purity) use OpenMP's reduction, whose
 * rounding may differ with the thread count at the level of one ulp per
 * partial sum.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

/* offset of member u of a group: sum_j bit_j(u) 2^{q_j} */
static void group_offsets(int k, const int *qubits, uint64_t *off, uint64_t *mask)
{
    uint64_t m = 0;
    for (int j = 0; j < k; ++j) m |= (uint64_t)1 << qubits[j];
    for (int u = 0; u < (1 << k); ++u) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((u >> j) & 1) o |= (uint64_t)1 << qubits[j];
        off[u] = o;
    }
    *mask = m;
}

/* psi <- U psi for a k-qubit U (k <= 3), U row-major 2^k x 2^k. */
void ora_sv_apply(cplx *psi, int n, int k, const int *qubits, const cplx *U)
{
    uint64_t off[8], mask;
    group_offsets(k, qubits, off, &mask);
    const int d = 1 << k;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if ((uint64_t)i & mask) continue;
        cplx in[8], out[8];
        for (int u = 0; u < d; ++u) in[u] = psi[i + off[u]];
        for (int u = 0; u < d; ++u) {
            cplx s = 0;
            for (int v = 0; v < d; ++v) s += U[u * d + v] * in[v];
            out[u] = s;
        }
        for (int u = 0; u < d; ++u) psi[i + off[u]] = out[u];
    }
}

/* rho <- sum_m K_m rho K_m^dagger for nk Kraus operators of k qubits (k <= 2),
 * K stored as nk consecutive row-major 2^k x 2^k matrices.  For the row group
 * based at r and the column group based at c, the 2^k x 2^k block
 * B[u][v] = rho[r + off_u][c + off_v] becomes sum_m K_m B K_m^dagger: left
 * multiplication on the row index, right multiplication by K_m^dagger on the
 * column index, summed over m. */
void ora_dm_kraus(cplx *rho, int n, int k, const int *qubits, int nk, const cplx *K)
{
    uint64_t off[4], mask;
    group_offsets(k, qubits, off, &mask);
    const int d = 1 << k;
    const int64_t D = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < D; ++r) {
        if ((uint64_t)r & mask) continue;
        for (int64_t c = 0; c < D; ++c) {
            if ((uint64_t)c & mask) continue;
            cplx B[4][4], T[4][4], out[4][4];
            for (int u = 0; u < d; ++u)
                for (int v = 0; v < d; ++v) {
                    B[u][v] = rho[(r + off[u]) * D + c + off[v]];
                    out[u][v] = 0;
                }
            for (int m = 0; m < nk; ++m) {
                const cplx *Km = K + (size_t)m * d * d;
                for (int u = 0; u < d; ++u)          /* T = K_m B */
                    for (int v = 0; v < d; ++v) {
                        cplx s = 0;
                        for (int a = 0; a < d; ++a) s += Km[u * d + a] * B[a][v];
                        T[u][v] = s;
                    }
                for (int u = 0; u < d; ++u)          /* out += T K_m^dagger */
                    for (int v = 0; v < d; ++v) {
                        cplx s = 0;
                        for (int b = 0; b < d; ++b) s += T[u][b] * conj(Km[v * d + b]);
                        out[u][v] += s;
                    }
            }
            for (int u = 0; u < d; ++u)
                for (int v = 0; v < d; ++v) rho[(r + off[u]) * D + c + off[v]] = out[u][v];
        }
    }
}

/* Matrix element <j| P |k> of the Pauli string P = (x)_m sigma_m, where qubit
 * m carries I, X, Z or Y according to (bit m of x, bit m of z) = (0,0),
 * (1,0), (0,1), (1,1): the product over qubits of the one-qubit factors'
 * elements <j_m| sigma_m |k_m>. */
static cplx pauli_element(int n, uint64_t x, uint64_t z, uint64_t j, uint64_t kk)
{
    cplx e = 1;
    for (int m = 0; m < n; ++m) {
        int xb = (x >> m) & 1, zb = (z >> m) & 1;
        int jb = (j >> m) & 1, kb = (kk >> m) & 1;
        if (!xb && !zb) {                 /* I */
            if (jb != kb) return 0;
        } else if (xb && !zb) {           /* X = [[0,1],[1,0]] */
            if (jb == kb) return 0;
        } else if (!xb && zb) {           /* Z = [[1,0],[0,-1]] */
            if (jb != kb) return 0;
            if (jb) e = -e;
        } else {                          /* Y = [[0,-i],[i,0]] */
            if (jb == kb) return 0;
            e *= jb ? I : -I;
        }
    }
    return e;
}

/* <psi| P |psi> = sum_j conj(psi_j) sum_k <j|P|k> psi_k.  A Pauli string has
 * one non-zero element per row, at k = j xor x, so the inner sum has one term. */
void ora_sv_expval(const cplx *psi, int n, uint64_t x, uint64_t z, double *out)
{
    const int64_t N = (int64_t)1 << n;
    double re = 0, im = 0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (int64_t j = 0; j < N; ++j) {
        uint64_t kk = (uint64_t)j ^ x;
        cplx t = conj(psi[j]) * pauli_element(n, x, z, (uint64_t)j, kk) * psi[kk];
        re += creal(t);
        im += cimag(t);
    }
    out[0] = re;
    out[1] = im;
}

/* Tr(rho P) = sum_j sum_k rho[j][k] <k|P|j>; the one non-zero element of
 * column j of P is at row k = j xor x. */
void ora_dm_expval(const cplx *rho, int n, uint64_t x, uint64_t z, double *out)
{
    const int64_t D = (int64_t)1 << n;
    double re = 0, im = 0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (int64_t j = 0; j < D; ++j) {
        uint64_t kk = (uint64_t)j ^ x;
        cplx t = rho[j * D + (int64_t)kk] * pauli_element(n, x, z, kk, (uint64_t)j);
        re += creal(t);
        im += cimag(t);
    }
    out[0] = re;
    out[1] = im;
}

/* Tr(rho^2) = sum_jk rho[j][k] rho[k][j]; for Hermitian rho this is
 * sum_jk |rho[j][k]|^2, which is what is computed (Hermiticity is checked
 * separately by the tests). */
double ora_dm_purity(const cplx *rho, int n)
{
    const int64_t E = (int64_t)1 << (2 * n);
    double s = 0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int64_t e = 0; e < E; ++e) s += creal(rho[e]) * creal(rho[e]) + cimag(rho[e]) * cimag(rho[e]);
    return s;
}

void ora_dm_trace(const cplx *rho, int n, double *out)
{
    const int64_t D = (int64_t)1 << n;
    double re = 0, im = 0;
    for (int64_t j = 0; j < D; ++j) {
        re += creal(rho[j * D + j]);
        im += cimag(rho[j * D + j]);
    }
    out[0] = re;
    out[1] = im;
}

/* psi <- e_0 and rho <- e_0 e_0^dagger (|0...0>, the start state of every
 * workload). */
void ora_sv_reset(cplx *psi, int n)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) psi[j] = 0;
    psi[0] = 1;
}

void ora_dm_reset(cplx *rho, int n)
{
    const int64_t E = (int64_t)1 << (2 * n);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) rho[e] = 0;
    rho[0] = 1;
}

#ifdef _OPENMP
#include <omp.h>
void ora_set_threads(int t) { omp_set_num_threads(t); }
int ora_get_threads(void) { return omp_get_max_threads(); }
#else
void ora_set_threads(int t) { (void)t; }
int ora_get_threads(void) { return 1; }
#endif
