/* Variational Monte Carlo around block SR on MI355X (gfx950): sampling,
 * local energies and the parameter step for an RBM on the spin-1/2
 * Heisenberg chain (paper, Sec. 3, Heisenberg paragraph: H = J sum_i
 * S_i . S_{i+1}, S = sigma / 2; Eq. 1 for the energy as an average of local
 * energies over samples from |psi|^2).  With qgt_rbm_jacobian (O) and
 * qgt_block_form / qgt_block_solve (delta), one VMC iteration runs on the
 * device from theta to theta - eta delta.
 *
 * RBM: log psi(x) = sum_i a_i x_i + sum_h logcosh(b_h + sum_i W_hi x_i) with
 * N visible and M hidden units; theta device complex128 [W (M x N, row-major)
 * | b (M) | a (N)], the layout of qgt_rbm_jacobian.  logcosh as in
 * qgt_jacobian.h.  Configurations: device int8, one row of N spins (+1 or -1
 * only) per chain or sample, row stride ldx >= N.  Limits: N in [2, 64], M in
 * [1, 65535].  Every call runs on the given stream, allocates nothing and does
 * not synchronise; argument errors return synchronously
 * (QGT_ERR_INVALID_ARGUMENT, QGT_ERR_UNSUPPORTED), a failed launch
 * QGT_ERR_HIP (detail: qgt_last_error()).
 */
#ifndef QGT_VMC_H
#define QGT_VMC_H

#include "qgt_block.h"

#ifdef __cplusplus
extern "C" {
#endif

/* n_steps Metropolis steps of n_chains independent chains (x updated in
 * place).  Step s of chain c proposes the exchange of spins
 * pairs[2 (s n_chains + c)] and pairs[2 (s n_chains + c) + 1] (device int32;
 * a no-op when the spins are equal or an index is outside [0, N)) and
 * accepts it when u[s n_chains + c] < |psi(x') / psi(x)|^2 (device double,
 * the caller's uniforms in [0, 1)); exchange moves keep the magnetisation.
 * accepted (device int32, n_chains entries, may be null) receives the number
 * of accepted moves of each chain in this call. */
qgt_status qgt_rbm_metropolis(int32_t n_visible, int32_t n_hidden, const void* theta, int8_t* x, int64_t ldx,
                              int64_t n_chains, int32_t n_steps, const int32_t* pairs, const double* u,
                              int32_t* accepted, hipStream_t stream);

/* Local energies e_loc[s] (device complex128, n_s entries) of the samples x:
 * E_loc(x) = J sum_bonds [x_i x_j / 4 + [x_i != x_j] psi(x^{ij}) / (2 psi(x))],
 * bonds (i, i + 1) and, when periodic != 0 and N > 2, (N - 1, 0); x^{ij} is x
 * with spins i and j exchanged. */
qgt_status qgt_rbm_heisenberg_eloc(int32_t n_visible, int32_t n_hidden, const void* theta, const int8_t* x,
                                   int64_t ldx, int64_t n_s, double J, int32_t periodic, void* e_loc,
                                   hipStream_t stream);

/* theta[k] <- theta[k] - eta delta[k], k < n_p (device complex128): the SR
 * step with the update direction delta returned by qgt_block_solve (paper,
 * Sec. 2: the block updates concatenated, scaled by the learning rate). */
qgt_status qgt_sr_update(void* theta, const void* delta, int64_t n_p, double eta, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QGT_VMC_H */
