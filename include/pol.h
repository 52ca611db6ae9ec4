/* Thole-damped polarizable point-charge model on top of the PME library.
 *
 * This is the self-consistent induced-dipole teacher of the learned dipole head.
 * - The paper's own polarization is not self-consistent (Sec. 4), and it cites Thole
 *   damping without giving its form.
 * - Damping here is exponential with exponent A: s = (a_i a_j)^(1/6), u = r/s,
 *   e = exp(-A u^3), and the damped Ewald functions are
 *       B1t = B1 - e / r^3
 *       B2t = B2 - 3 (1 + A u^3) e / r^5
 *       B3t = B3 - 15 (1 + A u^3 + 0.6 A^2 u^6) e / r^7.
 *
 * Model:
 *     U(mu) = E_lr(q, mu) + E_real(q, mu) + sum_i |mu_i|^2 / (2 a_i)
 *
 * - E_lr is the PME long-range energy (pme_forward; Secs. 2.3.1-2.3.5).
 * - E_real is the real-space Ewald pair sum within the cutoff r_c. Its
 *   charge-charge term is undamped, with B0 = erfc(alpha r)/r.
 * - Its charge-dipole and dipole-dipole terms use the Thole-damped B_l^t above,
 *   in the pair form of the explicit Ewald sum:
 *       q_i q_j B0 + (q_i mu_j - q_j mu_i).R B1t + (mu_i.mu_j) B1t
 *         - (mu_i.R)(mu_j.R) B2t
 *
 * Conventions, as in pme.h:
 * - Per-atom arrays are device FP32; pos is [n][3], pol (the polarizabilities
 *   a_i, in Angstrom^3) is [n].
 * - Outputs are overwritten; a NULL output is skipped; a NULL q or mu means zero.
 * - Calls are asynchronous on `stream`, except pol_scf, which synchronises once
 *   per iteration to test convergence (unless POL_F_FIXED_ITERS).
 * - A plan's workspaces are shared by its calls: calls on one plan must not
 *   overlap in time (one stream, or ordered by events).
 * - Every energy and gradient is multiplied by `prefactor`, including the
 *   polarization term, so the dipoles do not depend on it. It must equal the
 *   prefactor of the PME plan used with pol_scf.
 * - Return codes are the PME_* codes of pme.h.
 */
#ifndef POL_MI355X_H
#define POL_MI355X_H

#include <stdint.h>

#include "pme.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pol_plan_s* pol_plan_t;

typedef struct {
    int32_t max_atoms;   /* capacity, >= 1                                        */
    int32_t flags;       /* POL_F_* bits                                           */
    double  box[9];      /* host copy of the cell (rows = lattice vectors); it fixes
                            the cell-list grid, and every call uses this cell      */
    double  alpha;       /* Ewald splitting parameter, equal to the PME plan's    */
    double  cutoff;      /* real-space cutoff r_c: > 0 and below half the smallest
                            perpendicular width of the cell (minimum image)       */
    double  thole_a;     /* Thole exponent A (0.39), >= 0; 0 disables damping     */
    double  prefactor;   /* energy unit factor, equal to the PME plan's           */
} pol_desc_t;

/* pol_scf: start from the dipoles in `mu` instead of zero. */
#define POL_F_WARM_START 1
/* pol_scf: run exactly max_iter iterations and never synchronise the stream (no
 * host-side convergence test), so that a solve can be captured into a HIP graph;
 * *iters receives max_iter and *resid -1 (the caller checks the solution, e.g. by
 * the stationarity dU/dmu = 0 of pol_model).  The PME plan's binnings in such a
 * solve are 1 + max_iter (2 + max_iter with POL_F_WARM_START). */
#define POL_F_FIXED_ITERS 2

/* Validate `desc`, build the cell grid and allocate the workspaces.  Returns
 * PME_EINVAL for a bad cell, cutoff, alpha or exponent. */
int pol_plan_create(const pol_desc_t* desc, pol_plan_t* out);
void pol_plan_destroy(pol_plan_t plan);

/* Real-space pair sum E_real and its gradients (pair form above; each pair
 * within r_c under the minimum image).
 *   energy   device double[1] or NULL
 *   dE_dpos  device float[n*3] or NULL
 *   dE_dq    device float[n] or NULL: sum_j [q_j B0 + (mu_j . R_ij) B1t]
 *   dE_dmu   device float[n*3] or NULL */
int pol_real(pol_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
             const float* mu, const float* pol, double* energy, float* dE_dpos, float* dE_dq,
             float* dE_dmu);

/* Mixed second derivative of E_real applied to a position cotangent:
 * g_mu = d/dmu (grad_r E_real . v_pos).  Used for the force-loss gradient of
 * learned dipoles. */
int pol_real_mixed(pol_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                   const float* mu, const float* pol, const float* v_pos, float* g_mu);

/* U(q, mu) of the model and its gradients at the given charges and dipoles
 * (pme_forward + pol_real + the polarization term sum |mu|^2 / (2 a)).  The
 * teacher's forces are -dU_dpos at the self-consistent dipoles; a student's
 * Hellmann-Feynman forces the same at its predicted ones.
 *   energy   device double[1] or NULL
 *   dU_dpos  device float[n*3] or NULL
 *   dU_dq    device float[n] or NULL (the electrostatic potential at each atom)
 *   dU_dmu   device float[n*3] or NULL */
int pol_model(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
              const float* q, const float* mu, const float* pol, const double* box,
              double* energy, float* dU_dpos, float* dU_dq, float* dU_dmu);

/* The q and mu rows of the Hessian of U in (r, q, mu) applied to the tangent
 * (v_pos, v_q, v_mu) (each NULL = zero):
 *   g_q  = d/dq  (grad U . t),  device float[n]
 *   g_mu = d/dmu (grad U . t),  device float[n*3]
 * PME part: pme_backward with the three cotangents (Sec. 2.3.5).  Real-space
 * part: E_real is bilinear in (q, mu), so its (q, mu) columns are the pol_real
 * gradients with charges v_q and dipoles v_mu; its r column differentiates
 * dE/dq_i and dE/dmu_i along w = v_i - v_j (grad B0 = -R B1 undamped, grad
 * B_l^t = -R B_{l+1}^t).  The polarization term adds (prefactor / a) v_mu.
 * These rows are what training a charge and dipole head on forces needs
 * (Eq. loss with the forces of Eq. forces). */
int pol_model_hvp(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
                  const float* q, const float* mu, const float* pol, const double* box,
                  const float* v_pos, const float* v_q, const float* v_mu, float* g_q,
                  float* g_mu);

/* Self-consistent induced dipoles by preconditioned conjugate gradients.
 *
 * The system is (diag(1/a) + H_real + H_pme) mu = -(dE_lr/dmu + dE_real/dmu) at mu = 0.
 * - H_pme v is pme_backward with a dipole cotangent v.
 * - H_real v is pol_real with the dipoles v and no charges.
 * - The preconditioner is diag(a).
 *
 * Iterations stop when the RMS of the preconditioned residual, in e*Angstrom,
 * falls below `tol`, or after `max_iter` iterations.
 *
 * Arguments:
 * - pme: a plan with the same alpha and prefactor (PME_F_KEEP_PHI saves one
 *   potential per iteration).
 * - box: the device copy of the cell, as for pme_forward.
 * - mu: the solution (device float[n*3]); also the initial guess under
 *   POL_F_WARM_START.
 * - iters, resid: host outputs (the iterations taken and the final RMS), or NULL.
 */
int pol_scf(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
            const float* q, const float* pol, const double* box, double tol, int32_t max_iter,
            float* mu, int32_t* iters, double* resid);

#ifdef __cplusplus
}
#endif
#endif /* POL_MI355X_H */
