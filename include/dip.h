/* Learned induced-dipole head trained through the PME model.
 *
 * The head follows the dipole readout of Sec. 2.2 (Eq. dipole_pred): an
 * invariant-weighted sum of equivariant vector features of the neighbourhood.
 * Fixed local features within r_c replace the paper's message-passing backbone.
 *
 * Features of atom i (neighbours j within r_c, minimum image, R_ij = r_i - r_j):
 *     R_k(r)    = sqrt(2 / r_c) sin(k pi r / r_c) / r * f(r / r_c),   k = 1..8
 *     f(x)      = 1 - 21 x^5 + 35 x^6 - 15 x^7 for x < 1, else 0
 *     G_i[s,k]  = sum_{j of species s} R_k(r_ij)
 *     V_i[s,k]  = sum_{j of species s} q_j R_k(r_ij) R_ij / r_ij
 * Species are cation (q > 0) and anion (q <= 0); channel c = 8 s + k - 1.
 *
 * Inputs and network:
 * - feat[i] = [G_i (16), |V_i[c]|^2 (16), one-hot species of i (2)] (34 values);
 *   vec[i] = V_i as [16][3].
 * - An MLP 34 -> 64 -> 64 -> 16 with SiLU on the two hidden layers gives the
 *   channel weights w_i, and mu_i = sum_c w_ic V_i[c].
 * - Parameters are one float array of DIP_NPARAM values:
 *   W1 [64][34], b1 [64], W2 [64][64], b2 [64], W3 [16][64], b3 [16].
 *
 * Training loss (Eq. loss, with teacher values from the polarizable model of pol.h):
 *     L = lE ((U_s - U_t)/n)^2 + lF mean (dU/dr_s - dU/dr_t)^2 + lmu mean (mu - mu_t)^2
 * so forces enter as -dU/dr.  Its dipole gradient is
 *     dL/dmu = dL/dU dU/dmu + H_{mu r} v + 2 lmu (mu - mu_t)/(3n),
 *     v = dL/d(dU/dr).
 * dip_loss returns v and the first and last terms.  H_{mu r} v is the dipole
 * output of pme_backward with position cotangent v, plus pol_real_mixed.
 *
 * Conventions as in pme.h: device FP32 arrays, asynchronous on `stream`,
 * PME_* return codes.
 */
#ifndef DIP_MI355X_H
#define DIP_MI355X_H

#include <stdint.h>

#include "pme.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DIP_NFEAT 34
#define DIP_NCH 16
#define DIP_HIDDEN 64
#define DIP_NPARAM 7440

typedef struct dip_plan_s* dip_plan_t;

typedef struct {
    int32_t max_atoms;   /* capacity, >= 1                                        */
    int32_t flags;       /* 0                                                      */
    double  box[9];      /* host cell (rows are lattice vectors) of every call     */
    double  cutoff;      /* feature cutoff r_c, below half the smallest width      */
} dip_desc_t;

int dip_plan_create(const dip_desc_t* desc, dip_plan_t* out);
void dip_plan_destroy(dip_plan_t plan);

/* Features of n atoms: feat [n][34], vec [n][16][3] (device outputs). */
int dip_features(dip_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                 float* feat, float* vec);

/* Dipoles mu [n][3] of the network with parameters `params` [DIP_NPARAM]. */
int dip_forward(dip_plan_t plan, void* stream, int32_t n, const float* params, const float* feat,
                const float* vec, float* mu);

/* Parameter gradient g_params [DIP_NPARAM] (overwritten) from dipole gradients
 * dL/dmu = g_mu0 + g_mu1 + g_mu2 (each [n][3], NULL = zero); the network is
 * re-evaluated, nothing from dip_forward is kept.  Deterministic: per-workgroup
 * partial sums are reduced in a fixed order. */
int dip_backward(dip_plan_t plan, void* stream, int32_t n, const float* params, const float* feat,
                 const float* vec, const float* g_mu0, const float* g_mu1, const float* g_mu2,
                 float* g_params);

/* Position vector-Jacobian product of the dipole head: g_pos[j] = sum_i (d mu_i /
 * d r_j)^T u_i (overwritten), for u [n][3] (device).  With u = dU/dmu it is the
 * term that turns the Hellmann-Feynman force of Eq. loss into the conservative
 * student force F = -dU(r, mu_NN(r))/dr = -(dU/dr + g_pos) (the total derivative
 * through the dipole prediction, Eq. forces).  feat and vec are dip_features of
 * the same (pos, q); the network runs back to its inputs, then the position
 * derivatives of the features are summed per atom over its pairs (each pair is
 * visited from both atoms; no atomics).  Uses the plan's cell list (rebuilt
 * here) and its [max_atoms][64] cotangent workspace; calls on one plan must not
 * overlap. */
int dip_position_vjp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* pos, const float* q, const float* feat, const float* vec,
                     const float* u, float* g_pos);

/* Loss of the student (U_s, dUdr_s at dipoles mu, with dU/dmu dUdmu_s) against
 * the teacher (U_t, dUdr_t, mu_t; mu_t may be NULL when lmu = 0).
 *   loss   device double[1]
 *   v_pos  device float[n][3]: dL/d(dU/dr), the cotangent for H_{mu r}
 *   g_mu   device float[n][3]: dL/dU dU/dmu + 2 lmu (mu - mu_t)/(3n) */
int dip_loss(dip_plan_t plan, void* stream, int32_t n, const double* U_s, const double* U_t,
             const float* dUdr_s, const float* dUdr_t, const float* mu, const float* mu_t,
             const float* dUdmu_s, double lE, double lF, double lmu, double* loss,
             float* v_pos, float* g_mu);

/* One Adam step (t = 1, 2, ...) on `count` parameters:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int dip_adam(void* stream, int32_t count, int32_t t, double lr, double beta1, double beta2,
             double eps, float* params, const float* grad, float* m, float* v);

#ifdef __cplusplus
}
#endif
#endif /* DIP_MI355X_H */
