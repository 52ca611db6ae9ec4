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
 * Charge head (Sec. 2.2, Eq. charge_pred): a two-layer perceptron with SiLU on
 * the same 34 inputs, c_i = w2 . silu(W1q feat_i + b1q), and
 *     q_i = z_i + c_i - (1/n) sum_k c_k,
 * the formal charges z (the q of dip_features, which fix the species and the
 * vector weights) plus a centred correction, so the cell keeps its total charge
 * (the PME energy assumes a neutral cell).  An output bias would cancel in the
 * centring and is left out.  Parameters: W1q [64][34], b1q [64], w2q [64]
 * (DIP_NQPARAM values).
 *
 * Conservative forces (Eq. forces) of U(r, q(r), mu(r)) add the head channels
 * J_q^T dU/dq + J_mu^T dU/dmu to dU/dr (dip_position_vjp).  Training on them
 * needs the parameter derivative of v . dU/dr, v = dL/d(dU/dr), which is
 * second order: with t = (v, q_dot, mu_dot) the tangent of (r, q, mu) along v,
 *     dL/dtheta = [a U_q + H_q. t]^T dq/dtheta + [a U_mu + H_mu. t]^T dmu/dtheta
 *               + U_q^T d(q_dot)/dtheta + U_mu^T d(mu_dot)/dtheta,
 * a = dL/dU, U_q = dU/dq, U_mu = dU/dmu, H_q. and H_mu. the q and mu rows of the
 * model Hessian (pol_model_hvp).  The calls in order: dip_features_jvp (the
 * feature tangent along v), dip_charges and dip_forward_jvp (q_dot, mu_dot),
 * pol_model_hvp, dip_backward_jvp (reverse mode through the forward-mode
 * networks).
 *
 * Conventions as in pme.h: device FP32 arrays, asynchronous on `stream`,
 * PME_* return codes.  A plan's workspaces are shared by its calls: calls on one
 * plan must not overlap in time.
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
#define DIP_NQPARAM 2304

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

/* Position vector-Jacobian product of the heads: g_pos[j] = base[j] + sum_i
 * [(d mu_i / d r_j)^T u_i + (d q_i / d r_j) c_i] (overwritten), for cotangents u
 * [n][3] on the dipoles and c [n] on the charges (either may be NULL, not both;
 * base NULL = zero).  With u = dU/dmu, c = dU/dq and base = dU/dr (pol_model) it
 * is the conservative student gradient dU(r, q_NN(r), mu_NN(r))/dr = -F of
 * Eq. forces.  feat and vec are dip_features of the same (pos, q = formal
 * charges); params (dipole head) is needed with u, qparams (charge head) with c.
 * The networks run back to their inputs (the charge cotangent centred first),
 * then the position derivatives of the features are summed per atom over its
 * pairs (each pair is visited from both atoms; no atomics).  Uses the plan's
 * cell list (rebuilt here) and its [max_atoms][64] cotangent workspace. */
int dip_position_vjp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* qparams, const float* pos, const float* q, const float* feat,
                     const float* vec, const float* u, const float* c, const float* base,
                     float* g_pos);

/* Directional derivative of dip_features along the position tangent v [n][3]:
 *     G_dot  = sum_j R_k'(r) r_dot
 *     V_dot  = sum_j q_j [R_k'(r) r_dot u + R_k(r)/r (w - r_dot u)]
 * (w = v_i - v_j, u = R/r, r_dot = u . w), the |V_c|^2 entries 2 V_c . V_dot_c
 * and zeros for the species one-hot.  vec is dip_features' output for the same
 * (pos, q).  Outputs feat_dot [n][34], vec_dot [n][16][3]. */
int dip_features_jvp(dip_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                     const float* vec, const float* v, float* feat_dot, float* vec_dot);

/* Charges of the charge head q [n] from the formal charges z [n] and features,
 * and (feat_dot non-NULL) the tangent q_dot [n] = centred directional
 * derivative along feat_dot (NULL feat_dot: q_dot = 0).  Either output may be
 * NULL, not both. */
int dip_charges(dip_plan_t plan, void* stream, int32_t n, const float* qparams, const float* z,
                const float* feat, const float* feat_dot, float* q, float* q_dot);

/* Dipoles mu (as dip_forward) and their tangent mu_dot_i = sum_c (w_dot_ic V_ic +
 * w_ic V_dot_ic), w_dot the network's directional derivative along feat_dot
 * (NULL feat_dot, vec_dot = zero tangents).  Either output may be NULL. */
int dip_forward_jvp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                    const float* feat, const float* vec, const float* feat_dot,
                    const float* vec_dot, float* mu, float* mu_dot);

/* Parameter gradients of both heads (overwritten; either may be NULL, not both)
 * for a loss of the heads' outputs and their tangents along one position
 * direction, given
 *   on mu:      g_mu0 + g_mu1   [n][3]    on mu_dot: u [n][3]
 *   on q:       g_q0 + g_q1     [n]       on q_dot:  c [n]
 * (NULL = zero) and the feature tangents of dip_features_jvp (NULL = zero: then
 * u and c have no effect and this is the first-order gradient).  Reverse mode
 * through the forward-mode networks, so silu'' couples the two passes; charge
 * cotangents are centred as the charges are.  Deterministic: at most 512
 * workgroups each sum their tiles, then the partial rows are added in order. */
int dip_backward_jvp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* qparams, const float* feat, const float* vec,
                     const float* feat_dot, const float* vec_dot, const float* g_mu0,
                     const float* g_mu1, const float* u, const float* g_q0, const float* g_q1,
                     const float* c, float* g_params, float* g_qparams);

/* Loss of the student (U_s, dUdr_s at dipoles mu, with dU/dmu dUdmu_s and dU/dq
 * dUdq_s) against the teacher (U_t, dUdr_t, mu_t; mu_t may be NULL when lmu = 0).
 * dUdr_s is the Hellmann-Feynman gradient or the conservative one of
 * dip_position_vjp.
 *   loss   device double[1]
 *   v_pos  device float[n][3]: dL/d(dU/dr), the cotangent for the Hessian rows
 *   g_mu   device float[n][3]: dL/dU dU/dmu + 2 lmu (mu - mu_t)/(3n)
 *   g_q    device float[n]: dL/dU dU/dq (with dUdq_s; both NULL or neither) */
int dip_loss(dip_plan_t plan, void* stream, int32_t n, const double* U_s, const double* U_t,
             const float* dUdr_s, const float* dUdr_t, const float* mu, const float* mu_t,
             const float* dUdmu_s, const float* dUdq_s, double lE, double lF, double lmu,
             double* loss, float* v_pos, float* g_mu, float* g_q);

/* One Adam step (t = 1, 2, ...) on `count` parameters:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int dip_adam(void* stream, int32_t count, int32_t t, double lr, double beta1, double beta2,
             double eps, float* params, const float* grad, float* m, float* v);

#ifdef __cplusplus
}
#endif
#endif /* DIP_MI355X_H */
