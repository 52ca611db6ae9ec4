/*
 * pme.h -- C ABI of the MI355X (gfx950) differentiable particle-mesh Ewald
 * for per-atom charges q and point dipoles mu.
 *
 * What is computed (paper: "Differentiable Particle-Mesh Ewald with Cartesian
 * Tensor Message Passing ...", Sec. 2.3):
 *
 *   rho(n)  = sum_i sum_stencil [ q_i W + sum_a N_a (mu_i . C^-1[:,a]) dW/dx_a ]
 *                                                       (Eq. charge_dipole_assign)
 *             W = M_p(x_x - n_x) M_p(x_y - n_y) M_p(x_z - n_z), x = N * frac(r C^-1),
 *             M_p the centered cardinal B-spline of order p (Sec. 2.3.2, Eq. w3d)
 *   phi     = IDFT[ g(k) DFT[rho] ]  (unnormalised inverse, real part)
 *             g = 4 pi/|k|^2 exp(-|k|^2/4a^2) / |B(n)|^(2 gamma), g(0) = 0,
 *             B(n) = prod_a sinc^p(n_a/N_a), k = sum_a n_a b_a, b = 2 pi C^-T
 *                                      (Eqs. fft, Bk, influence, green, potential_k,
 *                                       ifft)
 *   E_recip = (1/2V) sum_n rho(n) phi(n)                     (Eq. energy_recip)
 *   E_self  = -a/sqrt(pi) sum q^2 - 2a^3/(3 sqrt(pi)) sum |mu|^2
 *                                                  (Eqs. self_q, self_mu)
 *   E^lr    = E_recip + E_self                               (Eq. E_lr_total)
 *
 * and its exact derivatives (what autograd of the paper's pipeline yields,
 * Sec. 2.3.5 and Eq. forces): dE/dr, dE/dq, dE/dmu, and the Hessian-vector
 * product, which is also the force-loss double backward of training
 * (Eq. loss).
 *
 * Units: positions in Angstrom, q in e, mu in e*Angstrom; energies are
 * e^2/Angstrom times `prefactor` (14.3996454784 gives eV).
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory (hipMalloc / torch CUDA tensors),
 *     contiguous, float32 unless stated; the caller owns them and keeps them
 *     alive until the stream work completes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - No call synchronises the stream except pme_status.  Device-detected
 *     problems (non-finite positions or box) are reported by pme_status.
 *   - Outputs are overwritten, never accumulated.  A NULL output is skipped.
 *   - A plan owns all of its workspaces; it is not thread safe and must not be
 *     used by two streams at once.
 *   - Return codes are PME_OK or a negative PME_E* value; pme_strerror maps
 *     them to text.  Host-side checks run before anything is launched, so a
 *     failed call leaves the outputs untouched.
 */
#ifndef PME_MI355X_H
#define PME_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define PME_OK          0
#define PME_EINVAL     -1   /* NULL required pointer, n < 0, bad flag or strategy */
#define PME_EORDER     -2   /* assignment order p outside 1..7                    */
#define PME_EMESH      -3   /* a mesh dimension is not 5-smooth or outside 2..1024 */
#define PME_EALPHA     -4   /* alpha <= 0, non-finite alpha/gamma/prefactor, gamma < 0 */
#define PME_ECAPACITY  -5   /* n > max_atoms of the plan                          */
#define PME_ENOMEM     -6   /* device allocation failed                           */
#define PME_EHIP       -7   /* a HIP runtime call failed (see pme_last_hip_error) */
#define PME_ENONFINITE -8   /* device saw NaN/Inf in positions or box (pme_status) */
#define PME_ESCRATCH   -9   /* pme_forward_noalloc: workspace above its fixed scratch */

/* ---- plan flags ------------------------------------------------------ */
/* Keep phi (the potential mesh) of the last pme_forward; a following
 * pme_backward with the same (pos, q, mu, box) then reuses it instead of
 * recomputing it.  The caller asserts the inputs are unchanged. */
#define PME_F_KEEP_PHI  1
/* Allocate a second set of atom records, counters, density and spectrum (about
 * doubling the plan's workspace) and a second stream, so that pme_step runs the
 * forward chain and the cotangent's chain (its density, transform and potential)
 * concurrently. */
#define PME_F_CONCURRENT 2
/* Use the energy-optimal influence function with aliasing sums instead of the
 * sinc^(-2 gamma p) deconvolution of Eq. influence (influence_power is then
 * unused):  g(f) = sum_m U^2(f + m N) G(k(f + m N)) / (sum_m U^2(f + m N))^2,
 * U(f) = prod_a sinc(f_a / N_a)^p, m in {-1, 0, 1}^3.  Not with pme_forward_cell
 * (PME_EINVAL); in a batch, every box or none. */
#define PME_F_OPT_INFLUENCE 4
/* Spread the density by mesh tiles and transform it in a separate pass.  Without
 * this flag, a plan whose y-z plane, padded by p - 1 rows and columns, fits in LDS
 * beside a transform buffer (meshes up to about 110 points in y and z, and N >= p
 * plus the bin size on every axis) spreads by x-planes and transforms each plane
 * in the same workgroup (Sec. 2.3.2 and Eq. fft); a larger mesh with N >= p plus
 * the bin size on every axis and p <= 7 spreads by bands of y-rows of each x-plane
 * and transforms in separate passes.  All three give the same density and spectrum
 * bit for bit; the flag exists for comparison and measurement. */
#define PME_F_SEPARATE_SPREAD 8

/* ---- mesh strategies for pme_mesh_dims (Sec. 2.3.1) ------------------- */
#define PME_MESH_POW2    0   /* N = 2^ceil(log2 N_target)                       */
#define PME_MESH_SMOOTH  1   /* smallest N >= N_target with factors {2,3,5}      */
#define PME_MESH_CEIL    2   /* N = N_target (may be rejected by pme_plan) */

typedef struct pme_plan_s* pme_plan_t;

typedef struct {
    int32_t mesh[3];          /* N_x, N_y, N_z: 5-smooth, each in 2..1024        */
    int32_t order;            /* assignment order p, 1..7                         */
    int32_t max_atoms;        /* capacity of the workspaces, >= 1                 */
    int32_t flags;            /* PME_F_* bits                                     */
    double  alpha;            /* Ewald splitting parameter [1/Angstrom], > 0      */
    double  influence_power;  /* gamma of Eq. influence, >= 0 (1 = default,
                                 0 = no assignment deconvolution)                 */
    double  prefactor;        /* energy unit factor (1, or 14.3996454784 for eV)  */
    int32_t tile[3];          /* spread/gather tile target per axis in mesh points
                                 (all 0 = default: per axis the tile near 8, 8, 16
                                 that divides N with an atom-bin size dividing it;
                                 a given target is rounded to the atom-bin size);
                                 shrunk to fit LDS (set by autotuning)            */
    int32_t fft_lines;        /* FFT lines per workgroup of the x pass and of the
                                 pencil y pass, 0..1024 (0 = default: 16 for axes
                                 up to 64 points, 24 up to 160, 4 above); clamped
                                 to the LDS budget and to N_z/2 + 1 columns, then
                                 evened out over the columns (set by autotuning)  */
} pme_desc_t;

/* Eq. mesh_target, N_a = ceil(2 |a_a| / spacing + 1), mapped by `strategy`
 * (PME_MESH_*).  box: host, 3x3 row-major, rows are the lattice vectors.
 * out: host int32[3].  Returns PME_OK or PME_EINVAL (spacing <= 0, singular
 * box, unknown strategy, or a dimension above 2^30). */
int pme_mesh_dims(const double box[9], double spacing, int strategy, int32_t out[3]);

/* The plan of Sec. 2.3.1: mesh dimensions, assignment order p, alpha and the
 * influence power gamma fixed once; the per-axis deconvolution factors
 * |sinc(f/N_a)|^(-2 gamma p) of Eqs. Bk and influence (signed frequency f) are
 * tabulated here, the cell inverse is formed on the device from the caller's box
 * at every call.  Validates `desc` and allocates every workspace on the current
 * HIP device (meshes, spectrum, atom bins, FFT tables, deconvolution tables).
 *   desc   host pointer, read only during the call
 *   out    host pointer; *out receives the plan (NULL on failure), owned by the
 *          caller until pme_plan_destroy
 * Returns PME_OK, PME_EINVAL, PME_EORDER, PME_EMESH, PME_EALPHA, PME_ENOMEM or
 * PME_EHIP; on failure nothing stays allocated. */
int pme_plan(const pme_desc_t* desc, pme_plan_t* out);

/* Release a plan and its device memory (synchronises the device first).
 * NULL is ignored. */
void pme_plan_destroy(pme_plan_t plan);

/* Device bytes held by the plan's workspaces (0 for NULL). */
int64_t pme_plan_workspace_bytes(pme_plan_t plan);

/* Identifier of the evaluation whose potential phi (Eqs. potential_k, ifft) the
 * plan keeps for a following pme_backward under PME_F_KEEP_PHI: every call that
 * writes the kept phi (pme_forward, pme_forward_cell, pme_step, pme_step_replay,
 * and pme_backward when it recomputes phi) gives it a new identifier, unique per
 * plan and increasing; 0 when no phi is kept (after pme_forward_quad, or before
 * the first evaluation).  A caller that evaluates several frames on one plan
 * (the batch loss of Sec. 2.4, Eq. loss) records the identifier after each
 * forward and, before the backward of an earlier frame, calls pme_plan_drop_phi
 * when the identifier has changed, so that phi is recomputed from that frame's
 * inputs.  Host-side state: no synchronisation.  Returns 0 for NULL. */
int64_t pme_plan_phi_id(pme_plan_t plan);

/* Forget the kept phi: the next pme_backward recomputes it from its own
 * (pos, q, mu, box).  Host-side state only.  PME_OK, or PME_EINVAL for NULL. */
int pme_plan_drop_phi(pme_plan_t plan);

/* Forward evaluation (Secs. 2.3.2-2.3.5).
 *   n                atoms, 0 <= n <= max_atoms
 *   pos              device float[n*3], Cartesian, any periodic image
 *   q                device float[n] or NULL (all charges zero)
 *   mu               device float[n*3] or NULL (all dipoles zero)
 *   box              device double[9], row-major, rows a_x, a_y, a_z
 *   energy           device double[3] or NULL: E_recip, E_self_q, E_self_mu
 *                    (their sum is E^lr), each times prefactor
 *   dE_dpos          device float[n*3] or NULL  (forces are -dE_dpos)
 *   dE_dq            device float[n]   or NULL
 *   dE_dmu           device float[n*3] or NULL
 */
int pme_forward(pme_plan_t plan, void* stream, int32_t n,
                const float* pos, const float* q, const float* mu, const double* box,
                double* energy, float* dE_dpos, float* dE_dq, float* dE_dmu);

/* pme_forward (same arguments and outputs) that also returns the gradient of E^lr
 * with respect to the cell at fixed Cartesian positions, charges and dipoles, what
 * the virial/stress loss of Sec. 2.4 differentiates.  The self terms do not depend
 * on the cell; E_recip does through the volume, the k-vectors of the Green's
 * function and the density (mesh coordinates N (r_i C^-1) and x-space dipoles
 * N (mu_i C^-1)):
 *   dE/dC = -E_recip C^-T + (1/V) C^-T T - (1/V) (P + Q) C^-T
 *   T = sum_k |rho~|^2 g (1/k^2 + 1/(4 alpha^2)) k k^T          (the x pass)
 *   P + Q = sum_i s_i (x) N (q_i G_i + H_i J mu_i) + (mu_i C^-1) (x) N G_i
 *           with s_i = r_i C^-1 from the caller's (unwrapped) position  (the gather)
 * (times the prefactor; G_i, H_i the stencil sums of phi with grad W and
 * grad grad W).  The result depends on which periodic image a position is given
 * in: moving atom i by n C changes it by -n (x) dE/dr_i.
 *   dE_dbox   device double[9], row-major like box: dE_dbox[3a+b] = dE/dbox[a][b]
 *   energy    may be NULL (E_recip is then formed in the plan's workspace)
 * Uses the plan's workspace; calls on one plan must not overlap. */
int pme_forward_cell(pme_plan_t plan, void* stream, int32_t n,
                     const float* pos, const float* q, const float* mu, const double* box,
                     double* energy, float* dE_dpos, float* dE_dq, float* dE_dmu,
                     double* dE_dbox);

/* Charges, dipoles and quadrupoles: pme_forward with a third channel, the
 * symmetric Cartesian second moment Theta_i of each atom (the quadrupolar PME
 * channel that Sec. 4 names as the next extension of the method; readings:
 * the density of atom i is q_i delta - mu_i . grad delta + (1/2) Theta_i : grad
 * grad delta, the limit of a point-charge cluster with sum q r r^T = Theta_i, so
 * the mesh density gains (1/2) (J Theta_i J^T) : grad_x grad_x W; the self terms
 * extend Eqs. self_q and self_mu by the screened self-interaction of the
 * quadrupole: + 2a^3/(3 sqrt(pi)) q tr Theta - a^5/(5 sqrt(pi)) (tr^2 Theta +
 * 2 Theta:Theta)).  Theta need not be traceless.
 *   theta     device float[n][6]: xx, yy, zz, xy, xz, yz (e Angstrom^2), or NULL (= 0)
 *   energy    device double[4] or NULL: E_recip, E_self_q, E_self_mu, E_self_theta
 *             (the last holds the q-Theta cross term); E^lr is their sum
 *   dE_dtheta device float[n][6] or NULL: gradient with respect to the six stored
 *             entries (an off-diagonal entry stands for both Theta_ab and Theta_ba)
 *   other arguments and outputs as pme_forward.
 * Needs order p >= 4 (PME_EINVAL otherwise): the density takes second
 * derivatives of the weights, which are discontinuous for p <= 3, and the force
 * third ones.  No
 * Hessian-vector product, cell gradient or batch form for this channel; its
 * potential is not kept for pme_backward.  Launches are timed under the
 * PME_K_BIN, PME_K_SPREAD and PME_K_GATHER kinds.  Uses the plan's workspace;
 * calls on one plan must not overlap. */
int pme_forward_quad(pme_plan_t plan, void* stream, int32_t n,
                     const float* pos, const float* q, const float* mu, const float* theta,
                     const double* box, double* energy, float* dE_dpos, float* dE_dq,
                     float* dE_dmu, float* dE_dtheta);

/* Hessian-vector product of E^lr in (r, q, mu): the derivative of the gradient
 * of Eq. forces (and of the q and mu derivatives of Eqs. energy_recip, self_q,
 * self_mu) that autograd through the pipeline of Sec. 2.3.5 takes when a loss on
 * the forces is trained (Sec. 2.4, Eq. loss).  With the gradient
 * (dE/dr, dE/dq, dE/dmu) of pme_forward and cotangents (v_pos, v_q, v_mu)
 * on it, returns H v, which equals the vector-Jacobian product of the
 * gradient because H is symmetric.  With v_q = v_mu = 0 and v_pos = -dL/dF it
 * is the double backward of a force loss L(F).
 *   pos, q, mu, box  as pme_forward (the point the Hessian is taken at)
 *   v_pos, v_q, v_mu device cotangents (shapes as pos, q, mu) or NULL (= 0)
 *   g_pos, g_q, g_mu device outputs (shapes as pos, q, mu) or NULL (skip)
 * With PME_F_KEEP_PHI the kept potential (pme_plan_phi_id) is reused: the caller
 * asserts that it came from these same inputs.  Without the flag, or after
 * pme_plan_drop_phi, phi is recomputed from (pos, q, mu, box) and kept.
 * Returns PME_OK, PME_EINVAL, PME_ECAPACITY or PME_EHIP. */
int pme_backward(pme_plan_t plan, void* stream, int32_t n,
                 const float* pos, const float* q, const float* mu, const double* box,
                 const float* v_pos, const float* v_q, const float* v_mu,
                 float* g_pos, float* g_q, float* g_mu);

/* pme_forward followed by pme_backward of the same (pos, q, mu, box) in one call
 * (arguments and outputs as there; the backward reuses the forward's phi).  The
 * forward gradient and H v of one evaluation, as a training step with a force
 * loss needs them (Sec. 2.4).  With PME_F_CONCURRENT the cotangent's binning,
 * spread and mesh transform run on the plan's second stream, forked from
 * `stream`, beside the forward chain on `stream`; the second stream is joined back
 * into `stream`, where one gather over the cotangent's records forms H v and the
 * forward outputs from both potentials, so all work is ordered before later work
 * on `stream`.
 * Without the flag the two run in sequence on `stream`.  Calls on one plan must
 * not overlap (they share its workspaces). */
int pme_step(pme_plan_t plan, void* stream, int32_t n,
             const float* pos, const float* q, const float* mu, const double* box,
             double* energy, float* dE_dpos, float* dE_dq, float* dE_dmu,
             const float* v_pos, const float* v_q, const float* v_mu,
             float* g_pos, float* g_q, float* g_mu);

/* Capture `steps` consecutive pme_step calls with these arguments into a HIP
 * graph held by the plan (replacing any earlier one), without running them;
 * pme_step_replay launches it.  Replaying costs one launch instead of about ten
 * per step (the per-step launch overhead and the gaps between dependent kernels
 * shrink), and gives the same results bit for bit as the eager calls.
 * The pointers are baked into the graph: the caller keeps those buffers alive
 * and updates their contents in place between replays.  Each binning alternates
 * between two counter sets, so the captured steps must leave the plan's set
 * parity unchanged (with PME_F_CONCURRENT an even `steps`; PME_EINVAL
 * otherwise), and a replay requires the calls made on the plan since the
 * capture (or the last replay) to have done the same (PME_EINVAL otherwise; one
 * more eager call restores it).  Launches captured into the graph are not
 * timed by pme_plan_timer.
 * Returns PME_OK, PME_EINVAL, PME_ECAPACITY, or PME_EHIP (capture or
 * instantiation failed). */
int pme_step_capture(pme_plan_t plan, int32_t steps, int32_t n,
                     const float* pos, const float* q, const float* mu, const double* box,
                     double* energy, float* dE_dpos, float* dE_dq, float* dE_dmu,
                     const float* v_pos, const float* v_q, const float* v_mu,
                     float* g_pos, float* g_q, float* g_mu);

/* Launch the captured step graph on `stream` (ordered like any other work on
 * it).  PME_EINVAL without a graph or when the counter-set parity differs from
 * the capture's. */
int pme_step_replay(pme_plan_t plan, void* stream);

/* pme_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results as pme_forward on a plan made from `desc` with
 * max_atoms = n, but with no plan.  Every workspace (atom bins and records,
 * counters, density, spectrum, potential, per-axis twiddle and deconvolution
 * tables, energy partials) is carved from one fixed device array of
 * PME_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first use of that
 * GPU until the process ends; the call makes no device or host allocation and
 * does not synchronise.  The tables are rebuilt on the device by every call.
 *   desc     host, read during the call; desc->max_atoms is ignored (sized for n);
 *            PME_F_OPT_INFLUENCE is rejected (PME_EINVAL), the other flags have
 *            no effect
 *   other arguments and outputs as pme_forward
 * Returns PME_ESCRATCH when the workspace of (desc, n) exceeds the array (about
 * 27 MB for 32,000 atoms on 100^3), else as pme_forward.  All calls on one GPU
 * share the array: calls that overlap on one GPU (two streams, or two host
 * threads) race and give wrong results; calls ordered on one stream do not.
 * Non-finite inputs are not reported (there is no plan for pme_status to read). */
#define PME_NOALLOC_SCRATCH_BYTES (64 << 20)
int pme_forward_noalloc(const pme_desc_t* desc, void* stream, int32_t n,
                        const float* pos, const float* q, const float* mu, const double* box,
                        double* energy, float* dE_dpos, float* dE_dq, float* dE_dmu);

/* Synchronise `stream`, then return PME_ENONFINITE if any kernel of this plan
 * saw a non-finite position or box since the last pme_status call, or
 * PME_EHIP if the stream reported an error; else PME_OK.  Clears the flag. */
int pme_status(pme_plan_t plan, void* stream);

/* Text for a return code. */
const char* pme_strerror(int code);

/* Text of the last HIP runtime error seen by the library (thread-local). */
const char* pme_last_hip_error(void);

/* Device pointer of the potential mesh phi (float[N_x*N_y*N_z], z fastest)
 * left by the last pme_forward, and of the density rho it was built from.
 * For inspection and tests; valid until the plan is destroyed.  A plan that
 * spreads by x-planes fused with the transform (the default where it fits, see
 * PME_F_SEPARATE_SPREAD) never stores the density: pme_plan_rho returns NULL. */
const float* pme_plan_phi(pme_plan_t plan);
const float* pme_plan_rho(pme_plan_t plan);

/* How a plan spreads the density (Sec. 2.3.2, Eq. charge_dipole_assign): by mesh
 * tiles, by bands of y-rows of each x-plane, or by x-planes fused with the
 * transform (see PME_F_SEPARATE_SPREAD).  Returns one of the values below, or
 * PME_EINVAL for a NULL plan.  For inspection, tests and measurement. */
#define PME_SPREAD_TILE  0
#define PME_SPREAD_BAND  1
#define PME_SPREAD_FUSED 2
int pme_plan_spread_kind(pme_plan_t plan);

/* ---- batches of boxes ---------------------------------------------------
 * The training loss of Sec. 2.4 (Eq. loss) sums energy and force errors over a
 * batch of structures; each structure is an independent cell with its own PME
 * evaluation (Secs. 2.3.1-2.3.5).  Many such cells of uneven atom count and mesh
 * are evaluated together here: every kernel kind runs once for all boxes, over a
 * list of (box, work item) pairs, instead of once per box.  Per-atom arrays are packed:
 * the atoms of box b occupy [off_b, off_b + n_b), off = exclusive prefix sum of
 * n_atoms; cells are packed as [nbox][9] doubles and energies as [nbox][3].
 * Results equal those of one plan per box, bit for bit (same kernels, same
 * tiles).  A batch needs one order p for all boxes and meshes whose y-z planes
 * fit in LDS (at most about 130 x 130). */
typedef struct pme_batch_s* pme_batch_t;

/* The plan of a batch (Sec. 2.3.1 per box, Sec. 2.4 for the batch): descs[b]
 * describes box b (of its flags only PME_F_OPT_INFLUENCE counts, and it must be
 * set on every box or none; the backward always reuses the potential of the
 * preceding pme_batch_forward); n_atoms[b] >= 0 is its atom count.  Host arrays
 * of nbox entries, read during the call; *out receives the batch (NULL on
 * failure), released by pme_batch_destroy.  PME_EORDER if the orders differ,
 * PME_EMESH if a mesh does not fit, PME_EINVAL if the boxes disagree on the
 * optimal influence function or hold more than 2^31 - 1 atoms in all,
 * PME_ENOMEM/PME_EHIP. */
int pme_batch_plan(const pme_desc_t* descs, int32_t nbox, const int32_t* n_atoms,
                     pme_batch_t* out);
void pme_batch_destroy(pme_batch_t batch);

/* pme_forward of every box (Secs. 2.3.2-2.3.5 and Eq. forces per box; packed
 * device arrays as above; NULL outputs skipped). */
int pme_batch_forward(pme_batch_t batch, void* stream, const float* pos, const float* q,
                      const float* mu, const double* box, double* energy, float* dE_dpos,
                      float* dE_dq, float* dE_dmu);

/* pme_backward of every box (the Hessian-vector product that the force term of
 * Eq. loss needs) with the potentials of the last pme_batch_forward, which the
 * caller asserts came from the same pos, q, mu, box. */
int pme_batch_backward(pme_batch_t batch, void* stream, const float* pos, const float* q,
                       const float* mu, const double* box, const float* v_pos, const float* v_q,
                       const float* v_mu, float* g_pos, float* g_q, float* g_mu);

/* The buffers of one captured training step (all packed, device). */
typedef struct {
    const float* pos; const float* q; const float* mu; const double* box;
    double* energy; float* dE_dpos; float* dE_dq; float* dE_dmu;      /* forward        */
    const float* v_pos; const float* v_q; const float* v_mu;          /* generic H v    */
    float* g_pos; float* g_q; float* g_mu;
    const float* vf_pos;                                              /* force-loss H v */
    float* gf_pos; float* gf_q; float* gf_mu;                         /* (v_q = v_mu = 0) */
} pme_batch_step_t;

/* Capture one training step of Eq. loss over the whole batch -- forward,
 * Hessian-vector product and force-loss double backward -- into one HIP graph
 * owned by the batch (replacing any previous one); nothing runs.  The buffer
 * addresses in `step` (host struct, read during the call) are fixed at capture,
 * their contents are read at every launch.  Capture runs on a stream of the
 * batch's own.  PME_OK, PME_EINVAL or PME_EHIP. */
int pme_batch_graph_capture(pme_batch_t batch, const pme_batch_step_t* step);

/* Launch the graph of pme_batch_graph_capture on `stream` (ordered like other
 * work on it).  PME_EINVAL without a captured graph, PME_EHIP on a launch error. */
int pme_batch_graph_launch(pme_batch_t batch, void* stream);

/* pme_status over every box of the batch (synchronises `stream`). */
int pme_batch_status(pme_batch_t batch, void* stream);

/* ---- launch timing (measurement support) ------------------------------ */
/* Kernel kinds that pme_plan_timer can bracket.  Each kind is one launch (or, in
 * the pencil FFT layout, the two launches of one transform half) per call. */
#define PME_K_NONE           -1
#define PME_K_BIN             0   /* forward binning: stencil anchors, records     */
#define PME_K_BIN_TANGENT     1   /* binning of the tangent density (backward)     */
#define PME_K_SPREAD          2   /* spread of q and mu onto the mesh (Eq.
                                     charge_dipole_assign)                          */
#define PME_K_SPREAD_TANGENT  3   /* spread of the tangent density (backward)      */
#define PME_K_FFT_R2C         4   /* forward real-to-complex passes before the x
                                     pass (Eq. fft)                                 */
#define PME_K_FFT_X           5   /* x pass: forward x FFT, influence multiply
                                     (Eqs. influence, potential_k), energy, inverse */
#define PME_K_FFT_C2R         6   /* inverse complex-to-real passes (Eq. ifft)      */
#define PME_K_GATHER          7   /* gradient gather + energy (Eqs. energy_recip,
                                     forces)                                        */
#define PME_K_GATHER_HVP      8   /* Hessian-vector product gather (backward)       */
#define PME_K_COUNT           9

/* Time every later launch of kernel kind `kind` (PME_K_*) by this plan: the
 * launch records its kernel's own begin and end timestamps into a HIP event
 * pair (hipExtLaunchKernel), so the interval excludes queueing and dispatch.
 * PME_K_NONE stops timing.  Switching kinds discards what was recorded.  Up to
 * 65536 launches are kept between reads; later ones are not timed.  Returns
 * PME_OK, PME_EINVAL (bad kind or plan) or PME_EHIP (event creation failed). */
int pme_plan_timer(pme_plan_t plan, int kind);

/* Wait for the recorded events, then return the number of timed launches in
 * *launches and their summed duration in milliseconds in *total_ms, and clear
 * the record (the kind stays armed).  Host pointers; either may be NULL. */
int pme_plan_timer_read(pme_plan_t plan, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* PME_MI355X_H */
