/*
 * crk.h -- C ABI of the MI355X (gfx950) library for the CRK-SPH particle-pair
 * passes and short-range particle-particle gravity.
 *
 * The paper (Rangel et al., "A Performance-Portable SYCL Implementation of
 * CRK-HACC for Exascale") names the hot GPU kernels of CRK-HACC's adiabatic
 * hydrodynamics -- Geometry (particle volumes), Corrections (reproducing-kernel
 * coefficients), Acceleration (momentum derivative) and Energy (internal
 * energy derivative) -- in Sec. 5, and the short-range gravity evaluated by
 * direct particle-particle interaction after the particle-mesh force split in
 * Sec. 3.1.  Interactions are evaluated between leaves of a recursive
 * coordinate bisection (RCB) tree (Sec. 3.1; Sec. 5.3, Figs. 3-4).  Two
 * species exist: gas feels hydrodynamic and gravitational forces, dark matter
 * gravity only (Sec. 3.1).  The paper does not print the equations; the ones
 * implemented here are linear conservative reproducing-kernel SPH (the method
 * it cites) with a Wendland C4 kernel of support H = 2h, spelled out per call.
 *
 * Conventions for every call
 *  - Particle indices are int32 (n < 2^31).  Pair counts are int64.
 *  - Positions x, y, z are FP64 device arrays in the unit periodic box.  They
 *    are wrapped into [0, 1) and rounded to the 2^-32 grid on entry; inputs on
 *    that grid are used exactly.  Separations use the minimum image.
 *  - Every other particle field, and every output, is a device array of the
 *    precision `prec`: float for CRK_F32, double for CRK_F64.  Vector fields
 *    are row-major per particle: a[3*i + c], B[3*i + a], dB[9*i + 3*a + c].
 *  - Inputs and outputs are in the caller's particle order; the library
 *    reorders internally along the tree.
 *  - The library allocates no device memory.  All device buffers passed in
 *    are owned by the caller and must not alias each other.  A crk_leaves
 *    handle is host metadata pointing into a caller-owned device workspace
 *    (`ws` of crk_build_leaf_pairs): tree order, fixed-point positions,
 *    interaction lists and the per-pass scratch (sized at the build for
 *    passes in either precision) all live there.  The workspace must stay
 *    allocated, and must not be written by the caller, until the handle is
 *    freed and the work queued on it is done.
 *  - Work is enqueued on `stream` (a hipStream_t).  crk_build_leaf_pairs,
 *    crk_leaves_stats, crk_timing and crk_kernel_times synchronise with the
 *    host; no pass call synchronises.  Calls that use the same handle share
 *    its scratch and must not run concurrently.
 *  - Return value: CRK_OK (0) or a negative code; crk_last_error() then
 *    returns a message (thread-local).  Asynchronous device errors surface at
 *    a later call.
 *
 * Precision modes
 *  - CRK_F32: pair arithmetic in FP32 with compensated (Kahan-type) FP32
 *    accumulation; the per-particle 3x3 correction solve and the global
 *    momentum/energy totals in FP64.
 *  - CRK_F64: the same kernels instantiated in FP64 with plain sums.
 */
#ifndef CRK_H
#define CRK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CRK_OK = 0,
    CRK_EINVAL = -1, /* invalid argument (null pointer, size, radius >= half the box, ...) */
    CRK_EHIP = -3,   /* a HIP runtime or launch error */
    CRK_ESTATE = -4, /* handle built in the wrong mode for this call */
    CRK_ENOSPC = -5  /* the caller's workspace is too small (crk_build_leaf_pairs sets *ws_needed) */
};

typedef enum { CRK_F32 = 0, CRK_F64 = 1 } crk_prec;

/* Gas particles.  x, y, z: FP64 device arrays of n.  vx..m: device arrays of n
 * in the precision of the call.  Fields a call does not use may be NULL. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    const void *vx, *vy, *vz; /* velocity */
    const void *u;            /* specific internal energy */
    const void *h;            /* smoothing length; kernel support H = 2h */
    const void *m;            /* mass */
} crk_gas;

/* Reproducing-kernel corrections (device, precision of the call):
 * A[n], B[3n], dA[3n] (dA[3i+c] = d_c A), dB[9n] (dB[9i+3a+c] = d_c B^a).
 * M (optional, NULL = unused): device double[30 n], caller-owned, row-major
 * [30][n] in caller order: the 29 independent moment sums of each particle
 * (m0 with the self term, m1[3], m2[6], g0[3], the symmetric t1[6] and t3[10]
 * of the gradient moments) and its neighbour count.  crk_corrections fills it;
 * crk_accel_energy_backward reads it instead of recomputing the moments. */
typedef struct {
    void *A, *B, *dA, *dB;
    double* M;
} crk_corr;

/* Opaque handle: tree order, leaf and tile interaction lists, scratch. */
typedef struct crk_leaves crk_leaves;

/* Launch and tiling choices (the autotuner's search space). */
typedef struct {
    int persistent;      /* 1: persistent grid draining an atomic work queue; 0: one tile per wave */
    int waves_per_cu;    /* persistent grid size = CUs * waves_per_cu waves */
    int kahan_chunk;     /* FP32 pair sums (all passes): plain sums over this many pairs, compensated across chunks
                            (1 = every pair); a power of two in [1, 64] */
    int block_waves;     /* waves per workgroup for the list-driven pair passes (1, 2, 4) */
    int xcd_groups;      /* tile order is cut into this many contiguous chunks, one per XCD (1..16) */
    int tile_order;      /* 0: tree order (locality); 1: longest tiles first */
    int addr64;          /* 0: staged record loads use 32-bit offsets from the array base while the records
                            span at most 4 GiB, 64-bit addresses beyond; 1: 64-bit addresses always
                            (same results bit for bit; kept to exercise the wide form on small inputs) */
    int exchange;        /* sr_gravity and its adjoint: how a block's kept candidates reach the lanes
                            (Sec. 5.3's variants): 0 compacted into LDS and read as LDS broadcasts,
                            1 scalar-register broadcast (v_readlane), 2 cross-lane permute (ds_bpermute);
                            same results bit for bit */
    int stage16;         /* volume and moments passes (16-byte FP32 neighbour records): 0 gathered lane by
                            lane, 1 each slot's distinct particles staged through LDS like the larger
                            records (same results bit for bit) */
} crk_tuning;

/*
 * Build the tree and interaction lists (Sec. 3.1 RCB tree; Sec. 5.3 leaf-pair
 * interaction).  Copies positions (and h) to the host, bisects recursively
 * along the longest axis at the median until a node holds at most leaf_max
 * particles (and, when split_extent > 0, until its longest side is at most
 * split_extent, never producing leaves below leaf_min), then forms tiles of
 * 64 consecutive particles in tree order and, per tile, the list of leaves
 * whose boxes come within the interaction radius of the tile's box.
 *
 *  h != NULL (hydro mode): radius max(2h_i, 2h_j); a per-particle neighbour
 *    list (j != i, |x_ij| < max(2h_i, 2h_j)) is built on the GPU for the CRK
 *    passes, then ordered per tile so that lanes sharing a neighbour take it
 *    at the same list position (each particle's neighbours with |x_ij| < 2h_i
 *    first; deterministic).  The order changes only the summation order of the
 *    passes, never which pairs they sum.  In this mode r_fixed >= 0 is a list
 *    skin: every support is widened by it for the lists (pairs beyond a
 *    particle's support add exactly zero in every pass), so the handle serves
 *    positions that moved since the build as long as no particle moved by
 *    skin / 2 or more (the passes re-read positions at every call; see
 *    crk_kick_drift's disp).  Requires 2 max(h) + skin < 1/2.
 *  h == NULL (fixed-radius mode): radius r_fixed (< 1/2), for sr_gravity.
 *
 * Workspace: ws is caller-owned device memory of ws_bytes bytes, 256-byte
 * aligned (NULL with ws_bytes = 0 asks for the size).  *ws_needed (host,
 * required) receives the bytes the handle needs.  If ws_bytes is smaller the
 * call returns CRK_ENOSPC with *out = NULL (what it wrote into ws is then of
 * no use); the caller allocates *ws_needed bytes and calls again with the
 * same arguments.
 * The size of the neighbour lists is known only after they are counted on
 * the GPU, which needs the rest of the workspace: a first CRK_ENOSPC may
 * therefore report that rest alone (the lists come on top), and the retry
 * with that much then reports the exact total; a repeated call resumes from
 * the host tree and list counts of the one that stopped.  On success the
 * handle uses the first *ws_needed bytes of ws.
 *
 * prec gives the precision of h.  leaf_max in [1, 1<<20].  Synchronises
 * `stream`.
 */
int crk_build_leaf_pairs(int64_t n, const double* x, const double* y, const double* z,
                         const void* h, double r_fixed, int leaf_max, int leaf_min,
                         double split_extent, crk_prec prec, void* ws, size_t ws_bytes,
                         size_t* ws_needed, crk_leaves** out, hipStream_t stream);

/*
 * The same handle built on the GPU (the paper's code builds its tree on the
 * host, Sec. 3.1; this build keeps the positions on the device).  Leaves are
 * the cells of an octree over the 2^-32 grid: the particles are sorted by the
 * Morton key of their top 21 bits per axis, and each particle's leaf is the
 * largest octree cell around it that holds at most leaf_max particles (a
 * finest-level cell holding more is cut into runs of leaf_max).  Tiles of 64
 * consecutive particles in that order find their candidate leaves by looking
 * up the octree cells that cover the tile's box widened by the largest
 * interaction radius and testing every leaf found there box against box.  In
 * hydro mode each leaf is then ordered by decreasing list length (deterministic
 * ties), and the lists are built and scheduled as by crk_build_leaf_pairs.
 *
 * Arguments, modes, the skin, the workspace protocol and the handle are those
 * of crk_build_leaf_pairs except: no leaf_min or split_extent; leaf_max in
 * [1, 1024]; the workspace also holds the build's temporaries (its per-pass
 * scratch is at least about 100 bytes per particle); a call that returns
 * CRK_ENOSPC keeps no state (the repeated call rebuilds and reaches the same
 * sizes).  Every particle's neighbour list holds the same set of particles as
 * with crk_build_leaf_pairs (the list test does not depend on the tree); the
 * tree order, tiles and list order differ, so pass results agree to rounding
 * of the summation order.  Invalid positions or h are reported as CRK_EINVAL
 * from a device check.  Synchronises `stream`.
 */
int crk_build_leaf_pairs_device(int64_t n, const double* x, const double* y, const double* z,
                                const void* h, double r_fixed, int leaf_max, crk_prec prec, void* ws,
                                size_t ws_bytes, size_t* ws_needed, crk_leaves** out, hipStream_t stream);

/*
 * Geometry pass (Sec. 5, "Geometry": particle volumes).
 *   S_i = sum_{j: |x_ij| < 2h_i} W(|x_ij|, h_i)   (j = i included)
 *   V_i = 1 / S_i,  rho_i = m_i S_i
 * Reads gas x, y, z, h, m.  Writes V[n], rho[n].
 */
int crk_volume(crk_leaves* leaves, const crk_gas* gas, crk_prec prec, void* V, void* rho,
               hipStream_t stream);

/*
 * Corrections pass (Sec. 5, "Corrections": reproducing-kernel coefficients).
 * Over j with |x_ij| < 2h_i (j = i included), with W_ij = W(r_ij, h_i) and
 * d_c W_ij its x_i^c derivative, the 40 moments
 *   m0 = sum V_j W, m1^a = sum V_j x^a W, m2^ab = sum V_j x^a x^b W,
 *   g0^c = sum V_j d_cW, g1^ac = d_c m1^a, g2^abc = d_c m2^ab
 * give, per particle in FP64,
 *   B = -m2^-1 m1,  A = 1/(m0 + B.m1),
 *   d_cB = -m2^-1 (g1[.,c] + g2[.,.,c] B),  d_cA = -A^2 (g0^c + B.g1[.,c] + m1.d_cB),
 * so that sum_j V_j A_i(1 + B_i.x_ij) W_ij reproduces constant and linear fields.
 * If particle i has fewer than 4 neighbours or det m2 <= 1e-12 (tr m2 / 3)^3 the
 * zeroth-order form A = 1/m0, B = 0, dA = -g0/m0^2, dB = 0 is used and counted.
 * Reads gas x, y, z, h and V[n].  Writes A, B, dA, dB of *out, and out->M when
 * it is not NULL.  If n_fallback (device int64) is not NULL the number of
 * fallbacks is added to it.
 */
int crk_corrections(crk_leaves* leaves, const crk_gas* gas, const void* V, crk_prec prec,
                    const crk_corr* out, int64_t* n_fallback, hipStream_t stream);

/*
 * Acceleration and Energy passes, fused (Sec. 5, "Acceleration", "Energy").
 * With P_i = (gamma - 1) rho_i u_i and, for j != i with r_ij < max(2h_i, 2h_j),
 *   G_ij = grad of the corrected kernel of i (A_i, B_i, dA_i, dB_i, h_i) at x_ij,
 *   G_ji = the same for j at x_ji = -x_ij,
 *   F_ij = -1/2 V_i V_j (P_i + P_j) (G_ij - G_ji)          (= -F_ji),
 *   a_i = (1/m_i) sum_j F_ij,   du_i/dt = -(1/(2 m_i)) sum_j F_ij . (v_i - v_j).
 * Reads gas x, y, z, vx, vy, vz, u, h, m, V, rho and the corrections.
 * Writes a[3n] and dudt[n].  If totals (device double[8]) is not NULL it
 * receives, in FP64, [sum m a_x, sum m a_y, sum m a_z, sum m (v.a + du/dt),
 * sum m |a|, sum m (|v.a| + |du/dt|), sum m du/dt, sum m v.a].
 */
int crk_accel_energy(crk_leaves* leaves, const crk_gas* gas, const void* V, const void* rho,
                     const crk_corr* corr, double gamma, crk_prec prec, void* a, void* dudt,
                     double* totals, hipStream_t stream);

/*
 * crk_accel_energy without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and results (bit for bit) as
 * crk_accel_energy, but the pass's scratch -- the neighbour records and the
 * FP64 totals partials -- lives in a fixed device array of 80 MiB compiled
 * into the library, one per GPU, held from the first call on that GPU until
 * the process ends, instead of in the handle's workspace.  Scratch needed:
 * n x 128 bytes (FP32; 256 in FP64) plus 64 bytes per 64 particles plus
 * 8 KiB, i.e. up to about 640k particles in FP32 and 320k in FP64; larger
 * inputs are refused with CRK_EINVAL before anything is launched.  Allocates
 * nothing and enqueues no memset.  Every call on a GPU shares that GPU's array
 * (it keeps the last call's contents; every byte a call reads it first
 * writes): calls that overlap on one GPU -- concurrent streams, threads or
 * handles -- race, and the caller must order them.
 */
int crk_accel_energy_noalloc(crk_leaves* leaves, const crk_gas* gas, const void* V, const void* rho,
                             const crk_corr* corr, double gamma, crk_prec prec, void* a, void* dudt,
                             double* totals, hipStream_t stream);

/*
 * Extras pass (Sec. 5, "Extras": the density and the state gradients), over
 * each particle's gather support (j with |x_ij| < 2h_i), with the corrected
 * kernel W^R_ij = A_i (1 + B_i.x_ij) W_ij and its x_i-gradient G_ij (as in
 * crk_accel_energy):
 *   rhoR_i     = sum_j m_j W^R_ij                       (j = i included)
 *   dv_i[a][c] = sum_{j != i} V_j (v_j^a - v_i^a) G_ij^c   (= d_c v^a)
 *   du_i[c]    = sum_{j != i} V_j (u_j - u_i) G_ij^c
 * (the reproducing conditions make both gradients exact for linear fields).
 * Reads gas x, y, z, vx, vy, vz, u, h, m, V[n] and the corrections.  Writes
 * rhoR[n], dv[9n] (dv[9i + 3a + c]) and du[3n].
 */
int crk_extras(crk_leaves* leaves, const crk_gas* gas, const void* V, const crk_corr* corr, crk_prec prec,
               void* rhoR, void* dv, void* du, hipStream_t stream);

/* Artificial viscosity constants (see crk_accel_energy_visc). */
typedef struct {
    double Cl;    /* linear coefficient (>= 0) */
    double Cq;    /* quadratic coefficient (>= 0) */
    double eps_q; /* softening of mu, relative to h^2 (> 0) */
} crk_visc;

/*
 * crk_accel_energy with an artificial viscosity fed by the Extras pass's
 * velocity gradients dv (the step between Corrections and Acceleration in the
 * paper's kernel sequence, Sec. 5).  For each force pair, with D_k = dv_k x_ij
 * and s_k = x_ij . D_k (k = i, j), the van Leer limiter
 *   Phi = max(0, 4 s_i s_j / (s_i + s_j)^2)
 * weights the linear reconstruction of both velocities to the pair's midpoint,
 *   w = v_i - v_j - Phi/2 (D_i + D_j),
 *   mu_k = min(0, h_k (w.x_ij) / (r_ij^2 + eps_q h_k^2)),
 *   Q_k = rho_k (-Cl c_k mu_k + Cq mu_k^2),  c_k = sqrt(gamma (gamma - 1) u_k),
 * and P_i + P_j in F_ij becomes P_i + P_j + Q_i + Q_j (still F_ij = -F_ji, so
 * momentum and total energy stay conserved).  A linear velocity field gives
 * Phi = 1 and w = 0: no viscosity.  dv: [9n] as written by crk_extras.  Other
 * arguments, outputs and totals as crk_accel_energy.  (No adjoint: the
 * backward call covers the inviscid pass.)
 */
int crk_accel_energy_visc(crk_leaves* leaves, const crk_gas* gas, const void* V, const void* rho,
                          const crk_corr* corr, const void* dv, const crk_visc* visc, double gamma,
                          crk_prec prec, void* a, void* dudt, double* totals, hipStream_t stream);

/*
 * Force pass with the compatible energy partition (the paper's hydrodynamics
 * is CRK-SPH, Sec. 3.1, whose energy equation splits every pair's work
 * between the two particles; the paper prints no formula).  The accelerations
 * are those of crk_accel_energy (dv, visc NULL) or crk_accel_energy_visc (both
 * given); only du/dt changes.  With W_ij = (v_j - v_i) . F_ij the work of the
 * pair force on i (W_ji = W_ij):
 *   du_i/dt = (1/m_i) sum_j f_ij W_ij,
 *   f_ij = 1/2 [1 + sgn(W_ij) (u_j - u_i) / (|u_j - u_i| + eps_u (u_i + u_j))]
 * (f_ij = 1/2 where the denominator is 0).  f_ij + f_ji = 1, so total energy
 * is conserved as with the symmetric split (f_ij = 1/2, crk_accel_energy);
 * heating goes mostly to the colder particle and cooling comes mostly from the
 * hotter one, and equal u gives the symmetric split exactly.  eps_u >= 0
 * (finite) sets how sharply the share follows the energy difference.
 * Arguments and outputs otherwise as crk_accel_energy_visc; timed as the
 * force pass it extends (CRK_K_ACCEL or CRK_K_ACCEL_VISC).
 */
int crk_accel_energy_compatible(crk_leaves* leaves, const crk_gas* gas, const void* V, const void* rho,
                                const crk_corr* corr, const void* dv, const crk_visc* visc, double eps_u,
                                double gamma, crk_prec prec, void* a, void* dudt, double* totals,
                                hipStream_t stream);

/*
 * Short-range particle-particle gravity (Sec. 3.1 force split; all species).
 *   a_i = -G sum_{j != i, r_ij < r_cut} m_j x_ij [ (r^2 + eps^2)^(-3/2) - sum_k p_k r^(2k) ]
 * poly: host array of 6 coefficients p_0..p_5 or NULL (no polynomial term).
 * Needs a handle built in fixed-radius mode with r_fixed >= r_cut.
 * Reads x, y, z and m[n] (precision prec).  Writes a[3n].
 */
int sr_gravity(crk_leaves* leaves, int64_t n, const double* x, const double* y, const double* z,
               const void* m, double G, double eps, double r_cut, const double* poly,
               crk_prec prec, void* a, hipStream_t stream);

/*
 * Adjoint of sr_gravity with respect to positions (masses held fixed).  Given
 * ga = dL/da [3n], writes gx = dL/dx [3n]:
 *   gx_i = -G sum_{j != i, r_ij < r_cut} [phi d + 2 phi'(s) (x_ij . d) x_ij],
 *   d = m_j ga_i - m_i ga_j,  s = r_ij^2,  phi(s) = (s + eps^2)^(-3/2) - P(s),
 * the derivative of every a_k with x_i in it.  Each particle's adjoint is
 * accumulated by its own lane (no atomics; bitwise reproducible).  Arguments
 * otherwise as sr_gravity.  (The paper has no adjoint.)
 */
int sr_gravity_backward(crk_leaves* leaves, int64_t n, const double* x, const double* y, const double* z,
                        const void* m, double G, double eps, double r_cut, const double* poly,
                        const void* ga, crk_prec prec, void* gx, hipStream_t stream);

/*
 * The polynomial of the particle-mesh force split (Sec. 3.1; the build option
 * HACC_CUDA_POLY_ORDER=5, appendix), for a mesh potential filtered by
 * exp(-k^2 r_s^2): the long-range force per unit mass is that of a Gaussian
 * cloud, f_L(r) = [erf(x) - (2x/sqrt(pi)) exp(-x^2)] / r^2 with x = r/(2 r_s),
 * and poly[0..5] (host) receives the p_k of P(s) = sum_k p_k s^k that
 * minimise sum_k [r_k^3 (f_L(r_k)/r_k - P(r_k^2))]^2 -- the error of the pair
 * force relative to the Newtonian one -- at s_k = r_cut^2 (k + 1/2) / samples,
 * k < samples (Householder least squares in s / r_cut^2).  sr_gravity with
 * these p_k then evaluates the short-range remainder of the split.  Host only.
 */
int sr_gravity_fit_poly(double r_s, double r_cut, int samples, double* poly);

/*
 * Adjoint of crk_accel_energy together with the corrections and volume passes
 * it depends on (reverse mode of the chain x, v, u -> V, rho -> A, B, dA, dB ->
 * a, du/dt; h and m held fixed; the interaction lists are those of the handle).
 * Given ga = dL/da [3n] and gdudt = dL/d(du/dt) [n], writes gx = dL/dx [3n],
 * gv = dL/dv [3n] and gu = dL/du [n].  V, rho and the corrections must be the
 * ones the forward passes produced for this gas (they are reused, not
 * recomputed).  The moments are taken from corr->M when it is not NULL (it
 * must then hold what crk_corrections wrote for this gas and V), else
 * recomputed per tile over the lists.  Pair terms are
 * recomputed per tile and never stored; each particle's adjoints are
 * accumulated by its own lane, so the result is bitwise reproducible.
 * FP32: pair arithmetic in FP32 with compensated sums, the adjoint of the 3x3
 * solve in FP64.  (The paper has no adjoint; this is the derivative of the
 * passes defined above.)
 */
int crk_accel_energy_backward(crk_leaves* leaves, const crk_gas* gas, const void* V,
                              const void* rho, const crk_corr* corr, double gamma, const void* ga,
                              const void* gdudt, crk_prec prec, void* gx, void* gv, void* gu,
                              hipStream_t stream);

/*
 * Adjoint of the viscous chain: volume -> corrections -> Extras (the velocity
 * gradients dv, Sec. 5) -> forces with the artificial viscosity
 * (crk_accel_energy_visc).  Same upstream adjoints and outputs as
 * crk_accel_energy_backward (gx, gv, gu: dL/dx, dL/dv, dL/du in caller
 * order), plus dv (the Extras pass's output the forward used, caller order,
 * 9 per particle) and the viscosity constants of the forward.  The force
 * adjoint also takes the viscosity's dependence on x, v, dv, rho and u; an
 * Extras adjoint pass (timed as CRK_K_EXTRAS_ADJ) then carries dL/d dv to x,
 * v, V and the corrections before the corrections, moments and volume
 * adjoints.  corr.M (the forward's stored moment sums) is used when given.
 */
int crk_accel_energy_visc_backward(crk_leaves* leaves, const crk_gas* gas, const void* V, const void* rho,
                                   const crk_corr* corr, const void* dv, const crk_visc* visc, double gamma,
                                   const void* ga, const void* gdudt, crk_prec prec, void* gx, void* gv,
                                   void* gu, hipStream_t stream);

/*
 * Global time step (the paper's port reduces floating-point minima with atomic
 * fetch_min, Sec. 5.1): dt = min_i min(c_cfl 2h_i / (c_i + |v_i|),
 * c_acc sqrt(2h_i / |a_i|)), c_i = sqrt(gamma (gamma - 1) u_i), the second limit
 * only where |a_i| > 0.  h, u, vx, vy, vz [n] and a [3n] are device arrays of
 * the precision `prec`; dt is one device value of that precision, written on
 * `stream` (reduced per workgroup, then with atomic minima on the bits of the
 * positive values: deterministic).  n = 0 gives +inf.  No host synchronisation.
 */
int crk_timestep(int64_t n, const void* h, const void* u, const void* vx, const void* vy, const void* vz,
                 const void* a, double gamma, double c_cfl, double c_acc, crk_prec prec, void* dt,
                 hipStream_t stream);

/*
 * Kick-drift update with the device time step dt (one value, as written by
 * crk_timestep): v += a dt, u += du/dt dt, then x += v dt (the updated v) with
 * each position wrapped into [0, 1).  x, y, z: FP64 device arrays [n], updated
 * in place; vx, vy, vz, u [n] updated in place, a [3n] and dudt [n] read, all
 * in the precision `prec`.
 * disp (optional, device double[2]): disp[0] += the step's largest drift
 * max_i |v_i dt| (disp[1] is scratch, left at 0).  Zeroed by the caller after
 * each build, disp[0] bounds how far any particle has moved since: a handle
 * built with a list skin (crk_build_leaf_pairs) stays valid while
 * disp[0] < skin / 2.
 */
int crk_kick_drift(int64_t n, double* x, double* y, double* z, void* vx, void* vy, void* vz, void* u,
                   const void* a, const void* dudt, const void* dt, double* disp, crk_prec prec,
                   hipStream_t stream);

/*
 * Statistics of a handle (host int64[8]):
 *   [0] leaves, [1] tiles, [2] candidate pairs scanned by the list build
 *   (tile particles x candidate-leaf particles), [3] neighbour-list entries,
 *   [4] ordered pairs j != i with r < 2h_i, [5] with r < max(2h_i, 2h_j)
 *   ([4], [5] counted in FP64 on the device; hydro mode only, else 0),
 *   [6] padded list slots, [7] host build time in microseconds.
 * Synchronises the device.
 */
int crk_leaves_stats(crk_leaves* leaves, int64_t* host_out);

/*
 * Tree order of a handle: perm[s] = caller index of the particle at position s
 * of tree order (device int32[n], written on `stream`).  Callers that keep
 * their particle arrays in this order (x_tree[s] = x[perm[s]]) and rebuild get
 * the identity permutation -- the median splits keep the existing order -- and
 * every pass then reads and writes particle fields with coalesced accesses.
 */
int crk_leaves_perm(const crk_leaves* leaves, int32_t* perm, hipStream_t stream);

/*
 * Work-distribution check: launches the pair passes' work distribution with
 * the handle's tuning (persistent atomic queue or one tile per wave, XCD
 * chunks, order) and adds 1 to visits[t] (device int32[tiles], zeroed by the
 * caller) for every tile t a wave is handed.  Every entry must read 1: each
 * tile processed exactly once, whatever the schedule.
 */
int crk_queue_visits(crk_leaves* leaves, int32_t* visits, hipStream_t stream);

/* Read or set the launch/tiling choices of a handle (set validates them). */
int crk_get_tuning(const crk_leaves* leaves, crk_tuning* out);
int crk_set_tuning(crk_leaves* leaves, const crk_tuning* in);

/*
 * Kernel timing, for measurement.  While enabled on a handle, every kernel a
 * call launches is bracketed by HIP events recorded on the call's stream.
 * crk_kernel_times waits for the recorded events and returns, per kernel kind,
 * the summed milliseconds and the number of launches since timing was last
 * enabled (ms and launches: host arrays of CRK_K_COUNT).
 */
enum {
    CRK_K_CULL = 0,    /* neighbour-list build (count, fill and schedule passes) */
    CRK_K_VOLUME = 1,  /* volume pair kernel */
    CRK_K_MOMENTS = 2, /* correction moments + FP64 solve (and their recomputation in the backward) */
    CRK_K_ACCEL = 3,   /* acceleration/energy pair kernel */
    CRK_K_GRAVITY = 4, /* short-range gravity */
    CRK_K_PACK = 5,    /* per-particle packing, gathers and the totals reduction */
    CRK_K_ACCEL_ADJ = 6,   /* force adjoint pair kernel */
    CRK_K_MOMENTS_ADJ = 7, /* moments adjoint pair kernel */
    CRK_K_VOLUME_ADJ = 8,  /* volume adjoint pair kernel */
    CRK_K_SOLVE_ADJ = 9,   /* per-particle solve adjoint from stored moment sums (crk_corr.M) */
    CRK_K_GRAVITY_ADJ = 10, /* short-range gravity adjoint */
    CRK_K_EXTRAS = 11,      /* Extras pass (CRK density, gradients of v and u) */
    CRK_K_ACCEL_VISC = 12,  /* acceleration/energy pair kernel with the artificial viscosity */
    CRK_K_EXTRAS_ADJ = 13,  /* Extras adjoint pair kernel (viscous backward) */
    CRK_K_COUNT = 14
};
int crk_timing(crk_leaves* leaves, int enable);
int crk_kernel_times(crk_leaves* leaves, double* ms, int64_t* launches);

/* Release a handle's host metadata (NULL is ignored).  Its workspace stays the
 * caller's: free it once the work queued on the handle is done. */
void crk_leaves_free(crk_leaves* leaves);

/* Message for the last non-zero return on this thread ("" if none). */
const char* crk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CRK_H */
