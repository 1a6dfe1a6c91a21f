/*
 * lbm.h - C ABI of the MI355X (gfx950) D3Q19 LBM-LES library (liblbm.so).
 *
 * The library advances the weakly compressible lattice-Boltzmann model of
 * arXiv 2607.04516, Appendix D ("Lattice Boltzmann method in FluidX3D"):
 * D3Q19 velocities, second-order Hermite equilibrium (eq. D.4), single
 * relaxation time BGK collision (eq. D.2) with the Smagorinsky-Lilly eddy
 * viscosity obtained locally from the non-equilibrium momentum flux
 * (eqs. D.7-D.11), streaming (eq. D.3) with halfway bounce-back at solid
 * cells and at wall faces (App. D, last paragraph), and equilibrium-velocity
 * inflow cells (Sec. 3, boundary conditions).  Zero-gradient outflow,
 * free-slip and periodic faces complete the face set.  An optional uniform
 * body force enters through Guo's forcing scheme (the scheme App. E names).
 *
 * Conventions for every entry point
 *  - Return value: LBM_OK (0) or a negative LBM_E* code; no exception or
 *    longjmp crosses the ABI.  lbm_last_error() gives the message.
 *  - Cell order: n = x + nx*(y + ny*z), x fastest.  "Canonical" population
 *    arrays are [19][nz][ny][nx] in the direction order below, holding the
 *    shifted pre-collision populations h_i = f_i - w_i*rho0 of time t.
 *  - Direction order: 0 rest; 1/2 = +-x; 3/4 = +-y; 5/6 = +-z; 7/8 = +-(1,1,0);
 *    9/10 = +-(1,0,1); 11/12 = +-(0,1,1); 13/14 = +-(1,-1,0);
 *    15/16 = +-(1,0,-1); 17/18 = +-(0,1,-1).  Weights 1/3, 1/18, 1/36.
 *  - Element type of device arrays: "real" is double for an LBM_F64 context
 *    and float otherwise; "store" is the storage type of the context
 *    (double, float, IEEE binary16, bfloat16).  LBM_F16S stores 256*h (a
 *    power-of-two scale that keeps the shifts in binary16's normal range);
 *    every other codec stores h itself.  Stores round to nearest even.
 *  - Host pointers are read during the call and copied; device pointers are
 *    borrowed for the duration of the enqueued work only.  The context owns
 *    every allocation it makes (populations, mask bits, ghost planes,
 *    reduction scratch) and frees them in lbm_destroy().
 *  - All work is enqueued on the context's HIP stream (params.hip_stream,
 *    or the null stream).  Only lbm_probe, lbm_mass and lbm_step with the
 *    watchdog on synchronise with the host.
 *  - A context is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* bad dimensions, tau0 <= 1/2, unpaired periodic face, null pointer */
#define LBM_ENOMEM (-2)    /* device allocation failed */
#define LBM_EHIP (-3)      /* HIP runtime error; text in lbm_last_error() */
#define LBM_EUNSTABLE (-4) /* watchdog: NaN/Inf, |u| > 0.5 or |rho - rho0| > 0.5 somewhere */
#define LBM_ESTATE (-5)    /* call out of order, e.g. stepping with an inflow face lacking a profile */

enum lbm_storage { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 };

enum lbm_face_kind {
    LBM_PERIODIC = 0,   /* wraps to the opposite face; both faces of the axis must be periodic */
    LBM_INFLOW_EQ = 1,  /* the face layer holds feq(rho0, u_in(z)) cells */
    LBM_OUTFLOW_ZG = 2, /* zero-gradient: entering populations copy the inner layer */
    LBM_FREESLIP = 3,   /* specular reflection at the half plane outside the face */
    LBM_WALL = 4,       /* halfway bounce-back at the half plane outside the face */
    LBM_HALO = 5        /* y faces only: the face row is a ghost row holding a copy of the
                           neighbouring slab's boundary row (slab decomposition along y);
                           see lbm_halo_pack / lbm_halo_unpack */
};

enum lbm_face { LBM_XM = 0, LBM_XP = 1, LBM_YM = 2, LBM_YP = 3, LBM_ZM = 4, LBM_ZP = 5 };

typedef struct lbm_ctx lbm_ctx;

typedef struct {
    int32_t nx, ny, nz; /* each >= 3 */
} lbm_grid;

typedef struct {
    double tau0;          /* molecular relaxation time, > 1/2 (eq. D.5: nu0 = (tau0 - 1/2)/3) */
    double c_smag;        /* Smagorinsky constant C (eq. D.7); 0 disables the closure */
    double delta;         /* filter width Delta in lattice units (eq. D.7) */
    double rho0;          /* reference density; inflow cells hold feq(rho0, u_in) */
    double body_force[3]; /* uniform force per unit volume, Guo scheme */
    double u_init[3];     /* uniform initial velocity used by lbm_create */
    double noise_amp;     /* initial noise: u += amp*(2*U - 1), U from splitmix64 */
    uint64_t noise_seed;  /* U for component c of cell n = splitmix64(seed + 3n + c) >> 11 * 2^-53 */
    int32_t storage;      /* enum lbm_storage */
    int32_t face[6];      /* enum lbm_face_kind per face, order x-, x+, y-, y+, z-, z+ */
    int32_t watchdog_stride; /* check for blow-up every this many steps; 0 = off */
    void *hip_stream;     /* hipStream_t borrowed from the caller; NULL = null stream */
} lbm_params;

/* Create a context.  solid: host uint8 [nz][ny][nx], nonzero = solid cell
 * (buildings and terrain voxels, Sec. 2.1); copied and bit-packed on the
 * device.  Allocates the population array (19 * nx_pitch * ny_pad * nz * sizeof(store))
 * and initialises the state at t = 0 to feq(rho0, u_init + noise) in fluid
 * cells and h = 0 in solid cells.  The array is laid out in row blocks
 * (R consecutive rows (y, z) keep their 19 populations together, R = 2^k <=
 * 32 the largest block whose padding of each xy plane to ny_pad rows, a
 * multiple of R, stays within ny / 16 rows), so the step kernels' 32-bit
 * slot offsets span one xy plane of all 19 populations: size limit
 * (19 * nx_pitch * ny_pad + 1282 * nx_pitch) * sizeof(store) < 4 GiB,
 * nx_pitch = nx rounded up to 64; larger grids return EINVAL.
 * lbm_push_step and lbm_adjoint_step have a tighter limit (below).  Errors:
 * EINVAL, ENOMEM, EHIP; *out is NULL on error and lbm_last_error(NULL) gives
 * the message. */
int lbm_create(const lbm_grid *grid, const uint8_t *solid, const lbm_params *params, lbm_ctx **out);

/* Set the velocity profile of an INFLOW_EQ face: host double [nz][3]; every
 * cell of the face layer at height z gets the boundary state u[z] (the z+
 * face: u[nz - 1]), so an inflow cell there takes feq(rho0, u[z]) (Sec. 3:
 * equilibrium velocity boundaries; App. F: the boundary velocity array).  A
 * cell on two inflow faces takes the state of the lower-numbered face.
 * Replaces the face's states set by either call.  Takes effect at the next
 * step.  Errors: EINVAL (face not INFLOW_EQ, NULL u, non-finite value). */
int lbm_set_inflow(lbm_ctx *ctx, int32_t face, const double *u);

/* Set the boundary state of every cell of an INFLOW_EQ face (Sec. 2.3: the
 * boundary states come from a face-wise mapping of the mesoscale field onto
 * the faces; App. F: the mean boundary velocity U_b,i of each cell).  u: host
 * double [n2][n1][3], cell (j1, j2) of the face being (y, z) on the x faces,
 * (x, z) on the y faces and (x, y) on the z faces, n1 and n2 their extents;
 * copied.  The entry of a cell that is solid or belongs to a lower-numbered
 * inflow face is kept but only read as a sponge target.  The state is what
 * the inflow cells impose (feq(rho0, u)), the sponge / buffer layers relax
 * toward (at each cell's projection onto the face), flux balancing (mode 1)
 * corrects and the synthetic turbulence fluctuates around.  Takes effect at
 * the next step.  Errors: EINVAL (face not INFLOW_EQ, NULL u, non-finite
 * value). */
int lbm_set_inflow_face(lbm_ctx *ctx, int32_t face, const double *u);

/* Set the rotation vector Omega of the frame in lattice units (App. E:
 * Omega_lbm = Omega_SI * dt_SI, for the Earth Omega_SI = 7.292115e-5 rad/s
 * times (0, cos phi, sin phi) in the east-north-up frame at latitude phi,
 * rotated into the grid axes by the caller).  host double [3], components
 * along x, y, z.  Every fluid cell then adds the Coriolis force
 * F_c = -2 Omega x m (m = sum_i c_i f_i, the momentum recovered before the
 * force enters) to the uniform body force in the Guo source; the sign is
 * that of the rotating-frame acceleration.  Zero (the default) disables it.
 * Applies to lbm_step, lbm_push_step, lbm_macros, the probes and
 * lbm_adjoint_step from the next call on.  Errors: EINVAL (NULL, a
 * component not finite or of magnitude above 0.25). */
int lbm_set_rotation(lbm_ctx *ctx, const double *omega);

/* The Earth's rotation vector in lattice units for lbm_set_rotation (App. E):
 * Omega_ENU = LBM_OMEGA_EARTH * (0, cos phi, sin phi) rad/s in the
 * east-north-up frame at latitude phi = latitude_deg, times the time step
 * dt_si in seconds, expressed in grid axes whose x axis is turned
 * counterclockwise from east by grid_angle_deg (y likewise from north; z up).
 * out: host double [3].  Host arithmetic only, no context.  Errors: EINVAL
 * (NULL out, an argument not finite, dt_si <= 0, |latitude_deg| > 90). */
#define LBM_OMEGA_EARTH 7.292115e-5
int lbm_earth_rotation(double latitude_deg, double dt_si, double grid_angle_deg, double *out);

/* Synthetic von Karman inflow turbulence (App. F).  Before every step from
 * time t the boundary velocity of each active cell becomes
 *   U_i(t) = U_b,i + sigma_i q(x_i, t),
 *   q_a(x, t) = sum_m A_m,a cos(k_m . x - omega_m t + phi_m,a),
 * with U_b,i the cell's boundary state (lbm_set_inflow, lbm_set_inflow_face) and x the global
 * lattice coordinates of the cell (origin + index), so grids that tile one
 * domain see one field.  Active cells: cells of the INFLOW_EQ faces x-, x+,
 * y-, y+, z+ (never z-), not solid, on one face each (the lower-numbered
 * one), optionally only where U_b . n_f > 0 (n_f inward normal); faces whose
 * mean velocity has characteristic speed |U_f| (or |U_f . n_f|) <= 1e-7 are
 * dropped.  u_ref = mean |U_b| and e_c = sum U_b / |sum U_b| over the active
 * cells (e_c = x when the sum vanishes); omega_m = u_ref k_m . e_c, so the
 * pattern is carried along the mean flow.  Modes: k_m log-stratified in
 * [2 pi / (10 L), pi] (k_min = 0.1 pi if that band is empty), isotropic
 * directions, amplitude sqrt(W(k_m)) with W(k) = k^4 / (1 + (k L)^2)^(17/6),
 * normalised to unit RMS per component, times gain[a].  sigma_i = intensity
 * times |U_b,i| (or |U_b,i . n_f|) when intensity > 0, else sigma0.  With a
 * stride s > 1, q is taken at anchors t_a = s floor(t / s), held or
 * interpolated linearly to t_a + s.  Random draws: U = (splitmix64(seed +
 * 2^32 (r + 1) + 6 m + j) >> 11) 2^-53 for realization r (the face, or 0
 * when shared), mode m, draw j: r_m, mu = 2U - 1, theta = 2 pi U, then the
 * phases of x, y, z, each 2 pi U.  The field is evaluated in double
 * precision on the device.  Profiles set later rebuild the generator.
 * p = NULL turns the generator off (boundaries back to the profiles).
 * While it is on, lbm_push_step and lbm_adjoint_step return ESTATE.
 * Errors: EINVAL (n_modes outside [1, 4096], stride < 1, length_scale not
 * positive, a non-finite value), ENOMEM, EHIP. */
typedef struct {
    int32_t n_modes;      /* N_m modes per realization */
    int32_t stride;       /* s >= 1 */
    int32_t interpolate;  /* with s > 1: 0 hold q(t_a), 1 linear between t_a and t_a + s */
    int32_t char_normal;  /* 0: characteristic speed |U|, 1: |U . n_f| (faces and sigma_i) */
    int32_t inflow_only;  /* 1: only cells with U_b . n_f > 0 */
    int32_t shared;       /* 1: one realization for every face */
    double length_scale;  /* integral length L, lattice units */
    double intensity;     /* I; <= 0 selects sigma0 */
    double sigma0;        /* fluctuation level when intensity <= 0 */
    double gain[3];       /* component gains g_x, g_y, g_z */
    double origin[3];     /* global lattice coordinates of cell (0, 0, 0) */
    uint64_t seed;
} lbm_turbulence;

int lbm_set_turbulence(lbm_ctx *ctx, const lbm_turbulence *p);

/* Sponge and buffer nudging (Sec. 2.2: relaxation layers next to the top and
 * lateral open faces, toward the target boundary state).  Next to every
 * INFLOW_EQ face except z-, a fluid cell at distance d = 1..width from the
 * face layer gets s = strength ((width + 1 - d) / width)^2 (the largest over
 * the faces, the lower-numbered face on ties), and after its collision
 *   f*_i += s (feq_i(rho, u_t) - feq_i(rho, u)),
 * with rho, u the cell's collision moments and u_t the face's boundary state
 * at the cell's projection onto the face (for a profile: its value at the
 * cell's height; the z+ face: its single row).  Mass is unchanged; the
 * momentum relaxes by s rho (u_t - u).  Widths and strengths are not printed
 * in the paper; the ramp is this library's choice.  width 0 or strength 0
 * turns it off.  While it is on, lbm_adjoint_step returns ESTATE.
 * Errors: EINVAL (width outside [0, min(nx, ny, nz) - 2], strength outside
 * [0, 1]). */
int lbm_set_sponge(lbm_ctx *ctx, int32_t width, double strength);

/* Global flux balancing over the INFLOW_EQ faces (Sec. 2.2 and 2.3: mass-flux
 * consistency of the boundary data).  Over the non-solid cells of those
 * faces (each on its owning face) the net outward volume flux is
 * Phi = sum_i U_i . n_i; the least-squares smallest change of the normal
 * velocities that zeroes it is U_i -= (Phi / N) n_i for every cell.
 *   mode 1: apply it to the boundary states now (host, double): every entry
 *           of every INFLOW_EQ face moves by -(Phi / N) n; the
 *           synthetic-turbulence generator is rebuilt on the new states;
 *   mode 2: apply it to the whole per-cell boundary field (states plus
 *           synthetic turbulence) now and on the device before every step;
 *   mode 0: stop the per-step balancing.
 * phi_before, phi_after (host, may be NULL): the net flux before and after
 * this call's correction (mode 0: the current field's, twice).
 * Errors: EINVAL (mode), ENOMEM, EHIP. */
int lbm_balance_flux(lbm_ctx *ctx, int32_t mode, double *phi_before, double *phi_after);

/* Net outward flux of the current per-cell boundary field (device sum in a
 * fixed order, deterministic).  Synchronises. */
int lbm_net_flux(lbm_ctx *ctx, double *phi);

/* The generator's active cell count, u_ref and e_c (zeros when it is off). */
int lbm_turbulence_info(lbm_ctx *ctx, int64_t *n_active, double *u_ref, double *e_c);

/* Copy the current boundary velocity of one INFLOW_EQ face to host double
 * out[n2][n1][3] (x faces [nz][ny], y faces [nz][nx], z faces [ny][nx]):
 * the velocity the inflow cells of that face took in the last step (the
 * profile, or profile plus synthetic turbulence).  Solid cells hold the
 * profile value.  Synchronises.  Errors: EINVAL (face not INFLOW_EQ, NULL). */
int lbm_get_inflow(lbm_ctx *ctx, int32_t face, double *out);

/* Re-initialise the state at t = 0 to feq(rho0, u0[z] + noise) in fluid
 * cells.  u0: host double [nz][3], or NULL for params.u_init. */
int lbm_reset(lbm_ctx *ctx, const double *u0);

/* Advance n >= 0 steps of collide-and-stream (eqs. D.2, D.3 with D.4, D.11).
 * Asynchronous unless the watchdog fires inside the n steps (then it
 * synchronises and returns EUNSTABLE with the state at the failing check).
 * Errors: ESTATE (an inflow face has no profile), EUNSTABLE, EHIP. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* As lbm_step, and after every step adds u(x_p, t+1) of each registered
 * probe cell (lbm_set_probes) to acc: device real [2][np][3], a
 * Neumaier-compensated sum: acc[0] the running sum, acc[1] the accumulated
 * rounding errors; the accumulated value is acc[0] + acc[1].  The caller
 * zeroes acc before the first call of a sum.  The step kernels take the
 * samples of the states they start from when every probe is a fluid,
 * non-inflow cell off the x faces in a row the fast kernels run; the other
 * samples go through the probe kernel (lbm_probe_accumulate); both give the
 * same bits. */
int lbm_step_probed(lbm_ctx *ctx, int64_t n, void *acc);

/* Macroscopic fields of the current state (eq. D.1; nu_t from eqs. D.6, D.11
 * as (tau_eff - tau0)/3, the value the next collision uses).  Device real
 * arrays rho [N], u [3][N], nu_t [N], N = nx*ny*nz; any may be NULL.  Inflow
 * cells report (rho0, u_in, 0), solid cells (rho0, 0, 0). */
int lbm_macros(lbm_ctx *ctx, void *rho, void *u, void *nu_t);

/* Sample rho and u at np points: pts host float [np][3] in lattice
 * coordinates (cell centres at integers); out host float [np][4] =
 * (rho, ux, uy, uz).  Integer points return that cell; other points are
 * trilinear in the cell values (solid cells count as rho0, u = 0); points
 * outside [0, n-1] are clamped.  Synchronises. */
int lbm_probe(lbm_ctx *ctx, const float *pts, int32_t np, float *out);

/* lbm_probe for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sampling, arguments and results, staged through a fixed per-GPU
 * scratch array of LBM_PROBE_NOALLOC_MAX * 7 floats (448 KiB) that the
 * library holds until the process ends, so the call makes no hipMalloc,
 * hipFree or other allocating call.  np > LBM_PROBE_NOALLOC_MAX returns
 * LBM_EINVAL.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (several host threads, or contexts on different
 * streams) race and must be serialised by the caller.  Synchronises. */
#define LBM_PROBE_NOALLOC_MAX 16384
int lbm_probe_noalloc(lbm_ctx *ctx, const float *pts, int32_t np, float *out);

/* Mass sum(rho) and kinetic energy sum(rho |u|^2 / 2) over fluid cells
 * (solid and inflow cells excluded).  Per-lane compensated sums of
 * rho - rho0 in real precision, then a deterministic double-precision tree
 * over lanes and blocks.  Synchronises. */
int lbm_mass(lbm_ctx *ctx, double *mass, double *kinetic_energy);

/* Export the canonical state of time t (see conventions) into dst: device
 * store [19][N].  Inflow cells hold h_eq(rho0, u_in), solid cells 0. */
int lbm_get_state(lbm_ctx *ctx, void *dst, int64_t *t);

/* Import a canonical state (device store [19][N]) as time t.  Values of
 * solid and inflow cells are ignored.  With the watchdog on
 * (watchdog_stride > 0) the imported state is checked at once (synchronises):
 * EUNSTABLE for a non-finite value, |u| > 0.5 or |rho - rho0| > 0.5 in a
 * fluid cell (a corrupt checkpoint); the state stays imported. */
int lbm_set_state(lbm_ctx *ctx, const void *src, int64_t t);

/* Register integer probe cells: host int32 [np][3] = (x, y, z), each a
 * non-solid cell inside the grid; np <= 4096.  Used by lbm_step_probed,
 * lbm_probe_accumulate and lbm_adjoint_step. */
int lbm_set_probes(lbm_ctx *ctx, const int32_t *cells, int32_t np);

/* acc (device real [2][np][3], compensated as in lbm_step_probed) += u of
 * the registered probe cells in the current state. */
int lbm_probe_accumulate(lbm_ctx *ctx, void *acc);

/* Time statistics: while set, every step from a time t with t % stride == 0
 * adds u(t) and u(t)^2 into acc (device real [6][N]: sum ux, uy, uz, then
 * sum ux^2, uy^2, uz^2) inside the step kernel.  acc NULL or stride <= 0
 * turns the statistics off. */
int lbm_set_stats(lbm_ctx *ctx, void *acc, int32_t stride);

/* One step from a canonical state to a canonical state, out of place:
 * src, dst device store [19][N], distinct.  Uses the context's geometry,
 * parameters and inflow boundary states; does not touch its state or time.
 * This is the recompute step of the checkpointed adjoint.  Size limit (the
 * kernel's 32-bit slot offsets span up to two population slices, or eight
 * when a y or z face is LBM_FREESLIP): nx * ny * nz *
 * sizeof(store) below 2 GiB, or below 512 MiB with such faces; else EINVAL. */
int lbm_push_step(lbm_ctx *ctx, const void *src, void *dst);

/* One discrete-adjoint step (transpose of the linearised update, eqs. D.2-D.4
 * and D.11 differentiated by hand):
 *   lam = J_C(f_t)^T S^T lam_next + d(loss)/d f(t),
 * where S is the streaming with its boundary rules and J_C the Jacobian of
 * the local collision at the canonical state f_t (device store [19][N]).
 * lam_next, lam: device real [19][N] canonical layout, distinct.
 * probe_src: device real [np][3] = dL/du(x_p, t) for the registered probes,
 * or NULL.  g_inflow: device real [2][6][nz][3], or NULL; [0] += the
 * gradient of the loss with respect to each inflow face profile u_in(face, z)
 * through the step t -> t+1 (the sum over the face's inflow cells at height z
 * of the derivative with respect to their own velocity, i.e. with respect to
 * a uniform shift of that row), as a compensated (Neumaier) sum with [1] the
 * compensation.  Solid and inflow cells get lam = 0.  One kernel launch on
 * the context's stream.  Size limit as for lbm_push_step, with the real
 * type's size (nx * ny * nz * sizeof(real) below 2 GiB, or 512 MiB with
 * free-slip y/z faces); else EINVAL. */
int lbm_adjoint_step(lbm_ctx *ctx, const void *f_t, const void *lam_next, void *lam,
                     const void *probe_src, void *g_inflow);

/* Voxelize closed triangle meshes into the solid mask (Sec. 4.1: rays cast
 * along the grid axes through the cell centres, ray-triangle intersections
 * and the odd-even parity rule along each ray, independent passes along
 * other ray directions corroborating the labels; Sec. 2.1: the mask is the
 * Boolean union of its layers).  tri: host double [nt][3][3], the vertices
 * (x, y, z) of each triangle in lattice units (cell (x, y, z) is the unit
 * cube from (x, y, z) to (x + 1, y + 1, z + 1)); starts: host int32 [nm + 1],
 * mesh m owns triangles starts[m] .. starts[m + 1] - 1 and must be closed.
 * Each mesh is tested on its own and the meshes are united.  A ray crosses a
 * triangle where its foot lies in the triangle's projection (counter-
 * clockwise; a foot on an edge counts only for an edge running upward or
 * horizontally toward -u, so shared edges count once); a cell centre is
 * inside a mesh when an odd number of crossings lies below it along the ray.
 * passes 1: rays along z; 3: rays along z, x and y, solid where at least two
 * agree.  solid: host uint8 [nz][ny][nx], in/out: voxelized cells are set to
 * 1, others keep their value.  Synchronous; allocates and frees its device
 * buffers.  Errors: EINVAL (NULL, counts, starts not running from 0 to nt,
 * non-finite vertices, passes, a ray longer than 1024 cells), ENOMEM, EHIP;
 * the message is in lbm_last_error(NULL). */
int lbm_voxelize(const lbm_grid *grid, const double *tri, int32_t nt, const int32_t *starts, int32_t nm,
                 int32_t passes, uint8_t *solid);

/* Halo exchange of a slab decomposition along y (one context per slab, the
 * decomposition of the paper's multi-GPU runs).  A slab has a ghost row on
 * each LBM_HALO side (y = 0 for y-, y = ny - 1 for y+) that mirrors the
 * neighbour's boundary row; the kernels update ghost rows like free-slip
 * face rows, and two exchanges keep the real rows exact: only the five
 * populations with c_y toward the neighbour cross an interface.
 *   After an even step (A-A swapped layout): the post-collision values of the
 *   real boundary row moving toward the neighbour fill the neighbour's ghost
 *   row, which its odd step gathers from.
 *   After an odd step: the values this slab's odd step pushed into its ghost
 *   row go back into the neighbour's real boundary row (where the pull there
 *   came from a non-solid ghost cell).
 * lbm_halo_pack writes what this context sends through `side` (0: y-, 1: y+)
 * at its current phase; lbm_halo_unpack writes what the neighbour on `side`
 * sent.  buf: device store [5][nz][nx] (directions with c_y = -1 for a y-
 * send, +1 for a y+ send, ascending).  Call both after every step, all packs
 * of the step before any unpack, and only between steps of all slabs in
 * lockstep; the state then equals the undecomposed run's, bit for bit.  Ghost
 * rows are counted by the diagnostics (mass, macros).  Contexts with a HALO
 * face refuse the push step, the adjoint, the synthetic inflow and flux
 * balancing (they would need quantities summed over all slabs).
 * Errors: EINVAL (side not a HALO face, NULL buf). */
int lbm_halo_pack(lbm_ctx *ctx, int32_t side, void *buf);
int lbm_halo_unpack(lbm_ctx *ctx, int32_t side, const void *buf);

/* Kernel timing for measurement: while enabled, a pair of HIP events on the
 * context's stream brackets every launch of the fused collide-and-stream
 * kernel (not the outflow passes).  Enabling resets the record. */
int lbm_profile(lbm_ctx *ctx, int32_t enable);

/* Synchronise, then return the summed duration in ms of the bracketed
 * step-kernel launches recorded since lbm_profile(ctx, 1) or the previous
 * read, and their number; resets the record. */
int lbm_profile_read(lbm_ctx *ctx, double *total_ms, int64_t *launches);

/* Current time step t of the context's state. */
int64_t lbm_time(const lbm_ctx *ctx);

/* Number of fluid cells (non-solid, including inflow cells) and of the
 * cells counted by lbm_mass (non-solid, non-inflow). */
int lbm_cell_counts(const lbm_ctx *ctx, int64_t *fluid, int64_t *interior);

/* Layout of the context's in-place population array (see lbm_create):
 * rows per block R, rows per xy plane ny_pad (ny rounded up to a multiple of
 * R) and the x pitch nx_pitch; any may be NULL. */
int lbm_layout(const lbm_ctx *ctx, int32_t *rows_per_block, int32_t *ny_pad, int32_t *nx_pitch);

/* Replace the HIP stream work is enqueued on (NULL = null stream). */
int lbm_set_stream(lbm_ctx *ctx, void *hip_stream);

/* Message of the last error of ctx (ctx-owned string), or of the last
 * failed lbm_create on this thread when ctx is NULL. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Free every allocation of the context (synchronises its stream). */
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
