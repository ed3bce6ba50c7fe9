/*
 * vlb.h -- C ABI of the coupled vortex-filament / lattice-Boltzmann step
 * (S. Inui and M. Tsubota, arXiv:2108.04435, Sec. II) on AMD gfx950.
 *
 * One "run" is one simulation: a D3Q19 normal-fluid lattice (Sec. II.B)
 * plus a set of closed vortex filaments (Sec. II.A), coupled through the
 * mutual-friction force (Sec. II.B).  All state lives in ONE caller-owned
 * block of device memory (the workspace); the library never allocates
 * device memory.  Device work is ordered on ONE caller-owned HIP stream,
 * given at creation: inside vlb_step and a graph, the lattice part of a
 * step runs on a second, library-owned stream (default priority) forked
 * from the caller's stream at the start of the call and joined back to it
 * at the end, so to the caller every call is ordered on its stream.
 *
 * Conventions
 *  - Every function returns a vlb_status (0 = success, negative = error);
 *    no C++ exception crosses this boundary.  After an error,
 *    vlb_last_error(run) returns a message (NULL-run errors go to
 *    vlb_last_error(NULL)).
 *  - "host" pointers are ordinary CPU memory, read or written synchronously
 *    before the call returns.  "device" pointers are device memory on the
 *    run's GPU; the copy is enqueued on the run's stream and the call
 *    synchronises that stream before returning.
 *  - Lattice fields are stored z-major: index = (z * ny + y) * nx + x.
 *    Vector fields are three such blocks (x, y, z components).
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. II.B, Step 1).
 *  - Deferred device errors (capacity overflow, non-finite values) are
 *    latched on the device and returned by the next vlb_sync /
 *    vlb_read_* call.
 *  - A run is not thread-safe; different runs may be used from different
 *    threads.
 */
#ifndef VLB_H
#define VLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlb_run vlb_run; /* opaque host handle, owned by the library */

typedef enum {
  VLB_OK = 0,
  VLB_EINVAL = -1,    /* invalid argument; nothing was changed             */
  VLB_ENOSPACE = -2,  /* workspace smaller than vlb_query_footprint        */
  VLB_EDEVICE = -3,   /* a HIP call failed                                  */
  VLB_ESTATE = -4,    /* call out of order (e.g. step before any fields)    */
  VLB_ECAPACITY = -5, /* filament points or reconnection candidates
                         exceeded their capacity (n_cap; recon_cap in the
                         step, or 8 candidates at one point); the step that
                         overflowed skipped the operation that needed the
                         room                                               */
  VLB_ENUMERIC = -6   /* NaN/Inf met in the normal-fluid or line velocity   */
} vlb_status;

/* Precision of the normal-fluid populations and of the Biot-Savart sum.  */
typedef enum {
  VLB_F64 = 0, /* plain path: populations, LBM and Biot-Savart in FP64     */
  VLB_F32 = 1, /* populations stored as FP32 deviations f_i - w_i (rho0=1),
                  FP32 LBM arithmetic, FP32 Biot-Savart                    */
  VLB_F16 = 2  /* populations stored as FP16 deviations scaled by 2^10,
                  FP32 arithmetic, FP32 Biot-Savart                        */
} vlb_precision;

/* Lattice and normal fluid (Sec. II.B).                                    */
typedef struct {
  int32_t nx, ny, nz;     /* nodes per axis, each >= 4                      */
  int32_t precision;      /* vlb_precision                                  */
  double tau;             /* BGK relaxation time (Sec. II.B, Eq. BGK), > 1/2 */
  uint32_t wall_axes;     /* bit a (0=x,1=y,2=z): axis a is closed by two
                             halfway bounce-back walls half a cell outside
                             its first and last node; otherwise periodic   */
  int32_t plane_lo;       /* 1: nodes z = 0 carry f^eq(1, plane_u) before
                             each collision (heater plane, Sec. III.C, IV)  */
  int32_t plane_hi;       /* 1: the same on z = nz-1 (cooler plane)         */
  int32_t reserved0;
  double plane_u[3];      /* velocity imposed on the planes                 */
  double body_force[3];   /* uniform Guo body force added at every node     */
} vlb_lattice_desc;

/* Vortex filaments and coupling (Sec. II.A, II.B, III.B, III.C).            */
typedef struct {
  double kappa;           /* circulation quantum in lattice units           */
  double core_a;          /* vortex core radius a                           */
  double core_c;          /* LIA core constant C in ln(2 sqrt(l+ l-)/(e^C a)) */
  double alpha, alpha_p;  /* mutual friction coefficients (Eq. E of M)      */
  double rho_s_over_rho_n;/* rho_s / rho_n                                  */
  double dxi_min, dxi_max;/* remeshing bounds on segment length (Sec. II.A) */
  double reconnect_dist;  /* leg exchange below this distance (Sec. III.B)  */
  double vs_applied[3];   /* externally applied superflow v_s,a (Eq. B-S)   */
  int32_t remesh;         /* 1: keep segments inside [dxi_min, dxi_max]     */
  int32_t reconnect;      /* 1: reconnection on                             */
  int32_t min_loop_pts;   /* loops with fewer points are removed (>= 3)     */
  int32_t coupling;       /* 1: the mutual-friction force acts on the
                             normal fluid; 0: prescribed normal fluid       */
  int32_t mass_balance;   /* 1: superflow V_s from mass conservation
                             along the flow axis mass_balance_axis (Sec.
                             III.C, Eq. mass cons): minus rho_n/rho_s times
                             the mean of u_n along that axis over each
                             cross-section normal to it, added to v_s along
                             it (linear between cross-sections); that axis
                             must be periodic                               */
  int32_t force_model;    /* reaction on the normal fluid per length
                             (Sec. II.B, Eq. f): 0 = rho_s kappa s' x
                             (ds/dt - v_s), the Magnus balance; 1 = rho_s
                             kappa (ds/dt - v_s), the relation as printed
                             (for ablation)                                 */
  int32_t wall_images;    /* 1: superfluid wall term v_s,b (Sec. II.A, Eq.
                             Biot-Savart) from image filaments: on every
                             closed axis the filaments are mirrored in the
                             wall planes -1/2 and n - 1/2 with circulation
                             -kappa per reflection, every combination of
                             reflections across the closed axes (3^w - 1
                             copies for w closed axes, each summed like the
                             real filaments, none excluded); 0: v_s,b = 0.
                             The Biot-Savart work grows 3^w-fold.           */
  int32_t mass_balance_axis; /* flow axis of the mass balance: 0, 1, 2 for
                             x, y, z (the paper's channel flows along x)    */
  int64_t n_cap;          /* capacity in filament points (>= 1)             */
  int64_t recon_cap;      /* capacity in reconnection candidates per step   */
  int32_t ff_cell;        /* 0: the non-local sum of every stage is the
                             direct sum over all segment pairs (Sec. II.A);
                             > 0: its far-field approximation (the
                             definition at vlb_biot_savart_farfield) with
                             cells of this edge, for large tangles; needs a
                             periodic box, FP32 or FP16 precision and no
                             wall images                                    */
  int32_t ff_levels;      /* levels of cells of that approximation (0, 1, 2) */
  double ff_theta;        /* its opening parameter, 0 < ff_theta < 1        */
  int32_t rk_stages;      /* time integration of the filaments over one
                             lattice step (Sec. II.A, Eq. E of M; the paper
                             names no method): an explicit Runge-Kutta
                             method of 1 (forward Euler), 2 (the midpoint
                             rule) or 4 (the classical method) stages; 0
                             means 4.  Each stage is one Biot-Savart sum    */
  int32_t vfm_substeps;   /* that method applied this many times per
                             lattice step with steps of 1/vfm_substeps, in
                             [1, 64] (0 means 1), for stiff filaments (large
                             kappa, short segments).  The normal-fluid
                             velocity and the superflow stay those of the
                             step's start; the force on the normal fluid is
                             that of the step's start positions; remeshing
                             and reconnection follow the last substep       */
  int32_t reserved2;      /* 0                                              */
} vlb_vortex_desc;

/* Bytes of device workspace a run with these descriptors needs.           */
int vlb_query_footprint(const vlb_lattice_desc* lat, const vlb_vortex_desc* vor,
                        uint64_t* bytes);

/* Create a run inside the caller's device workspace (>= footprint bytes,
 * 256-byte aligned) on the caller's stream (hipStream_t, may be NULL for the
 * null stream); the library creates its side stream and four events here
 * (VLB_EDEVICE if that fails) and releases them in vlb_destroy.
 * Populations start at equilibrium f^eq(rho = 1, u = 0); there are no
 * filaments.  The workspace and stream must outlive the run.               */
int vlb_create_lattice(const vlb_lattice_desc* lat, const vlb_vortex_desc* vor,
                       void* dev_workspace, uint64_t ws_bytes, void* hip_stream,
                       vlb_run** out);

/* Populations <- f^eq(rho, u) (Sec. II.B, Step 1).  rho: device, nx*ny*nz
 * doubles; u: device, 3*nx*ny*nz doubles.  Resets the step counter and the
 * spread force field.                                                      */
int vlb_write_fields(vlb_run* run, const double* rho_dev, const double* u_dev);

/* Replace the filaments by n_pts points (host xyz[n][3], lattice units)
 * linked by next (host, n ints, the successor of each point).  A filament
 * is a closed loop or an open line bound to the walls (Sec. IV: lines bound
 * to the solid walls): its last point links to itself (next[e] = e) and no
 * point links to its first; both ends must lie exactly on a wall plane
 * (-1/2 or L - 1/2) of a closed axis and stay on it (they slide along the
 * wall).  Every point has at most one predecessor besides itself.
 * Positions on periodic axes are wrapped into [0, L) by one shift of L; a
 * wall axis mirrors a point beyond the wall plane once.  VLB_EINVAL when
 * that leaves a coordinate outside the box (more than one length L away),
 * for a non-finite coordinate, an index out of range, a point with two
 * predecessors, a one-point line or an end off the wall planes.            */
int vlb_seed_vortices(vlb_run* run, int64_t n_pts, const double* xyz_host,
                      const int32_t* next_host);

/* Enqueue n_steps coupled steps (Sec. II): filament RK4 with the
 * Biot-Savart + LIA velocity and the Schwarz equation of motion, force
 * spreading, one forced LBM update, remeshing / reconnection.  Returns
 * after enqueueing (asynchronous).  The filament stages stay on the run's
 * stream; the moments, the spreading and the LBM update go to the side
 * stream, with event dependencies where the two parts exchange data.      */
int vlb_step(vlb_run* run, int64_t n_steps);

/* Several runs advanced together (the served form): n_steps coupled steps
 * of each of the n_runs distinct runs, enqueued step by step across the
 * runs (step s of every run before step s + 1 of any), each run on its own
 * stream, so that runs on different streams overlap on the GPU.  Each
 * run's result is the one vlb_step(run, n_steps) gives, bit for bit.
 * Returns after enqueueing; the first failing run's code is returned
 * (runs before it may have been advanced).                                 */
int vlb_step_many(vlb_run* const* runs, int32_t n_runs, int64_t n_steps);

/* Wait for the run's streams; return a latched device error if any.       */
int vlb_sync(vlb_run* run);

/* Density and bare velocity sum(c_i f_i)/sum(f_i) of the current
 * populations (velocity planes applied).  Device outputs: rho (cells) and
 * u (3*cells) doubles; either may be NULL.                                  */
int vlb_read_fields(vlb_run* run, double* rho_dev, double* u_dev);

/* Current populations f_i (full value, not deviation) as doubles, device
 * output of 19*cells, population-major (i slowest), in the library's fixed
 * D3Q19 order: rest, +x,-x,+y,-y,+z,-z, (+1,+1,0),(-1,-1,0),(+1,-1,0),
 * (-1,+1,0), (+1,0,+1),(-1,0,-1),(+1,0,-1),(-1,0,+1), (0,+1,+1),(0,-1,-1),
 * (0,+1,-1),(0,-1,+1).                                                      */
int vlb_read_populations(vlb_run* run, double* f_dev);

/* Checkpoint of the normal fluid: the stored populations as they are kept
 * (deviations f_i - w_i in the run's precision: FP64, FP32, or FP16 scaled
 * by 2^10), population-major in the D3Q19 order above, natural layout
 * (population i of node c at index i * cells + c); device output of
 * 19 * cells elements of 8, 4 or 2 bytes.  Together with
 * vlb_read_filaments and vlb_get_step this is the whole state of a run:
 * vlb_write_state and vlb_seed_vortices (and the friction profile, if one
 * was set) on a run created with the same descriptors continue it bit for
 * bit.  Synchronises the run's stream.                                     */
int vlb_read_state(vlb_run* run, void* pops_dev);

/* Restore populations saved by vlb_read_state (device input, same size and
 * format) and set the step counter to step (>= 0); clears the spread force
 * field, as vlb_write_fields.  Synchronises the run's stream.              */
int vlb_write_state(vlb_run* run, const void* pops_dev, int64_t step);

/* The force field spread by the last step (or vlb_eval_line_velocity):
 * device output of 3*cells doubles (body force not included).               */
int vlb_read_force(vlb_run* run, double* force_dev);

/* Current filaments: up to cap points into host xyz[cap][3] and next[cap];
 * *n_pts receives the point count (also when it exceeds cap, then
 * VLB_ENOSPACE and nothing is copied).                                     */
int vlb_read_filaments(vlb_run* run, int64_t cap, double* xyz_host, int32_t* next_host,
                       int64_t* n_pts);

/* Evaluate, at the current positions and normal fluid and without
 * advancing, what the first RK stage of a step computes: per point the
 * superfluid velocity v_s (non-local Biot-Savart + LIA + applied +
 * mass-balance superflow), the interpolated normal-fluid velocity v_n, the
 * line velocity ds/dt and the mutual-friction force g on the normal fluid;
 * host outputs of n_pts*3 doubles each (any may be NULL).  When coupling is
 * on, the force is also spread into the force field (see vlb_read_force). */
int vlb_eval_line_velocity(vlb_run* run, double* vs_host, double* vn_host,
                           double* sdot_host, double* force_host);

/* Apply only the topology phase of a step (remeshing, reconnection,
 * small-loop removal, compaction) to the current filaments.  stats_host
 * (may be NULL) receives 4 int64: deleted, inserted, reconnections, points
 * removed with small loops.                                                */
int vlb_apply_topology(vlb_run* run, int64_t* stats_host);

/* Mutual-friction coefficients varying along the channel (Sec. IV: alpha
 * and alpha' depend on the temperature, which varies along the channel).
 * alpha_z_host and alpha_p_z_host (nz doubles each, finite) replace the
 * constants alpha and alpha' of the vortex descriptor: at a point of height
 * z each is interpolated linearly between the slices floor(z) and
 * floor(z) + 1 (a periodic z axis wraps; on a wall z axis the end slices'
 * values extend to the walls).  Both NULL restores the constants; one NULL
 * is VLB_EINVAL.  Applies to every later step, graph launch and
 * vlb_eval_line_velocity (also of graphs captured before the call).
 * Synchronises the run's stream.                                           */
int vlb_set_friction_profile(vlb_run* run, const double* alpha_z_host,
                             const double* alpha_p_z_host);

/* Vortex line length of the current filaments (Sec. III.C and IV: the line
 * density the paper follows in time and along the channel).  *total_host
 * receives the sum of the segment lengths |s_next - s| (nearest periodic
 * image); per_slab_host (nz doubles) the length inside each slab
 * [z - 1/2, z + 1/2) along z (a periodic z axis wraps), every straight
 * segment split in proportion to its z extent, a segment without z extent
 * counted in the slab of its start point.  Either may be NULL, not both.
 * Divide by the volume nx*ny*nz (resp. the slab volume nx*ny) for the line
 * density.  Synchronises the run's stream.                                 */
int vlb_line_length(vlb_run* run, double* total_host, double* per_slab_host);

/* Statistics of the normal-fluid velocity (Sec. III.C: the mean flow V_n
 * and its fluctuations delta v_n = v_n - V_n, component by component) of
 * the bare velocity sum(c_i f_i)/sum(f_i) of the current populations
 * (velocity planes applied, as vlb_read_fields).  Host outputs, any may be
 * NULL: slice_mean and slice_rms ([nz][3]) the mean of each component over
 * each z slice and the root mean square of its deviation from that mean;
 * mean and rms ([3]) the same over the whole lattice.  All sums in FP64 in
 * a fixed order.  Synchronises the run's stream.                          */
int vlb_flow_stats(vlb_run* run, double* slice_mean_host, double* slice_rms_host,
                   double* mean_host, double* rms_host);

/* Vorticity of the normal fluid, omega = curl v (Sec. III.A).  u_dev
 * (3*cells doubles, device, as vlb_read_fields) receives the bare velocity
 * and omega_dev (3*cells doubles, device) its curl by central differences;
 * periodic axes wrap and a node beyond a wall counts as u = 0.  Both
 * required.  Synchronises the run's stream.                                */
int vlb_read_vorticity(vlb_run* run, double* u_dev, double* omega_dev);

/* Cylindrical components of a vector field about an axis (Sec. III.A: the
 * vorticity of a ring in the frame of its axis): omega_dev (3*cells doubles,
 * device, e.g. from vlb_read_vorticity) in, out_dev (3*cells doubles,
 * device) receives (omega.rho_hat, omega.phi_hat, omega.axis) per node, the
 * axis through point (3 doubles, host, lattice units) along direction (3
 * doubles, host, normalised here); a node's offset from the point is taken
 * at the nearest periodic image, rho_hat is the unit offset perpendicular
 * to the axis and phi_hat = axis x rho_hat; on the axis both are 0.
 * VLB_EINVAL for a zero or non-finite direction or a non-finite point.
 * Synchronises the run's stream.                                           */
int vlb_vorticity_cylindrical(vlb_run* run, const double* point_host,
                              const double* direction_host, const double* omega_dev,
                              double* out_dev);

/* Number of completed steps.                                               */
int vlb_get_step(vlb_run* run, int64_t* step);

/* Kernel timing with HIP events recorded on the run's stream around every
 * launch of the named kernel class: 0 = Biot-Savart pair sum, 1 = LBM
 * collide+stream.  vlb_set_timing(run, e) clears the totals and enables
 * timing for e > 0 (e > 1 also pre-creates e events so that no event is
 * created while the timed steps are enqueued), disables it for e = 0; the
 * totals are read (after a sync) with vlb_get_timing.                      */
int vlb_set_timing(vlb_run* run, int32_t enable);
int vlb_get_timing(vlb_run* run, int32_t kernel_class, double* total_ms, int64_t* launches);

/* Average duration of one launch of a kernel class (0 = Biot-Savart pair
 * sum at the current positions, 1 = LBM collide+stream) over reps >= 1
 * launches enqueued back to back between two HIP events on the run's
 * stream.  The Biot-Savart timing leaves the state unchanged; the LBM one
 * advances the normal fluid by reps updates (force field as last spread).
 * Synchronises the stream.                                                 */
int vlb_time_kernel(vlb_run* run, int32_t kernel_class, int32_t reps, double* avg_ms);

/* Algorithmic work of the last step: lattice node updates and Biot-Savart
 * (target, segment) pairs summed over the RK stages.                      */
int vlb_get_work(vlb_run* run, int64_t* node_updates, int64_t* bs_pairs);

/* Graph-captured steps.  vlb_graph_create records n_steps coupled steps of
 * the run (n_steps even, so that the population layout returns to the same
 * AA parity) into an executable HIP graph by stream capture on the run's
 * stream (which must not be the null stream); nothing is executed.  Each
 * vlb_graph_launch enqueues the whole graph on the run's stream and
 * advances the run's step counter by n_steps; it returns VLB_ESTATE if the
 * run was stepped by an odd number of steps since the capture, or if the
 * first filaments were seeded after a capture of lattice-only steps.  The
 * graph holds the run's pointers: destroy it before the run.              */
typedef struct vlb_graph vlb_graph;
int vlb_graph_create(vlb_run* run, int64_t n_steps, vlb_graph** out);
int vlb_graph_launch(vlb_graph* graph);
int vlb_graph_destroy(vlb_graph* graph);

/* Stand-alone Biot-Savart sum (Sec. II.A, Eq. Biot-Savart), without a
 * lattice: the non-local superfluid velocity of a caller's closed
 * filaments, the same kernels as the first term of a step's line velocity.
 * Point j receives v_j = kappa/(4 pi) times the sum, over every segment
 * k -> next(k) except the two that touch j (k = prev(j) and k = j, the
 * divergent local part that the LIA term replaces), of the exact integral
 * over the straight segment, at the nearest periodic image decided on the
 * library's 32-bit position grid.
 *  - d: box of nx, ny, nz lattice units; an axis whose bit is set in
 *    wall_axes is closed (no images; positions in [-1/2, n - 1/2]), the
 *    others are periodic of length n (positions anywhere: the grid wraps).
 *    precision VLB_F64 sums in FP64, VLB_F32 and VLB_F16 in FP32 (chunk
 *    partials added in FP64 in a fixed order: bitwise reproducible).
 *  - xyz_dev: device, n_pts x 3 doubles ([n][3], lattice units);
 *    next_dev: device, n_pts int32, the successor of each point: closed
 *    loops, or open lines whose last point links to itself (its zero
 *    segment adds nothing; not checked: invalid links give meaningless
 *    velocities, each entry is clamped into [0, n_pts) so no access leaves
 *    the arrays);
 *    v_dev: device output, n_pts x 3 doubles.
 *  - dev_workspace: device scratch of at least vlb_biot_savart_workspace
 *    bytes, 256-byte aligned, owned by the caller; the call only enqueues
 *    work on hip_stream (NULL: the null stream) and returns: inputs,
 *    output and workspace must stay untouched until that work completes.
 *  - VLB_EINVAL for a bad descriptor, n_pts outside [0, 2^26] or a NULL
 *    pointer (n_pts > 0); VLB_ENOSPACE for a small workspace; VLB_EDEVICE
 *    if a launch fails.  Messages go to vlb_last_error(NULL).              */
typedef struct {
  int32_t nx, ny, nz;     /* box extent per axis, each in [1, 2^24]         */
  uint32_t wall_axes;     /* bit a: axis a closed by walls; else periodic   */
  int32_t precision;      /* vlb_precision of the sum                       */
  int32_t reserved;       /* 0                                              */
  double kappa;           /* circulation quantum, > 0                       */
} vlb_bs_desc;

int vlb_biot_savart_workspace(const vlb_bs_desc* d, int64_t n_pts, uint64_t* bytes);
int vlb_biot_savart(const vlb_bs_desc* d, int64_t n_pts, const double* xyz_dev,
                    const int32_t* next_dev, double* v_dev, void* dev_workspace,
                    uint64_t ws_bytes, void* hip_stream);

/* Allocation-free vlb_biot_savart, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the same sum, kernels and bits as vlb_biot_savart, with its
 * scratch (grid coordinates, links, chunk partials) in a fixed device array
 * of the library (about 4.5 MB per GPU, held until the process ends)
 * instead of a caller workspace.  Arguments as vlb_biot_savart; call with
 * the GPU of hip_stream current.  n_pts is limited to 16384 (VLB_EINVAL
 * above).  Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (other streams, other threads) race and give wrong
 * results; calls ordered on one stream are safe.  The call itself
 * allocates nothing (the first call on a device looks up the array's
 * address, also nothing allocated).                                        */
int vlb_biot_savart_noalloc(const vlb_bs_desc* d, int64_t n_pts, const double* xyz_dev,
                            const int32_t* next_dev, double* v_dev, void* hip_stream);

/* Far-field approximation of the stand-alone sum (an extension of Sec. II.A
 * for large tangles: the paper sums the full non-local integral, which
 * grows as the square of the point count).  The box (periodic on all three
 * axes) is cut into cells of edge `cell`; each segment belongs to the cell
 * of its midpoint, and each cell carries the monopole, dipole and
 * quadrupole moments of its segments' vorticity about its centre.  For
 * each target point and cell: every segment sits at the periodic image of
 * its start that vlb_biot_savart takes; when the cell's segments share one
 * image of the centre at distance R with R theta >= the cell radius (the
 * largest |midpoint - centre| + |segment| / 2), the cell adds its
 * expansion there; when the plane half a box from the target cuts the
 * cell's segment starts on exactly one axis, each of the two image
 * classes adds the expansion of its own segments at its own image
 * (provided both pass the same test); every other cell adds the exact
 * straight-segment integral of each segment, the target's own two
 * segments excluded.  Positions are first reduced into [0, L) per axis
 * (one box length of shift either way; farther positions give
 * meaningless results, never an access outside the buffers).
 * Approximation error: relative L2 of the non-local velocity about 5e-4
 * at theta = 0.25 on tangles of random rings (it grows with theta).
 *  With p->levels = 2 the cells of edge 2 p->cell are taken first: a coarse
 *  cell that is neither far nor split is opened and its 8 children follow
 *  the same rule (fewer expansions per target; error 7e-4 at theta = 0.25
 *  on a 256^3 tangle of 1e5 points, 2.7x faster than vlb_biot_savart
 *  there with cells of 16, 4.9x at 3.8e5 points).
 *  - d: as vlb_biot_savart with wall_axes 0 and precision VLB_F32 (the
 *    sum is FP32; chunk partials added in FP64 in a fixed order, bitwise
 *    reproducible); p->cell >= 1 divides nx, ny and nz (2 p->cell does with
 *    two levels), at most 2^22 cells of edge p->cell; 0 < p->theta < 1
 *    (which keeps each target's own segments in cells it sums directly).
 *  - xyz_dev, next_dev, v_dev, dev_workspace, hip_stream: as
 *    vlb_biot_savart, the workspace sized by
 *    vlb_biot_savart_farfield_workspace (about 620 bytes per point, 700
 *    per cell and 12 per point per cell chunk, up to 64 chunks).
 *  - VLB_EINVAL for a bad descriptor or parameters, n_pts outside
 *    [0, 2^26] or a NULL pointer (n_pts > 0); VLB_ENOSPACE for a small
 *    workspace; VLB_EDEVICE if a launch fails.                             */
typedef struct {
  int32_t cell;           /* finest cell edge in lattice units               */
  int32_t levels;         /* 1 (or 0): one grid of cells; 2: cells of edge   */
                          /* 2 cell first, opened ones handing their 8       */
                          /* children of edge cell to the same rule          */
  double theta;           /* opening parameter, 0 < theta < 1               */
} vlb_ff_params;

int vlb_biot_savart_farfield_workspace(const vlb_bs_desc* d, const vlb_ff_params* p,
                                       int64_t n_pts, uint64_t* bytes);
int vlb_biot_savart_farfield(const vlb_bs_desc* d, const vlb_ff_params* p, int64_t n_pts,
                             const double* xyz_dev, const int32_t* next_dev, double* v_dev,
                             void* dev_workspace, uint64_t ws_bytes, void* hip_stream);

/* Release the host handle.  The workspace is the caller's to free.         */
int vlb_destroy(vlb_run* run);

const char* vlb_last_error(const vlb_run* run);

#ifdef __cplusplus
}
#endif

#endif /* VLB_H */
