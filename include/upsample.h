/*
 * upsample.h -- C ABI of the MI355X (gfx950) library for the high-resolution
 * (HR) upsampling step of "Interactive High-Resolution Simulation of Granular
 * Material" (arXiv 2308.01629), Section 4.
 *
 * One step advances every HR particle i against a frame of low-resolution (LR)
 * guide particles j:
 *   w_ij  = max(0, (1 - |X_j - x_i|^2 / (9 r_LR^2))^3)              (Section 4, weight)
 *   v~_i  = sum_j w_ij V_j / sum_j w_ij                             (Section 4, Shepard average)
 *   a_i   = 1 - max_j w_ij if max w <= c1 or max w / sum w >= c2, else 0   (Section 4, blend)
 *   v_i'  = (1 - a_i) v~_i + a_i (v_i + dt g)                        (Section 4, velocity)
 *   x_i'  = x_i + dt v_i'                                           (Section 4, position)
 * LR particles flagged rigid count only when a granular LR particle is within
 * the support of HR particle i (Section 4, last paragraph).  Afterwards the
 * planar walls of the scene are applied in order (a contract of this library;
 * the paper gives no HR boundary step).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Particle arrays are caller-owned DEVICE memory, float32 structure-of-arrays
 *   [3][n] (x row, then y row, then z row), contiguous.  lr_rigid is a device
 *   uint8 array [n_lr] (0 granular, 1 rigid or boundary sample) or NULL for
 *   "all granular".
 * - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *   null stream).  Calls return as soon as the work is enqueued; results are
 *   ready when the stream reaches that point.  Step functions never allocate:
 *   all scratch is allocated by upsample_init (or upsample_autotune).
 * - Return value: UPSAMPLE_OK (0) or one of the UPSAMPLE_ERR_* codes below.
 *   Argument errors are detected on the host before any device work is
 *   enqueued, so a rejected call has no effect.  upsample_last_error() gives a
 *   message for the last failing call on a handle.
 * - A handle is not thread-safe; separate handles are independent.  Calls on
 *   one handle that overlap on different streams race on its scratch.
 */
#ifndef UPSAMPLE_H
#define UPSAMPLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UPSAMPLE_OK                 0
#define UPSAMPLE_ERR_INVALID_ARG    1  /* null handle/pointer, bad size or parameter   */
#define UPSAMPLE_ERR_CAPACITY       2  /* n_lr > max_lr or n_hr > max_hr               */
#define UPSAMPLE_ERR_GRID_TOO_LARGE 3  /* cell count >= 2^31 or an axis > 2^20 cells   */
#define UPSAMPLE_ERR_NO_DEVICE      4  /* no HIP device visible                       */
#define UPSAMPLE_ERR_OOM            5  /* device allocation failed                    */
#define UPSAMPLE_ERR_HIP            6  /* a HIP runtime call or kernel launch failed  */
#define UPSAMPLE_ERR_NONFINITE      7  /* VALIDATE flag: non-finite input found       */
#define UPSAMPLE_ERR_STATE          8  /* call order: e.g. advance before build_grid  */

#define UPSAMPLE_MAX_WALLS          32
#define UPSAMPLE_WALL_FLOATS        12
#define UPSAMPLE_DEFAULT_CELL_FACTOR 1.0001f

/* flags */
#define UPSAMPLE_FLAG_VALIDATE      1u  /* scan inputs for NaN/Inf (synchronises the stream) */
/* Deterministic LR gradients in upsample_step_backward(_taped): the HR pass
 * records each particle's adjoint coefficients instead of adding to the LR
 * gradients, the HR particles are sorted by cell (stable), and each LR
 * particle's gradient is summed by one wave over its HR neighbours in a fixed
 * order with a fixed lane reduction, then added by one writer.  No float
 * atomics: repeated calls give the same bits.  Costs a per-lane HR pass, the HR
 * sort and the LR pass; init allocates 8 B per cell and 76 B per HR particle
 * (max_hr) more. */
#define UPSAMPLE_FLAG_DETERMINISTIC_BWD 2u

typedef struct upsample_handle_s* upsample_handle;

/*
 * Parameters of one scene (Section 4 symbols in brackets).
 *   r_lr         LR radius [r_LR] > 0; the kernel support is h = 3 r_lr.
 *   r_hr         HR radius [r_HR] >= 0; used only as the wall offset.
 *   dt           HR time step [dt_HR] >= 0 (Section 5.2 uses 0.0167 s).
 *   g            gravity [g], default (0, -9.81, 0) (Algorithm 1: |g| = 9.81).
 *   c1, c2       blend thresholds, default 512/729 and 0.6 (Section 4).
 *   domain_lo/hi axis-aligned box covered by the neighbour grid; particles
 *                outside it are clamped into the edge cells (results stay exact).
 *   cell_factor  grid cell size = cell_factor * h; 0 = UPSAMPLE_DEFAULT_CELL_FACTOR.
 *                The stencil reach R is the smallest integer with
 *                R >= h / cell_size + 16 * max_axis_cells * 2^-24.
 *   n_walls, walls  host array [n_walls][12]: n(3), d, a(3), b, o(3), R.  Plane
 *                n.x = d, unit normal n into the admissible side.  After
 *                integration, for each wall in order, the wall acts on HR particle
 *                i when a.x' >= b, the in-plane distance of x' from o is >= R
 *                (R = 0: no hole) and n.x - d >= 0 for the pre-step x.  An acting
 *                wall with n.x' - d < r_hr sets x' += (r_hr - (n.x' - d)) n and, if
 *                n.v' < 0, v' -= (n.v') n.  Copied at init.
 *   max_lr, max_hr  capacities; scratch is sized for them at init.
 *   flags        UPSAMPLE_FLAG_*.
 */
typedef struct {
  float r_lr;
  float r_hr;
  float dt;
  float g[3];
  float c1;
  float c2;
  float domain_lo[3];
  float domain_hi[3];
  float cell_factor;
  int32_t n_walls;
  const float* walls;
  int64_t max_lr;
  int64_t max_hr;
  uint32_t flags;
} upsample_params;

/* Integer grid contract, identical on every device and on the host.
 *   cell coordinate c_a = clamp(floor(fl32(fl32(X_a - lo_a) * inv_cell_size)), 0, dims_a - 1)
 *   cell key        k   = c_x + dims_x (c_y + dims_y c_z)
 *   membership      fl32(fl32(fl32(dx dx) + fl32(dy dy)) + fl32(dz dz)) < h2,
 *                   d = fl32(X_j - x_i), each operation rounded separately.
 *   inv_cell_size = fl32(1 / cell_size), h2 = fl32(9 r_lr^2), inv_h2 = fl32(1 / (9 r_lr^2)). */
typedef struct {
  int32_t dims[3];
  int32_t reach;
  int64_t n_cells;
  double cell_size;
  float inv_cell_size;
  float h2;
  float inv_h2;
  float lo[3];
} upsample_grid_info;

/* Fill *p with the defaults above (r_lr = 0.02, r_hr = 0.005, dt = 1/60, unit
 * box, no walls, capacities 0).  Host only.  Returns INVALID_ARG for p == NULL. */
int upsample_default_params(upsample_params* p);

/* Validate *p and compute its grid on the host; touches no device.  Returns
 * INVALID_ARG or GRID_TOO_LARGE for a bad *p. */
int upsample_grid_info_for(const upsample_params* p, upsample_grid_info* out);

/* Create a handle on the current HIP device and allocate its scratch.  Returns
 * INVALID_ARG / GRID_TOO_LARGE for bad parameters (checked first), NO_DEVICE
 * when no device is visible, OOM when allocation fails.  *out is set only on
 * success. */
int upsample_init(const upsample_params* p, upsample_handle* out);

/* Release a handle (NULL is a no-op).  The caller must make sure no enqueued
 * work still uses it. */
int upsample_destroy(upsample_handle h);

/* Static message for an error code; message of the last failing call on h. */
const char* upsample_strerror(int code);
const char* upsample_last_error(upsample_handle h);

/* The handle's grid (as upsample_grid_info_for of its current parameters). */
int upsample_get_grid_info(upsample_handle h, upsample_grid_info* out);

/*
 * Uniform-grid rebuild of one LR frame (the neighbour search of Section 5.1,
 * compact-hashing style): cell keys, counting sort stable in the original index,
 * cell ranges, and an LR copy in sorted order kept in the handle.  lr_x, lr_v:
 * [3][n_lr]; n_lr may be 0 (every HR particle then falls freely).
 */
int upsample_build_grid(upsample_handle h, const float* lr_x, const float* lr_v,
                        const uint8_t* lr_rigid, int64_t n_lr, void* stream);

/*
 * Advance n_hr HR particles one step against the LR frame of the last
 * upsample_build_grid on this handle (Section 4).  hr_x, hr_v: state at t,
 * [3][n_hr]; hr_x_out, hr_v_out: state at t+1, may alias hr_x, hr_v (in place).
 * Returns STATE if no grid has been built.
 */
int upsample_advance(upsample_handle h, const float* hr_x, const float* hr_v,
                     float* hr_x_out, float* hr_v_out, int64_t n_hr, void* stream);

/* upsample_build_grid followed by upsample_advance: one full step. */
int upsample_step(upsample_handle h,
                  const float* lr_x, const float* lr_v, const uint8_t* lr_rigid, int64_t n_lr,
                  const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                  int64_t n_hr, void* stream);

/*
 * Adjoint of upsample_step (not in the paper): given dL/dx' and dL/dv' for the
 * step that took (hr_x, hr_v) to (x', v') against the LR frame (lr_x, lr_v,
 * lr_rigid), write dL/dx and dL/dv (gx_in, gv_in, [3][n_hr], may alias gx_out,
 * gv_out) and ADD dL/dX, dL/dV into g_lr_x, g_lr_v ([3][n_lr], caller-zeroed).
 * The alpha branch, neighbour membership, the argmax of the weights (ties: the
 * smallest LR index) and the wall activations are held at their forward values.
 * Rebuilds the grid from lr_x (so the handle's grid afterwards is that frame's).
 * LR gradients are accumulated with float atomics: summation order, and so the
 * last bits, may differ between runs -- unless the handle was created with
 * UPSAMPLE_FLAG_DETERMINISTIC_BWD (then they are bitwise reproducible).
 */
int upsample_step_backward(upsample_handle h,
                           const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                           int64_t n_lr, const float* hr_x, const float* hr_v, int64_t n_hr,
                           const float* gx_out, const float* gv_out,
                           float* gx_in, float* gv_in, float* g_lr_x, float* g_lr_v,
                           void* stream);

/*
 * Taped step and adjoint.  upsample_step_taped is upsample_step that also
 * records, per HR particle, the forward sums the adjoint needs: tape is a
 * device float array [6][n_hr] receiving S, U_x, U_y, U_z, M and the argmax
 * of the weights (original LR index as float bits; ties: smallest index;
 * 0xffffffff when the support is empty), with the rigid rule applied (a
 * rigid-only support is recorded as zero sums).  upsample_step_backward_taped
 * is upsample_step_backward reading these sums from tape instead of
 * recomputing them; it must get the same LR frame and HR state as the taped
 * step.  The results agree with the untaped adjoint to float32 rounding.
 * The tape is caller-owned and must not alias any other argument.
 */
int upsample_step_taped(upsample_handle h,
                        const float* lr_x, const float* lr_v, const uint8_t* lr_rigid, int64_t n_lr,
                        const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                        int64_t n_hr, float* tape, void* stream);
int upsample_step_backward_taped(upsample_handle h,
                                 const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                                 int64_t n_lr, const float* hr_x, const float* hr_v, int64_t n_hr,
                                 const float* tape, const float* gx_out, const float* gv_out,
                                 float* gx_in, float* gv_in, float* g_lr_x, float* g_lr_v,
                                 void* stream);

/*
 * Saved grids (not in the paper): the adjoint of a step needs that step's LR
 * grid (the uniform-grid neighbour search of Section 5.1: cell ranges and the
 * LR copy in sorted order).  upsample_step_backward(_taped) rebuilds it from
 * the LR frame; a caller that keeps the taped forward's grid skips that
 * rebuild.
 *
 * upsample_grid_snapshot_bytes: bytes of one snapshot for this handle (the
 * sorted LR copy for max_lr particles, 32 B each, then the n_cells + 1 cell
 * starts, each part padded to 256 B).  It depends on max_lr and on the grid
 * dimensions, so a change of the cell size (upsample_set_tuning,
 * upsample_autotune) changes it and invalidates earlier snapshots.
 *
 * upsample_grid_snapshot: copy the handle's current grid (that of the last
 * upsample_build_grid, step or backward) into grid, caller-owned device
 * memory of upsample_grid_snapshot_bytes bytes, 256-byte aligned, on stream.
 * Returns STATE if no grid has been built, INVALID_ARG for a NULL or
 * misaligned pointer.
 *
 * upsample_step_backward_taped_grid: upsample_step_backward_taped with the
 * grid read from a snapshot of the same LR frame (taken on this handle, with
 * the same grid parameters, after the taped step) instead of rebuilt.  Only
 * whether lr_rigid is NULL is read (the rigid flags are in the snapshot's LR
 * copy); n_lr must be the frame's particle count.  The handle's own grid is
 * left as it was.  Results are bitwise those of upsample_step_backward_taped
 * on the same inputs (the same grid, the same kernels).  A snapshot of
 * another frame or handle gives wrong gradients; its contents are not checked.
 */
int upsample_grid_snapshot_bytes(upsample_handle h, int64_t* bytes);
int upsample_grid_snapshot(upsample_handle h, void* grid, void* stream);
int upsample_step_backward_taped_grid(upsample_handle h, const void* grid,
                                      const uint8_t* lr_rigid, int64_t n_lr,
                                      const float* hr_x, const float* hr_v, int64_t n_hr,
                                      const float* tape, const float* gx_out, const float* gv_out,
                                      float* gx_in, float* gv_in, float* g_lr_x, float* g_lr_v,
                                      void* stream);

/*
 * Multi-step run: advances the HR state in place through n_frames
 * consecutive LR frames (lr_x, lr_v: device [n_frames][3][n_lr]; lr_rigid, if
 * given, applies to every frame), i.e. n_frames upsample_step calls.  Before
 * step t the state is reordered as by upsample_sort_hr when sort_every > 0
 * and t % sort_every == 0.  The grids are built on an internal stream in
 * batches of 4 frames, into two sets of 4 grid buffers: batch k + 1 is built
 * while the step kernels of batch k run.  HIP events order the two streams
 * once per batch, and everything is done when the caller's stream reaches the
 * call's end.  perm_io (device int32 [n_hr], may be NULL) maps positions to
 * particles: on entry the particle at each position (for instance 0, 1, 2,
 * ...), on return the same after the reorders.  The handle's grid afterwards
 * is the last frame's.  The first call allocates seven more grid buffers and
 * the internal stream.  Results per particle equal
 * those of the step-by-step loop up to float32 rounding (reorders change the
 * waves).
 */
int upsample_run(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                 int64_t n_lr, int32_t n_frames, float* hr_x, float* hr_v, int64_t n_hr,
                 int32_t sort_every, int32_t* perm_io, void* stream);

/*
 * Multi-rate run (Section 5.2): LR frames at their own time step dt_lr (the
 * paper's LR simulation steps at 0.005 s, the HR upsampling at 0.0167 s), HR
 * steps of the handle's dt.  lr_x, lr_v: device [n_frames][3][n_lr], frame k
 * at time t_lr0 + k dt_lr (n_frames >= 2).  HR step n (0 <= n < n_steps)
 * advances the state from t_hr0 + n dt to t_hr0 + (n + 1) dt against the LR
 * state at its end (Section 4's time level t + 1): with
 *   s = (t_hr0 + (n + 1) dt - t_lr0) / dt_lr,  k = floor(s),  theta = s - k
 * (in double; a step ending on the last frame takes k = n_frames - 2,
 * theta = 1), the LR state is the linear interpolation in time between frames
 * k and k + 1, in float32 with theta rounded to float32 and each operation
 * rounded separately:  X = X_k + fl(theta fl(X_{k+1} - X_k)),  V likewise.
 * The interpolation is fused into the grid build (the keys and the sorted
 * copy compute it identically); otherwise the run is upsample_run's: grids
 * built on the internal stream in batches, a reorder every sort_every steps,
 * perm_io composed through the reorders, the state advanced in place.  A
 * step ending before frame 0 or after the last frame is INVALID_ARG (checked
 * before any work is enqueued).
 */
int upsample_run_multirate(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                           int64_t n_lr, int32_t n_frames, double t_lr0, double dt_lr, double t_hr0,
                           int32_t n_steps, float* hr_x, float* hr_v, int64_t n_hr, int32_t sort_every,
                           int32_t* perm_io, void* stream);

/*
 * Reorder HR particles by the key that upsample_tuning's sort_mode selects
 * over cells split into sort_sub^3 sub-cells (by default the Hilbert index of
 * the sub-cells), so that consecutive particles -- the lanes of one wave of
 * the step kernel -- occupy a compact box.  Reads hr_x,
 * hr_v [3][n_hr]; writes the reordered arrays to hr_x_out, hr_v_out (both
 * alias their inputs for an in-place reorder through scratch, or neither).
 * perm_out (device int32 [n_hr], may be NULL) receives, for each new position,
 * the particle's old index.  The order inside a sub-cell is unspecified.
 * Later steps compute the same per-particle results in any order, up to
 * float32 rounding (the weights of a compact wave are taken relative to its
 * box centre).  In the Hilbert mode the first reorder (and the first after
 * the tuning changes sort_sub) also ranks the grid's fine cells along the
 * curve on the stream, into a table the handle allocates then
 * (4 B per fine cell) and keeps: later reorders count one bin per fine cell.
 */
int upsample_sort_hr(upsample_handle h, const float* hr_x, const float* hr_v, float* hr_x_out,
                     float* hr_v_out, int64_t n_hr, int32_t* perm_out, void* stream);

/*
 * Apply a permutation to the columns of a [3][n] array a and, optionally, of
 * a second one b (positions and velocities, or their gradients), so that a
 * caller can keep HR particles in reordered form between steps and map
 * results and gradients back.  mode UPSAMPLE_PERMUTE_GATHER:
 * a_out[:, i] = a[:, perm[i]]; UPSAMPLE_PERMUTE_SCATTER: a_out[:, perm[i]] =
 * a[:, i] (the inverse; the adjoint of the gather).  perm (device int32 [n])
 * must be a permutation of 0..n-1, as upsample_sort_hr writes; columns whose
 * index lies outside [0, n) are skipped, and with UPSAMPLE_FLAG_VALIDATE the
 * call then synchronises and returns UPSAMPLE_ERR_INVALID_ARG.  b and b_out
 * are both NULL or both set; outputs alias no input.  All device pointers.
 */
#define UPSAMPLE_PERMUTE_GATHER 0
#define UPSAMPLE_PERMUTE_SCATTER 1
int upsample_permute(upsample_handle h, const float* a, const float* b, float* a_out, float* b_out,
                     int64_t n, const int32_t* perm, int mode, void* stream);

/*
 * Debug exports (for parity tests).
 * upsample_debug_grid copies the last build's cell keys [n_lr] (original
 * order), sorted order perm [n_lr] and cell_start [n_cells + 1] into device
 * buffers (any may be NULL).
 * upsample_debug_neighbors runs the step's stencil walk for hr_x/hr_v against
 * the last grid and writes, per HR particle, the member count (float32
 * predicate above, all types), up to max_k member LR ids (original indices,
 * walk order) into ids[i * max_k + c], and a branch byte: bit 0 = alpha branch
 * taken, bit 1 = a granular LR is within the support, bit 2 = the sum of
 * weights is positive.  Any output pointer may be NULL.
 */
int upsample_debug_grid(upsample_handle h, uint32_t* keys, uint32_t* perm,
                        uint32_t* cell_start, void* stream);
int upsample_debug_neighbors(upsample_handle h, const float* hr_x, const float* hr_v,
                             int64_t n_hr, uint32_t* count, uint32_t* ids, int64_t max_k,
                             uint8_t* branch, void* stream);

/* upsample_debug_lr_sorted copies the last build's LR state in sorted order --
 * the positions and velocities the step kernel reads, after any interpolation
 * in time -- into device [3][n_lr] arrays (either may be NULL). */
int upsample_debug_lr_sorted(upsample_handle h, float* x_sorted, float* v_sorted, void* stream);

/*
 * upsample_debug_step_members runs the step kernel of upsample_advance --
 * the same template instance path for this handle's tuning and scene (wave
 * tiles, box cull of the candidates, weight form, matrix-core sums, per-lane
 * walk for spread-out waves) with the same arithmetic -- against the last
 * grid, writes the stepped state to hr_x_out, hr_v_out ([3][n_hr], equal bit
 * for bit to upsample_advance's), and exports per HR particle what its walk
 * saw:
 *   count[i]       entries of its candidate list meeting the membership
 *                  predicate above (so: the size of its neighbour set (Section
 *                  4's sums run over it), if the cull kept every member)
 *   ids[i * max_k + c]  their original LR indices, in walk order (max_k > 0
 *                  when ids is given; entries past max_k are counted only)
 *   count_w[i]     entries whose weight, as the kernel computed it, is > 0
 *                  (the entries that enter the sums)
 *   w_disagree[i]  the largest weight over entries on which those two tests
 *                  disagree: the kernel's weight, or the separately rounded
 *                  direct form max(0, 1 - s / h2)^3 of the exact s; 0 if none
 * Any export pointer may be NULL.  All device pointers; errors as
 * upsample_advance.  For parity tests: the kernel timed by upsample_advance
 * and upsample_run is checked here member by member.
 */
int upsample_debug_step_members(upsample_handle h, const float* hr_x, const float* hr_v,
                                float* hr_x_out, float* hr_v_out, int64_t n_hr, uint32_t* count,
                                uint32_t* ids, int64_t max_k, uint32_t* count_w, float* w_disagree,
                                void* stream);

/*
 * Launch-shape knobs of a handle (results do not depend on them beyond float
 * summation order).  gather_groups: lane groups per wave in the gather kernel
 * (1, 2 or 4); each group of 64/G lanes walks its own LDS candidate list, culled
 * against the group's bounding box.  Default 1.  sort_sub: sub-cells per axis
 * of the HR reorder key (1, 2 or 4, at most what the grid's bins allow).
 * sort_mode: 0 orders HR by grid cell then by the Morton order of its
 * sub-cells, 1 by the global Morton (Z-order) code of the sub-cells, 2 by the
 * global Hilbert index of the sub-cells (bins for it are allocated at the
 * default sort_sub when they fit in 2^24).  A sort_sub / sort_mode pair whose
 * bins exceed the handle's allocation is rejected with INVALID_ARG.
 * adjoint_tiled: 1 (default) runs the adjoint as wave tiles with block-summed
 * LR gradients, 0 one particle per lane with per-pair atomics (scenes with
 * rigid LR particles always use the latter).  tile_max: a wave of the step
 * kernel whose stencil rows hold more LR candidates than this walks per lane
 * when its longest per-lane stencil holds fewer than a quarter of them (a
 * compact wave in dense LR keeps its shared list); 0 sends every wave with
 * candidates to the per-lane walk.  adjoint_tile_max: the same for the
 * adjoint's waves, with a share of an eighth.
 * wall_cull: 1 (default) lets a wave of the step kernel skip the walls whose
 * planes lie farther than r_hr from the neighbourhood of the cells its
 * particles occupy (a per-cell table built at init for grids of up to 2^22
 * cells); 0 tests every wall for every particle.  Results are the same.
 */
typedef struct {
  int32_t gather_groups;
  int32_t sort_sub;
  int32_t adjoint_tiled;
  int32_t sort_mode;
  int32_t tile_max;
  int32_t adjoint_tile_max;
  int32_t wall_cull;
} upsample_tuning;
int upsample_set_tuning(upsample_handle h, const upsample_tuning* t);
int upsample_get_tuning(upsample_handle h, upsample_tuning* t);

/*
 * Kernel-time probe for one handle: when enabled, HIP events on the call's
 * stream bracket the step kernels -- each launch of upsample_advance, and in
 * upsample_run each stretch of consecutive step kernels of a batch (a reorder
 * ends a stretch), so that no event packets sit between them -- and
 * upsample_timing_read returns the summed milliseconds and the number of
 * kernel launches since the last read (it synchronises on the last event).
 */
int upsample_timing_enable(upsample_handle h, int enable);
int upsample_timing_read(upsample_handle h, double* advance_ms, int64_t* launches);

/*
 * Autotuner.  Times the step kernel (upsample_advance) for candidate cell
 * factors kappa in {0.51, 0.6, 0.75, 1.0001, 1.25} (cs = kappa * 3 r_lr;
 * below 1 the stencil reaches two cells) and for the launch knobs (sort_sub,
 * sort_mode) in {(1, Hilbert), (2, Hilbert), (2, cell then Morton)},
 * gather_groups and tile_max, by replaying a short stretch of the caller's
 * run: lr_x, lr_v hold n_frames consecutive LR frames ([n_frames][3][n_lr],
 * device); a copy of the HR state is reordered at the first frame, as a run
 * reorders at the start of each interval, and carried along the frames; each
 * setting is scored by its mean kernel time over the frames (waves spread as
 * particles drift between reorders, so the fresh state alone favours the
 * wrong knobs; n_frames of about the reorder interval is a good choice).
 * The fastest setting is returned.  It does not change what a step computes:
 * it depends on the grid and launch shape only (the membership predicate is
 * exact at any kappa).  Inputs are not modified.  The call allocates
 * temporary device memory and synchronises the stream; it is meant for
 * set-up, not for the timed path.
 *
 * cache_path (may be NULL) names a JSON-lines file: a result is looked up
 * there by a key made of the device architecture and a hash of the counts,
 * n_frames, the parameters and the wall table (from_cache = 1, nothing is
 * measured), and a new measurement is appended.  Errors: as upsample_init,
 * plus UPSAMPLE_ERR_INVALID_ARG for n_frames outside [1, 1024] and
 * UPSAMPLE_ERR_GRID_TOO_LARGE if no candidate grid fits.
 */
typedef struct {
  float cell_factor;       /* kappa for upsample_params.cell_factor */
  upsample_tuning tuning;  /* knobs for upsample_set_tuning */
  float advance_ms;        /* its mean step-kernel time per launch over the frames */
  int32_t from_cache;      /* 1: read from cache_path */
} upsample_autotune_result;

int upsample_autotune(const upsample_params* p, const float* lr_x, const float* lr_v,
                      const uint8_t* lr_rigid, int64_t n_lr, int32_t n_frames, const float* hr_x,
                      const float* hr_v, int64_t n_hr, const char* cache_path, void* stream,
                      upsample_autotune_result* out);

/*
 * One step without a handle and without allocating: for callers that cannot
 * call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  It computes what upsample_step computes
 * on a handle made from *p with the default tuning, bit for bit, from the
 * same arguments (p: as for upsample_init; max_lr, max_hr are ignored).  The
 * LR grid's scratch is a fixed device array inside the library, one per
 * device it runs on (taken at the first call on a device, with that device
 * current, and held until the process ends): it admits at most
 * UPSAMPLE_NOALLOC_MAX_LR LR particles and a grid of at most
 * UPSAMPLE_NOALLOC_MAX_CELLS cells (upsample_grid_info_for gives the count);
 * larger inputs are rejected with UPSAMPLE_ERR_CAPACITY before any work is
 * enqueued.  n_hr is not limited (the HR arrays are the caller's).  Every call
 * on one device uses that device's array, so calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller.
 * The flag UPSAMPLE_FLAG_VALIDATE is rejected (INVALID_ARG): it would
 * synchronise.  Other errors: as upsample_step; a failure inside HIP is
 * UPSAMPLE_ERR_HIP (no handle holds a message).
 */
#define UPSAMPLE_NOALLOC_MAX_LR    65536
#define UPSAMPLE_NOALLOC_MAX_CELLS 262144
int upsample_step_noalloc(const upsample_params* p,
                          const float* lr_x, const float* lr_v, const uint8_t* lr_rigid, int64_t n_lr,
                          const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                          int64_t n_hr, void* stream);

/*
 * Randomized volume sampling of an initial particle state (Section 4, the
 * sampling paragraph).  The box [lo, hi] (host float[3] each) is cut into
 * cubic cells of side 2 r / sqrt(3), G_a = ceil((hi_a - lo_a) / side) per
 * axis in double, so a cell's diagonal is 2 r; each candidate (device
 * float32 [3][n_cand], random positions inside the hull, drawn by the caller)
 * belongs to the cell clamp(floor(fl(fl(x - lo) fl32(1 / side))), 0, G - 1)
 * per axis.  Each cell then takes the first of its candidates, in input
 * order, whose squared distance to every position already taken is at least
 * fl32(4 r^2) (squared distance rounded as in the membership predicate), so
 * no two samples overlap as spheres of radius r.  The paper leaves the order
 * of the cells open: here it is 27 colour phases, colour (cx mod 3) +
 * 3 (cy mod 3) + 9 (cz mod 3), cell-key order inside a phase (cells of one
 * colour cannot conflict, so a phase's cells choose in parallel).  The samples
 * are written to out (device float32 [3][max_out]) in cell-key order, and
 * *n_out (host) receives their number; when it exceeds max_out the first
 * max_out are written and UPSAMPLE_ERR_CAPACITY is returned.  A set-up routine,
 * not a step: it allocates temporary device memory (about 36 B per cell and
 * 40 B per candidate) and synchronises the stream.  Errors: INVALID_ARG (bad
 * r, box or pointers), GRID_TOO_LARGE (2^31 cells or more, or an axis of 2^20),
 * CAPACITY, NO_DEVICE, OOM, HIP.
 */
int upsample_sample_volume(const float* cand, int64_t n_cand, float r, const float* lo, const float* hi,
                           float* out, int64_t max_out, int64_t* n_out, void* stream);

/*
 * Batched step: many independent scenes (each the problem of Section 4 with
 * its own parameters) advanced together.
 *
 * Particles of all scenes sit column-wise in shared device arrays: LR arrays
 * are [3][total_lr] with scene s in columns lr_offset .. lr_offset + n_lr - 1,
 * HR arrays [3][total_hr] likewise, where total_lr / total_hr are the largest
 * offset + count over the scenes; the column ranges of two scenes must not
 * overlap.  lr_rigid, when given, is uint8 [total_lr].  Each scene keeps its
 * own upsample_params (grid, dt, gravity, blend constants, walls; max_lr,
 * max_hr and flags are ignored); its counts are fixed at init.
 *
 * One step rebuilds the grids of all scenes with one counting sort over the
 * cells of every scene and advances all HR particles with one kernel over a
 * table of (scene, 256-particle tile) entries, one block per entry, laid out
 * so that each of the chip's XCDs works through a contiguous range of tiles.  The
 * launches are captured into a HIP graph (on an internal stream) once per
 * distinct set of buffer pointers -- the last four sets are kept -- and the
 * graph is replayed on the caller's stream; with UPSAMPLE_BATCH_EAGER they
 * are launched directly.  A captured step allocates nothing and holds no
 * memset node.  Per scene, results are bit-identical to upsample_step on a
 * handle with the same parameters.  The HR outputs may alias the inputs.
 *
 * Errors: UPSAMPLE_ERR_INVALID_ARG (bad scene table, overlapping ranges,
 * NULL buffers), UPSAMPLE_ERR_GRID_TOO_LARGE (all scenes' cells or LR
 * particles reach 2^31), UPSAMPLE_ERR_NO_DEVICE, UPSAMPLE_ERR_OOM,
 * UPSAMPLE_ERR_HIP.  A batch, like a handle, is not thread-safe; calls on one
 * batch must be ordered on one stream.
 */
typedef struct upsample_batch_s* upsample_batch;

typedef struct {
  upsample_params params;
  int64_t lr_offset, n_lr;
  int64_t hr_offset, n_hr;
} upsample_scene;

#define UPSAMPLE_BATCH_EAGER 1u
#define UPSAMPLE_MAX_SCENES 65535

int upsample_batch_init(const upsample_scene* scenes, int32_t n_scenes, uint32_t flags,
                        upsample_batch* out);
int upsample_batch_step(upsample_batch b, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                        const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                        void* stream);
/* HR reorder of every scene of the batch (the upsample_sort_hr of Section 4's
 * grid, per scene): each scene's HR columns [hr_offset, hr_offset + n_hr) of
 * hr_x, hr_v (device float32 [3][total_hr]) are permuted in place into the
 * order of the single-scene handle's default key (Hilbert order of the grid
 * cells split in two per axis), so that each scene's new order is the one
 * upsample_sort_hr gives its columns alone.  perm (device int32 [total_hr], or
 * NULL) receives for each new column the column it came from.  Long batched
 * runs call it every few steps to keep each wave's particles close together.
 * Scenes that own consecutive column ranges in scene order are sorted by one
 * counting sort over all of them (bins: the scenes' fine cells, ranked along
 * the Hilbert curve); other layouts by one sort per scene.  The first call
 * allocates the sort scratch (about 40 B per HR column plus 12 B per fine
 * cell of all scenes), builds the rank tables and synchronises; later calls
 * only enqueue.  Errors: INVALID_ARG, GRID_TOO_LARGE (a scene's grid is too fine
 * for the key bins), OOM/HIP (last_error says which). */
int upsample_batch_sort_hr(upsample_batch b, float* hr_x, float* hr_v, int32_t* perm, void* stream);
int upsample_batch_destroy(upsample_batch b);  /* waits for the device; NULL is a no-op */
const char* upsample_batch_last_error(upsample_batch b);
/* out[0] total_lr, out[1] total_hr, out[2] HR tiles, out[3] launch positions
 * of the step kernel's grid (one per tile; each runs as one one-wave block
 * per 64 particles of its tile), out[4] graphs captured so far */
int upsample_batch_info(upsample_batch b, int64_t* out);

/*
 * The LR simulation step (Section 3, Algorithm 1): position-based dynamics of
 * LR particles of radius r with contact and friction constraints, constraint
 * averaging (each particle's displacements of an iteration summed and divided
 * by its number of active constraints, all evaluated at the positions the
 * iteration starts from), stabilization iterations, masses scaled by
 * exp(-h) (h the height above ground_y), and shape matching of rigid bodies.
 *
 * Particles are typed by body[i]: UPSAMPLE_PBD_GRANULAR (-1), UPSAMPLE_PBD_STATIC
 * (-2: boundary samples that never move, inverse mass 0), or a rigid body id
 * 0 .. B-1 (dense).  One step of dt:
 *   1. dynamic particles v += dt g; x~ = x + dt v; w* = w exp(y - ground_y);
 *   2. contact pairs of x (closer than 2r, no static-static and no same-body
 *      pairs); stab_iters times: each overlapping pair (i, j) gives i the
 *      displacement -w*_i/(w*_i + w*_j) (2r - d) x_ij/d, x_ij = x_j - x_i;
 *      the averages are added to x and to x~;
 *   3. contact pairs of x~; solve_iters times: each overlapping pair gives
 *      the contact displacement plus friction on the tangential part Dt of
 *      the relative displacement (x'_i - x0_i) - (x'_j - x0_j) (x' after the
 *      contact displacement, x0 the stabilized start positions): the whole
 *      of Dt if |Dt| < 2 r mu_s, else Dt min(2 r mu_k / |Dt|, 1), shared in
 *      the inverse-mass ratio; each rigid particle gets R o_i + c - x~_i with
 *      c the mean of its body's x~ and R the rotation of the polar
 *      decomposition of sum (x~_i - c) o_i^T (o_i the rest offsets);
 *   4. v = (x~ - x0) / dt, x = x~ (static particles keep x, v = 0).
 * Pairs are found on a uniform grid of cells 2r (1.0001) wide over
 * [domain_lo, domain_hi] (particles outside are clamped into the border
 * cells: correct, only slower); the pair predicate is the float32 squared
 * distance (each operation rounded) against fl32(4 r^2).  Each particle keeps
 * at most max_neighbors pairs per phase; a longer list sets a sticky overflow
 * flag read by upsample_pbd_status (the extra pairs are dropped, which ones
 * unspecified).
 */
#define UPSAMPLE_PBD_GRANULAR (-1)
#define UPSAMPLE_PBD_STATIC   (-2)

typedef struct {
  float r;                 /* LR particle radius (m), > 0 */
  float dt;                /* LR time step (s), > 0 (Section 5.2: 0.005) */
  float g[3];              /* gravity (m/s^2) */
  float mu_s, mu_k;        /* static / kinetic friction (Section 5.2: 0.35, 0.3) */
  float ground_y;          /* height origin of the mass scaling */
  int32_t stab_iters;      /* stabilization iterations (Algorithm 1: 2) */
  int32_t solve_iters;     /* solver iterations (Algorithm 1: 5) */
  int32_t mass_scaling;    /* 1: w* = w exp(y - ground_y); 0: w */
  float domain_lo[3];      /* the pair grid's box */
  float domain_hi[3];
  int32_t max_neighbors;   /* pairs kept per particle and phase, 1 .. 1024 */
} upsample_pbd_params;

typedef struct upsample_pbd_s* upsample_pbd;

/* The defaults above, r = 0.02, domain [0, 1]^3, max_neighbors 32. */
int upsample_pbd_default_params(upsample_pbd_params* p);
/* body (int32 [n]), inv_mass (float32 [n], >= 0; ignored for static) and
 * rest (float32 [3][n], rest offsets o_i of rigid particles from their body's
 * centre of mass, equal masses within a body; ignored for others) are HOST
 * arrays, copied.  The handle owns device scratch of about (120 + 4 K) B per
 * particle plus 12 B per grid cell.  Errors: INVALID_ARG (bad parameters,
 * body ids below -2 or not dense, negative or non-finite inverse masses),
 * GRID_TOO_LARGE, NO_DEVICE, OOM, HIP. */
int upsample_pbd_init(const upsample_pbd_params* p, int64_t n, const int32_t* body, const float* inv_mass,
                      const float* rest, upsample_pbd* out);
/* Advances the device state x, v (float32 [3][n] each, in place) by n_steps
 * steps on the stream.  frames_x / frames_v (device float32 [n_steps][3][n],
 * both or neither) receive the state after each step.  Enqueues work only;
 * no synchronisation.  Errors: INVALID_ARG, HIP (the handle's last_error
 * says which call). */
int upsample_pbd_step(upsample_pbd h, float* x, float* v, int32_t n_steps, float* frames_x, float* frames_v,
                      void* stream);
/* Synchronises the stream; *overflow (host) = 1 if some particle had more
 * than max_neighbors pairs in a phase since init. */
int upsample_pbd_status(upsample_pbd h, int64_t* overflow, void* stream);
/* out[0] n, out[1] rigid bodies, out[2] max_neighbors, out[3] grid cells,
 * out[4] the trace length in floats of upsample_pbd_debug_step. */
int upsample_pbd_info(upsample_pbd h, int64_t* out);
/* One step, as upsample_pbd_step, that also records every stage (float32,
 * device): w* [n]; v and x~ after step 1 [3][n] each; per stabilization
 * iteration x and x~ [3][n] each; per solver iteration the bodies' c and R
 * (12 floats per body: c, then R row-major) and x~ [3][n]; the final x and v
 * [3][n] each.  trace_len must equal out[4] of upsample_pbd_info.  pair_cnt
 * (device uint32 [2][n]) and pair_ids (device uint32 [2][n][max_neighbors])
 * receive the pair lists of the stabilization (0) and solver (1) phases:
 * particle i's partners are pair_ids[phase][i][0 .. pair_cnt[phase][i]) (a
 * static particle keeps no list: every constraint moves it by zero, and its
 * partners list the pair); with stab_iters = 0 no stabilization pairs are
 * formed and phase 0's counts are 0.
 * Synchronises the stream.  A debug entry point. */
int upsample_pbd_debug_step(upsample_pbd h, float* x, float* v, float* trace, int64_t trace_len,
                            uint32_t* pair_cnt, uint32_t* pair_ids, void* stream);
int upsample_pbd_destroy(upsample_pbd h);  /* waits for the device; NULL is a no-op */
const char* upsample_pbd_last_error(upsample_pbd h);

#ifdef __cplusplus
}
#endif

#endif /* UPSAMPLE_H */
