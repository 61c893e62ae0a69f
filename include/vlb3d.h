/* vlb3d.h -- C ABI of the three-dimensional (D3Q19 or D3Q27) form of the coupled
 * viscoelastic lattice Boltzmann step (arXiv:2508.16997 extended to three dimensions,
 * which the paper calls straightforward in Sec. 3.1).
 *
 * One step is the two-dimensional method of Sec. 3.1-3.3 with every tensor index over
 * x, y, z: a hydrodynamic TRT regularized collision with the Galilean correction G_i
 * for the three diagonal cubic defects d_a(rho u_a^3), the body force F_i and the
 * polymer stress T_i; six convection-diffusion lattices (A_xx, A_xy, A_xz, A_yy, A_yz,
 * A_zz) with the auxiliary term, the constitutive source Phi = -(A - I)/lambda + A L +
 * (A L)^T + A tr L (Oldroyd-B, L = grad u by central differences; the other closures
 * of vlb.h through vlb3_set_closure) and half its time difference; half-way bounce-back of f and CNEBB of the conformation lattices at flat
 * walls.  The third order of the hydrodynamic lattice is expanded and projected in an
 * orthogonal basis with its lattice norms: on D3Q19 the six combinations H_aab -+ H_bcc,
 * on D3Q27 the six H_aab and H_xyz.
 *
 * Geometry: x and z periodic; y periodic (VLB_PERIODIC) or bounded by half-way walls
 * half a spacing outside rows 0 and ny - 1 (VLB_WALL); optionally solid nodes from a mask,
 * whose faces are half-way walls too (vlb3_set_solid).  Uniform body force.  Fields are
 * [nz][ny][nx] arrays, x fastest, in the simulation's precision (float for VLB_FP32,
 * double for VLB_FP64).  Arithmetic is double in both.
 *
 * Conventions as in vlb.h: every call returns VLB_OK (0) or a negative VLB_E_* code with
 * a thread-local detail string (vlb_last_error_detail); the caller owns the device
 * workspace and the stream; calls are asynchronous on that stream except where noted.
 */
#ifndef VLB3D_H
#define VLB3D_H

#include <stddef.h>
#include <stdint.h>

#include "vlb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlb3_sim vlb3_sim;

/* Host object for an nx x ny x nz grid on the lattice q (19: D3Q19, 27: D3Q27); each
 * size >= 1, ny >= 3 with VLB_WALL, nz <= 65535, ny <= 65535, 7 q (nx * ny * nz + 4224)
 * below 2^31.  prec: VLB_FP32 or VLB_FP64; ymode: VLB_PERIODIC or VLB_WALL.
 * Errors: VLB_E_INVALID_ARG. */
int vlb3_create(int nx, int ny, int nz, int q, int prec, int ymode, vlb3_sim** out);
/* Device workspace the simulation needs: two buffers of 7 q population planes, 9
 * history planes (S of the six components and u), 4 planes of rho and u, one 32-bit
 * plane of solid-link bits (256-byte aligned sections; each plane nx * ny * nz rounded up
 * to 64 elements plus 4160 of padding). */
int vlb3_workspace_bytes(const vlb3_sim* sim, size_t* bytes);
/* Attach the caller's 256-byte aligned device workspace of at least
 * vlb3_workspace_bytes and the HIP stream (NULL: the null stream) all work goes to.
 * Errors: VLB_E_WORKSPACE. */
int vlb3_bind(vlb3_sim* sim, void* workspace_dev, size_t bytes, void* hip_stream);
/* Solid nodes (host mask [nz][ny][nx], nonzero = solid; NULL removes them).  A fluid
 * node's pull from a solid node is the half-way bounce-back of f and the CNEBB input of
 * the conformation lattices (Sec. 3.3), a difference toward a solid neighbour takes the
 * no-slip value half a spacing away; solid nodes are read out at rest (rho = 1, u = 0,
 * A = I).  Call after vlb3_bind and before vlb3_init_equilibrium (it clears the state).
 * Synchronizes the stream.  Errors: VLB_E_STATE (not bound), VLB_E_HIP. */
int vlb3_set_solid(vlb3_sim* sim, const unsigned char* mask);
/* Lattice-unit parameters (Sec. 2.4, 3.1-3.2): solvent viscosity nu_s, polymer
 * viscosity eta_p, relaxation time lambda, conformation diffusivity kappa, the two magic
 * parameters, the uniform body force.  flags: VLB_FLAG_NO_SOURCE or 0.
 * Errors: VLB_E_INVALID_ARG (nu_s, kappa, lambda <= 0, eta_p < 0, magic parameters <= 0,
 * non-finite values, unknown flags). */
int vlb3_set_params(vlb3_sim* sim, double nu_s, double eta_p, double lambda, double kappa,
                    double Lambda_s, double Lambda_p, double Fx, double Fy, double Fz,
                    int flags);
/* Constitutive closure (Sec. 2.2; the enum and functions of vlb.h with every tensor
 * index over x, y, z and the 3-D trace, tr A = 3 at rest: Giesekus alpha (A - I)^2,
 * PTT factor of eps (tr A - 3), FENE-P f = (L^2 - 3) / (L^2 - tr A)).  The default
 * is VLB_OLDROYD_B; model_param is ignored for it.  Host call, takes effect at the next
 * vlb3_step.  Errors: VLB_E_INVALID_ARG (null sim, unknown model, non-finite parameter,
 * Giesekus alpha outside [0, 1], PTT eps < 0, FENE-P L^2 <= 3). */
int vlb3_set_closure(vlb3_sim* sim, int model, double model_param);
/* State at equilibrium of the given fields (device pointers in the simulation's
 * precision, [nz][ny][nx]; any may be NULL for its rest value rho = 1, u = 0, A = I), in
 * the order rho, u_x, u_y, u_z, A_xx, A_xy, A_xz, A_yy, A_yz, A_zz.  Resets the step
 * counter; the first step takes S and u of the previous step equal to its own.
 * Errors: VLB_E_STATE (not bound or no parameters). */
int vlb3_init_equilibrium(vlb3_sim* sim, const void* const fields_dev[10]);
/* Advance nsteps coupled steps (two launches per step). Errors: VLB_E_STATE, VLB_E_HIP. */
int vlb3_step(vlb3_sim* sim, int64_t nsteps);
/* rho, u (with the half-force shift) and the six conformation components of the
 * current state into ten device arrays in the order of vlb3_init_equilibrium (NULL to
 * skip one).  Errors: VLB_E_STATE, VLB_E_HIP. */
int vlb3_read_fields(vlb3_sim* sim, void* const fields_dev[10]);
/* Steps taken since vlb3_init_equilibrium. */
int vlb3_get_step(const vlb3_sim* sim, int64_t* step);
void vlb3_destroy(vlb3_sim* sim);

#ifdef __cplusplus
}
#endif

#endif /* VLB3D_H */
