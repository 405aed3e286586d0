/*
 * pod.h -- C ABI of the MI355X (gfx950) fast proper orthogonal descriptor
 * library, libpod.so.
 *
 * The operations follow N.-C. Nguyen, "Fast proper orthogonal descriptors for
 * many-body interatomic potentials" (arXiv:2212.14446):
 *   - radial snapshots Phi_l = f_c(r) psi(r; mu_l)          Sec. II.B, eqs. (3)-(8), (11)
 *   - POD radial basis R_k = sum_l Q_lk Phi_l                Sec. II.B, eq. (12)
 *   - atomic basis B_imnl = sum_j R_m(r_ij) A_nl(rhat_ij)    Sec. II.E, eq. (24b)
 *   - 2/3/4-body descriptors by the fast contractions        Sec. II.E, eqs. (25)-(30a)
 *   - linear energy E_i = sum_m c_m D_im, E = c . G          Sec. IV.A, eqs. (57a), (58a)
 *   - forces and virial from the descriptor derivatives      Sec. II.G, eqs. (26c), (24c)
 *   - batched descriptor matrices and the linear fit         Sec. IV.A, eqs. (58a), (63a)
 *   - network surrogate of the 4-body term                   Sec. IV.D
 *   - exclusive-sum descriptors (cost comparison)            Sec. II.C-D, eqs. (15b), (20a)
 *   - five-body descriptors (higher body order)              Sec. II.F
 *   - atom-centred symmetry functions                        Sec. III.B, eqs. (21c)-(22d)
 *   - molecular dynamics and neighbour lists                 Sec. V, Sec. II.A
 *
 * Conventions shared by every call
 *   - Descriptor vector of one atom (length M):
 *       [ 1 | D2_k, k < K2 | D3_mn, m < K3, n = 0..P3 (m-major) | D4_mp, m < K4, p < Ka(P4) (m-major) ]
 *     with M = 1 + K2 + K3 (P3 + 1) + K4 Ka(P4) (caption of Table 6); the 4-body
 *     index p runs over (a, b, c), a >= b >= c >= 0, a + b + c <= P4, in the
 *     order of Table 1.  The 3- and 4-body sums run over all ordered neighbour
 *     pairs / triples, coincident indices included (eqs. (15), (18a)).
 *   - Neighbour list (CSR, device memory, int32): offsets[N+1] (offsets[0] = 0,
 *     offsets[N] = P, non-decreasing), nbr_j[P] in [0, N), shift[P] packing the
 *     periodic image n as three signed bytes (n_x | n_y << 8 | n_z << 16).
 *     r_ij = pos[j] + n_x a1 + n_y a2 + n_z a3 - pos[i], a_k the rows of cell.
 *     The list is full (both directions).  Pairs with |r_ij| >= rcut are not
 *     neighbours (Sec. II.A) and contribute nothing, so a list built with a
 *     skin distance can be reused while atoms move; a pair with
 *     |r_ij| <= rin is a data error.  Periodic self-images (i == j, n != 0)
 *     are allowed.
 *   - pos: N x 3 row-major device array in the handle's dtype.
 *   - cell: 9 doubles in HOST memory, lattice vectors as rows; NULL for an open
 *     system (all shifts must then be zero).
 *   - Device pointers are caller-owned; the library never frees them.  All
 *     compute calls are asynchronous on the handle's HIP stream.
 *   - Errors: 0 = OK, negative POD_E* codes.  Argument errors are reported by
 *     the call itself; errors found in the data on the device (a pair at or
 *     inside rin, a non-finite coordinate, a malformed list) are latched in a
 *     device error word and reported by pod_check().  Offending pairs or atoms
 *     are skipped, never read out of bounds.  Nothing aborts across the ABI.
 *   - One handle per stream; calls on one handle must not overlap.
 */
#ifndef POD_H
#define POD_H

#ifdef __cplusplus
extern "C" {
#endif

#define POD_OK 0
#define POD_EINVAL (-1)      /* invalid argument or parameter */
#define POD_ERANGE (-2)      /* a pair distance at or below rin */
#define POD_ENONFINITE (-3)  /* a non-finite coordinate */
#define POD_ENOMEM (-4)      /* device allocation failed */
#define POD_EHIP (-5)        /* a HIP runtime call failed */
#define POD_ENOTSUP (-6)     /* parameters beyond what the kernels are built for */
#define POD_ENEIGH (-7)      /* malformed neighbour list (offsets, index, shift) */
#define POD_ESINGULAR (-8)   /* fit matrix not positive definite */
#define POD_ETOOBIG (-9)     /* problem larger than the static scratch of pod_energy_forces_noalloc */

#define POD_F64 0
#define POD_F32 1

/* Compile-time limits of the kernels.  Models up to angular degree 6 run on
 * the register-resident per-atom kernel; degrees 7 to 10 (the largest
 * models of Table 6) on a kernel that keeps each atom's basis in LDS. */
#define POD_MAX_L 16   /* snapshots */
#define POD_MAX_K 12   /* radial functions, max(K2, K3, K4) */
#define POD_MAX_P 10   /* angular degree of the 3-body terms, P3 */
#define POD_MAX_P4 6   /* angular degree of the 4-body terms, P4 (K_a <= 23) */

/*
 * Parameters (Sec. II.B-II.D).  One snapshot tuple mu_l = (rin, rcut, alpha_l,
 * beta_l, gamma_l, kappa_l) per l < L (eq. (11)); psi = kappa phi + (1 - kappa)
 * varphi with phi = sin(alpha pi x)/(r - rin), varphi = r^-gamma (eq. (3)).
 * Requirements: 0 <= rin < rcut; 1 <= L <= POD_MAX_L; 0 <= kappa_l <= 1;
 * beta_l >= 0; 0 <= K2, K3, K4 <= min(L, POD_MAX_K) with at least one > 0;
 * 0 <= P3 <= POD_MAX_P; 0 <= P4 <= POD_MAX_P4.  Q: NULL to compute the POD basis (method of
 * snapshots on n_quad midpoint nodes of (rin, rcut), unit eigenvectors of the
 * snapshot correlation matrix, decreasing eigenvalue, entry of largest
 * magnitude positive), or an L x K row-major matrix (K = max(K2, K3, K4)) to
 * use as given.  All arrays are host memory and are copied.
 */
typedef struct pod_params {
    double rin, rcut;
    int L;
    const double* alpha;
    const double* beta;
    const double* gamma;
    const double* kappa;
    int K2, K3, K4;
    int P3, P4;
    int dtype;          /* POD_F64 or POD_F32: type of pos, c, D, E_atom, F */
    const double* Q;    /* L x K row-major, or NULL */
    int n_quad;         /* quadrature nodes for the POD basis (>= 2L); 0 = 2000 */
} pod_params;

typedef struct pod_handle pod_handle;

/* Validate parameters, build the POD basis and tables, upload them.
 * hip_stream: a hipStream_t (NULL = default stream).  On success *out owns
 * device memory released by pod_free. */
int pod_init(const pod_params* p, void* hip_stream, pod_handle** out);

/* Host only (no device call): the POD basis of Sec. II.B, eq. (12) for the
 * given parameters.  Q: L x L row-major (columns = basis vectors, decreasing
 * eigenvalue), eigvals: L.  p->Q is ignored. */
int pod_compute_basis(const pod_params* p, double* Q, double* eigvals);

/* Descriptor counts: *M total; M_by_order[4] = {1, 2-, 3-, 4-body counts}
 * (either pointer may be NULL). */
int pod_num_descriptors(const pod_handle* h, int* M, int* M_by_order);

/* The basis in use: Q (L x K row-major, host) and eigvals (L, host; zeros when
 * Q was supplied by the caller).  Either pointer may be NULL. */
int pod_get_basis(const pod_handle* h, double* Q, double* eigvals);

/* Per-atom descriptors D (N x M row-major, device, handle dtype), eqs. (12b),
 * (15), (18a) evaluated by eqs. (24b)-(30a).  N >= 0 atoms, P pairs. */
int pod_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell,
                    const int* offsets, const int* nbr_j, const int* shift, void* D);

/* Reverse-pair index of a full neighbour list: rev[p] (device, P ints) is the
 * index of the pair (j -> i, -n) for pair p = (i -> j, n), searched in the
 * list of j.  Asynchronous on the handle's stream; a pair without its reverse
 * gets rev[p] = -1 and latches POD_ENEIGH (pod_check).  It depends on the list
 * only, so it is computed once per list, beside the list itself. */
int pod_neighbor_reverse(pod_handle* h, int N, int P, const int* offsets, const int* nbr_j,
                         const int* shift, int* rev);

/* Full neighbour list in the format above (Sec. II.A: the neighbours of atom
 * i are the atoms and periodic images closer than the cut-off), built on the
 * device with a cell list over fractional coordinates, so triclinic and
 * small cells (several images of one atom, self-images) are handled.
 *   pos      : N x 3 (device, handle dtype); atoms may lie outside the cell
 *   cell     : 9 doubles (HOST), lattice vectors as rows, or NULL for an
 *              open system (then pos is copied to the host once to bound it)
 *   rlist    : list radius (> 0), or 0 for the handle's rcut; a radius above
 *              rcut gives a skin list (see the cut-off contract above)
 *   offsets  : N + 1 ints (device), always written
 *   nbr_j, shift : capacity ints each (device), written when capacity >= the
 *              number of pairs; capacity 0 (with NULL arrays) only counts
 *   n_pairs  : host out, the number of directed pairs P
 * Pairs are kept when |r_ij| < rlist, in double (FP32 positions widened);
 * the only pair excluded is an atom with itself in the same image.  The
 * order of each atom's neighbours is fixed (bin scan order), so equal
 * inputs give equal lists.  Blocking: returns after the list is written.
 * POD_ENOTSUP if rlist spans more than 64 bins of a thin cell or P needs
 * more than 32-bit offsets.  Latched on the device (pod_check): a
 * non-finite coordinate (POD_ENONFINITE; the atom gets no neighbours), an
 * image shift beyond a signed byte (POD_ENEIGH).  Scratch grows in the
 * handle. */
int pod_build_neighbors(pod_handle* h, int N, const void* pos, const double* cell, double rlist,
                        int* offsets, int* nbr_j, int* shift, long capacity, long* n_pairs);

/* Linear POD energy and its derivatives (eqs. (57a), (58a), (26c), (24c)).
 * Three kernels on the handle's stream: the per-atom kernel (atomic basis,
 * contractions, energy, adjoint rows dE_i/dB_i), the pair kernel (g_p =
 * dE_i/dr_ij of every pair, virial) and the finalize kernel (totals, forces).
 *   rev    : reverse-pair index from pod_neighbor_reverse, or NULL.  With it,
 *            forces are gathered per atom, F_n = sum_{p in N(n)} (g_p - g_rev(p))
 *            with g_p = dE_i/dr_ij, in a fixed order (bitwise reproducible):
 *            each g_p is stored at its own slot p and at slot rev(p), so atom
 *            n's gather reads its own list range.  rev must be the list's
 *            reverse index (a pair without a reverse latches POD_ENEIGH).
 *            Without rev, forces are accumulated with FP64 atomics.
 *   c      : M coefficients (device, handle dtype)
 *   E_atom : N per-atom energies (device, handle dtype) or NULL
 *   E      : total energy (device, 1 double) or NULL
 *   F      : N x 3 forces F_n = -dE/dr_n (device, handle dtype) or NULL
 *   W      : 3 x 3 virial W_ab = -sum_pairs r_ij,a dE_i/dr_ij,b (device,
 *            9 doubles) or NULL
 *   G      : M global descriptors G = sum_i D_i = dE/dc (device, M doubles) or NULL
 * Totals (E, W, G) are accumulated in double on both dtypes. */
int pod_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell,
                      const int* offsets, const int* nbr_j, const int* shift, const int* rev,
                      const void* c, void* E_atom, double* E, void* F, double* W, double* G);

/* pod_energy_forces without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * dynamics loops, harnesses that forbid it.  Same arguments, kernels and
 * results as pod_energy_forces; its scratch (block partials, adjoint rows,
 * pair centres and vectors, pair gradients, and on the atomic path a
 * force accumulator that it clears with a fill kernel) lives in a static
 * device array of POD_STATIC_SCRATCH_BYTES per GPU, held from the first
 * pod_init on that GPU until the process ends.  Returns POD_ETOOBIG, with
 * nothing launched, when the call needs more: the 15,840-atom box of the
 * benchmark (397,508 pairs, K = 6, angular degree 4, FP64) needs about 59 MB.
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other handles,
 * other threads) race and must be ordered by the caller. */
#define POD_STATIC_SCRATCH_BYTES 67108864
int pod_energy_forces_noalloc(pod_handle* h, int N, int P, const void* pos, const double* cell,
                              const int* offsets, const int* nbr_j, const int* shift, const int* rev,
                              const void* c, void* E_atom, double* E, void* F, double* W, double* G);

/* Batched descriptor-matrix assembly for fitting (Sec. IV.A, eqs. (58a),
 * (63a)): many independent periodic cells in one persistent launch, FP64
 * handles only (POD_ENOTSUP otherwise).
 *   n_cfg        : number of cells; N, P: total atoms and pairs over all cells
 *   cfg_atom_off : n_cfg + 1 ints (device); cell c owns atoms
 *                  [cfg_atom_off[c], cfg_atom_off[c+1]), cfg_atom_off[0] = 0,
 *                  cfg_atom_off[n_cfg] = N
 *   pos          : N x 3 doubles (device), all cells stacked
 *   cells        : n_cfg x 9 doubles (DEVICE), lattice vectors as rows
 *   offsets, nbr_j, shift : one CSR list over the N stacked atoms as for the
 *                  single-system calls; nbr_j holds stacked indices, and every
 *                  neighbour of an atom of cell c must lie in cell c (else
 *                  POD_ENEIGH is latched and the pair skipped)
 *   D            : N x M per-atom descriptors (device) or NULL
 *   G            : n_cfg x M global descriptors G_c = sum_{i in c} D_i
 *                  (device) or NULL
 *   dGdR         : 3N x M (device) or NULL; row 3n + d, column k holds
 *                  dG_{c,k}/dr_{n,d} for the cell c that owns atom n, i.e. each
 *                  cell's (3 N_c) x M block of derivatives, stacked.
 *   tune         : launch shape (see pod_tune) or NULL for the defaults.
 * The library plans on the host from offsets and cfg_atom_off (a blocking
 * device-to-host copy of both), so the call returns after the plan, with the
 * kernel queued on the handle's stream.  A cell with more atoms than the
 * LDS accumulator holds (the limit depends on M and the tune) gives
 * POD_ENOTSUP.  Scratch grows in the handle (POD_ENOMEM on failure). */
typedef struct pod_tune {
    int cw;       /* descriptor columns per dG/dR chunk (0 = default 17; lowered
                     until the cell's LDS accumulator fits the device's LDS
                     per workgroup) */
    int nblocks;  /* persistent workgroups (0 = default 512, capped at n_cfg) */
    int threads;  /* threads per workgroup, a multiple of 64 up to 512
                     (0 = default 512; otherwise POD_EINVAL) */
} pod_tune;

int pod_batch_assemble(pod_handle* h, int n_cfg, int N, int P, const int* cfg_atom_off,
                       const void* pos, const double* cells, const int* offsets,
                       const int* nbr_j, const int* shift, double* D, double* G,
                       double* dGdR, const pod_tune* tune);

/* ---- Network surrogate of the 4-body energy (Sec. IV.D, eqs. (671a)-(673a)) ----
 * A network y(x) with two SiLU hidden layers of width POD_MLP_HIDDEN and a
 * linear output reads the standardised descriptors x = (X - mu) * inv_sigma
 * of one atom.  Parameters theta (FP32, device, caller-owned) are laid out as
 * W1 [64][n_in], b1 [64], W2 [64][64], b2 [64], w3 [64], b3, row-major and
 * concatenated (pod_mlp_num_params(n_in) floats).  Matrix products take
 * bfloat16 operands (round to nearest even: standardised inputs, W1, W2, the
 * first hidden activation and the back-propagated pre-activation gradients)
 * and accumulate in FP32; biases, the output layer and the activations stay
 * in FP32. */
#define POD_MLP_HIDDEN 64
#define POD_MLP_MAX_IN 64

/* Parameter count for n_in inputs (1 <= n_in <= POD_MLP_MAX_IN), or POD_EINVAL. */
int pod_mlp_num_params(int n_in);

/* Network output and its input gradient (eq. (673a)) for n rows.
 *   X        : n rows (device, handle dtype), row i holds its n_in inputs at
 *              X[i * ldx + k] (ldx >= n_in); e.g. a descriptor matrix from
 *              pod_descriptors offset by one column, ldx = M
 *   theta    : parameters (device FP32); mu, inv_sigma: n_in floats (device)
 *   y        : n floats (device) or NULL
 *   dydx     : n x n_in floats (device) dy/dX (inv_sigma applied) or NULL
 * Asynchronous on the handle's stream. */
int pod_mlp_forward(pod_handle* h, int n, int n_in, const void* X, long ldx, const float* theta,
                    const float* mu, const float* inv_sigma, float* y, float* dydx);

/* One training step on a batch of n rows: the mean squared error
 * L = (1/n) sum_i (y(x_i) - target_i)^2 (the energy part of eq. (63b), per
 * atom), its gradient by reverse differentiation, and one Adam update
 * (Kingma and Ba, 2015) of theta with moments adam_m, adam_v (device FP32,
 * same layout as theta, zero before step 1; step counts from 1).
 *   X      : n x n_in FP32 rows at X[i * ldx + k]; target: n floats (device)
 *   loss   : device float receiving L before the update, or NULL
 * The gradient is reduced in a fixed order: results are reproducible.
 * Asynchronous on the handle's stream; uses the handle's network scratch. */
int pod_mlp_train_step(pod_handle* h, int n, int n_in, const float* X, long ldx, const float* target,
                       const float* mu, const float* inv_sigma, float* theta, float* adam_m,
                       float* adam_v, int step, float lr, float beta1, float beta2, float eps,
                       float* loss);

/* Energies, forces and virial with the network in place of the 4-body term:
 *   E_i = c . D_i + y((D_i[1..M-1] - mu) * inv_sigma)
 * for a handle without 4-body descriptors (K4 = 0; n_in = M - 1 inputs,
 * else POD_EINVAL / POD_ENOTSUP).  Forces follow eq. (673a): the adjoint of
 * atom i takes the weights c + (0, dy/dX_i) on its descriptors, then the
 * pair sweep of eq. (24c) as in pod_energy_forces.  The per-atom kernel
 * runs the network on its own descriptors (the same products and rounding
 * as pod_mlp_forward, so the results equal those of pod_descriptors followed
 * by pod_mlp_forward); before it a small kernel packs the weights into the
 * handle's network scratch.  Arguments as for pod_energy_forces (no G);
 * theta, mu, inv_sigma as for pod_mlp_forward. */
int pod_energy_forces_surrogate(pod_handle* h, int N, int P, const void* pos, const double* cell,
                                const int* offsets, const int* nbr_j, const int* shift,
                                const int* rev, const void* c, const float* theta, const float* mu,
                                const float* inv_sigma, void* E_atom, double* E, void* F, double* W);

/* Exclusive-sum descriptors, the earlier POD form the paper compares its
 * fast descriptors with, evaluated by their defining sums on an FP64 handle
 * (POD_ENOTSUP otherwise): D2 by eq. (12b), D3 by eq. (15b) (neighbour pairs
 * j < k, O(N_i^2) per atom), D4 by eq. (20a) (triples j < k < l, O(N_i^3))
 * with the angular functions g_p of eq. (19a) as Table 2 prints them (each
 * distinct term of the cyclic orbit once; P4 <= 4, else POD_ENOTSUP).  Same
 * layout, arguments and M as pod_descriptors; the sums run in neighbour-
 * list order (the g_p with three distinct exponents are invariant under
 * cyclic permutations of j, k, l only).  An atom with more than 128
 * neighbours latches POD_ENEIGH and gets the row [1, 0, ...]. */
int pod_opod_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell,
                         const int* offsets, const int* nbr_j, const int* shift, void* D);

/* Energies, forces and virial of the 2/3-body exclusive model (OPOD of
 * Table 6): E_i = c . [1 | D2_i | D3_i] with D3 of eq. (15b), on an FP64
 * handle with K4 = 0 (POD_ENOTSUP otherwise).  Forces by the chain rule of
 * the pair sums (O(N_i^2) per atom), accumulated with FP64 atomics.
 * Arguments as for pod_energy_forces (no reverse index, no G); same
 * neighbour limit as pod_opod_descriptors. */
int pod_opod_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell,
                           const int* offsets, const int* nbr_j, const int* shift, const void* c,
                           void* E_atom, double* E, void* F, double* W);

/* Molecular dynamics, the use by which the paper measures the cost of its
 * potentials (Sec. V, Fig. 4): nsteps velocity Verlet steps
 *   v += dt/2 F/m;  x += dt v;  F = F(x) (pod_energy_forces);  v += dt/2 F/m
 * on the handle's stream, asynchronous.  Units: angstrom, fs, amu, eV.
 *   pos, vel, F : N x 3 (device, handle dtype), updated in place; F must hold
 *                 the forces of the initial positions on entry and holds those
 *                 of the final positions on return.  Updates are computed in
 *                 FP64 and stored in the handle's dtype.
 *   offsets, nbr_j, shift, rev : one list for all steps (rev as for
 *                 pod_energy_forces, or NULL).  It must be a skin list (radius
 *                 rcut + skin) that stays valid, i.e. no atom moves more than
 *                 skin / 2 from where the list was built during the call.
 *   c           : coefficients; mass > 0 (amu, all atoms); dt (fs)
 *   E_pot, E_kin: nsteps doubles each (device) or NULL: potential and kinetic
 *                 energy (eV) after every step.
 *   pos_ref, max_disp : the positions the list was built at (device, N x 3)
 *                 and 1 double (device), or both NULL: max_disp receives the
 *                 largest |x_n - x_ref_n| over all atoms and all steps of the
 *                 call (NaN if a coordinate became non-finite), so a caller
 *                 can verify that every step ran on a valid list.
 * Data errors are latched as for pod_energy_forces (pod_check). */
int pod_md_verlet(pod_handle* h, int N, int P, void* pos, void* vel, void* F, const double* cell,
                  const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* c,
                  double mass, double dt, int nsteps, double* E_pot, double* E_kin, const void* pos_ref,
                  double* max_disp);

/* max_n |pos_n - pos_ref_n| into *out (device double), for the rebuild
 * criterion of a skin list; NaN if a coordinate is not finite. */
int pod_md_max_displacement(pod_handle* h, int N, const void* pos, const void* pos_ref, double* out);

/* Linear fit (Sec. IV.A, eq. (63a)): normal equations of
 *   min_c  w_e sum_cells (G_c . c - E_ref_c)^2
 *        + w_f sum_rows (-dGdR_r . c - F_ref_r)^2 + gamma ||c||^2,
 * i.e. the weights multiply the squared residuals as in the loss of
 * eq. (63b), and forces are F = -dG/dR c (eq. (58a)).  FP64 on any handle.
 *   M        : descriptors per atom (M + 1 <= 128, else POD_ENOTSUP)
 *   G, E_ref : n_cfg x M global descriptors and n_cfg energies (device), as
 *              written by pod_batch_assemble; unused when n_cfg = 0
 *   dGdR, F_ref : n_frows x M derivative rows and n_frows forces (device),
 *              row r = 3 n + d holds dG/dr_{n,d} and F_ref[r] = F_{n,d}
 *              (the dGdR layout of pod_batch_assemble); unused when
 *              n_frows = 0
 *   w_e, w_f : finite, >= 0
 *   Z        : (M+1) x (M+1) row-major (device), symmetric on return:
 *              Z[:M,:M] = A^T W A, Z[:M,M] = A^T W b, Z[M,M] = b^T W b for the
 *              rows A = [G; -dGdR], b = [E_ref; F_ref]; accumulate != 0 adds
 *              to Z (so large sets can be streamed through in pieces).
 * Asynchronous on the handle's stream; the Gram sums run on the FP64 matrix
 * cores and are reduced in a fixed order (bitwise reproducible). */
int pod_fit_gram(pod_handle* h, int M, int n_cfg, const double* G, const double* E_ref, double w_e,
                 long n_frows, const double* dGdR, const double* F_ref, double w_f, int accumulate,
                 double* Z);

/* Solve (Z[:M,:M] + gamma I) c = Z[:M,M] (gamma >= 0) by a Cholesky
 * factorisation of the symmetrically scaled matrix, in one workgroup on the
 * handle's stream.  c: M doubles (device); loss: 1 double (device) or NULL,
 * the objective of eq. (63a) at c.  A matrix that is not positive definite
 * latches POD_ESINGULAR (pod_check), with c = 0 and loss = NaN. */
int pod_fit_solve(pod_handle* h, int M, const double* Z, double gamma, double* c, double* loss);

/* Five-body descriptors (the extension of Sec. II.F to higher body order,
 * built like the four-body descriptors of eqs. (16a)-(18a)):
 *   D5_{i m e} = sum_{j,k,l,n} R_m(r_ij) R_m(r_ik) R_m(r_il) R_m(r_in)
 *                w_jk^e1 w_jl^e2 w_jn^e3 w_kl^e4 w_kn^e5 w_ln^e6
 * with w_jk = rhat_ij . rhat_ik, over all ordered neighbour quadruples
 * (repeated indices included), for exponent tuples e >= 0 with |e| <= P5.
 * Relabelling the four neighbours permutes the six angle positions (order
 * (j,k), (j,l), (j,n), (k,l), (k,n), (l,n)) without changing the sum; there
 * is one descriptor per orbit, ordered by |e| ascending and, within a
 * degree, by the orbit's lexicographically largest tuple, descending (1, 2,
 * 5, 11, 22 descriptors for P5 = 0..4).  Evaluated through the atomic basis
 * of eq. (24b) as sums of products of four basis values, the five-body
 * counterpart of eq. (30a).
 *   K5 : radial functions used, 1 <= K5 <= max(K2, K3, K4) of the handle
 *   P5 : 0 <= P5 <= POD_FIVE_MAX_P (POD_ENOTSUP above)
 *   D5 : N x (K5 * count) row-major (device, handle dtype), m-major
 * Neighbour list, cut-off contract and data errors as for pod_descriptors;
 * asynchronous on the handle's stream. */
#define POD_FIVE_MAX_P 4
int pod_five_body_count(int P5, int* n);
int pod_five_body_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell,
                              const int* offsets, const int* nbr_j, const int* shift, int K5,
                              int P5, void* D5);

/* Energy E_i = sum_{m, e} c5[m count + e] D5_{i m e} of a linear five-body
 * term and its forces F = -dE/dx (E = sum_i E_i), for the descriptors above.
 * The adjoint dE_i/dB of each atom and radial function comes from the
 * merged products, then the pair derivative of eq. (24c) with R_m, R'_m.
 *   c5     : K5 x count coefficients (device, handle dtype), m-major
 *   rev    : reverse-pair index (pod_neighbor_reverse), required with F
 *   E_atom : N (device, handle dtype) or NULL; F : N x 3 or NULL (not both)
 * Four kernels on the handle's stream (pair records with R', basis and
 * adjoint, per-pair gradients, per-atom gather; no atomics, reproducible);
 * the handle's scratch holds the records, the adjoint rows and the pair
 * gradients.  Limits and data errors as for pod_five_body_descriptors. */
int pod_five_body_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell,
                                const int* offsets, const int* nbr_j, const int* shift,
                                const int* rev, int K5, int P5, const void* c5, void* E_atom,
                                void* F);

/* Atom-centred symmetry functions (Sec. III.B) through the atomic basis of
 * Sec. II.E, in work linear in the number of neighbours:
 *   G2_i = sum_j exp(-eta (r_ij - r_s)^2) f_c(r_ij)                eq. (21c)
 *   G3_i = 2^(1-zeta) sum_{j,k} (1 + lambda w_ijk)^zeta
 *          exp(-eta (r_ij^2 + r_ik^2)) f_c(r_ij) f_c(r_ik)          eq. (22c)
 *   G4_i = sum_{j,k,l} (1 + alpha w_ijk)^a (1 + beta w_ijl)^b (1 + gamma w_ikl)^c
 *          exp(-eta (r_ij^2 + r_ik^2 + r_il^2)) f_c f_c f_c          eq. (22d)
 * with f_c the cut-off of eq. (8) at the handle's rin and rcut (same
 * cut-off contract as the POD calls) and w_ijk = rhat_ij . rhat_ik.  The sums
 * run over all ordered neighbour tuples, repeated indices included, as the
 * POD sums of eqs. (15) and (18a) do.  Each function is a fixed combination
 * of the 3- and 4-body invariants (eqs. (26a), (27a), (30a)) of the atomic
 * basis of its radial function exp(-eta (r - r_s)^2) f_c(r); functions with
 * equal (eta, r_s) share one basis.
 *
 * pod_acsf_create builds a set for the handle's dtype (host arrays):
 *   g2 : n2 x 2 (eta, r_s)
 *   g3 : n3 x 3 (eta, zeta, lambda), zeta an integer in [0, 6]
 *   g4 : n4 x 7 (eta, a, b, c, alpha, beta, gamma), a, b, c non-negative
 *        integers with a + b + c <= 6
 * Functions are numbered G2 first, then G3, then G4, in the order given;
 * 1 <= n2 + n3 + n4 <= POD_ACSF_MAX_FUNCTIONS, at most POD_ACSF_MAX_CHANNELS
 * distinct (eta, r_s).  POD_EINVAL for non-finite or non-integral
 * parameters, POD_ENOTSUP beyond the limits.  *out owns device memory
 * released by pod_acsf_free; it is used only with handles of its dtype. */
#define POD_ACSF_MAX_FUNCTIONS 1024
#define POD_ACSF_MAX_CHANNELS 64
#define POD_ACSF_MAX_DEGREE 6
typedef struct pod_acsf pod_acsf;
int pod_acsf_create(pod_handle* h, int n2, const double* g2, int n3, const double* g3, int n4,
                    const double* g4, pod_acsf** out);

/* Number of functions and of distinct radial channels of a set (host). */
int pod_acsf_num_functions(const pod_acsf* a, int* n_functions, int* n_channels);

/* G (N x n_functions row-major, device, handle dtype) for the list of the
 * POD calls.  Asynchronous on the handle's stream; data errors are latched
 * as for pod_descriptors (pod_check). */
int pod_acsf_descriptors(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos,
                         const double* cell, const int* offsets, const int* nbr_j,
                         const int* shift, void* G);

/* Forces of E = sum_i W_i . G_i (the vector-Jacobian product of the
 * functions, i.e. the force of a network potential given dE/dG_i):
 *   W   : weights (device, handle dtype), row i at W + i * ldw; ldw = 0 uses
 *         one row for every atom (a linear model), else ldw >= n_functions
 *   rev : reverse-pair index from pod_neighbor_reverse (required when P > 0)
 *   G   : N x n_functions (device) or NULL: the functions, written as well
 *   F   : N x 3 (device, handle dtype): F = -dE/dx
 * Three kernels on the handle's stream (basis and adjoint per radial
 * channel, per-pair gradients, per-atom gather: no atomics, the result is
 * reproducible); the handle's scratch holds N x (sum of the basis sizes)
 * adjoint values and P x 3 pair gradients.  Data errors as above. */
int pod_acsf_forces(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos,
                    const double* cell, const int* offsets, const int* nbr_j, const int* shift,
                    const int* rev, const void* W, long ldw, void* G, void* F);

/* Release a set (no device call may still use it). NULL is allowed. */
void pod_acsf_free(pod_acsf* a);

/* Diagnostics.  pod_set_kernel_timing(h, n) with n > 0 makes the next n
 * compute calls record pairs of HIP events on the handle's stream around each
 * of their kernels (n = 0 switches recording off).  pod_get_kernel_time waits
 * for the stream and returns the summed elapsed time (ms) and the number of
 * recorded launches of one kernel -- kind 1: the per-atom kernel (radial
 * basis, atomic basis, contractions, energy, adjoint rows) and the
 * batched-assembly kernel; kind 4: the pair-gradient kernel of the energy
 * calls (per-pair gradients, own-atom sums, virial); kind 0: the finalize
 * kernel (totals E, W, G and the force gather or copy-out); kind 2: the
 * network kernels (for the surrogate: its weight packing; its network runs
 * inside the per-atom kernel, kind 1); kind 3: the Gram kernels of
 * pod_fit_gram; for the symmetry functions, kind 1 times the basis kernels
 * and kind 0 the pair-gradient and gather kernels -- then resets that
 * count. */
int pod_set_kernel_timing(pod_handle* h, int n);
int pod_get_kernel_time(pod_handle* h, int kind, double* total_ms, int* launches);

/* Wait for the handle's stream, return and clear the device error word
 * (POD_OK, POD_ERANGE, POD_ENONFINITE, POD_ENEIGH or POD_ESINGULAR), or
 * POD_EHIP. */
int pod_check(pod_handle* h);

/* Static description of an error code. */
const char* pod_strerror(int code);

/* Release the handle (waits for its stream). NULL is allowed. */
void pod_free(pod_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* POD_H */
