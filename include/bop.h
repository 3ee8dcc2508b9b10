/*
 * bop.h — C ABI of the MI355X (gfx950) analytic-BOP energy path.
 *
 * The path follows Hammerschmidt et al., "BOPfox program for tight-binding
 * and analytic bond-order potential calculations" (arXiv:1803.07491):
 *
 *   bop_build_neighbours   periodic neighbour list          (Sec. II "Initialisation")
 *   bop_build_H            two-centre Slater-Koster blocks  (App. A.2.1, App. D)
 *   bop_moments_plan / bop_moments
 *                          orbital moments <ia|H^n|ia>      (App. B.3, Eqs. momDOS,
 *                                                            xi_rec, xi_invert, xi_merge)
 *   bop_recursion          recursion coefficients + band    (App. B.3 Eqs. momtoa,
 *                          edges (Gershgorin terminator)     momtob; App. B.5)
 *   bop_energy             expansion coefficients, Jackson  (App. B.2-B.4, App. A.1
 *                          damping, Fermi level, N and U     Eq. TB-Ubond, Sec. II)
 *   bop_scf_step           one local-charge-neutrality step (App. A.3 Eq. BOP_LCN)
 *
 * Conventions (all calls):
 *  - Array arguments are device pointers to caller-owned, contiguous, row-major
 *    memory unless marked [host].  The library allocates no device memory; any
 *    scratch comes from a caller buffer whose size a *_workspace_size /
 *    *_plan call reports (bop_energy_noalloc instead uses a fixed device
 *    array of the library).
 *  - Every call takes the HIP stream last, only enqueues work on it and returns;
 *    exceptions (documented per call) read a count back to the host.
 *    Buffers must stay alive until the stream's work has completed.
 *  - Return value: BOP_OK or a negative BOP_E_* code; bop_last_error() gives a
 *    thread-local message for the last failure.  Device-side conditions never
 *    abort: they set bits in per-row `flags` words (see BOP_FLAG_*).
 *  - Energies in eV, lengths in Angstrom.  Orbital order per atom: d-only
 *    (n_orb = 5): 3z^2-r^2, zx, yz, x^2-y^2, xy; s,p,d (n_orb = 9): s, p_z, p_x,
 *    p_y, then the five d orbitals (Eq. Hij).
 */
#ifndef BOP_H
#define BOP_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define BOP_OK                0
#define BOP_E_ARG            -1   /* null pointer, negative or inconsistent size */
#define BOP_E_CAPACITY       -2   /* output too small; the required size is reported */
#define BOP_E_HIP            -3   /* a HIP runtime call failed */
#define BOP_E_UNSUPPORTED    -4   /* n_orb, n_max, n_exp or dtype outside the supported set */
#define BOP_E_NOT_CONVERGED  -5

/* ---- per-row flags (int, set on the device) ------------------------------- */
#define BOP_FLAG_BREAKDOWN   1    /* recursion chain ended early; level in bits 8.. */
#define BOP_FLAG_NONFINITE   2    /* a non-finite moment was seen */
#define BOP_FLAG_OUTSIDE     4    /* E_F lies outside this orbital's band */
#define BOP_FLAG_NARROW      8    /* band width raised to its floor (1e-6 eV) */
#define BOP_FLAG_DIVERGENT  16    /* some |g_m sigma_m| > 1e4: the terminated chain has
                                     states far outside the estimated band */

/* ---- compute types for H and the H.X products ----------------------------- */
#define BOP_F64   0
#define BOP_F32   1
#define BOP_BF16  2
#define BOP_F16   3   /* H.X vectors stored in FP16, FP32 blocks in memory; Lanczos form only
                         (d band: products on FP16 MFMA; otherwise FP32 arithmetic) */

/* ---- tight-binding model (host struct, passed by value to kernels) -------- */
#define BOP_MAX_SPECIES 3
#define BOP_N_CHANNELS 14
/* channel order; first letter = orbital on the atom the bond starts from,
 * second = orbital on the atom it points to; last letter = sigma/pi/delta */
enum { BOP_SSS, BOP_SPS, BOP_PSS, BOP_SDS, BOP_DSS, BOP_PPS, BOP_PPP,
       BOP_PDS, BOP_DPS, BOP_PDP, BOP_DPP, BOP_DDS, BOP_DDP, BOP_DDD };
#define BOP_FORM_POWER 0          /* beta(r) = beta0 (r0 / r)^q          */
#define BOP_FORM_EXP   1          /* beta(r) = beta0 exp(-q (r - r0))    */

typedef struct bop_model {
    int n_species;                /* 1 .. BOP_MAX_SPECIES */
    int n_orb;                    /* 5 (d) or 9 (s, p, d) */
    double r_cut;                 /* bond cutoff */
    double d_cut;                 /* width of the cosine taper Eq. (cutoff); 0 = hard */
    double onsite[BOP_MAX_SPECIES][3];              /* s, p, d levels */
    unsigned char form[BOP_MAX_SPECIES * BOP_MAX_SPECIES][BOP_N_CHANNELS];
    double beta0[BOP_MAX_SPECIES * BOP_MAX_SPECIES][BOP_N_CHANNELS];
    double r0[BOP_MAX_SPECIES * BOP_MAX_SPECIES][BOP_N_CHANNELS];
    double q[BOP_MAX_SPECIES * BOP_MAX_SPECIES][BOP_N_CHANNELS];
} bop_model;                      /* index [si * n_species + sj][channel] */

/* ---- messages ------------------------------------------------------------ */
/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes); returns its full length. */
int bop_last_error(char *buf, size_t n);

/* =========================================================================
 * Neighbour list (Sec. II "Initialisation": pairs within the cutoff via cell
 * lists; the paper's ghost cells appear here as explicit image shifts).
 *
 * All (j, S) with 0 < |d|^2 < r_cut^2, d = (r_j - r_i) + S.A evaluated in FP64
 * in the fixed order (r_j - r_i) + ((s1 a1 + s2 a2) + s3 a3), |d|^2 =
 * (dx dx + dy dy) + dz dz, without contraction: the list is bit-exact and
 * deterministic.  The cell is periodic along all three vectors.  Rows are
 * atoms in input order; entries are sorted by (j, s1, s2, s3).  (i, i, 0) is
 * excluded; other images of i and repeated j with different S are included.
 *
 *  pos        [N][3]  positions (fractional coordinates need not be wrapped)
 *  cell       [host] [3][3], rows = a1, a2, a3
 *  capacity   entries the output arrays can hold
 *  row_ptr    [N+1], nbr_j [cap], nbr_shift [cap][3], nbr_d [cap][3]
 *  order      [N] or NULL: atoms along a 3-D Hilbert curve over a grid of
 *             cells a third of the cell-list width (index order inside a
 *             cell), so that consecutive atoms form compact moment tiles
 *  n_pairs    [host] out: number of entries.  This call waits for the count
 *             (one device-to-host copy).  If it exceeds `capacity` nothing is
 *             written and BOP_E_CAPACITY is returned.
 *  ws         scratch of bop_neighbours_workspace_size() bytes
 * ========================================================================= */
size_t bop_neighbours_workspace_size(int n_atoms, const double *cell, double r_cut);
int bop_build_neighbours(int n_atoms, const double *pos, const double *cell, double r_cut,
                         long capacity, int *row_ptr, int *nbr_j, int *nbr_shift,
                         double *nbr_d, int *order, long *n_pairs,
                         void *ws, size_t ws_bytes, hipStream_t stream);

/* =========================================================================
 * Hamiltonian (App. A.2.1 Eqs. Hij, cutoff, Hij_rot; App. D rotations).
 *
 *  H_on   [N][n_orb] FP64: onsite level of the atom's species for the
 *         orbital's l, plus shift[i] (shift may be NULL).
 *  H_bond in `dtype` (BOP_F64, BOP_F32 or BOP_BF16; BOP_F16 gives FP32 blocks):
 *         n_orb = 9: [P][9][ld], ld = 9 (FP64/FP32) or 16 (BF16, the MFMA slot
 *         width; columns beyond n_orb are zero);
 *         n_orb = 5, BF16: [P][5][8], columns 5..7 zero;
 *         n_orb = 5, FP64/FP32: [P][BOP_D_PACKED] packed.  A d-d block is
 *         symmetric (every Slater-Koster d-d matrix is), so only its upper
 *         triangle is stored: entry (a, b), a <= b, at a*5 - a(a-1)/2 + (b - a),
 *         and value 15 is zero.  This is the layout bop_moments and
 *         bop_lanczos read for n_orb = 5 in FP64/FP32.
 *         block p = <i a|H|j b> for pair p = (i -> j), built in the bond frame
 *         (z' along d) and rotated as R^T H^(b) R, where R[a][b] is App. D's
 *         matrix with a = bond-frame orbital, b = global orbital, theta the
 *         polar angle and phi the azimuth of d (taken from direction cosines).
 *         H_bond = NULL updates H_on only (self-consistency steps).
 * ========================================================================= */
#define BOP_D_PACKED 16     /* values per packed d-d block (15 + one zero) */
int bop_build_H(const bop_model *model /*[host]*/, int n_atoms, const int *species,
                const double *shift, const int *row_ptr, const int *nbr_j,
                const double *nbr_d, long n_pairs, int dtype,
                double *H_on, void *H_bond, hipStream_t stream);

/* =========================================================================
 * Moments (App. B.3).  mu[i][a][n] = <i a|H^n|i a>, n = 0..n_max, where H is
 * the folded periodic (Gamma-point) Hamiltonian: H[i][j] = sum over the
 * list's images of H_bond, plus diag(H_on).
 *
 * Interference paths are built iteratively, X^k = H X^(k-1) (Eq. xi_rec), for
 * tiles of `tile_atoms` atoms whose unit start vectors form the columns of X;
 * moments follow from merging path halves (Eqs. xi_invert, xi_merge):
 * mu_2k = <X^k, X^k>, mu_2k-1 = <X^(k-1), X^k>, and mu_2K+1 = <X^K, H X^K>.
 * X is stored and multiplied in `dtype`; mu is accumulated and returned in FP64.
 *
 * Three calls:
 *  bop_moments_plan     walks the neighbour graph once (device breadth-first
 *                       search per tile), waits for it, and fills `plan` with the
 *                       sizes, including plan->ws_bytes.  Uses `scratch` of
 *                       bop_moments_plan_scratch_size bytes.
 *  bop_moments_prepare  stores every tile's support, layers and layer-sorted
 *                       neighbour slots in `ws`.  Redo both when the neighbour
 *                       list changes; not when only H_on or H_bond change.
 *  bop_moments          the H.X steps; reads the prepared supports from `ws`.
 * `order` (may be NULL = input order) groups atoms into tiles.  A tile whose
 * support outgrows the plan, or whose support holds a row with more neighbours
 * than the plan's deg_max (neighbour list changed without re-planning), gets
 * NaN moments.
 * ========================================================================= */
typedef struct bop_tuning {
    int tile_atoms;      /* atoms per tile; 0 = as many as fit one wavefront */
    int block_threads;   /* 256, 512 or 1024; 0 = default (512) */
    int batch_tiles;     /* tiles whose X buffers are live at once; 0 = 48 GiB worth (at most a
                            quarter of the free device memory) */
    int chunk_rows;      /* support rows per workgroup and step (the rows are dealt to the
                            workgroups of a tile in wave-sized groups, round robin); 0 = default
                            (64; 128 for BF16 and FP16 d-band plans).  The moment passes use it;
                            the force passes deal their rows in chunks of 16 whatever it is */
    int plan_search;     /* support sizes in bop_moments_plan: 0 = automatic, 1 = visited bitmap in
                            LDS (up to 524,288 atoms), 2 = per-workgroup map in `scratch`; both
                            give the same plan */
} bop_tuning;

#define BOP_MAX_NMAX 40
/* Maximum radius of the interference paths (Sec. III "Speed-ups" (iii), an
 * additional approximation): with r_max > 0 the moments of atom i keep only the
 * paths whose every atom lies within r_max of atom i (minimum-image distance
 * from the positions).  Needs r_max + r_cut below half the smallest height of
 * the cell (then each atom within r_max has one image there), else BOP_E_ARG;
 * FP64/FP32/FP16 forms only (BF16: BOP_E_UNSUPPORTED).  The tiles' supports
 * then hold only atoms within r_max of one of their atoms, and each column
 * keeps the rows within r_max of its own atom. */
typedef struct bop_path_radius {
    double r_max;          /* > 0 */
    double r_cut;          /* the neighbour list's cutoff */
    double cell[9];        /* rows a1, a2, a3 */
    const double *pos;     /* [N][3] device positions (those of the neighbour list) */
} bop_path_radius;

typedef struct bop_plan {
    int n_atoms, n_orb, n_max, dtype;
    int tile_atoms, n_tiles, block_threads, batch_tiles, chunk_rows;
    int deg_max;         /* longest neighbour row */
    int rows_cap;        /* largest tile support (rows of X) */
    int rows_k[BOP_MAX_NMAX / 2 + 1];   /* largest |support of X^k| per k */
    int search;          /* support search used by the plan and by bop_moments_prepare:
                            1 = bitmaps in LDS (rows of a layer in ascending atom index),
                            2 = per-workgroup map (rows in order of discovery) */
    size_t ws_bytes;     /* workspace bop_moments_prepare / bop_moments need */
    double r_max;        /* path radius of the plan (0: none) */
} bop_plan;

size_t bop_moments_plan_scratch_size(int n_atoms);
int bop_moments_plan(int n_atoms, int n_orb, int n_max, int dtype,
                     const int *row_ptr, const int *nbr_j, const int *order,
                     const bop_tuning *tuning /*[host] or NULL*/,
                     const bop_path_radius *radius /*[host] or NULL = all paths*/,
                     void *scratch, size_t scratch_bytes,
                     bop_plan *plan /*[host] out*/, hipStream_t stream);
int bop_moments_prepare(const bop_plan *plan /*[host]*/, const int *row_ptr,
                        const int *nbr_j, const int *order,
                        const bop_path_radius *radius /*[host]; the plan's, or NULL if it has none*/,
                        void *ws, size_t ws_bytes, hipStream_t stream);
int bop_moments(const bop_plan *plan /*[host]*/, const int *row_ptr, const double *H_on,
                const void *H_bond, double *mu, void *ws, size_t ws_bytes,
                hipStream_t stream);

/* =========================================================================
 * Batched form: many independent periodic structures as one block-diagonal
 * neighbour graph (moments of each structure are those of its own cell, Eq.
 * momDOS, since no pair joins two structures), so one plan / prepare /
 * bop_moments (or bop_lanczos) sequence covers the batch; bop_moments
 * enqueues kernels only (no synchronisation, no allocation) and can be
 * captured in a HIP graph and replayed.
 *
 * Joins per-structure neighbour lists (each from bop_build_neighbours on its
 * own cell) into global ones.  Structure s owns atoms [atom_off[s],
 * atom_off[s+1]) and pairs [pair_off[s], pair_off[s+1]).
 *   atom_off, pair_off [n_structs+1] (device, int)
 *   row_ptr_local [n_atoms + n_structs]: structure s's own row_ptr (n_s + 1
 *                 entries, local pair indices) at atom_off[s] + s
 *   nbr_j_local [P], order_local [n_atoms]: local atom indices, concatenated
 *   out: row_ptr [n_atoms+1], nbr_j [P], order [n_atoms] (global indices)
 * nbr_d and species concatenate unchanged.
 * ========================================================================= */
int bop_batch_concat(int n_structs, int n_atoms, const int *atom_off, const int *pair_off,
                     const int *row_ptr_local, const int *nbr_j_local, const int *order_local,
                     int *row_ptr, int *nbr_j, int *order, hipStream_t stream);

/* One call per batch step: bop_batch_concat, bop_moments_prepare and
 * bop_moments in sequence on `stream`, with no synchronisation and no
 * allocation, so that a serving loop can capture it in a HIP graph and
 * replay it for new per-structure neighbour lists of the batch.  `plan` is
 * made once (bop_moments_plan on a joined list of the batch; plan->n_atoms
 * is the batch's atom count) and must still fit the new lists: tiles whose
 * supports do not fit get NaN moments, as with bop_moments_prepare.  H_on
 * [N][n_orb] and H_bond [P] are in the joined order (structure by
 * structure, so each structure's blocks can be built from its own list).
 * Arguments as bop_batch_concat and bop_moments; ws is the plan's
 * workspace.  Errors: those of the three calls; BOP_E_UNSUPPORTED for a plan
 * with a path radius. */
int bop_moments_batched(const bop_plan *plan /*[host]*/, int n_structs, const int *atom_off,
                        const int *pair_off, const int *row_ptr_local, const int *nbr_j_local,
                        const int *order_local, int *row_ptr, int *nbr_j, int *order,
                        const double *H_on, const void *H_bond, double *mu, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* =========================================================================
 * Recursion coefficients straight from the H.X products: the Lanczos chain
 * (Sec. "Density of states" of App. B, the tridiagonal Hamiltonian of the
 * recursion method; App. B.3 for the coefficients' definition).
 *
 * Same plan, tiles, supports and workspace as bop_moments (prepare first).
 * Per orbital row: u_0 = the unit start vector, a_k = <u_k, H u_k - b_k
 * u_(k-1)>, b_(k+1) = |H u_k - a_k u_k - b_k u_(k-1)|, u_(k+1) = that vector /
 * b_(k+1), for a_k, k < n_a and b_k, 1 <= k <= n_b: in exact arithmetic the
 * coefficients bop_recursion derives from the moments up to n_max.  The
 * vectors are stored in the plan's dtype and kept orthonormal by construction,
 * so FP32 and BF16 rounding shows up in a_n, b_n at about the unit roundoff
 * times |H|, where the moment route amplifies it (ill-conditioned Hankel
 * map).  Inner products and coefficients are FP64.
 * Breakdown: b_(k+1)^2 <= thr * b_1^2 (thr = 1e-14 FP64, 1e-10 FP32, 1e-7
 * FP16, 1e-5 BF16) sets that and later b to 0, repeats a, and flags
 * BOP_FLAG_BREAKDOWN | level << 8, as the moment route does.  Seeds of a
 * failed tile get NaN coefficients and BOP_FLAG_NONFINITE.
 * 16-bit vectors: for the d band with at most 16 neighbours per atom, BF16
 * and FP16 plans run the products on MFMA over packed rows (two orbitals per
 * 32-bit word), with the blocks rounded to the vectors' format (FP16 plans
 * keep FP32 blocks in memory and round them as they are read), each column's
 * chain shifted by its own onsite level; otherwise BF16 takes a two-pass form
 * on padded rows and FP16 stores FP16 vectors with FP32 products.
 *
 *  a [N*n_orb][n_a], b [N*n_orb][n_b+1] (b[.][0] = 0), flags [N*n_orb] out.
 *  Follow with bop_recursion(mu = NULL) for the terminator and bop_energy(mu
 *  = NULL), which take every sigma_m from the chain.
 * ========================================================================= */
int bop_lanczos(const bop_plan *plan /*[host]*/, const int *row_ptr, const double *H_on,
                const void *H_bond, double *a, double *b, int *flags, void *ws,
                size_t ws_bytes, hipStream_t stream);

/* =========================================================================
 * Recursion coefficients and terminator (App. B.3, App. B.5), FP64.
 *
 * Per row (one orbital; mu normalised by its mu_0): a_n for n < n_a =
 * (n_max-1)/2 + 1 and b_n for 1 <= n <= n_b = n_max/2 (b[.][0] = 0), from the
 * moments via the c_j^n recursion, with b_(n+1) taken as the norm of the next
 * unnormalised Lanczos vector (the printed Eq. momtob needs c^n before b_n
 * is known).  Breakdown (b_(n+1)^2 <= 1e-14 (mu_2 - mu_1^2)) sets b_(n+1) = 0,
 * repeats a_n, and flags BOP_FLAG_BREAKDOWN | level << 8.
 * bw_mode (App. B.5 estimates of the centre a_inf = A and width b_inf = B):
 *  BOP_BW_GERSHGORIN (vii)  band edges of Eq. (gershogorin) over rows n < n_a
 *                       (b_0 = 0, b_(n_a) used only if computed); A = (top +
 *                       bottom)/2, B = (top - bottom)/4.  The default.
 *  BOP_BW_GLOBAL (viii) the given a_glob, b_glob for every row.
 *  BOP_BW_LOWEST (i)    A = a_0, B = b_1.
 *  BOP_BW_HIGHEST (ii)  the highest computed a_n and b_n.
 *  BOP_BW_AVERAGE (iii) A = mean a_n, B = sqrt(mean b_n^2).
 *  BOP_BW_AVERAGE_HIGHEST (iv)  A = mean a_n, B = highest computed b_n.
 *  BOP_BW_MINMAX (v)    A = (max a + min a)/2, B = (max a - min a + 4 max b)/4,
 *                       Eq. (findeminemax).
 *  BOP_BW_WEIGHTED      the weighted-average terminator of App. B.1 Eq.
 *                       (weighted), beta = a_glob >= 0: w_m = 1/(beta (M - m) +
 *                       1), m = 0..M for a and 1..M for b, M the highest
 *                       computed level; the averages serve as the constant
 *                       tail and as the expansion's centre and width.
 *  Options i-v and the weighted average use the levels computed before a
 *  breakdown only (flag level L: a_0..a_(L-1), b_1..b_(L-1)).
 *
 *  mu [n_rows][n_max+1] -> a [n_rows][n_a], b [n_rows][n_b+1],
 *  a_inf, b_inf, flags [n_rows].   n_max <= 40.
 *  mu = NULL: a, b (and flags) are inputs from bop_lanczos; only a_inf, b_inf
 *  and the flags the terminator adds are written.
 * ========================================================================= */
#define BOP_BW_GERSHGORIN      0
#define BOP_BW_GLOBAL          1
#define BOP_BW_LOWEST          2
#define BOP_BW_HIGHEST         3
#define BOP_BW_AVERAGE         4
#define BOP_BW_AVERAGE_HIGHEST 5
#define BOP_BW_MINMAX          6
#define BOP_BW_WEIGHTED        7
int bop_recursion(int n_rows, int n_max, const double *mu, int bw_mode,
                  double a_glob, double b_glob, double *a, double *b,
                  double *a_inf, double *b_inf, int *flags, hipStream_t stream);

/* =========================================================================
 * Bond energy (App. B.2-B.4, App. A.1 Eq. TB-Ubond; Fermi level Sec. II), FP64.
 *
 * Per orbital: sigma_m = sum_n p_mn mu^_n for m <= n_max (Eq. sigma_i) and, for
 * n_max < m <= n_exp, the chain recursion of App. B.4 with the constant
 * terminator (evaluated exactly on the computed levels plus one delay level,
 * since the free terminator tail only delays its input); damping g_m =
 * g^J_(m+1)/g^J_1 with the Jackson kernel of length n_exp.  Then with
 * cos(phi) = clamp((E - a_inf)/(2 b_inf), -1, 1):
 *   N_ia = sum_m g sigma_m chi^_(m+1)(phi),
 *   U_ia = b_inf sum_m g sigma_m [chi^_(m+2) + chi^_m](phi) + (a_inf - E_ia) N_ia
 *          (= integral up to E of (E' - E_ia) n_ia(E') dE'),
 *   n_ia(E) = sum_m g sigma_m sin((m+1) phi) / (pi b_inf).
 * Per atom, both spins: N_atom = 2 sum_a N_ia, U_atom = 2 sum_a U_ia,
 * dos_atom = 2 sum_a n_ia(E_F); U_total = sum_i U_atom.
 *
 *  ef_mode 0: E_F [device, 1 double] out: bisection (Sec. II) on
 *             2 sum N_ia(E) = n_elec over [min(a_inf - 2 b_inf), max(a_inf +
 *             2 b_inf)], halving while the midpoint differs from both ends (at
 *             most 64 times; four halvings are decided per pass over the
 *             coefficients, with exactly the midpoints and decisions of
 *             sequential bisection); E_F = midpoint of the final bracket.
 *  ef_mode 1: E_F [device] in: energies at the given level.
 *  ws: bop_energy_workspace_size(n_atoms, n_orb, n_exp) bytes.
 *  n_exp <= 1024 (default used by the paper's example: 200); n_orb <= 9
 *  (BOP_E_UNSUPPORTED beyond).
 *  mu = NULL (Lanczos form): sigma_m for every m from the chain, which equals
 *  the moment route for m <= n_max in exact arithmetic.
 * ========================================================================= */
size_t bop_energy_workspace_size(int n_atoms, int n_orb, int n_exp);
int bop_energy(int n_atoms, int n_orb, int n_max, int n_exp, const double *mu,
               const double *a, const double *b, const double *a_inf,
               const double *b_inf, const double *H_on, double n_elec /*[host]*/,
               int ef_mode, double *E_F, double *N_atom, double *U_atom,
               double *dos_atom, double *U_total, int *flags,
               void *ws, size_t ws_bytes, hipStream_t stream);

/* =========================================================================
 * Atom-averaged mode (the per-atom reading of the moments; the paper's DOS
 * and energy are per orbital, App. B.2, and that remains the default).
 *
 *  bop_atom_average          mu_avg[N][n_max+1] = sum_a mu[i][a][.] / n_orb and
 *                            H_avg[N] = the orbital-averaged onsite level.
 *  bop_energy_atom_averaged  bop_energy on one chain per atom (a, b, a_inf,
 *                            b_inf from bop_recursion on mu_avg with n_rows =
 *                            N), each chain standing for n_orb orbitals: the
 *                            Fermi level solves 2 n_orb sum_i N_i = n_elec and
 *                            N_atom, U_atom, dos_atom, U_total are 2 n_orb
 *                            times the chain's.  Workspace:
 *                            bop_energy_workspace_size(N, 1, n_exp).  Where
 *                            all orbitals of an atom share one local DOS it
 *                            equals the orbital-resolved result.
 * ========================================================================= */
int bop_atom_average(int n_atoms, int n_orb, int n_max, const double *mu, const double *H_on,
                     double *mu_avg, double *H_avg, hipStream_t stream);
int bop_energy_atom_averaged(int n_atoms, int n_orb, int n_max, int n_exp, const double *mu_avg,
                             const double *a, const double *b, const double *a_inf,
                             const double *b_inf, const double *H_avg, double n_elec /*[host]*/,
                             int ef_mode, double *E_F, double *N_atom, double *U_atom,
                             double *dos_atom, double *U_total, int *flags, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* =========================================================================
 * bop_energy without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, kernels and results as bop_energy;
 * the workspace is a fixed device array of BOP_ENERGY_NOALLOC_BYTES (64 MiB),
 * one per GPU the library runs on, kept until the process ends.  Fits n_atoms
 * * n_orb * (n_exp + 1) * 8 bytes plus small partials: about 8,000 d-band
 * atoms or 4,500 s,p,d atoms at n_exp = 200.  Larger inputs: BOP_E_CAPACITY
 * (nothing enqueued).  It calls no allocator.  All calls on one GPU share the
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (several streams or threads) race.
 * ========================================================================= */
#define BOP_ENERGY_NOALLOC_BYTES (64ull << 20)
int bop_energy_noalloc(int n_atoms, int n_orb, int n_max, int n_exp, const double *mu,
                       const double *a, const double *b, const double *a_inf,
                       const double *b_inf, const double *H_on, double n_elec /*[host]*/,
                       int ef_mode, double *E_F, double *N_atom, double *U_atom,
                       double *dos_atom, double *U_total, int *flags, hipStream_t stream);

/* =========================================================================
 * One local-charge-neutrality step (App. A.3 Eq. BOP_LCN with the linear
 * input/output mixing of Sec. II "Self-consistency").  One onsite shift per
 * atom: rebuild H_on from `shift`, then moments, recursion and energy as
 * above, then q_i = N_i - n0_i; if max|q_i| < tol: *converged = 1 and shift is
 * unchanged; else shift_i += mix q_i / max(n_i(E_F), n_floor) followed by
 * removal of the mean shift (shift + c with E_F + c is the same state).
 * Everything stays on the device; the host loops until *converged.
 * method 0: moments + bop_recursion; method 1: bop_lanczos (mu unused).
 * ========================================================================= */
typedef struct bop_system {
    bop_model model;
    int n_atoms, n_max, n_exp, dtype;
    int method;
    const int *species;            /* [N] */
    const double *n0;              /* [N] reference electrons per atom */
    const int *row_ptr, *nbr_j, *order;
    long n_pairs;
    double *H_on;                  /* [N][n_orb] (rebuilt each step) */
    const void *H_bond;            /* [P][n_orb][n_orb] in dtype */
    bop_plan plan;
    void *moments_ws; size_t moments_ws_bytes;
    double *mu, *a, *b, *a_inf, *b_inf;
    int *flags;
    void *energy_ws; size_t energy_ws_bytes;
    double n_elec;                 /* total electrons, both spins */
    double *E_F, *N_atom, *U_atom, *dos_atom, *U_total;   /* outputs */
} bop_system;

int bop_scf_step(const bop_system *sys /*[host]*/, double mix, double n_floor,
                 double tol, double *shift, double *q, double *max_dq,
                 int *converged, hipStream_t stream);

/* =========================================================================
 * The same step with Broyden mixing (Sec. II "Self-consistency", mixer (ii):
 * Broyden's second method, updating an approximation H of the inverse
 * Jacobian of the residual).  Residual F_i = q_i / max(n_i(E_F), n_floor), the
 * linear mixer's output step; H_0 = -mix I, so a step from H_0 is linear
 * mixing.  With s = shift_n - shift_(n-1), y = F_n - F_(n-1):
 *   H_n = H_(n-1) + (s - H_(n-1) y) y^T / (y.y),  shift_(n+1) = shift_n - H_n F_n,
 * then the mean shift is removed.  `iter` is the caller's 0-based iteration
 * count of this cycle: position j = iter % (hist + 1) in the history, j = 0
 * (the first step and every hist + 1 steps) starting again from H_0.  The
 * history lives in `ws` (bop_broyden_workspace_size(n_atoms, hist) bytes,
 * hist <= 64) and must be kept between the steps of one cycle.  Converged
 * (max |q_i| < tol): nothing changes.
 * ========================================================================= */
size_t bop_broyden_workspace_size(int n_atoms, int hist);
int bop_scf_step_broyden(const bop_system *sys /*[host]*/, double mix, double n_floor,
                         double tol, int iter, int hist, double *shift, double *q,
                         double *max_dq, int *converged, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* =========================================================================
 * Collinear magnetism (Sec. II "Hamiltonian": the up and down channels are
 * computed one after the other, each like a non-magnetic calculation; App.
 * A.2.2 collinear onsite levels; App. A.1 Eq. TB-UX).
 *
 * Channel onsite levels E_iav = H0_ia + shift_i - (-1)^v B_z
 * + (1/2) (-1)^v I_i m_i, with (-1)^v = -1 for the up channel (a positive
 * moment lowers the up levels by I_i m_i / 2).  The channels share H_bond.
 *
 *  bop_spin_shifts   shift_spin[2][N]: the per-atom onsite shifts of the up
 *                    and down channels (shift, moment may be NULL = 0).
 *  bop_mag_energy    both channels through the energy path with one Fermi
 *                    level: sum over channels, orbitals, atoms of N_iav = N_e
 *                    (sys->n_elec).  The bop_system buffers hold both channels
 *                    stacked, up atoms then down atoms: H_on [2N][n_orb], mu
 *                    [2N][n_orb][n_max+1] (method 0) or a, b, flags for 2N
 *                    n_orb rows (method 1), a_inf, b_inf, flags [2N n_orb],
 *                    N_atom, U_atom, dos_atom [2N] and energy_ws sized for 2N
 *                    atoms.  Outputs per channel (no spin factor): N_atom[v N
 *                    + i] = N_iv, U_atom[v N + i] = sum_a int^E_F (E - E_iav)
 *                    n_iav dE, dos_atom[v N + i] = n_iv(E_F); U_total = bond
 *                    energy of both channels; m_out[N] = N_iup - N_idown;
 *                    U_X[1] = -1/4 sum_i I_i m_out_i^2 (Eq. TB-UX).
 *  bop_mag_scf_step  bop_mag_energy, then q_i = N_iup + N_idown - n0_i and
 *                    dm_i = m_out_i - moment_i; converged (*converged = 1,
 *                    nothing updated) if max |q| < tol and max |dm| < tol_m;
 *                    else shift_i += mix q_i / max(n_i(E_F), n_floor) (total
 *                    DOS), minus the mean, and moment_i += mix_m dm_i.
 *                    max_d[2] = max |q|, max |dm|.
 * ========================================================================= */
typedef struct bop_magnetism {
    double stoner[BOP_MAX_SPECIES];   /* Stoner exchange integral I per species (eV) */
    double B_z;                       /* field term of the onsite levels (eV) */
} bop_magnetism;

int bop_spin_shifts(int n_atoms, const int *species, const bop_magnetism *mag /*[host]*/,
                    const double *shift, const double *moment, double *shift_spin,
                    hipStream_t stream);
int bop_mag_energy(const bop_system *sys /*[host]*/, const bop_magnetism *mag /*[host]*/,
                   const double *shift, const double *moment, double *m_out, double *U_X,
                   hipStream_t stream);
int bop_mag_scf_step(const bop_system *sys /*[host]*/, const bop_magnetism *mag /*[host]*/,
                     double mix, double mix_m, double n_floor, double tol, double tol_m,
                     double *shift, double *moment, double *m_out, double *q, double *U_X,
                     double *max_d, int *converged, hipStream_t stream);

/* =========================================================================
 * Learned warm start (not in the paper: its Sec. III speed-up (ii), starting
 * the self-consistency from earlier onsite levels, generalised to a learned
 * map from an atom's lowest moments to its converged onsite shift).  FP32.
 *
 * Network 6 -> 64 -> 64 -> 1 with tanh hidden layers; parameters are one
 * array of BOP_MLP_NPARAM floats: W1[64][6] b1[64] W2[64][64] b2[64] W3[64] b3.
 *
 *  bop_features        x[i][n-1] = (sum_a mu[i][a][n] / n_orb - mean[n-1]) /
 *                      std[n-1], n = 1..6 (mean/std [device 6] or both NULL =
 *                      raw traces).  Needs n_max >= 6.
 *  bop_mlp_forward     y[r] = network(x[r]) for n_rows rows.
 *  bop_mlp_train_step  one Adam step (lr, betas 0.9/0.999, eps 1e-8; `step` is
 *                      the 1-based step count, step <= 0 computes the gradient
 *                      only) on the mean squared error over `batch` rows of
 *                      (x, t), taken as x[idx[r]], t[idx[r]] when idx is given.
 *                      loss [device 1] and grad [device BOP_MLP_NPARAM] are
 *                      optional outputs (gradient before the update).
 * ========================================================================= */
#define BOP_MLP_NPARAM 4673
int bop_features(int n_atoms, int n_orb, int n_max, const double *mu, const float *mean,
                 const float *std, float *x, hipStream_t stream);
int bop_mlp_forward(int n_rows, const float *params, const float *x, float *y,
                    hipStream_t stream);
/*  bop_feature_stats   mean[6] and std[6] (n - 1 normalisation, floored at
 *                      1e-12) of the columns of x[n_rows][6]; FP64 sums in a
 *                      fixed order.
 *  bop_standardise     out[r][f] = (x[r][f] - mean[f]) / std[f] (may alias x).
 *  bop_mlp_shift       the warm-start shifts: y = network(x[r]) in FP64, minus
 *                      their mean (the gauge of the charge-neutrality cycle: a
 *                      shift common to all atoms moves E_F with it and changes
 *                      nothing else). */
int bop_feature_stats(int n_rows, const float *x, float *mean, float *std, hipStream_t stream);
int bop_standardise(int n_rows, const float *x, const float *mean, const float *std, float *out,
                    hipStream_t stream);
int bop_mlp_shift(int n_rows, const float *params, const float *x, double *shift,
                  hipStream_t stream);
size_t bop_mlp_train_workspace_size(int batch);
int bop_mlp_train_step(int batch, const int *idx, const float *x, const float *t,
                       float *params, float *adam_m, float *adam_v, int step, float lr,
                       float *loss, float *grad, void *ws, size_t ws_bytes,
                       hipStream_t stream);
/*  bop_mlp_backward    the training step's forward and backward passes
 *                      only: loss[1] and grad[4673] (same layout as params)
 *                      of the batch, params unchanged (bop_mlp_train_step
 *                      with step 0).  Workspace from bop_mlp_train_workspace_size.
 *  bop_mlp_adam        one Adam update (lr, beta1 0.9, beta2 0.999, eps 1e-8,
 *                      bias correction with `step` >= 1) of params, adam_m,
 *                      adam_v from a given grad[4673]: the update of
 *                      bop_mlp_train_step split out. */
int bop_mlp_backward(int batch, const int *idx, const float *x, const float *t,
                     const float *params, float *loss, float *grad, void *ws, size_t ws_bytes,
                     hipStream_t stream);
int bop_mlp_adam(const float *grad, float *params, float *adam_m, float *adam_v, int step,
                 float lr, hipStream_t stream);

/* =========================================================================
 * Forces of the d-band bond energy (App. C.1-C.2: Eqs. dUdLambda, weights,
 * theta-tilde, Theta_tilde_BOP, F_k), non-magnetic, Gershgorin terminator,
 * no path radius, n_max <= 20.
 *
 * bop_weights   w[r][n] = dU_bond/dmu_r^(n) (Eq. weights, both spins) of
 *               every orbital row r at the self-determined Fermi level: the
 *               partial derivative of the row's U at E_F plus the Fermi
 *               level's response, -(E_F - E_bar) dN_r/dmu with E_bar the
 *               DOS-weighted mean onsite level at E_F.  mu [n_rows][n_max+1]
 *               (bop_moments), H_on [n_rows], E_F [1] device (bop_energy's).
 *               w [n_rows][n_max+1], w[r][0] = 0.  n_exp as in bop_energy.
 * bop_bond_derivatives
 *               dH[p][x][16] = d H_p / d d_p,x for every directed pair p
 *               (d_p = nbr_d[p]), packed like the FP64 d-d blocks of
 *               bop_build_H (upper triangle row-major, entry 15 = 0).
 *               A species outside the model gives NaN.
 * bop_forces    F[k][3] = -dU_bond/dr_k (eV/A) from Theta~ = dU/dH (Eq.
 *               Theta_tilde_BOP) and the block derivatives (Eq. F_k):
 *               F_k = sum over k's pairs p of g_p - g_reverse(p), g_p =
 *               sum_ab Theta~_p,ab dH_p,ab/dd_p.  `plan` and `moments_ws` are
 *               the ones bop_moments used (plan dtype FP64 or FP32: the
 *               vectors' precision; H_bond in that dtype), after
 *               bop_moments_prepare; w from bop_weights.  nbr_shift locates
 *               each pair's reverse.  batch_tiles: tiles whose vectors are
 *               live at once (0: a default of at most 24 GiB, or a quarter of
 *               the free memory); pass the same value to
 *               bop_forces_workspace_size.  theta_on [N*5] (device, may be
 *               NULL): if given, also the onsite elements Theta~_(ia,ia) =
 *               dU/dE_ia through the moments (both spins), the first term
 *               of the self-consistency target of Eq. BOP_SCF; atoms of a
 *               failed tile get NaN.  Errors: BOP_E_UNSUPPORTED
 *               (not d band, BF16/FP16, path radius, n_max > 20),
 *               BOP_E_CAPACITY (workspace too small).  Tiles whose support
 *               did not fit the plan give NaN forces on their atoms and
 *               neighbours.  The pair gradients are summed with FP64
 *               atomics: results can differ in the last bits between runs.
 * bop_scf_target  Eq. BOP_SCF with one onsite shift per atom:
 *               delta[i] = sum_a theta_on[i*n_orb + a] - N_atom[i] =
 *               dU/d(shift_i) (eV per eV), from bop_forces' theta_on and
 *               the N_atom of the same energy call.  All arrays device,
 *               caller-owned.  Errors: BOP_E_ARG (NULL array, n_orb < 1).
 * ========================================================================= */
size_t bop_weights_workspace_size(int n_rows, int n_max);
int bop_weights(int n_rows, int n_max, int n_exp, const double *mu, const double *H_on,
                const double *E_F, double *w, void *ws, size_t ws_bytes, hipStream_t stream);
int bop_bond_derivatives(const bop_model *model, int n_atoms, const int *species,
                         const int *row_ptr, const int *nbr_j, const double *nbr_d, long n_pairs,
                         double *dH, hipStream_t stream);
size_t bop_forces_workspace_size(const bop_plan *plan, long n_pairs, int batch_tiles);
int bop_forces(const bop_plan *plan, const void *moments_ws, const int *row_ptr,
               const int *nbr_j, const int *nbr_shift, long n_pairs, const double *H_on,
               const void *H_bond, const double *dH, const double *w, int batch_tiles,
               double *F, double *theta_on, void *ws, size_t ws_bytes, hipStream_t stream);
int bop_scf_target(int n_atoms, int n_orb, const double *theta_on, const double *N_atom,
                   double *delta, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BOP_H */
