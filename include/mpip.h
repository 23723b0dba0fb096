/*
 * mpip.h -- C ABI of libmpip: one energy + forces + virial evaluation of an
 * equivariant message-passing interatomic potential on one AMD Instinct
 * MI355X (gfx950) GPU.
 *
 * Method (arxiv 2509.21694):
 *  - depth pruning, Methods "Message Passing Depth Pruning": a weight set
 *    holds T message-passing layers; an evaluation runs only the first K
 *    (1 <= K <= T) and reads the energy out from layer K;
 *  - partitions, Methods "Graph Partitioning" and "Global Output
 *    Integration": a system may be one partition of a larger structure --
 *    its first n_owned atoms are the root atoms, the rest are halo copies.
 *    The energy is summed over root atoms only; forces are -dE/dx for every
 *    local atom (halo rows hold partial forces, to be added to the atoms
 *    they copy); the virial decomposes the same way.
 *
 * The potential (layer equations, basis, harmonics, coupling tensors) is
 * the NequIP/MACE-style reading documented with the library: a Bessel
 * radial basis with polynomial envelope, component-normalised real
 * spherical harmonics up to l_max <= 2, real Gaunt coupling tensors with
 * natural parity, a bias-free SiLU radial MLP (n_basis -> hidden -> hidden
 * -> one channel vector per coupling path), gated non-linearity with
 * residual updates, and a linear per-species readout.
 *
 * Conventions for every entry point:
 *  - Pointers documented "device" are GPU global-memory addresses on the
 *    model's device; "host" pointers are CPU memory.  The caller owns every
 *    buffer it passes; the library never frees or retains them.
 *  - Asynchronous calls enqueue work on the given HIP stream (NULL = the
 *    legacy default stream) and return immediately; outputs are valid after
 *    the stream has been synchronised.
 *  - Every call returns an mpip_status; no C++ exception crosses the ABI.
 *    On failure mpip_last_error() describes the cause (thread-local string,
 *    valid until the next call on the same thread).
 */
#ifndef MPIP_H
#define MPIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPIP_OK = 0,
  MPIP_EINVAL = -1,        /* bad argument, species out of range, non-finite or coincident atoms */
  MPIP_ECELL = -2,         /* singular cell, or too many cell-list bins                          */
  MPIP_ECAPACITY = -3,     /* edge capacity or workspace too small (required size reported)      */
  MPIP_EDEVICE = -4,       /* HIP runtime error                                                  */
  MPIP_ENOMEM = -5,        /* device allocation failed (model creation only)                     */
  MPIP_EUNSUPPORTED = -6   /* valid input outside what this library implements                   */
} mpip_status;

typedef enum {
  MPIP_FP32 = 0,           /* all arithmetic in FP32 (FP32 MFMA for the dense contractions)       */
  MPIP_BF16_MIXED = 1      /* radial MLP and channel mixing as BF16 MFMA with FP32 accumulation.
                              In the specialised first and last layers (64 or 128 channels) the
                              radial MLP's second hidden layer a(r) is read from a per-layer
                              table instead (built at model creation in FP64 from the FP32
                              weights: 4096 intervals over [0, r_c], BF16 value and increment
                              per interval, linear interpolation, the interval's slope as
                              da/dr); the tensor-product contractions run on BF16 MFMA with
                              BF16 operands and FP32 accumulation (first layer: Q = a2 (x) YC
                              and its adjoint; last layer: X = ht . YC, dE/dYC and the
                              sender-side pull), and the last layer's ht and per-edge messages
                              are stored in BF16; generic (middle) layers evaluate the MLP on
                              BF16 MFMA and form the tensor product on the VALU in FP32.
                              Geometry (basis, harmonics) in FP32; r_e is the FP64 displacement
                              rounded to FP32 (also in the virial); energy, force and virial
                              sums in FP64                                                        */
} mpip_precision;

typedef struct {
  int32_t n_species;       /* >= 1                                                  */
  int32_t n_layers;        /* T, number of layers in the weight set, >= 1           */
  int32_t l_max;           /* 1 or 2                                                */
  int32_t channels;        /* C: 32, 64 or 128                                      */
  int32_t n_basis;         /* 8                                                     */
  int32_t envelope_p;      /* polynomial envelope order, >= 2                        */
  int32_t radial_hidden;   /* 64                                                    */
  double r_cut;            /* cutoff radius, Angstrom, > 0                           */
  double inv_avg_neighbors;/* message normalisation 1/n_avg                          */
} mpip_hparams;

typedef struct {
  int64_t n_atoms;         /* N >= 1                                                 */
  int64_t n_owned;         /* 0 <= n_owned <= N: root atoms are the first n_owned    */
  const double* positions; /* device [N,3] row-major, Angstrom; may lie outside the cell */
  const int32_t* species;  /* device [N], values 0..n_species-1                      */
  double cell[9];          /* host, row-major; rows are lattice vectors              */
  uint8_t pbc[3];          /* host, 1 = periodic along that lattice vector           */
} mpip_system;

typedef struct {
  double* energy;          /* device [1]: sum of root-atom energies, eV              */
  double* forces;          /* device [N,3]: -dE/dx_i, eV/Angstrom, input atom order  */
  double* virial;          /* device [9]: W = -sum_e r_e (x) dE/dr_e, eV, row-major  */
  double* atom_energy;     /* device [N] per-atom energies E_i (input order), or NULL;
                              zero on the non-root atoms of a trimmed share
                              (see mpip_evaluate)                                      */
} mpip_outputs;

typedef struct mpip_model mpip_model;

/* Number of float32 values in a weight set for these hyper-parameters.
 * Blob order: W_emb [S,C]; per layer t=1..T: W_up[l] [C,C] for each input
 * degree l ({0} at t=1, else 0..l_max), W1 [n_basis,H], W2 [H,H],
 * W3 [H, P_t*C] (path-major columns; paths (l1,l2,l3) ordered by l1, l2, l3
 * with l1+l2+l3 even and |l1-l2| <= l3 <= l1+l2), W_down[0] [C, C*(1+l_max)]
 * (C features then one gate block per l >= 1), W_down[l] [C,C] for
 * l = 1..l_max; then w_read [C], e0 [S].  Matrices are row-major and map
 * rows (inputs) to columns (outputs).  Returns 0 for invalid hparams. */
size_t mpip_weights_count(const mpip_hparams* hp);

/* Validate hparams, build the coupling tables and upload the weights
 * (host float32 [n]) to `device`.  The model owns its device memory
 * (weights in FP32 and BF16 operand layouts, coupling tables, the BF16
 * form's radial tables: 1 MiB per layer) until
 * mpip_model_destroy.  Synchronous.  Errors: EINVAL (bad hparams or n),
 * ENOMEM, EDEVICE. */
mpip_status mpip_model_create(const mpip_hparams* hp, const float* weights_host, size_t n,
                              int32_t device, mpip_model** out);
mpip_status mpip_model_destroy(mpip_model* model);

/* Workspace bytes needed by mpip_evaluate for this system size, precision,
 * depth K and edge capacity `max_edges` (directed edges).  Host only. */
mpip_status mpip_workspace_size(const mpip_model* model, const mpip_system* sys,
                                mpip_precision prec, int32_t K, int64_t max_edges,
                                size_t* bytes);

/* One evaluation: cell list, neighbour list, K layers forward, readout, the
 * hand-written adjoint of all K layers (edge intermediates recomputed), and
 * forces / virial.  Asynchronous on `stream`; never allocates; the caller's
 * `workspace` (device, >= mpip_workspace_size bytes for the same max_edges)
 * must not be used concurrently.  Host-detectable errors are returned at
 * once.  Data-dependent errors (edge capacity exceeded, species out of range,
 * non-finite positions, coincident atoms) are recorded in the workspace and
 * reported by mpip_workspace_status after the stream is synchronised; the
 * energy and virial are then NaN and the other outputs undefined.  Orthorhombic cells only (else EUNSUPPORTED).
 *
 * Partition shares (0 < n_owned < n_atoms, n_atoms >= 64): the energy of the
 * root atoms after K layers depends only on their K-hop neighbourhood
 * (Methods "Graph Partitioning"), so layer t is evaluated only on atoms
 * within K - t hops of a root (receptive-field trimming).  The hop classes
 * are found on the device by a breadth-first expansion over the built list
 * and read back once: such a call synchronises `stream` once, after the
 * neighbour list is built.  Energy, forces (including the partial forces on
 * halo atoms) and virial are those of the root energy, as without trimming;
 * atom_energy holds E_i on the roots and zero on every other atom. */
mpip_status mpip_evaluate(mpip_model* model, const mpip_system* sys, mpip_precision prec,
                          int32_t K, void* stream, void* workspace, size_t workspace_bytes,
                          int64_t max_edges, const mpip_outputs* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of mpip_evaluate, with the workspace taken from a fixed array of
 * MPIP_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends.  The caller passes inputs and outputs only;
 * the call allocates no device memory and clears what must start at zero
 * itself.  Systems whose workspace (mpip_workspace_size for the same
 * arguments) exceeds MPIP_NOALLOC_SCRATCH_BYTES are rejected with ECAPACITY
 * before anything is enqueued.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (two streams, two threads,
 * two models) race and give undefined outputs; serialise them.  A
 * data-dependent error (as for mpip_evaluate, e.g. more than max_edges edges)
 * leaves NaN in the energy and virial; the status word sits in the array, so
 * mpip_workspace_status cannot read it.  Otherwise as mpip_evaluate
 * (asynchronous on `stream`; partition shares synchronise once). */
#define MPIP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
mpip_status mpip_evaluate_noalloc(mpip_model* model, const mpip_system* sys, mpip_precision prec,
                                  int32_t K, void* stream, int64_t max_edges, const mpip_outputs* out);

/* Batched evaluation of B independent structures (atoms concatenated):
 * structure b owns atoms atom_ptr[b] .. atom_ptr[b+1]-1 (host int64 [B+1],
 * atom_ptr[0] = 0), with cell cells[9b..9b+8] and periodicity pbc[3b..3b+2]
 * (host; orthorhombic; periodic directions thinner than the cutoff are
 * searched over all images).  positions device [N,3], species device [N].
 * Outputs (device): energy [B], forces [N,3] (input order), virial [B,9].
 * Every atom is a root atom.  One pass of each kernel covers all structures
 * (the neighbour list is block diagonal).  Asynchronous; never allocates;
 * data-dependent errors via mpip_workspace_status as for mpip_evaluate. */
mpip_status mpip_batch_workspace_size(const mpip_model* model, int64_t n_atoms_total, int32_t B,
                                      mpip_precision prec, int32_t K, int64_t max_edges, size_t* bytes);
mpip_status mpip_evaluate_batch(mpip_model* model, int32_t B, const int64_t* atom_ptr,
                                const double* positions, const int32_t* species, const double* cells,
                                const uint8_t* pbc, mpip_precision prec, int32_t K, void* stream,
                                void* workspace, size_t workspace_bytes, int64_t max_edges,
                                double* energy, double* forces, double* virial);

/* Synchronise `stream` and read the status word of `workspace` written by
 * the last mpip_evaluate / mpip_neighbor_list on it.  *n_edges receives the
 * number of directed edges found (also when it exceeded the capacity). */
mpip_status mpip_workspace_status(const void* workspace, void* stream, int64_t* n_edges);

/* Neighbour list only (Methods "Graph Partitioning" builds its subgraphs on
 * this adjacency): all (i, j, S) with |x_j - x_i + S.cell| < r_cut, decided
 * in FP64 with a fixed operation order, in input atom indices.  Synchronous.
 * edge_i/edge_j (device int32 [capacity]) and edge_shift (device int32
 * [capacity,3]) receive the edges in an unspecified order; *n_edges the count.
 * If the count exceeds `capacity` nothing is written past it and ECAPACITY
 * is returned with *n_edges set to the required capacity.  The workspace must
 * hold mpip_workspace_size(.., max_edges = capacity) bytes of any model or
 * mpip_neighbor_workspace_size bytes. */
size_t mpip_neighbor_workspace_size(int64_t n_atoms, int64_t capacity);
mpip_status mpip_neighbor_list(const mpip_system* sys, double r_cut, void* stream,
                               void* workspace, size_t workspace_bytes, int64_t capacity,
                               int32_t* edge_i, int32_t* edge_j, int32_t* edge_shift,
                               int64_t* n_edges);

/* One partition of a structure (Methods "Graph Partitioning", stage 1
 * spatial grid and the halo that keeps every root atom's K-hop
 * neighbourhood).  Atoms are binned along lattice axis `axis` of the
 * orthorhombic `cell` (host [9]) by b = min(floor((x/L) P), P-1) with x the
 * coordinate wrapped into [0, L); slab `part` holds the root atoms.  Every
 * periodic image of every atom whose coordinate lies within `halo` of the
 * slab (and outside it) is added as a halo atom at its unwrapped position.
 * Output (device, capacity rows): root atoms first by increasing index (at
 * their wrapped coordinate), then halo images by increasing image shift and
 * index; out_index = the input atom each row copies.  The share is
 * evaluated with pbc[axis] = 0 and n_owned = *n_owned.  Synchronous.  If the
 * share has more rows than `capacity`, ECAPACITY with *n_local set. */
size_t mpip_slab_workspace_size(int64_t n_atoms, double axis_length, double halo);
mpip_status mpip_slab_share(const double* positions, const int32_t* species, int64_t n_atoms,
                            const double* cell, int32_t axis, int32_t n_parts, int32_t part,
                            double halo, void* stream, void* workspace, size_t workspace_bytes,
                            int64_t capacity, double* out_positions, int32_t* out_species,
                            int32_t* out_index, int64_t* n_local, int64_t* n_owned);

/* One partition with a graph halo (Methods "Graph Partitioning", stage 2:
 * each subgraph grown by a breadth-first expansion of depth K so that every
 * root atom keeps its K-hop neighbourhood).  The roots are the atoms of slab
 * `part` of n_parts along `axis` (the stage-1 rule of mpip_slab_share); the
 * halo holds every atom within K hops of a root in the neighbour graph of
 * the whole structure at cutoff r_cut, as the image that lies within K r_cut
 * of the slab.  Equivalently: the share mpip_slab_share builds with halo
 * K r_cut, without the images of atoms more than K hops from every root
 * (same row order: roots by index, then halo images by image shift and
 * index).  sys: the whole structure (orthorhombic, periodic along `axis`,
 * n_owned ignored); the slab plus 2 K r_cut must not exceed the cell length
 * along `axis` (one image per atom; else EUNSUPPORTED).  max_edges: capacity
 * of the whole structure's list (ECAPACITY with *n_edges = the count when
 * exceeded); capacity: rows of the outputs (ECAPACITY with *n_local set when
 * exceeded).  Workspace: mpip_bfs_share_workspace_size bytes (device).
 * Synchronous.  The halo growth factor of the share is
 * (*n_local - *n_owned) / *n_owned. */
size_t mpip_bfs_share_workspace_size(int64_t n_atoms, double axis_length, int32_t K, double r_cut,
                                     int64_t max_edges);
mpip_status mpip_bfs_share(const mpip_system* sys, double r_cut, int32_t axis, int32_t n_parts, int32_t part,
                           int32_t K, void* stream, void* workspace, size_t workspace_bytes, int64_t max_edges,
                           int64_t capacity, double* out_positions, int32_t* out_species, int32_t* out_index,
                           int64_t* n_local, int64_t* n_owned, int64_t* n_edges);

/* Sequential evaluation of a whole structure in n_parts partitions on one GPU
 * (the one-GPU mode of the paper's pipeline: Methods "Graph Partitioning"
 * and "Global Output Integration").  For part = 0 .. n_parts-1: the slab and
 * its halo along `axis` are built on the device, as by mpip_slab_share with
 * depth `halo` (graph_edges < 0) or as by mpip_bfs_share with K hops
 * (graph_edges >= 0: the capacity of the whole structure's neighbour list,
 * built once for all parts; `halo` is then unused), evaluated as a share (its root atoms owned, pbc[axis] = 0,
 * receptive-field trimming as in mpip_evaluate), and integrated into `out`:
 * energy and virial summed over parts, every share row's partial force added
 * to the atom it copies, root-atom energies stored (atom_energy optional).
 * With halo >= K r_cut and a cutoff shorter than every slab, the outputs are
 * those of one evaluation of the whole structure (up to summation order).
 * sys: the whole structure, n_owned == n_atoms, orthorhombic, periodic along
 * `axis`.  max_local bounds the rows of one share, max_edges its directed
 * edges; the workspace (device) holds mpip_partitioned_workspace_size bytes
 * for the same arguments, and is reused for every part, so the structure
 * itself may be far larger than one evaluation's workspace allows.
 * part_sizes: NULL or host int64 [3 n_parts] receiving per part (rows,
 * roots, directed edges): halo growth H = rows / roots - 1.
 * Synchronous (each share's size and status are read back).  Errors: those of
 * mpip_slab_share (ECAPACITY: a share has more than max_local rows, its size
 * in part_sizes), of mpip_bfs_share (ECAPACITY: the whole structure's list
 * has more than graph_edges edges, the count in part_sizes[2]) and of
 * mpip_evaluate / mpip_workspace_status (ECAPACITY: a share has more than
 * max_edges edges, the count in part_sizes); the outputs are then
 * incomplete. */
mpip_status mpip_partitioned_workspace_size(const mpip_model* model, const mpip_system* sys,
                                            mpip_precision prec, int32_t K, int32_t n_parts, int32_t axis,
                                            double halo, int64_t graph_edges, int64_t max_local,
                                            int64_t max_edges, size_t* bytes);
mpip_status mpip_evaluate_partitioned(mpip_model* model, const mpip_system* sys, mpip_precision prec,
                                      int32_t K, int32_t n_parts, int32_t axis, double halo, int64_t graph_edges,
                                      void* stream, void* workspace, size_t workspace_bytes, int64_t max_local,
                                      int64_t max_edges, const mpip_outputs* out, int64_t* part_sizes);

/* Output integration (Methods "Global Output Integration"): dst[index[k]]
 * += src[k] for rows of 3 doubles (device pointers), e.g. a partition's
 * force rows (root and halo) into the full structure's forces.
 * Asynchronous on `stream`; rows with an index outside [0, n_dst) are
 * skipped; repeated indices are summed atomically. */
mpip_status mpip_accumulate_rows(const double* src, const int32_t* index, int64_t n_rows, int64_t n_dst,
                                 double* dst, void* stream);

/* The library's coupling tensor for (l1,l2,l3), derived from Wigner 3j
 * symbols and the complex-to-real change of basis, Frobenius-normalised.
 * Host only, no GPU needed.  out: host [(2l1+1)*(2l2+1)*(2l3+1)] row-major
 * (m1, m2, m3).  EINVAL for l > 2 or a triple without natural parity. */
mpip_status mpip_coupling_tensor(int32_t l1, int32_t l2, int32_t l3, double* out);

#define MPIP_RADIAL_TABLE_INTERVALS 4096

/* The BF16 form's radial table of layer `layer` (1-based), as
 * mpip_model_create builds it: the radial MLP's second hidden layer
 * a(d) = silu(W2^T silu(W1^T e(d))) (e: Bessel basis times envelope) at the
 * knots d_k = k r_cut / MPIP_RADIAL_TABLE_INTERVALS, in FP64 from the FP32
 * weights.  Host only, no GPU needed.  out: host
 * [MPIP_RADIAL_TABLE_INTERVALS][radial_hidden] words; word (k, h) holds
 * BF16 a_h(d_k) in bits 0..15 and BF16 (a_h(d_k+1) - a_h(d_k)) in bits
 * 16..31.  The specialised layers interpolate it linearly in d and take
 * the interval's slope as da/dd.  EINVAL for bad hparams, weight count or
 * layer. */
mpip_status mpip_radial_table(const mpip_hparams* hp, const float* weights_host, size_t n, int32_t layer,
                              uint32_t* out);

/* Molecular dynamics on the device around mpip_evaluate (the MD runs of
 * the results section use Langevin dynamics).  Each of n_steps steps is the
 * BAOAB splitting (Leimkuhler and Matthews): v += a dt/2; x += v dt/2;
 * v = c1 v + sqrt(1 - c1^2) sqrt(kB T / m) xi with c1 = exp(-friction dt);
 * x += v dt/2; forces at the new x; v += a dt/2, with a = F/m.  friction
 * = 0 gives velocity Verlet (NVE).  Neighbour list: with skin = 0 it is
 * rebuilt at every step; with skin > 0 a list of radius r_cut + skin is
 * built and kept while no atom has moved more than skin/2 since (checked on
 * the device each step, one 8-byte read by the host), and every step
 * selects from it, in FP64 with the same predicate as a fresh build, the
 * pairs closer than r_cut -- the same edge set as a rebuild.  xi: three standard normal numbers per atom and step from
 * Philox4x32-10 (Salmon et al., SC'11) with key = seed and counter
 * (atom index, step index), through the Box-Muller transform of
 * u = (word + 1) / 2^32 (radius) and (word + 0.5) / 2^32 (angle).
 * Units: Angstrom, fs, eV, amu, K. */
typedef struct {
  double dt;               /* time step, fs, > 0                                      */
  int64_t n_steps;         /* >= 0                                                    */
  double friction;         /* Langevin friction, 1/fs, >= 0 (0: NVE)                  */
  double temperature;      /* Langevin bath temperature, K, >= 0                      */
  uint64_t seed;           /* key of the noise generator                              */
  double skin;             /* Angstrom, >= 0: neighbour-list reuse (see above)         */
} mpip_md_params;

/* Workspace bytes needed by mpip_md_run (the evaluation's plus the
 * integrator's scratch).  Host only. */
mpip_status mpip_md_workspace_size(const mpip_model* model, const mpip_system* sys,
                                   const mpip_md_params* params, mpip_precision prec, int32_t K,
                                   int64_t max_edges, size_t* bytes);

/* n_steps MD steps of the system `sys` (its positions field is ignored;
 * species, cell, pbc and n_owned are used as in mpip_evaluate) on `stream`.
 * positions, velocities (Angstrom / fs) and forces: device FP64 [N,3] in
 * input order, updated in place; on entry `forces` must hold the forces at
 * `positions` (e.g. from mpip_evaluate), on return they are those at the
 * final positions.  masses: device FP64 [n_species], amu.  epot, ekin:
 * device FP64 [n_steps] or NULL, the root-atom potential energy and the
 * kinetic energy (eV) after each step.  Asynchronous; never allocates; the
 * workspace (>= mpip_md_workspace_size bytes for the same params) must not
 * be used concurrently; with skin > 0 the host waits for each step's
 * displacement check.  max_edges bounds the edges closer than r_cut; the
 * list of radius r_cut + skin gets max_edges ((r_cut + skin) / r_cut)^3 * 1.5.
 * Data-dependent errors of any step are reported by mpip_workspace_status
 * after the run (the trajectory is then undefined from that step on). */
mpip_status mpip_md_run(mpip_model* model, const mpip_system* sys, double* positions, double* velocities,
                        double* forces, const double* masses, const mpip_md_params* params,
                        mpip_precision prec, int32_t K, void* stream, void* workspace, size_t workspace_bytes,
                        int64_t max_edges, double* epot, double* ekin);

/* Per-phase GPU timing of mpip_evaluate (tracing aid).  When enabled, each
 * evaluation records HIP events around its kernel phases on the evaluation
 * stream (no synchronisation); mpip_timing_read synchronises those events,
 * adds their durations to per-phase totals and returns the totals since the
 * last enable.  Phase names: "neighbors", "trim", "node_gemm", "gates", "outputs",
 * "node_fused", "node_last", "edge_fwd_t<k>", "edge_sum_t<k>",
 * "edge_bwd_t<k>" (k = layer).  Host-side only; the model
 * must not be evaluated concurrently on two streams while enabled. */
#define MPIP_MAX_PHASES 48
typedef struct {
  int32_t n;                          /* number of phases filled            */
  char name[MPIP_MAX_PHASES][24];     /* NUL-terminated phase names         */
  double ms[MPIP_MAX_PHASES];         /* summed duration, milliseconds      */
  int64_t calls[MPIP_MAX_PHASES];     /* number of recorded intervals       */
} mpip_timing;
mpip_status mpip_timing_enable(mpip_model* model, int32_t on);
mpip_status mpip_timing_read(mpip_model* model, mpip_timing* out);

const char* mpip_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPIP_H */
