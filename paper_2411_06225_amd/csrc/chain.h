// chain.h -- launchers of the sequential sweeps and the training-pair kernel
// (chain.hip).
#pragma once

#include "common.h"
#include "randnet.h"
#include "rkgen.h"

namespace rpr {

// Work-group size of the wide form of the sweep segments over a tiled grid
// (forward-Euler G).
constexpr int SWEEP_WIDE = 1024;

enum { CHAIN_SWEEP = 0, CHAIN_RANDNET = 1, CHAIN_PARAREAL = 2, CHAIN_RANDNET_NN = 3 };

// Largest number of nearest neighbours of the refit-per-prediction mode.
constexpr int NN_MAX = 32;

template <typename T>
struct ChainArgs {
    Geom g;
    int mode;                  // CHAIN_*
    int N, M, act;
    int k_max;                 // iteration cap: the sweep that reaches it raises the stop flag
    int G_method;
    long long G_steps;
    double dtG;
    double inv_s;              // 1 / input scale
    double eps;                // tolerance of the stopping rule
    T *U;                      // (N+1) x d slot states, updated in place
    const T *Fv;               // (N+1) x d fine values F(U_{i-1}^{k-1}) (row i)
    T *Gc;                     // (N+1) x d coarse values G(U_{i-1}) (row i)
    T *gtmp;                   // d: coarse value of the current slot
    double *phi;               // M: hidden layer of the current slot
    double *hpart;             // grid x M: per-work-group partial sums of A x / s
    TiledWork<T> gw;           // work arrays of the tiled or generic coarse solver (d values each)
    Tableau tbG;               // the coarse solver's tableau (generic form)
    const double *A, *zeta;
    const T *W;                // M x d readout weights (state precision: FP32 copies in reduced plans)
    const T *At;               // d x M: A^T (state precision)
    // nearest-neighbour mode: the store of every pair so far (rows 0 ..
    // ctrl->nn_rows + *nrows; the last *nrows are this iteration's)
    int m_nn;                  // neighbours per prediction
    double lambda;             // ridge penalty
    const T *Xs, *Ys;          // n_cap x d: inputs and targets
    const double *Ps;          // n_cap x M: features of the inputs
    const int *oks;            // n_cap: 1 if the pair is finite
    const int *nrows;          // pairs added this iteration
    int n_cap;                 // rows of the store
    double *dpart;             // grid x n_cap: per-work-group partial squared distances
    double *dist;              // n_cap: squared distances of the current slot input
    double *part;              // (N+1) x grid: per-work-group change maxima
    Ctrl *ctrl;
    int *L_hist;               // (N+1)
    double *chg_hist;          // (N+1)
};

// Dynamic LDS of the chain kernel for coarse-solver shape sh and M neurons.
size_t chain_lds(const OnchipShape &sh, int M);

// Cooperative launch of one sweep on nwg work-groups (CHAIN_SWEEP on chip:
// work-group 0 runs it alone, so nwg = 1).  With max_wg non-null nothing is launched and *max_wg receives
// the number of work-groups that can be co-resident on the device.
template <typename T>
rpr_status launch_chain(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st,
                        int *max_wg = nullptr);

// Per right-hand side instance (chain.hip, one object per kind and precision).
template <int KIND, typename T>
rpr_status launch_chain_kind(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st,
                             int *max_wg);

// One sweep as a sequence of kernels, one per segment (prologue; phase 1 of
// every slot i = 2..N, the tiled coarse solver's passes one kernel each;
// phase 2 of every slot; stopping rule), on nwg work-groups, for capture in
// a graph: the kernel boundaries take the place of the grid barriers, and a
// segment of a final slot returns at once.  args_dev: device copy of a (read
// by the kernels when they run); a: the host copy (sizes, mode, coarse
// propagator).  Same arithmetic as launch_chain with nwg work-groups.
// The k = 0 sweep (a.mode == CHAIN_SWEEP) of a grid-wide coarse solver
// (tiled or generic shape) as one kernel per pass of every slot on nwg
// work-groups; the values of launch_chain's sweep.
template <typename T>
rpr_status launch_sweep_segments(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st);
template <int KIND, typename T>
rpr_status launch_sweep_segments_kind(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st);

template <typename T>
rpr_status launch_chain_graph(const ChainArgs<T> *args_dev, const ChainArgs<T> &a, const OnchipShape &sh, int nwg,
                              hipStream_t st);
template <int KIND, typename T>
rpr_status launch_chain_graph_kind(const ChainArgs<T> *args_dev, const ChainArgs<T> &a, const OnchipShape &sh,
                                   int nwg, hipStream_t st);

// Independent instances in one launch, one work-group each (nwg = 1 sweeps).
// args_dev: device array of n_inst argument blocks; every instance must be
// served by the generic kernel instance of shape sh (built for geometry gmax).
template <typename T>
rpr_status launch_chain_multi(const ChainArgs<T> *args_dev, int n_inst, const Geom &gmax, const OnchipShape &sh,
                              int M, hipStream_t st);
template <int KIND, typename T>
rpr_status launch_chain_multi_kind(const ChainArgs<T> *args_dev, int n_inst, const Geom &gmax, const OnchipShape &sh,
                                   int M, hipStream_t st);

}  // namespace rpr
