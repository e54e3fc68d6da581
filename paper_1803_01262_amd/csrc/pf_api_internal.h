// Host-side internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "pf_internal.h"
#include "phasefield.h"

namespace pf {

constexpr int kGraphSteps = 8;  // steps per captured graph (steady velocity)
// A time-varying velocity gives every step its own launch arguments (the time factor at the
// stage times), so such a run is captured whole: one graph of the nsteps-step loop from t0,
// replayed when the same loop is asked for again. Shorter loops launch eagerly; longer ones too
// (a graph of more than kLoopGraphMax steps would hold tens of thousands of nodes).
constexpr int kLoopGraphMin = 16;
constexpr int kLoopGraphMax = 4096;

struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* phi = nullptr;
    const void* U = nullptr;
    const void* V = nullptr;
    const void* W = nullptr;
    hipStream_t stream = nullptr;
    int variant = -1;
    // whole-loop graphs (time-varying velocity): the loop they hold
    double t0 = 0.0;
    int nsteps = 0;
};

// A handle's non-uniform mesh (phasefield_set_spacing): per axis a device table of kNuCols
// storage-dtype values per cell index, the cell widths as doubles for the volume-weighted mass
// (1 on an axis of one cell), and the eps rule.
struct NuMesh {
    void* tab[3] = {nullptr, nullptr, nullptr};
    double* width[3] = {nullptr, nullptr, nullptr};
    int eps_mode = 0;
    bool on() const { return tab[0] != nullptr; }
};

pf_status fail(pf_status st, const char* fmt, ...);
pf_status hip_fail(hipError_t e, const char* what);
pf_status validate_params(const pf_params* p);
int wall_mask(const pf_params& p);  // bit a set: walls on axis a
pf_status check_field_ptr(const void* ptr, const char* name);
int scheme_stage_count(int scheme);  // stage inputs an RK step keeps for its adjoint
int tuned_variant(int dtype, const int32_t n[3]);
int default_variant(const pf_params& p);  // variant -1: walled grids by rule, else tuned_variant
void release_graph(StepGraph& g);
double time_factor(const pf_params& p, double t);

// nu: a non-uniform mesh (null or off: the uniform mesh of p)
template <typename T>
StageArgs<T> make_stage(const pf_params& p, double svel, const T* y, const T* base1,
                        const T* base2, T* out1, T* out2, double c1, double c2, const T* U,
                        const T* V, const T* W, const NuMesh* nu = nullptr);

template <typename T>
hipError_t enqueue_step(const pf_params& p, int variant, T* phi, const T* U, const T* V,
                        const T* W, T* ya, T* yb, T* acc, double t, hipStream_t st,
                        const NuMesh* nu = nullptr);

template <typename T>
hipError_t enqueue_steps(const pf_params& p, int variant, T* phi, const T* U, const T* V,
                         const T* W, T* ya, T* yb, T* acc, double t0, int nsteps,
                         hipStream_t st, const NuMesh* nu = nullptr);

template <typename T>
FusedArgs<T> make_fused(const pf_params& p, bool sweep_b, double t, const T* phi_cur, T* phi_next,
                        const T* U, const T* V, const T* W, T* yb);

// One stage launch with the per-stage kernel of a variant (fused variants use the per-stage
// default for the grid).
template <typename T>
hipError_t run_stage(int variant, const StageArgs<T>& a, hipStream_t st);

// One sweep of a fused variant.
template <typename T>
hipError_t run_fused_sweep(int variant, const FusedArgs<T>& a, bool sweep_b, hipStream_t st);

}  // namespace pf

struct pf_solver {
    pf_params p{};
    size_t N = 0;       // cells
    size_t esz = 0;     // bytes per element
    int variant = 0;
    int adjoint_form = -1;  // reverse RK4 stages: -1 chosen per grid, 0 one per launch, 1 two
    void* ya = nullptr;  // RK stage buffers
    void* yb = nullptr;
    void* acc = nullptr;
    void* adj[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // adjoint scratch
    double* red_part = nullptr;
    double* red_out = nullptr;
    double* red_host = nullptr;  // pinned
    void* vel_scratch = nullptr;
    pf::StepGraph graph;
    pf::NuMesh nu;
};
