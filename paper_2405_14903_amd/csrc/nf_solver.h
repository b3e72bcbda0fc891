// Host-side declarations shared by the library's translation units.
#pragma once

#include "nf_internal.h"

namespace nf {

struct Level {
  Dims d;
  void* a[3];   // face fractions (storage type of the level)
  void* invd;   // inverse diagonal
  void* r;      // restricted residual (levels >= 1)
  void* z;      // correction (levels >= 1)
  void* ta;     // smoother temporaries
  void* tb;
};

struct Solver {
  int nlev = 0;
  int precision = SIM_FP32;
  int check_every = 2;
  Level lev[kMaxLevels];
  const float* ax = nullptr;   // fine FP32 fractions (CG operator)
  const float* ay = nullptr;
  const float* az = nullptr;
  float* r = nullptr;
  float* z = nullptr;
  float* q = nullptr;
  float* p0 = nullptr;
  float* p1 = nullptr;
  CGScalars* sc = nullptr;
  CGScalars* host_sc = nullptr;  // pinned
  double* partials = nullptr;
  float* scratch_a = nullptr;    // FP32 coarse fractions while building a mixed hierarchy
  float* scratch_inv = nullptr;
  size_t scratch_off[kMaxLevels] = {};
};

// nf_geom.hip
void launch_phi_nodes(const Domain& D, const GeomParams& G, double* phi, hipStream_t s);
void launch_alpha(const Domain& D, const double* phi, float* alpha, hipStream_t s);
void launch_invdiag(const Dims& d, const float* ax, const float* ay, const float* az, float* invd, hipStream_t s);
void launch_coarsen_alpha(const Dims& fd, const Dims& cd, const float* fax, const float* fay, const float* faz,
                          float* cax, float* cay, float* caz, hipStream_t s);
// nf_advect.hip
void launch_fill(float* p, size_t n, float v, hipStream_t s);
void launch_advect(const Dims& d, double dx, double dt, const double* grav, const float* u, float* out,
                   hipStream_t s);
void launch_advect_adjoint(const Dims& d, double dx, double dt, const float* u, const float* gout, float* gin,
                           hipStream_t s);
// nf_project.hip
void launch_rhs(const Domain& D, const GeomParams& G, double inv_k, const float* alpha, const float* uhat,
                float* b, hipStream_t s);
void launch_update(const Domain& D, const GeomParams& G, double kk, const float* alpha, const float* uhat,
                   const float* p, float* out, hipStream_t s);
void launch_adj_div(const Dims& d, const float* alpha, const float* g, float* rhs, hipStream_t s);
size_t adj_faces_partials(const Dims& d);
void launch_adj_faces(const Domain& D, const GeomParams& G, bool grad, const float* alpha, const double* phi,
                      const float* g, const float* y, const float* un1, float* gu, double* partials,
                      unsigned* ticket, double* g_theta, double* g_ctrl, hipStream_t s);
// nf_solver.hip
void solver_setup_levels(Solver& S, const float* fine_alpha, hipStream_t st);
int solver_solve(Solver& S, const float* b, float* x, double tol, int maxit, sim_stats* stats, hipStream_t st);

}  // namespace nf
