// C ABI of the library: handle management, argument validation and the
// orchestration of one step (NeuralFluid, Sec. Numerical Simulation:
// advection -> body force -> projection) and of its adjoint (Sec.
// Back-propagation through Time: projection first, then advection), plus the
// host-side rigid pose dynamics used to drive the ellipsoid.
#include "nf_solver.h"
#include "nf_tile.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

using namespace nf;

struct sim_ctx {
  sim_desc desc;
  Domain dom;
  int device = 0;
  Solver S;
  // fine-grid buffers
  float* alpha = nullptr;   // face fractions (velocity layout)
  double* phi = nullptr;    // SDF at nodes
  float* uhat = nullptr;    // advected field
  float* gu = nullptr;      // dJ/dU^ (adjoint)
  float* b = nullptr;       // right-hand side
  float* P = nullptr;       // pressure (when the caller passes none)
  float* y = nullptr;       // adjoint pressure
  float* stage = nullptr;   // per-brick LDS windows of the advection adjoint
  double* trace = nullptr;  // back-traced positions (6 FP64 per face) for the advection adjoint
  double* knots = nullptr;      // B-spline wall: control amplitudes of the current call
  double* wall_cols = nullptr;  // B-spline wall: per-column totals of its adjoint
  double* solids = nullptr;     // parametric solids: the packed solids of the current call
  double* solids_part = nullptr;  // parametric solids: partial sums of their gradient
  unsigned char* solid_term = nullptr;  // parametric solids: CSG term of every node
  std::vector<double> solids_host;  // host staging of the packed solids
  std::vector<void*> allocs;
  GeomParams last_geom;
  bool have_geom = false;
  bool levels_current = false;   // the solver's hierarchy was built from the current fractions
  // warm start (sim_set_warm_start): P and y hold the last step's pressure and
  // the last adjoint pressure, the initial guesses of the next solves of their kind
  int warm = 0;          // SIM_WARM_* bits
  bool warm_p = false;   // h->P holds the previous step's pressure
  bool warm_y = false;   // h->y holds the previous adjoint pressure
  unsigned* maxbits = nullptr;   // bits of the largest |u_f| (sim_max_speed)
  Profiler prof;
};

namespace {

struct Plan {
  int nlev = 0;
  Dims dims[kMaxLevels];
  size_t bytes = 0;
};

bool plan_levels(const sim_desc* d, Plan& p) {
  Dims cur{d->n[0], d->n[1], d->n[2]};
  p.nlev = 0;
  p.dims[p.nlev++] = cur;
  while (p.nlev < kMaxLevels && cur.nx % 2 == 0 && cur.ny % 2 == 0 && cur.nz % 2 == 0 && cur.nx >= 4 &&
         cur.ny >= 4 && cur.nz >= 4) {
    cur = Dims{cur.nx / 2, cur.ny / 2, cur.nz / 2};
    p.dims[p.nlev++] = cur;
  }
  return p.dims[p.nlev - 1].cells() <= (size_t)kCoarseMaxCells;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int validate_desc(const sim_desc* d) {
  if (!d) return SIM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (d->n[a] < 2 || d->n[a] > 4096) return SIM_EINVAL;
  if ((long)d->n[0] * d->n[1] * d->n[2] > (1L << 30)) return SIM_EINVAL;
  if (!(d->dx > 0) || !(d->dt > 0) || !(d->rho > 0) || !(d->tol > 0) || d->max_iter <= 0) return SIM_EINVAL;
  if (d->precision < SIM_FP32 || d->precision > SIM_MIXED_BF16) return SIM_EINVAL;
  for (int s = 0; s < 6; ++s) {
    if (d->bc[s] < SIM_BC_WALL || d->bc[s] > SIM_BC_PERIODIC) return SIM_EINVAL;
    if (d->bc[s] == SIM_BC_PERIODIC) return SIM_EUNSUPPORTED;
  }
  if (!(d->nu >= 0.0) || !std::isfinite(d->nu)) return SIM_EINVAL;
  if (!std::isfinite(d->gravity[0]) || !std::isfinite(d->gravity[1]) || !std::isfinite(d->gravity[2]))
    return SIM_EINVAL;
  switch (d->geom) {
    case SIM_GEOM_NONE:
      if (d->n_params != 0 || d->n_ctrl != 0) return SIM_EINVAL;
      break;
    case SIM_GEOM_SPHERES:
      if (d->n_params < 4 || d->n_params % 4 || d->n_params > 4 * SIM_MAX_SPHERES || d->n_ctrl != 0)
        return SIM_EINVAL;
      break;
    case SIM_GEOM_ELLIPSOID:
      if (d->n_params != 15 || d->n_ctrl != 6) return SIM_EINVAL;
      break;
    case SIM_GEOM_WALL:
      if (d->n_params != SIM_WALL_KNOTS_Y * SIM_WALL_KNOTS_Z || d->n_ctrl != 3) return SIM_EINVAL;
      break;
    case SIM_GEOM_BEZIER: {
      const int per = 1 + SIM_BEZIER_SHAPE_PARAMS;
      if (d->n_ctrl != 0 || d->n_params < 1 + per || (d->n_params - 1) % per ||
          (d->n_params - 1) / per > SIM_MAX_SOLIDS)
        return SIM_EINVAL;
      break;
    }
    default:
      return SIM_EINVAL;
  }
  Plan p;
  if (!plan_levels(d, p)) return SIM_EINVAL;
  return SIM_OK;
}

// Every device buffer of a handle, in allocation order.  `alloc` is called
// with the byte size and the address of the pointer to fill.
template <typename F>
void for_each_buffer(const sim_desc* d, const Plan& p, sim_ctx* t, F alloc) {
  const Dims& d0 = p.dims[0];
  const size_t C = d0.cells(), F_ = d0.faces();
  const size_t es = d->precision == SIM_FP32 ? 4 : 2;
  alloc(F_ * 4, (void**)&t->alpha);
  alloc(d0.nodes() * 8, (void**)&t->phi);
  alloc(F_ * 4, (void**)&t->uhat);
  alloc(F_ * 4, (void**)&t->gu);
  alloc(C * 4, (void**)&t->b);
  alloc(C * 4, (void**)&t->P);
  alloc(C * 4, (void**)&t->y);
  alloc(advect_stage_floats(d0) * 4, (void**)&t->stage);
  alloc(F_ * 6 * 8, (void**)&t->trace);
  alloc(C * 8, (void**)&t->S.x);
  alloc(C * 4, (void**)&t->S.r);
  alloc(C * 4, (void**)&t->S.z);
  alloc(C * 4, (void**)&t->S.q);
  alloc(C * 4, (void**)&t->S.p0);
  alloc(C * 4, (void**)&t->S.p1);
  size_t nb_faces = (F_ + kBlock - 1) / kBlock, nb_cells = (C + kBlock - 1) / kBlock;
  size_t npart = nb_faces * 21 > nb_cells * 4 ? nb_faces * 21 : nb_cells * 4;
  alloc(npart * 8, (void**)&t->S.partials);
  alloc(kUpdateBlocks * 8, (void**)&t->S.partials_rr);
  alloc(4 * kRzPartsMax * 8, (void**)&t->S.partials_rz);
  if (d->precision != SIM_FP32) alloc(C * (16 + 4), &t->S.rec0);   // records, then 1/diag in FP32
  alloc(sizeof(CGScalars), (void**)&t->S.sc);
  alloc(sizeof(unsigned), (void**)&t->maxbits);
  // connected-region labels of the pressure system
  alloc(C * 4, (void**)&t->S.comp.parent);
  alloc(C * 4, (void**)&t->S.comp.id);
  alloc(nb_cells * 4, (void**)&t->S.comp.blockcnt);
  alloc(nb_cells * 4, (void**)&t->S.comp.blockbase);
  alloc(2 * 4, (void**)&t->S.comp.info);
  alloc(kMaxComponents * 4, (void**)&t->S.comp.count);
  alloc(kMaxComponents * 4, (void**)&t->S.comp.ground);
  alloc(kMaxComponents * 8, (void**)&t->S.comp.sums);
  alloc(kMaxComponents * 8, (void**)&t->S.comp.mean);
  alloc(kMaxComponents * 4, (void**)&t->S.comp.zroot);
  if (d->geom == SIM_GEOM_WALL) {
    alloc(SIM_WALL_KNOTS_Y * SIM_WALL_KNOTS_Z * 8, (void**)&t->knots);
    alloc(wall_column_doubles(d0) * 8, (void**)&t->wall_cols);
  }
  if (d->geom == SIM_GEOM_BEZIER) {
    alloc(solids_buffer_doubles() * 8, (void**)&t->solids);
    alloc(solids_partials_doubles() * 8, (void**)&t->solids_part);
    alloc(d0.nodes(), (void**)&t->solid_term);
  }
  for (int l = 0; l < p.nlev; ++l) {
    const Dims& dl = p.dims[l];
    Level& L = t->S.lev[l];
    if (l > 0 || d->precision != SIM_FP32) {
      alloc(dl.nfx() * es, &L.a[0]);
      alloc(dl.nfy() * es, &L.a[1]);
      alloc(dl.nfz() * es, &L.a[2]);
    }
    alloc(dl.cells() * es, &L.invd);
    if (l > 0) {
      alloc(dl.cells() * es, &L.r);
      alloc(dl.cells() * es, &L.z);
    }
    // the finest level's smoother iterates stay FP32 in every precision
    const size_t ts = l == 0 ? 4 : es;
    alloc(dl.cells() * ts, &L.ta);
    alloc(dl.cells() * ts, &L.tb);
  }
  if (d->precision != SIM_FP32) {
    size_t tot = 0;
    for (int l = 1; l < p.nlev; ++l) {
      t->S.scratch_off[l] = tot;
      tot += p.dims[l].faces();
    }
    alloc((tot ? tot : 1) * 4, (void**)&t->S.scratch_a);
    alloc(C * 4, (void**)&t->S.scratch_inv);
  }
}

int make_geom(sim_ctx* c, const double* theta, const double* ctrl, GeomParams& g, hipStream_t st) {
  std::memset(&g, 0, sizeof(g));
  g.kind = c->desc.geom;
  if (g.kind == SIM_GEOM_BEZIER) {
    c->solids_host.assign(solids_buffer_doubles(), 0.0);
    const int v = pack_solids(c->desc, theta, c->solids_host.data(), g);
    if (v != SIM_OK) return v;
    // pageable source: the copy has taken the values when the call returns
    if (hipMemcpyAsync(c->solids, c->solids_host.data(), solids_buffer_doubles() * sizeof(double),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return SIM_EHIP;
    g.solids = c->solids;
    g.solid_term = c->solid_term;
    return SIM_OK;
  }
  if (g.kind == SIM_GEOM_WALL) {
    if (!theta || !ctrl) return SIM_EINVAL;
    constexpr int nk = SIM_WALL_KNOTS_Y * SIM_WALL_KNOTS_Z;
    double amax = 0.0;
    for (int s = 0; s < nk; ++s) {
      if (!std::isfinite(theta[s])) return SIM_EINVAL;
      amax = std::max(amax, std::fabs(theta[s]));
    }
    for (int s = 0; s < 3; ++s)
      if (!std::isfinite(ctrl[s])) return SIM_EINVAL;
    // pageable source: the copy has taken the values when the call returns
    if (hipMemcpyAsync(c->knots, theta, nk * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
      return SIM_EHIP;
    const double t = ctrl[0], f = ctrl[1], w = 2.0 * M_PI * f;
    g.knots = c->knots;
    g.amp = ctrl[2];
    g.wall_s = 0.5 * (1.0 - std::cos(w * t));
    g.wall_sd = M_PI * f * std::sin(w * t);
    g.ly = c->desc.n[1] * c->desc.dx;
    g.lz = c->desc.n[2] * c->desc.dx;
    // |d| <= |amp s| max|a| (the bases are non-negative and sum to one), and
    // a face with alpha < 1 has a corner with x <= d
    const double dmax = std::fabs(g.amp * g.wall_s) * amax;
    g.wall_imax = (int)std::min((double)c->desc.n[0], std::floor(dmax / c->desc.dx) + 1.0);
    return SIM_OK;
  }
  if (g.kind == SIM_GEOM_SPHERES) {
    if (!theta) return SIM_EINVAL;
    g.nsph = c->desc.n_params / 4;
    for (int s = 0; s < 4 * g.nsph; ++s) {
      if (!std::isfinite(theta[s])) return SIM_EINVAL;
      g.sph[s] = theta[s];
    }
  } else if (g.kind == SIM_GEOM_ELLIPSOID) {
    if (!theta || !ctrl) return SIM_EINVAL;
    for (int s = 0; s < 15; ++s)
      if (!std::isfinite(theta[s])) return SIM_EINVAL;
    for (int s = 0; s < 6; ++s)
      if (!std::isfinite(ctrl[s])) return SIM_EINVAL;
    for (int s = 0; s < 3; ++s) {
      g.c[s] = theta[s];
      g.a[s] = theta[3 + s];
      if (!(g.a[s] > 0)) return SIM_EINVAL;
      g.v[s] = ctrl[s];
      g.w[s] = ctrl[3 + s];
    }
    for (int s = 0; s < 9; ++s) g.R[s] = theta[6 + s];
  }
  return SIM_OK;
}

int last_hip_error() { return hipGetLastError() == hipSuccess ? SIM_OK : SIM_EHIP; }

// phi and the face fractions of g; with `levels`, also the solver's
// multigrid hierarchy (a step that reuses a stored pressure needs none).
void eval_geometry(sim_ctx* c, const GeomParams& g, hipStream_t st, bool levels = true) {
  NF_TIMED(&c->prof, SIM_K_GEOM_PHI, st, launch_phi_nodes(c->dom, g, c->phi, st));
  NF_TIMED(&c->prof, SIM_K_GEOM_ALPHA, st, launch_alpha(c->dom, c->phi, c->alpha, st));
  if (levels) solver_setup_levels(c->S, c->alpha, st);
  c->levels_current = levels;
  c->last_geom = g;
  c->have_geom = true;
}

double k_factor(const sim_desc& d) { return d.dt / (d.rho * d.dx); }

// U^ of a step into h->uhat: the advected field (with the body force), then,
// with nu > 0, the explicit viscosity (the advected field goes through h->gu,
// which holds nothing at this point of a step or of its adjoint).
void advect_and_diffuse(sim_ctx* h, const float* u_n, double* trace, hipStream_t stream) {
  const bool visc = h->desc.nu > 0.0;
  float* adv = visc ? h->gu : h->uhat;
  NF_TIMED(&h->prof, SIM_K_ADVECT, stream,
           launch_advect(h->dom.d, h->desc.dx, h->desc.dt, h->desc.gravity, u_n, adv, trace, stream));
  if (visc)
    NF_TIMED(&h->prof, SIM_K_VISCOSITY, stream,
             launch_viscosity(h->dom.d, h->desc.nu * h->desc.dt / (h->desc.dx * h->desc.dx), adv, h->uhat, stream));
}

// In the device solve mode the stats are written by a kernel: the pointer
// must be device memory or pinned host memory.
int check_stats_ptr(const sim_ctx* c, const sim_stats* st) {
  if (!st || !c->S.device_mode) return SIM_OK;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, st) != hipSuccess) {
    (void)hipGetLastError();
    return SIM_EINVAL;
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeHost && at.type != hipMemoryTypeManaged)
    return SIM_EINVAL;
  return SIM_OK;
}

// Keep the first warning of a call (positive solver status) while the call
// carries on; negative statuses end it.
int merge_status(int warn, int r) { return warn != SIM_OK ? warn : r; }

}  // namespace

extern "C" {

const char* sim_version(void) { return "neuralfluid-gfx950 1.0"; }

const char* sim_status_string(int32_t s) {
  switch (s) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ENOMEM: return "device allocation failed";
    case SIM_EHIP: return "HIP runtime error";
    case SIM_EUNSUPPORTED: return "unsupported configuration";
    case SIM_EBUSY: return "no free slot or budget in the pool now";
    case SIM_WNOCONV: return "a Poisson solve did not reach the tolerance";
    case SIM_WNONFINITE: return "a Poisson solve met a non-finite value";
    default: return "unknown status";
  }
}

int32_t sim_footprint(const sim_desc* desc, size_t* bytes) {
  int v = validate_desc(desc);
  if (v != SIM_OK) return v;
  if (!bytes) return SIM_EINVAL;
  Plan p;
  plan_levels(desc, p);
  size_t tot = 0;
  sim_ctx tmp;
  for_each_buffer(desc, p, &tmp, [&](size_t b, void**) { tot += align256(b); });
  *bytes = tot;
  return SIM_OK;
}

int32_t sim_create(const sim_desc* desc, sim_handle* out) {
  int v = validate_desc(desc);
  if (v != SIM_OK) return v;
  if (!out) return SIM_EINVAL;
  sim_ctx* c = new (std::nothrow) sim_ctx();
  if (!c) return SIM_ENOMEM;
  c->desc = *desc;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  Plan p;
  plan_levels(desc, p);
  c->dom.d = p.dims[0];
  for (int s = 0; s < 6; ++s) c->dom.bc[s] = desc->bc[s];
  c->dom.dx = desc->dx;
  c->dom.inflow = desc->inflow_speed;
  c->S.nlev = p.nlev;
  c->S.prof = &c->prof;
  {
    const char* tr = std::getenv("NF_TRACE_SOLVER");
    c->S.trace = tr && tr[0] == '1';
    const char* gr = std::getenv("NF_SOLVER_GRAPHS");
    c->S.use_graph = !(gr && gr[0] == '0');
    const char* fu = std::getenv("NF_MG_FUSED");
    c->S.fused = !(fu && fu[0] == '0');
    const char* bl = std::getenv("NF_MG_BOTTOM_LANES");
    c->S.bottom_lanes = !(bl && bl[0] == '0');
  }
  // the fused tile kernels need 31-bit byte offsets over a tile's region
  if (!views_fit(p.dims[0].nx, p.dims[0].ny)) c->S.fused = 0;
  c->S.precision = desc->precision;
  for (int l = 0; l < p.nlev; ++l) c->S.lev[l].d = p.dims[l];
  solver_init_device(c->S);
  c->S.project = 1;
  for (int s = 0; s < 6; ++s) {
    c->S.sides.out[s] = desc->bc[s] == SIM_BC_OUTFLOW ? 1 : 0;
    if (desc->bc[s] == SIM_BC_OUTFLOW) c->S.project = 0;
  }
  c->S.nbottom = p.nlev - 1;
  size_t bottom_cells = kBottomCells;
  if (const char* bc = std::getenv("NF_MG_BOTTOM_CELLS")) {
    const long v = std::atol(bc);
    if (v > 0 && v <= kCoarseMaxCells) bottom_cells = (size_t)v;
  }
  while (c->S.nbottom > 0 && p.dims[c->S.nbottom - 1].cells() <= bottom_cells) --c->S.nbottom;
  bool ok = true;
  // NF_POISON_BUFFERS=1 fills every buffer with all-ones bytes (NaN in every
  // float format) so that a read of a value no kernel wrote shows up
  const char* pz = std::getenv("NF_POISON_BUFFERS");
  const bool poison = pz && pz[0] == '1';
  for_each_buffer(desc, p, c, [&](size_t b, void** ptr) {
    if (!ok) return;
    void* q = nullptr;
    if (hipMalloc(&q, align256(b)) != hipSuccess) {
      ok = false;
      return;
    }
    c->allocs.push_back(q);
    *ptr = q;
    if (poison && hipMemset(q, 0xff, align256(b)) != hipSuccess) ok = false;
  });
  if (ok && poison && hipDeviceSynchronize() != hipSuccess) ok = false;
  if (ok && hipHostMalloc((void**)&c->S.host_sc, sizeof(CGScalars), hipHostMallocDefault) != hipSuccess) ok = false;
  if (ok && hipMemset(c->S.sc, 0, sizeof(CGScalars)) != hipSuccess) ok = false;
  if (!ok) {
    (void)hipGetLastError();
    sim_destroy(c);
    return SIM_ENOMEM;
  }
  // with 2-byte multigrid storage the finest fused kernels read packed
  // coefficient records where their views fit 31-bit offsets (NF_MG_RECORDS=0:
  // the separate arrays)
  {
    const char* rc = std::getenv("NF_MG_RECORDS");
    const bool want = !(rc && rc[0] == '0');
    if (!want || !c->S.fused || c->S.nbottom == 0 || !views_fit(p.dims[0].nx, p.dims[0].ny, 16)) c->S.rec0 = nullptr;
  }
  *out = c;
  return SIM_OK;
}

int32_t sim_destroy(sim_handle h) {
  if (!h) return SIM_EINVAL;
  solver_release(h->S);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->S.host_sc) (void)hipHostFree(h->S.host_sc);
  delete h;
  return SIM_OK;
}

int32_t sim_layout(sim_handle h, size_t* vel_elems, size_t* cell_elems) {
  if (!h) return SIM_EINVAL;
  if (vel_elems) *vel_elems = h->dom.d.faces();
  if (cell_elems) *cell_elems = h->dom.d.cells();
  return SIM_OK;
}

int32_t sim_set_geometry(sim_handle h, const double* theta, const double* ctrl, float* alpha_out,
                         hipStream_t stream) {
  if (!h) return SIM_EINVAL;
  GeomParams g;
  int v = make_geom(h, theta, ctrl, g, stream);
  if (v != SIM_OK) return v;
  eval_geometry(h, g, stream);
  if (alpha_out &&
      hipMemcpyAsync(alpha_out, h->alpha, h->dom.d.faces() * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return SIM_EHIP;
  return last_hip_error();
}

static int32_t project_common(sim_handle h, const float* uhat, const GeomParams& g, float* u_out, float* p_out,
                              sim_stats* st, hipStream_t stream) {
  const double kk = k_factor(h->desc);
  NF_TIMED(&h->prof, SIM_K_RHS, stream, launch_rhs(h->dom, g, 1.0 / kk, h->alpha, uhat, h->b, stream));
  // warm start: the solve runs in h->P, which holds the previous solve's
  // pressure, and the result is copied out
  const bool warm = (h->warm & SIM_WARM_PRESSURE) != 0;
  float* P = (p_out && !warm) ? p_out : h->P;
  const int r = solver_solve(h->S, kSolvePressure, h->b, P, h->desc.tol, h->desc.max_iter, st, stream,
                             !(warm && h->warm_p));
  if (r < 0) return r;
  h->warm_p = warm;
  if (p_out && P != p_out) launch_copy(P, p_out, h->dom.d.cells(), stream);
  NF_TIMED(&h->prof, SIM_K_UPDATE, stream, launch_update(h->dom, g, kk, h->alpha, uhat, P, u_out, stream));
  const int e = last_hip_error();
  return e != SIM_OK ? e : r;
}

int32_t sim_step(sim_handle h, const float* u_n, const double* theta, const double* ctrl, float* u_n1, float* p_n1,
                 sim_stats* st, hipStream_t stream) {
  if (!h || !u_n || !u_n1 || u_n == u_n1) return SIM_EINVAL;
  if (check_stats_ptr(h, st) != SIM_OK) return SIM_EINVAL;
  GeomParams g;
  int v = make_geom(h, theta, ctrl, g, stream);
  if (v != SIM_OK) return v;
  eval_geometry(h, g, stream);
  advect_and_diffuse(h, u_n, nullptr, stream);
  return project_common(h, h->uhat, g, u_n1, p_n1, st, stream);
}

int32_t sim_step_replay(sim_handle h, const float* u_n, const double* theta, const double* ctrl,
                        const float* p_n1, float* u_n1, hipStream_t stream) {
  if (!h || !u_n || !u_n1 || !p_n1 || u_n == u_n1) return SIM_EINVAL;
  GeomParams g;
  int v = make_geom(h, theta, ctrl, g, stream);
  if (v != SIM_OK) return v;
  eval_geometry(h, g, stream, false);
  advect_and_diffuse(h, u_n, nullptr, stream);
  NF_TIMED(&h->prof, SIM_K_UPDATE, stream,
           launch_update(h->dom, g, k_factor(h->desc), h->alpha, h->uhat, p_n1, u_n1, stream));
  return last_hip_error();
}

int32_t sim_project(sim_handle h, const float* u_in, const double* theta, const double* ctrl, float* u_out,
                    float* p_out, sim_stats* st, hipStream_t stream) {
  if (!h || !u_in || !u_out || u_in == u_out) return SIM_EINVAL;
  if (check_stats_ptr(h, st) != SIM_OK) return SIM_EINVAL;
  GeomParams g;
  int v = make_geom(h, theta, ctrl, g, stream);
  if (v != SIM_OK) return v;
  eval_geometry(h, g, stream);
  return project_common(h, u_in, g, u_out, p_out, st, stream);
}

int32_t sim_step_adjoint(sim_handle h, const float* u_n, const float* p_n1, const double* theta, const double* ctrl,
                         const float* g_u_n1, float* g_u_n, double* g_theta, double* g_ctrl, sim_stats* st,
                         hipStream_t stream) {
  if (!h || !u_n || !g_u_n1 || !g_u_n || g_u_n == g_u_n1 || (const float*)g_u_n == u_n) return SIM_EINVAL;
  if (check_stats_ptr(h, st) != SIM_OK) return SIM_EINVAL;
  GeomParams g;
  int v = make_geom(h, theta, ctrl, g, stream);
  if (v != SIM_OK) return v;
  const bool grad = (h->desc.geom == SIM_GEOM_ELLIPSOID && (g_theta || g_ctrl)) ||
                    ((h->desc.geom == SIM_GEOM_WALL || h->desc.geom == SIM_GEOM_BEZIER) && g_theta);
  const double kk = k_factor(h->desc);
  eval_geometry(h, g, stream);
  // the step's advected (and diffused) field (the fluid velocity W on cut
  // faces needs it) and the back-traced positions
  advect_and_diffuse(h, u_n, h->trace, stream);
  const float* P = p_n1;
  int warn = SIM_OK;
  if (!P && grad) {
    // no stored pressure: solve the forward system again
    launch_rhs(h->dom, g, 1.0 / kk, h->alpha, h->uhat, h->b, stream);
    int r = solver_solve(h->S, kSolvePressure, h->b, h->P, h->desc.tol, h->desc.max_iter, nullptr, stream, true);
    if (r < 0) return r;
    warn = r;
    P = h->P;
    h->warm_p = false;   // h->P no longer holds the last step's pressure
  }
  // dJ/dP and the adjoint pressure system (G^T S G) y = -G^T S g
  NF_TIMED(&h->prof, SIM_K_ADJ_DIV, stream, launch_adj_div(h->dom.d, h->alpha, g_u_n1, h->b, stream));
  const bool warm_adj = (h->warm & SIM_WARM_ADJOINT) != 0;
  int r = solver_solve(h->S, kSolveAdjoint, h->b, h->y, h->desc.tol, h->desc.max_iter, st, stream,
                       !(warm_adj && h->warm_y));
  if (r < 0) return r;
  h->warm_y = warm_adj;
  warn = merge_status(warn, r);
  NF_TIMED(&h->prof, SIM_K_ADJ_FACES, stream,
           launch_adj_faces(h->dom, g, grad, kk, h->alpha, h->phi, g_u_n1, h->y, h->uhat, P ? P : h->y, h->gu,
                            h->S.partials, g_theta, g_ctrl,
                            h->desc.geom == SIM_GEOM_BEZIER ? h->solids_part : h->wall_cols, stream));
  // through the viscosity (symmetric; h->uhat is no longer needed)
  const float* g_adv = h->gu;
  if (h->desc.nu > 0.0) {
    NF_TIMED(&h->prof, SIM_K_VISCOSITY, stream,
             launch_viscosity(h->dom.d, h->desc.nu * h->desc.dt / (h->desc.dx * h->desc.dx), h->gu, h->uhat,
                              stream));
    g_adv = h->uhat;
  }
  launch_fill(g_u_n, h->dom.d.faces(), 0.0f, stream);
  NF_TIMED(&h->prof, SIM_K_ADVECT_ADJ, stream,
           launch_advect_adjoint(h->dom.d, h->desc.dx, h->desc.dt, u_n, h->trace, g_adv, g_u_n, h->stage, stream));
  const int e = last_hip_error();
  return e != SIM_OK ? e : warn;
}

int32_t poisson_solve(sim_handle h, const float* alpha, const float* b, float* x, double tol, int32_t max_iter,
                      sim_stats* st, hipStream_t stream) {
  if (!h || !b || !x) return SIM_EINVAL;
  if (!alpha && !h->have_geom) return SIM_EINVAL;
  if (check_stats_ptr(h, st) != SIM_OK) return SIM_EINVAL;
  if (alpha) {
    if (hipMemcpyAsync(h->alpha, alpha, h->dom.d.faces() * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return SIM_EHIP;
    solver_setup_levels(h->S, h->alpha, stream);
    h->have_geom = true;
    h->levels_current = true;
  } else if (!h->levels_current) {
    solver_setup_levels(h->S, h->alpha, stream);
    h->levels_current = true;
  }
  int r = solver_solve(h->S, kSolveUser, b, x, tol > 0 ? tol : h->desc.tol, max_iter > 0 ? max_iter : h->desc.max_iter, st,
                       stream);
  if (r < 0) return r;
  const int e = last_hip_error();
  return e != SIM_OK ? e : r;
}

int32_t sim_set_regions(sim_handle h, int32_t mode) {
  if (!h || mode < SIM_REGIONS_AUTO || mode > SIM_REGIONS_NEVER) return SIM_EINVAL;
  h->S.comp.mode = mode;
  h->S.comp.valid = false;
  return SIM_OK;
}

int32_t sim_regions(sim_handle h, int32_t* region_out, int32_t* count, int32_t* floating, hipStream_t stream) {
  if (!h || !count || !h->have_geom) return SIM_EINVAL;
  if (!h->levels_current) {
    solver_setup_levels(h->S, h->alpha, stream);
    h->levels_current = true;
  }
  if (!h->S.comp.valid) components_label(h->S, stream);
  const size_t C = h->dom.d.cells();
  if (region_out &&
      hipMemcpyAsync(region_out, h->S.comp.id, C * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return SIM_EHIP;
  int info[2] = {0, 0};
  if (hipMemcpyAsync(info, h->S.comp.info, sizeof(info), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return SIM_EHIP;
  *count = info[0];
  if (floating) {
    *floating = -1;
    if (info[1]) {
      std::vector<int> cnt(info[0]), gr(info[0]);
      if (info[0] > 0 &&
          (hipMemcpy(cnt.data(), h->S.comp.count, info[0] * 4, hipMemcpyDeviceToHost) != hipSuccess ||
           hipMemcpy(gr.data(), h->S.comp.ground, info[0] * 4, hipMemcpyDeviceToHost) != hipSuccess))
        return SIM_EHIP;
      int f = 0;
      for (int q = 0; q < info[0]; ++q) f += (cnt[q] > 0 && !gr[q]) ? 1 : 0;
      *floating = f;
    }
  }
  return last_hip_error();
}

int32_t sim_set_dt(sim_handle h, double dt) {
  if (!h || !(dt > 0.0) || !std::isfinite(dt)) return SIM_EINVAL;
  h->desc.dt = dt;
  return SIM_OK;
}

int32_t sim_max_speed(sim_handle h, const float* u, double* vmax, hipStream_t stream) {
  if (!h || !u || !vmax) return SIM_EINVAL;
  launch_max_abs(h->dom.d.faces(), u, h->maxbits, stream);
  unsigned bits = 0;
  if (hipMemcpyAsync(&bits, h->maxbits, sizeof(bits), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return SIM_EHIP;
  float v;
  std::memcpy(&v, &bits, sizeof(v));
  *vmax = (double)v;
  return last_hip_error();
}

int32_t sim_set_warm_start(sim_handle h, int32_t kinds) {
  if (!h || kinds < 0 || kinds > (SIM_WARM_PRESSURE | SIM_WARM_ADJOINT)) return SIM_EINVAL;
  h->warm = kinds;
  h->warm_p = h->warm_y = false;   // the next solve of each kind starts from zero
  return SIM_OK;
}

int32_t sim_set_solve_mode(sim_handle h, int32_t mode, int32_t budget) {
  if (!h || (mode != SIM_SOLVE_HOST && mode != SIM_SOLVE_DEVICE)) return SIM_EINVAL;
  h->S.device_mode = mode == SIM_SOLVE_DEVICE ? 1 : 0;
  h->S.budget = budget > 0 ? budget : 0;
  return SIM_OK;
}

int32_t sim_loss_box(sim_handle h, const float* u, const double* lo, const double* hi, double* J, float* g,
                     hipStream_t stream) {
  if (!h || !u || !lo || !hi || !J || !g || (const float*)g == u) return SIM_EINVAL;
  launch_loss_box(h->dom, lo, hi, u, J, g, h->S.partials, stream);
  return last_hip_error();
}

}  // extern "C"

// Partial sums of the allocation-free box loss: one fixed array per GPU,
// shared by every call on that GPU (held until the process ends).  Host code
// reaches it only through the address hipGetSymbolAddress returns on each
// device; the array's own name is a host-side stand-in there.
static __device__ __align__(256) double scratch[kLossBlocks];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_lock;
double* g_scratch[kScratchDevices] = {};

// The current device's copy of the scratch array (looked up once per device).
double* scratch_on_device(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_lock);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = (double*)ptr;
  }
  return g_scratch[dev];
}
}  // namespace

extern "C" {

int32_t sim_loss_box_noalloc(const int32_t n[3], double dx, const float* u, const double* lo, const double* hi,
                             double* J, float* g, hipStream_t stream) {
  if (!n || !u || !lo || !hi || !J || !g || (const float*)g == u || !(dx > 0.0) || !std::isfinite(dx))
    return SIM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || n[a] > 4096) return SIM_EINVAL;
  if ((long)n[0] * n[1] * n[2] > (1L << 30)) return SIM_EINVAL;
  Domain D;
  std::memset(&D, 0, sizeof(D));
  D.d = Dims{n[0], n[1], n[2]};
  D.dx = dx;
  if (loss_box_blocks(D.d) > kLossBlocks) return SIM_EINVAL;   // the scratch holds kLossBlocks partials
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SIM_EHIP;
  if (dev < 0 || dev >= kScratchDevices) return SIM_EINVAL;
  double* part = scratch_on_device(dev);
  if (!part) return SIM_EHIP;
  launch_loss_box(D, lo, hi, u, J, g, part, stream);
  return last_hip_error();
}

int32_t sim_loss_outlet(sim_handle h, const float* u, const float* w, double scale, double* J, float* g,
                        hipStream_t stream) {
  if (!h || !u || !J || !g || (const float*)g == u || !std::isfinite(scale)) return SIM_EINVAL;
  launch_loss_outlet(h->dom.d, scale, w, u, J, g, h->S.partials, stream);
  return last_hip_error();
}

int32_t sim_profile(sim_handle h, int32_t kernel) {
  if (!h || kernel < -1 || kernel >= SIM_K_COUNT) return SIM_EINVAL;
  h->prof.active = kernel;
  h->prof.used = 0;
  return SIM_OK;
}

int32_t sim_profile_read(sim_handle h, double min_ms, double* total_ms, int64_t* count) {
  if (!h || !total_ms || !count || !(min_ms >= 0.0)) return SIM_EINVAL;
  double tot = 0.0;
  int64_t n = 0;
  for (size_t q = 0; q + 1 < h->prof.used; q += 2) {
    if (hipEventSynchronize(h->prof.ev[q + 1]) != hipSuccess) return SIM_EHIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->prof.ev[q], h->prof.ev[q + 1]) != hipSuccess) return SIM_EHIP;
    if ((double)ms < min_ms) continue;
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  h->prof.used = 0;
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// rigid pose dynamics (host, FP64)
// ---------------------------------------------------------------------------

static void skew3(const double v[3], double K[9]) {
  K[0] = 0; K[1] = -v[2]; K[2] = v[1];
  K[3] = v[2]; K[4] = 0; K[5] = -v[0];
  K[6] = -v[1]; K[7] = v[0]; K[8] = 0;
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  std::memcpy(C, T, sizeof(T));
}

// exp([r]x) by the Rodrigues formula.
static void expmap(const double r[3], double R[9]) {
  double t = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  if (t == 0.0) return;
  double K[9], K2[9];
  skew3(r, K);
  matmul3(K, K, K2);
  double s = std::sin(t) / t, c = (1.0 - std::cos(t)) / (t * t);
  for (int i = 0; i < 9; ++i) R[i] += s * K[i] + c * K2[i];
}

// dR/dr_i of the exponential map (Gallego & Yezzi 2015):
// (r_i [r]x + [r x ((I - R) e_i)]x) R / |r|^2, and [e_i]x at r = 0.
static void expmap_grad(const double r[3], double dR[3][9]) {
  double t2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  for (int i = 0; i < 3; ++i) {
    double e[3] = {0, 0, 0};
    e[i] = 1.0;
    if (t2 == 0.0) {
      skew3(e, dR[i]);
      continue;
    }
    double R[9], K[9];
    expmap(r, R);
    skew3(r, K);
    double ImRe[3];
    for (int a = 0; a < 3; ++a) ImRe[a] = e[a] - R[3 * a + i];
    double cr[3] = {r[1] * ImRe[2] - r[2] * ImRe[1], r[2] * ImRe[0] - r[0] * ImRe[2],
                    r[0] * ImRe[1] - r[1] * ImRe[0]};
    double Kc[9], M[9];
    skew3(cr, Kc);
    for (int a = 0; a < 9; ++a) M[a] = (r[i] * K[a] + Kc[a]) / t2;
    matmul3(M, R, dR[i]);
  }
}

int32_t sim_ellipsoid_poses(const double* theta0, const double* ctrl, int32_t T, double dt, double* out) {
  if (!theta0 || (!ctrl && T > 0) || !out || T < 0) return SIM_EINVAL;
  double c[3] = {theta0[0], theta0[1], theta0[2]};
  double R[9];
  expmap(theta0 + 6, R);
  for (int n = 0; n < T; ++n) {
    const double* v = ctrl + 6 * n;
    double rw[3] = {dt * v[3], dt * v[4], dt * v[5]}, E[9];
    expmap(rw, E);
    for (int a = 0; a < 3; ++a) c[a] += dt * v[a];
    matmul3(E, R, R);
    double* o = out + 15 * n;
    for (int a = 0; a < 3; ++a) {
      o[a] = c[a];
      o[3 + a] = theta0[3 + a];
    }
    for (int a = 0; a < 9; ++a) o[6 + a] = R[a];
  }
  return SIM_OK;
}

int32_t sim_ellipsoid_poses_adjoint(const double* theta0, const double* ctrl, int32_t T, double dt,
                                    const double* g_steps, const double* g_ctrl_direct, double* g_theta0,
                                    double* g_ctrl) {
  if (!theta0 || !g_theta0 || T < 0 || (T > 0 && (!ctrl || !g_steps || !g_ctrl_direct || !g_ctrl)))
    return SIM_EINVAL;
  std::vector<double> poses((size_t)15 * (T > 0 ? T : 1));
  if (T > 0) sim_ellipsoid_poses(theta0, ctrl, T, dt, poses.data());
  double R0[9];
  expmap(theta0 + 6, R0);
  double gc[3] = {0, 0, 0}, ga[3] = {0, 0, 0}, gR[9] = {0};
  for (int n = T - 1; n >= 0; --n) {
    const double* gs = g_steps + 15 * n;
    const double* v = ctrl + 6 * n;
    for (int a = 0; a < 3; ++a) {
      gc[a] += gs[a];
      ga[a] += gs[3 + a];
    }
    for (int a = 0; a < 9; ++a) gR[a] += gs[6 + a];
    double* go = g_ctrl + 6 * n;
    for (int a = 0; a < 6; ++a) go[a] = g_ctrl_direct[6 * n + a];
    // c^{n+1} = c^n + dt v^n
    for (int a = 0; a < 3; ++a) go[a] += dt * gc[a];
    // R^{n+1} = E R^n, E = exp([dt w]x): dJ/dE = gR R^n^T, dJ/dR^n = E^T gR
    const double* Rn = n > 0 ? poses.data() + 15 * (n - 1) + 6 : R0;
    double rw[3] = {dt * v[3], dt * v[4], dt * v[5]}, E[9], dE[3][9];
    expmap(rw, E);
    expmap_grad(rw, dE);
    double gE[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) gE[3 * i + j] = gR[3 * i] * Rn[3 * j] + gR[3 * i + 1] * Rn[3 * j + 1] +
                                                 gR[3 * i + 2] * Rn[3 * j + 2];
    for (int q = 0; q < 3; ++q) {
      double s = 0;
      for (int a = 0; a < 9; ++a) s += dE[q][a] * gE[a];
      go[3 + q] += dt * s;
    }
    double nR[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) nR[3 * i + j] = E[i] * gR[j] + E[3 + i] * gR[3 + j] + E[6 + i] * gR[6 + j];
    std::memcpy(gR, nR, sizeof(nR));
  }
  double dR0[3][9];
  expmap_grad(theta0 + 6, dR0);
  for (int a = 0; a < 3; ++a) {
    g_theta0[a] = gc[a];
    g_theta0[3 + a] = ga[a];
    double s = 0;
    for (int q = 0; q < 9; ++q) s += dR0[a][q] * gR[q];
    g_theta0[6 + a] = s;
  }
  return SIM_OK;
}

}  // extern "C"
