// C ABI entry points (include/dgnp.h).  Every function converts exceptions into
// status codes and records the message for dgnp_last_error().
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "context.hpp"
#include "kernels_jac.hpp"
#include "solver.hpp"

using namespace dgnp;

static thread_local std::string g_last_error;
thread_local const dgnp::DevAllocator* dgnp::t_dev_alloc = nullptr;

template <typename F>
static int guard(F&& f) {
  try {
    f();
    return DGNP_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DGNP_E_ALLOC;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DGNP_E_ARG;
  } catch (...) {
    g_last_error = "unknown failure";
    return DGNP_E_ARG;
  }
}

dgnp::KArgs dgnp_ctx::kargs() const {
  KArgs A{};
  A.E = E;
  for (int i = 0; i < 3; ++i) {
    A.n[i] = n[i];
    A.lo[i] = lo[i];
    A.h[i] = h[i];
  }
  A.detJ = 1.0;
  for (int i = 0; i < dim; ++i) A.detJ *= 0.5 * h[i];
  A.delta = delta;
  A.Pe = vel.Pe;
  A.vel_kind = vel.kind;
  for (int i = 0; i < 3; ++i) A.vel_param[i] = vel.param[i];
  A.vel_H = hi[1] - lo[1];
  A.vel_ylo = lo[1];
  for (int i = 0; i < 4; ++i) {
    A.z[i] = z[i];
    A.D[i] = D[i];
    A.a[i] = a[i];
    A.b[i] = b[i];
  }
  for (int t = 0; t < 6; ++t) {
    A.c_bc[t] = c_bc[t];
    A.phi_bc[t] = phi_bc[t];
    A.btag_off[t] = btag_off[t];
  }
  A.n_bface = n_bface;
  A.nbr = d_nbr.p;
  A.bcq = d_bcq.p;
  A.src = d_src.p;
  A.objective_tag = 1;
  A.objective_kind = 0;
  A.bv_r = bv_ion;
  A.bv_z = has_electrode ? z[bv_ion - 1] : 0.0;
  A.bv_aa = bv_aa;
  A.bv_ac = bv_ac;
  for (int k = 0; k < 4; ++k) A.bv_dc[k] = 0.0;
  for (int k = 1; k < m; ++k)
    A.bv_dc[k - 1] = bv_ion < m ? (k == bv_ion ? 1.0 : 0.0) : -z[k - 1] / z[m - 1];
  A.bv_prof = dim == 3 ? bv_prof : 0;
  A.bv_zc = 0.5 * (lo[2] + hi[2]);
  A.bv_zhalf = 0.5 * (hi[2] - lo[2]);
  A.vin_mask = ~0u;
  A.jbase = nullptr;
  return A;
}

// shape of the exchange current of electrode faces across the box in z
// (DGNP_J0_PARABOLIC_Z: the parabola of Sec. 5.2 with mean 1)
static double j0_profile(const dgnp_ctx& c, double z) {
  if (c.bv_prof != DGNP_J0_PARABOLIC_Z || c.dim < 3) return 1.0;
  const double t = (z - 0.5 * (c.lo[2] + c.hi[2])) / (0.5 * (c.hi[2] - c.lo[2]));
  return 0.6 * (2.0 - t * t);
}

// boundary data at the face Gauss points, [m][n_bface][nqf]
static void build_boundary_data(dgnp_ctx& c) {
  if (!c.dir_face.empty()) {  // the caller's data at the face points
    c.d_bcq.upload(c.dir_face, c.stream);
    if (!c.src_vol.empty()) c.d_src.upload(c.src_vol, c.stream);
    return;
  }
  const int d = c.dim, nq = c.nq, nn = c.nn;
  std::vector<double> bcq(static_cast<size_t>(c.m) * c.n_bface * c.nqf, 0.0);
  int64_t stride2 = int64_t(c.n[0]) * c.n[1];
  for (int t = 0; t < 2 * d; ++t) {
    const int a = t / 2, side = (t & 1) ? 1 : -1;
    const int t1 = d == 3 ? (a == 0 ? 1 : 0) : 1 - a;
    const int t2 = d == 3 ? (a == 2 ? 1 : 2) : 0;
    const bool phid = c.phi_bc[t] == DGNP_PHI_DIRICHLET;
    const bool cdat = c.c_bc[t] == DGNP_C_DIRICHLET || c.c_bc[t] == DGNP_C_INFLOW;
    const bool elec = c.c_bc[t] == DGNP_C_ELECTRODE;
    int64_t lin = 0;
    for (int64_t e = 0; e < c.E; ++e) {
      int id[3] = {int(e % c.n[0]), int((e / c.n[0]) % c.n[1]), d == 3 ? int(e / stride2) : 0};
      if (id[a] != (side < 0 ? 0 : c.n[a] - 1)) continue;
      const int64_t bf = c.btag_off[t] + lin;
      for (int qf = 0; qf < c.nqf; ++qf) {
        const int qi = qf % nq, qj = qf / nq;
        double x[3] = {0, 0, 0};
        x[a] = c.lo[a] + (id[a] + (side > 0 ? 1.0 : 0.0)) * c.h[a];
        x[t1] = c.lo[t1] + (id[t1] + 0.5 * (c.ref.xq[qi] + 1.0)) * c.h[t1];
        if (d == 3) x[t2] = c.lo[t2] + (id[t2] + 0.5 * (c.ref.xq[qj] + 1.0)) * c.h[t2];
        double ph = 0.0, c1 = 0.0;
        if (c.mms) mms_exact(c, x, &ph, &c1);
        if (phid) bcq[(0 * c.n_bface + bf) * c.nqf + qf] = c.mms ? ph : c.phi_val[t];
        if (elec) {  // applied potential, and the exchange current at the point
          bcq[(0 * c.n_bface + bf) * c.nqf + qf] = c.bv_phi_app[t];
          bcq[(1 * c.n_bface + bf) * c.nqf + qf] = c.bv_j0[t] * j0_profile(c, x[2]);
        }
        if (cdat) {
          for (int k = 1; k < c.m; ++k) {
            double g = 0.0;
            if (c.mms) {
              g = c1;
            } else {
              const double* nodal = c.bc_conc.data() + size_t(k - 1) * c.n_bnode + c.bnode_off[t] + lin * c.nfn;
              for (int jn = 0; jn < c.nfn; ++jn) {
                const int ji = jn % nn, jj = jn / nn;
                double psi = c.ref.B[qi * nn + ji];
                if (d == 3) psi *= c.ref.B[qj * nn + jj];
                g += psi * nodal[jn];
              }
            }
            bcq[(size_t(k) * c.n_bface + bf) * c.nqf + qf] = g;
          }
        }
      }
      ++lin;
    }
  }
  c.d_bcq.upload(bcq, c.stream);
  if (!c.src_vol.empty()) {
    c.d_src.upload(c.src_vol, c.stream);
  } else if (c.mms) {
    std::vector<double> src(static_cast<size_t>(c.m) * c.E * c.nqv, 0.0);
    for (int64_t e = 0; e < c.E; ++e) {
      int id[3] = {int(e % c.n[0]), int((e / c.n[0]) % c.n[1]), d == 3 ? int(e / stride2) : 0};
      for (int q = 0; q < c.nqv; ++q) {
        int qc[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
        double x[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) x[i] = c.lo[i] + (id[i] + 0.5 * (c.ref.xq[qc[i]] + 1.0)) * c.h[i];
        double sp, sc;
        mms_source(c, x, &sp, &sc);
        src[(0 * c.E + e) * c.nqv + q] = sp;
        src[(1 * c.E + e) * c.nqv + q] = sc;
      }
    }
    c.d_src.upload(src, c.stream);
  }
}

extern "C" {

int dgnp_setup(const dgnp_mesh* mesh, int32_t order, const dgnp_species* sp, const dgnp_velocity* vel,
               const dgnp_options* opt, void* stream, dgnp_ctx** out) {
  return guard([&] {
    DGNP_REQUIRE(mesh && sp && vel && out, DGNP_E_ARG, "NULL argument");
    DGNP_REQUIRE(mesh->dim == 2 || mesh->dim == 3, DGNP_E_ARG, "dim must be 2 or 3");
    DGNP_REQUIRE(order >= 1 && order <= 3, DGNP_E_ARG, "order must be 1..3");
    DGNP_REQUIRE(sp->m >= 2 && sp->m <= 3, DGNP_E_ARG, "number of ions must be 2 or 3");
    DGNP_REQUIRE(sp->z && sp->D, DGNP_E_ARG, "species arrays missing");
    DGNP_REQUIRE(sp->z[sp->m - 1] != 0.0, DGNP_E_ARG, "eliminated ion must be charged");
    DGNP_REQUIRE(!opt || (opt->alloc == nullptr) == (opt->free_ == nullptr), DGNP_E_ARG,
                 "allocator hook: both alloc and free_, or neither");
    auto c = std::make_unique<dgnp_ctx>();
    if (opt && opt->alloc) {
      c->allocator.alloc = opt->alloc;
      c->allocator.free_ = opt->free_;
      c->allocator.ctx = opt->alloc_ctx;
    }
    AllocScope as(c->allocator);
    c->dim = mesh->dim;
    c->p = order;
    c->m = sp->m;
    c->nn = order + 1;
    c->nq = order + 2;
    c->nb = c->dim == 3 ? c->nn * c->nn * c->nn : c->nn * c->nn;
    c->nqv = c->dim == 3 ? c->nq * c->nq * c->nq : c->nq * c->nq;
    c->nqf = c->dim == 3 ? c->nq * c->nq : c->nq;
    c->nfn = c->dim == 3 ? c->nn * c->nn : c->nn;
    c->E = 1;
    double diam2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      c->n[i] = i < c->dim ? mesh->n[i] : 1;
      c->lo[i] = i < c->dim ? mesh->lo[i] : 0.0;
      c->hi[i] = i < c->dim ? mesh->hi[i] : 1.0;
      DGNP_REQUIRE(c->n[i] >= 1, DGNP_E_ARG, "element counts must be positive");
      DGNP_REQUIRE(c->hi[i] > c->lo[i], DGNP_E_ARG, "empty box");
      c->h[i] = (c->hi[i] - c->lo[i]) / c->n[i];
      if (i < c->dim) diam2 += c->h[i] * c->h[i];
      c->E *= c->n[i];
    }
    DGNP_REQUIRE(c->E <= (int64_t(1) << 30), DGNP_E_ARG, "too many elements");
    c->Nf = c->E * c->nb;
    c->N = c->m * c->Nf;
    for (int k = 0; k < c->m; ++k) {
      c->z[k] = sp->z[k];
      c->D[k] = sp->D[k];
      DGNP_REQUIRE(sp->D[k] > 0.0, DGNP_E_ARG, "diffusivities must be positive");
    }
    const double zm = c->z[c->m - 1], Dm = c->D[c->m - 1];
    for (int k = 0; k < c->m - 1; ++k) {
      c->a[k] = c->z[k] * (c->D[k] - Dm);
      c->b[k] = c->z[k] * (c->z[k] * c->D[k] - zm * Dm);
    }
    c->c_ip = opt ? opt->c_ip : 10.0;
    c->delta = c->c_ip * order * order / std::sqrt(diam2);
    c->mms = opt ? opt->mms : 0;
    c->phi_mg = opt ? opt->phi_mg : DGNP_PHIMG_AUTO;
    DGNP_REQUIRE(c->phi_mg >= DGNP_PHIMG_AUTO && c->phi_mg <= DGNP_PHIMG_PG, DGNP_E_ARG, "unknown phi_mg");
    if (c->phi_mg == DGNP_PHIMG_AUTO) c->phi_mg = order >= 3 ? DGNP_PHIMG_PG : DGNP_PHIMG_Q1;
    c->conc_pc = opt ? opt->conc_pc : DGNP_CPC_BILU;
    DGNP_REQUIRE(c->conc_pc == DGNP_CPC_BILU || c->conc_pc == DGNP_CPC_GMG, DGNP_E_ARG,
                 "unknown concentration preconditioner");
    c->gmg_nu = opt && opt->gmg_nu != 0 ? opt->gmg_nu : 2;
    DGNP_REQUIRE(c->gmg_nu >= 1 && c->gmg_nu <= 8, DGNP_E_ARG, "gmg_nu must be 1..8 (0: 2)");
    DGNP_REQUIRE(c->phi_mg == DGNP_PHIMG_Q1 || order >= 2, DGNP_E_ARG, "p-multigrid needs order 2 or 3");
    DGNP_REQUIRE(c->mms == 0 || c->m == 2, DGNP_E_ARG, "manufactured solutions need two ions");
    DGNP_REQUIRE(c->mms >= 0 && c->mms <= 2, DGNP_E_ARG, "unknown manufactured solution");
    c->vel = *vel;
    DGNP_REQUIRE(vel->kind >= 0 && vel->kind <= 2, DGNP_E_ARG, "unknown velocity kind");
    for (int t = 0; t < 6; ++t) {
      c->c_bc[t] = t < 2 * c->dim ? mesh->c_bc[t] : 0;
      c->phi_bc[t] = t < 2 * c->dim ? mesh->phi_bc[t] : 0;
      c->phi_val[t] = t < 2 * c->dim ? mesh->phi_val[t] : 0.0;
      DGNP_REQUIRE(c->c_bc[t] >= 0 && c->c_bc[t] <= 4, DGNP_E_ARG, "unknown concentration boundary kind");
      DGNP_REQUIRE(c->phi_bc[t] >= 0 && c->phi_bc[t] <= 1, DGNP_E_ARG, "unknown potential boundary kind");
      if (c->c_bc[t] == DGNP_C_ELECTRODE) {
        c->has_electrode = true;
        DGNP_REQUIRE(c->phi_bc[t] == DGNP_PHI_NEUMANN0, DGNP_E_ARG, "the potential is free on an electrode face");
      }
    }
    if (c->has_electrode) {
      DGNP_REQUIRE(opt && opt->electrode, DGNP_E_ARG, "electrode faces need dgnp_options.electrode");
      const dgnp_electrode& el = *opt->electrode;
      DGNP_REQUIRE(el.ion >= 1 && el.ion <= c->m, DGNP_E_ARG, "reacting ion must be 1..m");
      DGNP_REQUIRE(el.j0_profile == DGNP_J0_CONST || el.j0_profile == DGNP_J0_PARABOLIC_Z, DGNP_E_ARG,
                   "unknown exchange-current profile");
      DGNP_REQUIRE(std::isfinite(el.alpha_a) && std::isfinite(el.alpha_c), DGNP_E_NONFINITE, "non-finite exponents");
      c->bv_ion = el.ion;
      c->bv_aa = el.alpha_a;
      c->bv_ac = el.alpha_c;
      c->bv_prof = el.j0_profile;
      for (int t = 0; t < 6; ++t) {
        DGNP_REQUIRE(std::isfinite(el.j0[t]) && std::isfinite(el.phi_app[t]), DGNP_E_NONFINITE,
                     "non-finite electrode data");
        c->bv_j0[t] = el.j0[t];
        c->bv_phi_app[t] = el.phi_app[t];
      }
    }
    // the potential enters the residual through its gradient only, except on
    // potential-Dirichlet faces and in the Butler-Volmer rate of electrode
    // faces: without either it is fixed only up to a constant
    {
      bool fixed = false;
      for (int t = 0; t < 2 * c->dim; ++t)
        fixed = fixed || c->phi_bc[t] == DGNP_PHI_DIRICHLET || c->c_bc[t] == DGNP_C_ELECTRODE;
      DGNP_REQUIRE(fixed, DGNP_E_ARG,
                   "the potential is not fixed: no potential-Dirichlet or electrode face (singular problem)");
    }
    c->stream = static_cast<hipStream_t>(stream);
    DGNP_HIP(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
    c->ref = make_ref_tables(order);
    {
      RefTables all[3] = {make_ref_tables(1), make_ref_tables(2), make_ref_tables(3)};
      upload_ref_tables(all, 3);
      upload_ref_tables_jac(all, 3);
    }
    c->jac_tab = getenv("DGNP_JAC_GENERAL") == nullptr;
    c->obj_scratch = objective_scratch_init();
    build_tables(*c);
    if (opt && opt->src_vol) {
      c->src_vol.assign(opt->src_vol, opt->src_vol + size_t(c->m) * c->E * c->nqv);
      for (double v : c->src_vol) DGNP_REQUIRE(std::isfinite(v), DGNP_E_NONFINITE, "non-finite volume sources");
    }
    if (opt && opt->dir_face) {
      DGNP_REQUIRE(!c->has_electrode, DGNP_E_ARG, "caller face data and electrode faces cannot be combined");
      c->dir_face.assign(opt->dir_face, opt->dir_face + size_t(c->m) * c->n_bface * c->nqf);
      for (double v : c->dir_face) DGNP_REQUIRE(std::isfinite(v), DGNP_E_NONFINITE, "non-finite boundary data");
    } else if (c->mms == 0 && c->n_bnode > 0) {
      DGNP_REQUIRE(opt && opt->bc_conc, DGNP_E_ARG, "boundary data (bc_conc or dir_face) required");
      c->bc_conc.assign(opt->bc_conc, opt->bc_conc + size_t(c->m - 1) * c->n_bnode);
      for (double v : c->bc_conc) DGNP_REQUIRE(std::isfinite(v), DGNP_E_NONFINITE, "non-finite boundary data");
    }
    c->d_nbr.upload(c->nbr, c->stream);
    build_boundary_data(*c);
    c->d_aux.alloc(size_t(std::max<int64_t>(4 * c->E, c->m * c->n_bface * c->nqf)));
    precond_symbolic(*c);
    DGNP_HIP(hipStreamSynchronize(c->stream));
    *out = c.release();
  });
}

int dgnp_set_params(dgnp_ctx* c, const double* bc_conc, double Pe) {
  return guard([&] {
    DGNP_REQUIRE(c, DGNP_E_ARG, "NULL context");
    DGNP_REQUIRE(c->mms == 0, DGNP_E_ARG, "parameters are fixed by the manufactured solution");
    DGNP_REQUIRE(c->dir_face.empty(), DGNP_E_ARG, "parameters are fixed by the caller's face data");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(std::isfinite(Pe), DGNP_E_NONFINITE, "non-finite Pe");
    if (bc_conc && c->n_bnode > 0) {
      for (int64_t i = 0; i < (c->m - 1) * c->n_bnode; ++i)
        DGNP_REQUIRE(std::isfinite(bc_conc[i]), DGNP_E_NONFINITE, "non-finite boundary data");
      c->bc_conc.assign(bc_conc, bc_conc + size_t(c->m - 1) * c->n_bnode);
    }
    c->vel.Pe = Pe;
    DGNP_HIP(hipDeviceSynchronize());
    build_boundary_data(*c);
    c->has_state = c->has_state32 = false;
    precond_invalidate(*c);
  });
}

int dgnp_set_electrode(dgnp_ctx* c, const dgnp_electrode* e) {
  return guard([&] {
    DGNP_REQUIRE(c && e, DGNP_E_ARG, "NULL argument");
    DGNP_REQUIRE(c->has_electrode, DGNP_E_ARG, "the problem has no electrode faces");
    DGNP_REQUIRE(e->ion == c->bv_ion && e->alpha_a == c->bv_aa && e->alpha_c == c->bv_ac &&
                     e->j0_profile == c->bv_prof,
                 DGNP_E_ARG, "only the exchange currents and applied potentials can change");
    for (int t = 0; t < 6; ++t)
      DGNP_REQUIRE(std::isfinite(e->j0[t]) && std::isfinite(e->phi_app[t]), DGNP_E_NONFINITE,
                   "non-finite electrode data");
    AllocScope as(c->allocator);
    for (int t = 0; t < 6; ++t) {
      c->bv_j0[t] = e->j0[t];
      c->bv_phi_app[t] = e->phi_app[t];
    }
    DGNP_HIP(hipDeviceSynchronize());
    build_boundary_data(*c);
    c->has_state = c->has_state32 = false;
    precond_invalidate(*c);
  });
}

int dgnp_sizes(const dgnp_ctx* c, int64_t* E, int64_t* nf, int32_t* nfields, int64_t* nbn) {
  return guard([&] {
    DGNP_REQUIRE(c, DGNP_E_ARG, "NULL context");
    if (E) *E = c->E;
    if (nf) *nf = c->Nf;
    if (nfields) *nfields = c->m;
    if (nbn) *nbn = c->n_bnode;
  });
}

int dgnp_n_faces(const dgnp_ctx* c, int64_t* ni, int64_t* nbd) {
  return guard([&] {
    DGNP_REQUIRE(c, DGNP_E_ARG, "NULL context");
    if (ni) *ni = c->F;
    if (nbd) *nbd = c->n_bface;
  });
}

int dgnp_connectivity(const dgnp_ctx* c, int32_t* elem_nbr, int32_t* face_elems, int32_t* face_axis) {
  return guard([&] {
    DGNP_REQUIRE(c, DGNP_E_ARG, "NULL context");
    if (elem_nbr) std::memcpy(elem_nbr, c->nbr.data(), c->nbr.size() * sizeof(int));
    if (face_elems) std::memcpy(face_elems, c->face_elems.data(), c->face_elems.size() * sizeof(int));
    if (face_axis) std::memcpy(face_axis, c->face_axis.data(), c->face_axis.size() * sizeof(int));
  });
}

int dgnp_residual(dgnp_ctx* c, const double* x, double* r, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && x && r, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    ScopeTimer tm(*c, "residual", static_cast<hipStream_t>(stream));
    launch_dg(c->dim, c->p, c->m, false, M_RES, c->kargs(), x, nullptr, r, nullptr,
              static_cast<hipStream_t>(stream));
  });
}

int dgnp_residual_dpe(dgnp_ctx* c, const double* x, double* r, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && x && r, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    launch_dg(c->dim, c->p, c->m, false, M_DPE, c->kargs(), x, nullptr, r, nullptr,
              static_cast<hipStream_t>(stream));
  });
}

int dgnp_set_state(dgnp_ctx* c, const double* x, int32_t prec, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && x, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    const bool asm_only = (prec & DGNP_STATE_ASSEMBLE_ONLY) != 0;
    const bool apply_only = (prec & DGNP_STATE_APPLY_ONLY) != 0;
    prec &= ~(DGNP_STATE_ASSEMBLE_ONLY | DGNP_STATE_APPLY_ONLY);
    DGNP_REQUIRE(prec == DGNP_F64 || prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
    set_state(*c, x, prec, static_cast<hipStream_t>(stream), asm_only, apply_only);
  });
}

int dgnp_jacobian_apply(dgnp_ctx* c, const void* v, void* y, int32_t prec, int32_t transpose,
                        void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && v && y, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(prec == DGNP_F64 || prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
    jac_apply(*c, v, y, prec == DGNP_F32, transpose != 0, static_cast<hipStream_t>(stream));
  });
}

int dgnp_coupling_apply(dgnp_ctx* c, const void* v, void* y, int32_t prec, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && v && y, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(prec == DGNP_F64 || prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
    jac_apply(*c, v, y, prec == DGNP_F32, false, static_cast<hipStream_t>(stream), ~1u, true, nullptr);
  });
}

int dgnp_phi_apply(dgnp_ctx* c, const void* v, void* y, int32_t prec, int32_t kind, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && v && y, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(prec == DGNP_F64 || prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
    DGNP_REQUIRE(kind == DGNP_PHIOP_ASSEMBLED || kind == DGNP_PHIOP_MATFREE, DGNP_E_ARG, "unknown kind");
    phi_apply(*c, v, y, prec == DGNP_F32, kind == DGNP_PHIOP_MATFREE, static_cast<hipStream_t>(stream));
  });
}

int dgnp_precond_apply(dgnp_ctx* c, const void* r, void* z, int32_t prec, int32_t transpose,
                       int32_t pc_kind, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && r && z, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(prec == DGNP_F64 || prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
    DGNP_REQUIRE(pc_kind == DGNP_PC_P2 || pc_kind == DGNP_PC_P1, DGNP_E_ARG, "unknown preconditioner");
    precond_apply(*c, r, z, prec == DGNP_F32, transpose != 0, pc_kind, static_cast<hipStream_t>(stream));
  });
}

int dgnp_solve(dgnp_ctx* c, double* x, const dgnp_solve_opts* opts, dgnp_solve_stats* stats) {
  return guard([&] {
    DGNP_REQUIRE(c && x, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    dgnp_solve_opts o = default_solve_opts();
    if (opts) o = *opts;
    dgnp_solve_stats st{};
    DGNP_HIP(hipStreamSynchronize(c->stream));
    DGNP_HIP(hipDeviceSynchronize());
    int code = newton_solve(*c, x, o, st);
    if (stats) *stats = st;
    if (code != DGNP_OK) throw Error(code, st.status == DGNP_E_NOCONV ? "Newton did not converge"
                                                                      : "solve failed");
  });
}

int dgnp_adjoint(dgnp_ctx* c, const double* x, int32_t objective, double* dJ_dbc, double* dJ_dPe,
                 double* J_out, double* lambda, const dgnp_solve_opts* opts, dgnp_solve_stats* stats) {
  return guard([&] {
    DGNP_REQUIRE(c && x, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(objective == 0 || objective == 1, DGNP_E_ARG, "objective must be 0 or 1");
    DGNP_REQUIRE(!dJ_dbc || c->dir_face.empty(), DGNP_E_ARG,
                 "no boundary-data gradient with caller face data (dir_face): pass dJ_dbc = NULL");
    dgnp_solve_opts o = default_solve_opts();
    if (opts) o = *opts;
    dgnp_solve_stats st{};
    DGNP_HIP(hipDeviceSynchronize());
    int code = adjoint_solve(*c, x, objective, dJ_dbc, dJ_dPe, J_out, lambda, o, st);
    if (stats) *stats = st;
    if (code != DGNP_OK) throw Error(code, "adjoint solve failed");
  });
}

int dgnp_objective(dgnp_ctx* c, const double* x, int32_t objective, double* J_out) {
  return guard([&] {
    DGNP_REQUIRE(c && x && J_out, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(objective == 0 || objective == 1, DGNP_E_ARG, "objective must be 0 or 1");
    *J_out = objective_value(*c, x, objective);
  });
}

int dgnp_objective_noalloc(dgnp_ctx* c, const double* x, int32_t objective, double* J_dev, void* stream) {
  return guard([&] {
    DGNP_REQUIRE(c && x && J_dev, DGNP_E_ARG, "NULL argument");
    DGNP_REQUIRE(objective == 0 || objective == 1, DGNP_E_ARG, "objective must be 0 or 1");
    objective_noalloc(c->dim, c->p, c->m, objective_args(*c, objective), x, c->obj_scratch, J_dev,
                      static_cast<hipStream_t>(stream));
  });
}

int dgnp_electrode_gradient(dgnp_ctx* c, const double* x, int32_t objective, const double* lambda, double* dJ_dj0,
                            double* dJ_dphi_app) {
  return guard([&] {
    DGNP_REQUIRE(c && x && lambda, DGNP_E_ARG, "NULL argument");
    DGNP_REQUIRE(objective == 0 || objective == 1, DGNP_E_ARG, "objective must be 0 or 1");
    AllocScope as(c->allocator);
    electrode_gradient(*c, x, objective, lambda, dJ_dj0, dJ_dphi_app);
  });
}

int dgnp_get_block(dgnp_ctx* c, int32_t field, int64_t elem, int32_t slot, double* out) {
  return guard([&] {
    DGNP_REQUIRE(c && out, DGNP_E_ARG, "NULL argument");
    AllocScope as(c->allocator);
    DGNP_REQUIRE(field >= 0 && field < c->m && elem >= 0 && elem < c->E && slot >= 0 &&
                     slot <= 2 * c->dim,
                 DGNP_E_ARG, "block index out of range");
    get_block(*c, field, elem, slot, out);
  });
}

int dgnp_timer(dgnp_ctx* c, const char* name, double* seconds, int64_t* calls, int32_t reset) {
  return guard([&] {
    DGNP_REQUIRE(c && name, DGNP_E_ARG, "NULL argument");
    c->ev_resolve();
    auto it = c->timers.find(name);
    if (seconds) *seconds = it == c->timers.end() ? 0.0 : it->second.first;
    if (calls) *calls = it == c->timers.end() ? 0 : it->second.second;
    if (reset) c->timers.clear();
  });
}

int dgnp_profile(dgnp_ctx* c, int32_t enable) {
  return guard([&] {
    DGNP_REQUIRE(c, DGNP_E_ARG, "NULL context");
    c->ev_resolve();
    c->profiling = enable != 0;
  });
}

void dgnp_destroy(dgnp_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();  // no kernel of the context is still running when its memory goes
  delete c;
}

const char* dgnp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
