// C ABI: validation, sizes, error state.  Kernels live in the other .hip files.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <utility>

#include "common.h"

namespace tl {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }

// Profiling hook: caller events attached to one stage's kernel launch.
static thread_local hipEvent_t g_stage_ev[TL_STAGE_COUNT][2] = {};

void stage_events(int stage, hipEvent_t* start, hipEvent_t* stop) {
  hipEvent_t a = g_stage_ev[stage][0], b = g_stage_ev[stage][1];
  *start = a && b ? a : nullptr;
  *stop = a && b ? b : nullptr;
}

static bool is_int_multiple(double v, double h) {
  double q = v / h;
  return std::fabs(q - std::round(q)) < 1e-9 * std::fmax(1.0, std::fabs(q));
}

tl_status digest(const tl_system* s, Geometry* g) {
  TL_REQUIRE(s != nullptr && g != nullptr, "null system");
  std::memset(g, 0, sizeof(*g));
  TL_REQUIRE(s->mode == TL_MODE_PERIODIC || s->mode == TL_MODE_BOX, "mode must be 0 or 1");
  TL_REQUIRE(s->m0 >= 1 && s->m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", s->m0, TL_MAX_M0);
  TL_REQUIRE(s->R >= 1 && s->R <= TL_MAX_R, "R = %d outside [1, %d]", s->R, TL_MAX_R);
  TL_REQUIRE(s->h > 0 && std::isfinite(s->h), "grid step h must be positive");
  TL_REQUIRE(s->n_nuc >= 1, "at least one nucleus is required");
  TL_REQUIRE(s->nuc_pos && s->nuc_Z && s->fn_center && s->fn_l && s->fn_alpha && s->fn_coef &&
                 s->t_q && s->w_q,
             "null host array in tl_system");
  g->mode = s->mode;
  g->h = s->h;
  g->m0 = s->m0;
  g->R = s->R;
  g->box_origin0 = s->box_origin0;
  for (int d = 0; d < 3; ++d) {
    g->L[d] = s->L[d];
    g->periodic[d] = s->periodic[d] ? 1 : 0;
    g->n[d] = s->n[d];
    g->cell_nodes[d] = s->cell_nodes[d];
    g->K[d] = s->K[d];
    g->x0[d] = s->x0[d];
    g->a[d] = s->a[d];
    TL_REQUIRE(s->L[d] >= 1, "L[%d] = %d < 1", d, s->L[d]);
    TL_REQUIRE(s->n[d] >= 2 && s->n[d] <= (1 << 24), "n[%d] = %d out of range", d, s->n[d]);
    if (g->periodic[d]) {
      TL_REQUIRE(s->mode == TL_MODE_PERIODIC, "box mode needs open dimensions");
      TL_REQUIRE(s->cell_nodes[d] >= 1, "cell_nodes[%d] must be >= 1", d);
      TL_REQUIRE(is_int_multiple(s->a[d], s->h) &&
                     (int)std::lround(s->a[d] / s->h) == s->cell_nodes[d],
                 "a[%d]/h must be the integer cell_nodes[%d]", d, d);
      TL_REQUIRE((int64_t)s->L[d] * s->cell_nodes[d] == s->n[d],
                 "n[%d] must equal L*cell_nodes on a torus", d);
      TL_REQUIRE(s->K[d] >= 0 && s->K[d] <= 4096, "K[%d] out of range", d);
      TL_REQUIRE(std::fabs(s->x0[d]) == 0.0, "torus dims start at x0 = 0");
    } else {
      TL_REQUIRE(s->mode == TL_MODE_BOX || s->L[d] == 1,
                 "open dimension %d must have L = 1 in periodic mode", d);
    }
  }
  for (int mu = 0; mu < s->m0; ++mu) {
    TL_REQUIRE(s->fn_alpha[mu] > 0 && std::isfinite(s->fn_alpha[mu]), "fn_alpha[%d] <= 0", mu);
    for (int d = 0; d < 3; ++d)
      TL_REQUIRE(s->fn_l[3 * mu + d] == 0 || s->fn_l[3 * mu + d] == 1,
                 "fn_l must be 0 or 1 per dimension");
  }
  for (int q = 0; q < s->R; ++q)
    TL_REQUIRE(s->t_q[q] > 0 && std::isfinite(s->t_q[q]) && std::isfinite(s->w_q[q]),
               "quadrature node %d invalid", q);
  // groups of nuclei sharing (y, z)
  std::map<std::pair<double, double>, int> groups;
  for (int nu = 0; nu < s->n_nuc; ++nu) {
    TL_REQUIRE(std::isfinite(s->nuc_Z[nu]), "nuc_Z[%d] not finite", nu);
    groups.emplace(std::make_pair(s->nuc_pos[3 * nu + 1], s->nuc_pos[3 * nu + 2]), 0);
  }
  g->n_groups = (int)groups.size();
  if (s->mode == TL_MODE_PERIODIC) {
    TL_REQUIRE(s->n_nuc <= TL_MAX_SITES, "at most %d sites per unit cell", TL_MAX_SITES);
    for (int nu = 0; nu < s->n_nuc; ++nu)
      for (int d = 0; d < 3; ++d)
        if (g->periodic[d])
          TL_REQUIRE(is_int_multiple(s->nuc_pos[3 * nu + d], s->h),
                     "site offsets must be multiples of h in periodic dims");
  } else {
    TL_REQUIRE(g->n_groups <= 16, "box mode: at most 16 distinct (y,z) nucleus lines");
  }
  g->pot_terms = (int64_t)s->R * g->n_groups;
  for (int d = 0; d < 3; ++d) {
    g->basis_rows[d] = (s->mode == TL_MODE_BOX && d == 0) ? (int64_t)s->L[0] * s->m0 : s->m0;
    g->shifts[d] = g->periodic[d] ? s->L[d] / 2 + 1 : 1;
  }
  int64_t bo = 0, po = 0;
  for (int d = 0; d < 3; ++d) {
    g->basis_off[d] = bo;
    bo += g->basis_rows[d] * s->n[d];
    g->pot_off[d] = po;
    po += g->pot_terms * s->n[d];
  }
  g->basis_elems = bo;
  g->pot_elems = po;
  if (s->mode == TL_MODE_PERIODIC) {
    g->block_elems = (int64_t)s->L[0] * s->L[1] * s->L[2] * s->m0 * s->m0;
  } else {
    TL_REQUIRE(s->L[1] == 1 && s->L[2] == 1, "box mode is a chain along x (L = (L0,1,1))");
    int64_t nb = (int64_t)s->L[0] * s->m0;
    TL_REQUIRE(nb <= 16384, "box mode: at most 16384 basis functions");
    g->block_elems = nb * nb;
  }
  return TL_OK;
}

}  // namespace tl

extern "C" {

const char* tl_version(void) { return "tl 0.1 (gfx950)"; }

const char* tl_status_string(tl_status s) {
  switch (s) {
    case TL_OK: return "ok";
    case TL_EINVAL: return "invalid argument";
    case TL_EUNSUPPORTED: return "unsupported";
    case TL_EHIP: return "HIP runtime error";
    case TL_EWORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* tl_last_error(void) { return tl::g_err; }

tl_status tl_set_stage_events(int stage, void* start_event, void* stop_event) {
  tl::clear_error();
  TL_REQUIRE(stage >= 0 && stage < TL_STAGE_COUNT, "stage %d outside [0, %d)", stage,
             TL_STAGE_COUNT);
  TL_REQUIRE((start_event == nullptr) == (stop_event == nullptr),
             "give both events or neither");
  tl::g_stage_ev[stage][0] = (hipEvent_t)start_event;
  tl::g_stage_ev[stage][1] = (hipEvent_t)stop_event;
  return TL_OK;
}

tl_status tl_query_sizes(const tl_system* sys, tl_sizes* out) {
  tl::clear_error();
  TL_REQUIRE(out != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  for (int d = 0; d < 3; ++d) out->basis_rows[d] = g.basis_rows[d];
  out->basis_elems = g.basis_elems;
  out->pot_terms = g.pot_terms;
  out->pot_elems = g.pot_elems;
  out->block_elems = g.block_elems;
  return TL_OK;
}

}  // extern "C"
