// Host-side validation of the parameter structs shared by several entry points.
#pragma once
#include <cmath>

#include "tred_internal.hpp"

static inline bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

static inline tred_status validate_grid(const tred_grid* g) {
    TRED_REQUIRE(g != nullptr, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        TRED_REQUIRE(std::isfinite(g->origin[a]), "grid.origin[%d] is not finite", a);
        TRED_REQUIRE(finite_pos(g->spacing[a]), "grid.spacing[%d] must be > 0", a);
    }
    for (int a = 0; a < 2; ++a) {
        TRED_REQUIRE(g->npix[a] > 0, "grid.npix[%d] must be > 0", a);
        TRED_REQUIRE(g->sub[a] > 0, "grid.sub[%d] must be > 0", a);
        TRED_REQUIRE((int64_t)g->npix[a] * g->sub[a] < (1 << 24), "grid is too large along %d", a);
    }
    TRED_REQUIRE(g->nticks > 0 && g->nticks < (1 << 24), "grid.nticks out of range");
    return TRED_OK;
}

static inline tred_status validate_physics(const tred_physics* p) {
    TRED_REQUIRE(p != nullptr, "physics is NULL");
    TRED_REQUIRE(finite_pos(p->v_drift), "physics.v_drift must be > 0");
    TRED_REQUIRE(finite_pos(p->lifetime), "physics.lifetime must be > 0");
    TRED_REQUIRE(std::isfinite(p->diff_T) && p->diff_T >= 0.0f, "physics.diff_T must be >= 0");
    TRED_REQUIRE(std::isfinite(p->diff_L) && p->diff_L >= 0.0f, "physics.diff_L must be >= 0");
    for (int a = 0; a < 3; ++a)
        TRED_REQUIRE(finite_pos(p->sigma_min[a]), "physics.sigma_min[%d] must be > 0", a);
    TRED_REQUIRE(finite_pos(p->n_sigma) && p->n_sigma <= 64.0f, "physics.n_sigma out of range");
    TRED_REQUIRE(std::isfinite(p->point_frac) && p->point_frac >= 0.0f,
                 "physics.point_frac must be >= 0");
    TRED_REQUIRE(p->n_gl >= 1 && p->n_gl <= 8, "physics.n_gl must be in [1, 8]");
    return TRED_OK;
}

static inline tred_status validate_blocking(const tred_blocking* b) {
    TRED_REQUIRE(b != nullptr, "blocking is NULL");
    TRED_REQUIRE(b->blk_pix[0] > 0 && b->blk_pix[1] > 0 && b->blk_ticks > 0,
                 "blocking sizes must be > 0");
    return TRED_OK;
}

#define TRED_TRY(expr)                          \
    do {                                        \
        tred_status _s = (expr);                \
        if (_s != TRED_OK) return _s;           \
    } while (0)

static inline int nblk_axis(const tred_grid* g, const tred_blocking* b, int a) {
    int nf = a == 0 ? g->npix[0] * g->sub[0] : a == 1 ? g->npix[1] * g->sub[1] : g->nticks;
    int bf = a == 0 ? b->blk_pix[0] * g->sub[0] : a == 1 ? b->blk_pix[1] * g->sub[1] : b->blk_ticks;
    return (nf + bf - 1) / bf;
}
