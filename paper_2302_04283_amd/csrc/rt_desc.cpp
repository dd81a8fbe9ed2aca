// Checks of a grid descriptor before any table is built or any device
// memory is touched (host only).
#include <cmath>
#include <string>

#include "rt_host.h"

namespace rt {

int check_desc(const rt_grid_desc *d, std::string &err) {
    auto fail = [&err](int code, const char *msg) {
        err = msg;
        return code;
    };
    if (!d) return fail(RT_EINVAL, "desc is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return fail(RT_EINVAL, "n[a] must be >= 1");
        if (d->geo_extent[a] != 1 && d->geo_extent[a] != d->n[a])
            return fail(RT_EINVAL, "geo_extent[a] must be 1 or n[a]");
        for (int s = 0; s < 2; ++s)
            if (d->bc[a][s] != RT_BC_PERIODIC && d->bc[a][s] != RT_BC_OUTFLOW_VACUUM)
                return fail(RT_EINVAL, "unknown boundary condition");
        if ((d->bc[a][0] == RT_BC_PERIODIC) != (d->bc[a][1] == RT_BC_PERIODIC))
            return fail(RT_EINVAL, "periodic boundaries must be periodic on both sides");
        if (!d->x_faces[a] || !d->area[a] || !d->gcov_f[a] || !d->tet_f[a])
            return fail(RT_EINVAL, "missing face geometry");
    }
    if ((long long)d->n[0] * d->n[1] * d->n[2] > (1LL << 31) - 1)
        return fail(RT_EINVAL, "too many cells");
    const bool latlong = d->n_zeta > 0;
    if (latlong) {
        if (d->n_zeta < 2 || d->n_psi < 2 || (d->n_psi & 1) || d->n_zeta * d->n_psi > 512)
            return fail(RT_EINVAL, "latitude-longitude grid needs n_zeta >= 2, an even n_psi >= 2 "
                                   "and n_zeta n_psi <= 512");
    } else if (d->nlev < 1 || d->nlev > 7) {
        return fail(RT_EINVAL, "nlev must be in 1..7 (nang <= 492)");
    }
    if (d->ang_recon < 0 || d->ang_recon > 2 || (d->ang_recon == 1 && !latlong) ||
        (d->ang_recon == 2 && latlong))
        return fail(RT_EINVAL, "ang_recon must be 0, 1 (PLM, latitude-longitude grid) or 2 (MAPR, "
                               "geodesic grid)");
    const int nang = latlong ? d->n_zeta * d->n_psi : 10 * d->nlev * d->nlev + 2;
    if (d->precision != RT_F32 && d->precision != RT_F64) return fail(RT_EINVAL, "bad precision");
    if (d->recon != RT_RECON_DC && d->recon != RT_RECON_PLM) return fail(RT_EINVAL, "bad recon");
    if (d->lum_axis < 0 || d->lum_axis > 2 || d->lum_side < 0 || d->lum_side > 1)
        return fail(RT_EINVAL, "bad luminosity face");
    if (!(d->gamma_gas > 1.0) || !(d->kb_mu_mp > 0.0) || !(d->a_rad >= 0.0) || !(d->n0_crit >= 0.0))
        return fail(RT_EINVAL, "bad physical constants");
    if (!d->vol || !d->gcov_c || !d->dgcov_c || !d->tet_c || !d->dtet_c)
        return fail(RT_EINVAL, "missing cell geometry");
    const int G = d->geo_extent[0] * d->geo_extent[1] * d->geo_extent[2];
    for (int c = 0; c < G; ++c)
        if (!(d->vol[c] > 0.0)) return fail(RT_EGEOM, "cell volumes must be positive");
    if (d->beam_mask) {
        if (d->beam_angle < 0 || d->beam_angle >= nang)
            return fail(RT_EINVAL, "beam_angle out of range");
    }
    if (d->integrator < 0 || d->integrator > 2) return fail(RT_EINVAL, "integrator must be 1 or 2");
    if (!(d->tau_coeff >= 0.0) || !std::isfinite(d->tau_coeff))
        return fail(RT_EINVAL, "tau_coeff must be finite and >= 0");
    if (d->rad_velocity < 0 || d->rad_velocity > 1) return fail(RT_EINVAL, "rad_velocity must be 0 or 1");
    if (d->kernel < 0 || d->kernel > 2)
        return fail(RT_EINVAL, "kernel must be 0 (fastest), 1 (general) or 2 (column where allowed)");
    if (d->seglen < 0) return fail(RT_EINVAL, "seglen must be >= 0");
    return RT_OK;
}

}  // namespace rt
