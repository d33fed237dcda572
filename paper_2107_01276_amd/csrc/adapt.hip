// Adaptive refinement on gfx950 (section 3): background m_ref lookup,
// split, mutual-closest merge, shifting with Taylor correction, h update,
// and the background-particle update.
#include "sph_device.h"

int mref_lookup_run(sph_ctx* c, const sph_particles*, const sph_background*)
{
    set_err(c, "mref lookup not available in this build");
    return SPH_E_INVAL;
}

int adapt_run(sph_ctx* c, sph_particles*, const sph_background*, sph_adapt_map*)
{
    set_err(c, "adaptation not available in this build");
    return SPH_E_INVAL;
}

int bg_update_run(sph_ctx* c, sph_background*, const sph_particles*, const double*, double, int,
                  int64_t*)
{
    set_err(c, "background update not available in this build");
    return SPH_E_INVAL;
}
