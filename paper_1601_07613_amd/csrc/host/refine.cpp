// Nonconforming refinement with the six-color child map (Section 3.2).
#include "internal.hpp"

extern "C" dgc_status dgc_mesh_refine(const dgc_mesh *parent, const uint8_t *flags, dgc_mesh **out,
                                      int64_t *n_closure) {
    (void)parent; (void)flags; (void)n_closure;
    if (out) *out = nullptr;
    return dgc::fail(DGC_E_UNSUPPORTED, "dgc_mesh_refine is not built yet");
}
