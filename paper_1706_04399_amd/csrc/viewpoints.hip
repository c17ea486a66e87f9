// Viewpoint selection (Sect. 2.1): camera footprint, image overlap and
// working distance (eq. fov, eq. premitive, eq. cameraDistance) and a grid of
// footprint cells over each planar surface. Host code: a few thousand
// viewpoints, no device work.
#include <stdint.h>

#include <vector>

#include "dpso.h"
#include "errors.hpp"

namespace {

// floor(a / b) for b > 0
int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Whole mm nearest to half2 / 2000 um (half2 = twice a length in um), halves up.
int64_t half_um_to_mm(int64_t half2) { return floor_div(half2 + 1000, 2000); }

}  // namespace

extern "C" dpso_status dpso_viewpoints(const dpso_surface *surfaces, int32_t count, const dpso_camera *camera,
                                       int32_t *vp_mm, int32_t max_n, int32_t *n_out)
{
    using dpso::fail;
    if (!n_out || !camera || count < 0 || (count > 0 && !surfaces) || max_n < 0)
        return fail(DPSO_E_INVAL, "dpso_viewpoints: NULL argument or negative count");
    const dpso_camera &c = *camera;
    if (c.resolution_px <= 0 || c.feature_um <= 0 || c.focal_um <= 0 || c.sensor_um <= 0 ||
        c.overlap_permille < 0 || c.overlap_permille > 999)
        return fail(DPSO_E_INVAL, "camera: resolution, feature, focal length and sensor must be positive, "
                                  "overlap 0..999 permille");
    const int64_t a_um = int64_t(c.resolution_px) * c.feature_um / 2;          // eq. fov
    const int64_t p_um = (1000 - int64_t(c.overlap_permille)) * a_um / 1000;   // eq. premitive
    if (a_um > INT32_MAX) return fail(DPSO_E_RANGE, "camera footprint above 2^31 um");
    const int64_t d_um = a_um * c.focal_um / c.sensor_um;                       // eq. cameraDistance
    if (p_um < 1) return fail(DPSO_E_INVAL, "cell size below 1 um");
    int64_t total = 0;
    std::vector<int64_t> cells(2 * size_t(count));
    for (int32_t s = 0; s < count; ++s) {
        const dpso_surface &f = surfaces[s];
        if (f.normal_axis < 0 || f.normal_axis > 2 || (f.normal_sign != 1 && f.normal_sign != -1) ||
            f.lo_mm[f.normal_axis] != f.hi_mm[f.normal_axis])
            return fail(DPSO_E_INVAL, "surface %d: not a rectangle in a plane normal to an axis", s);
        for (int k = 0, m = 0; k < 3; ++k) {
            if (k == f.normal_axis) continue;
            const int64_t len = int64_t(f.hi_mm[k]) - f.lo_mm[k];
            if (len < 0) return fail(DPSO_E_INVAL, "surface %d: hi below lo on axis %d", s, k);
            const int64_t cnt = (len * 1000 + p_um - 1) / p_um;
            cells[2 * size_t(s) + m++] = cnt > 1 ? cnt : 1;
        }
        total += cells[2 * size_t(s)] * cells[2 * size_t(s) + 1];
        if (total > INT32_MAX) return fail(DPSO_E_RANGE, "more than 2^31 viewpoints");
    }
    *n_out = int32_t(total);
    if (!vp_mm) return DPSO_OK;
    if (total > max_n) return fail(DPSO_E_RANGE, "%lld viewpoints do not fit in max_n = %d", (long long)total, max_n);
    // coordinates first (range check), then the copy
    std::vector<int32_t> out(3 * size_t(total));
    size_t at = 0;
    for (int32_t s = 0; s < count; ++s) {
        const dpso_surface &f = surfaces[s];
        int ax[2], m = 0;
        for (int k = 0; k < 3; ++k)
            if (k != f.normal_axis) ax[m++] = k;
        const int64_t nrm = half_um_to_mm(2 * (int64_t(f.lo_mm[f.normal_axis]) * 1000 + f.normal_sign * d_um));
        for (int64_t i = 0; i < cells[2 * size_t(s)]; ++i)
            for (int64_t j = 0; j < cells[2 * size_t(s) + 1]; ++j) {
                int64_t v[3];
                v[f.normal_axis] = nrm;
                v[ax[0]] = half_um_to_mm(2 * int64_t(f.lo_mm[ax[0]]) * 1000 + (2 * i + 1) * p_um);
                v[ax[1]] = half_um_to_mm(2 * int64_t(f.lo_mm[ax[1]]) * 1000 + (2 * j + 1) * p_um);
                for (int k = 0; k < 3; ++k) {
                    if (v[k] < INT32_MIN || v[k] > INT32_MAX)
                        return fail(DPSO_E_RANGE, "surface %d: a viewpoint coordinate is outside int32", s);
                    out[at++] = int32_t(v[k]);
                }
            }
    }
    for (size_t k = 0; k < out.size(); ++k) vp_mm[k] = out[k];
    return DPSO_OK;
}
