// Module compatibility map (host, FP64), built once per geometry.
//
// Sec. 2.1 of the paper restricts the modules a reference module can be
// linked to: those reachable by helices of both charges at the threshold
// p_T from the centre of the detector.  Here module B on the next logical
// layer is compatible with module A when
//   azimuth  |phi_B - phi_A| <= dphi_A + dphi_B
//                               + W (asin(rmax_B kh) - asin(rmin_A kh)) + margin,
//            i.e. the two azimuth ranges overlap once widened by the turning
//            angle of a threshold helix between the two radii, and
//   r-z      some straight line (in arc length) from the luminous region
//            |z0| <= W Z0MAX through a corner of A reaches B: extrapolated to
//            B's radii (barrel) or B's disk plane (endcap), with the
//            arc-over-chord factor q_B = asin(rmax_B kh)/(rmax_B kh) as slack
//            and a length margin.
// Every quantity is FP64 from the FP32 module table; the rows are sorted by
// module index.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace lst {

namespace {

struct ModInfo {
    double rmin, rmax, zmin, zmax, phi, dphi;
    double asin_lo, asin_hi, q;
    int layer, barrel, side;
};

struct MapPar {
    double w, z0m, dphi_margin, len_margin;
};

// logical layers a track can reach next: barrel l -> l+1 and the first disk
// of either side; disks -> the next disk of the same side
int successors(int layer, int out[3])
{
    int n = 0;
    if (layer >= 1 && layer <= 6) {
        if (layer < 6) out[n++] = layer + 1;
        out[n++] = 7;
        out[n++] = 12;
    } else if ((layer >= 7 && layer <= 10) || (layer >= 12 && layer <= 15)) {
        out[n++] = layer + 1;
    }
    return n;
}

bool azimuth_ok(const ModInfo &A, const ModInfo &B, const MapPar &p)
{
    double turn = (B.asin_hi - A.asin_lo) * p.w;
    double d = B.phi - A.phi;
    if (d > M_PI) d -= 2.0 * M_PI;
    if (d < -M_PI) d += 2.0 * M_PI;
    return std::fabs(d) <= ((A.dphi + B.dphi) + turn) + p.dphi_margin;
}

bool rz_ok(const ModInfo &A, const ModInfo &B, const MapPar &p)
{
    if (B.barrel) {
        // z reached at B's radii: z0 + (z - z0) t, t = r_B / r_A (times q_B at most)
        const double t_lo = B.rmin / A.rmax;
        const double t_hi = (B.rmax / A.rmin) * B.q;
        double lo = INFINITY, hi = -INFINITY;
        const double v0[2] = {-p.z0m, p.z0m};
        const double va[2] = {A.zmin, A.zmax};
        const double vt[2] = {t_lo, t_hi};
        for (double z0 : v0)
            for (double za : va)
                for (double t : vt) {
                    double z = z0 + (za - z0) * t;
                    lo = std::min(lo, z);
                    hi = std::max(hi, z);
                }
        return (B.zmin <= hi + p.len_margin) && (B.zmax >= lo - p.len_margin);
    }
    // endcap B: radius reached on B's plane, mirrored to positive z
    const double za_lo = (B.side > 0) ? A.zmin : -A.zmax;
    const double za_hi = (B.side > 0) ? A.zmax : -A.zmin;
    const double zd = std::fabs(B.zmin);
    if (za_hi + p.z0m <= 0.0) return false;  // every line leaves towards the other side
    const double r_lo = ((A.rmin * (zd + p.z0m)) / (za_hi + p.z0m)) / B.q;
    double r_hi = INFINITY;                   // lines nearly parallel to the disk
    if (za_lo - p.z0m > 0.0) r_hi = (A.rmax * (zd - p.z0m)) / (za_lo - p.z0m);
    return (B.rmin <= r_hi + p.len_margin) && (B.rmax >= r_lo - p.len_margin);
}

}  // namespace

// f32: [21][n] module table, i32: [4][n]; params: primary parameter vector.
void build_module_map(int n, const float *f32, const int32_t *i32, const double *params,
                      std::vector<int32_t> &row_ptr, std::vector<int32_t> &col)
{
    const double kmax = (0.0029979245800 * params[0]) / params[1];
    const double kh = 0.5 * kmax * (1.0 + params[6]);
    MapPar p;
    p.w = params[11];
    p.z0m = params[2] * p.w;
    p.dphi_margin = params[12];
    p.len_margin = params[13];

    std::vector<ModInfo> info(n);
    std::vector<std::vector<int>> by_layer(17);
    for (int m = 0; m < n; ++m) {
        ModInfo &x = info[m];
        x.rmin = f32[15 * n + m];
        x.rmax = f32[16 * n + m];
        x.zmin = f32[17 * n + m];
        x.zmax = f32[18 * n + m];
        x.phi = f32[19 * n + m];
        x.dphi = f32[20 * n + m];
        x.layer = i32[m];
        x.barrel = i32[n + m] == 0;
        x.side = i32[2 * n + m];
        const double slo = std::min(x.rmin * kh, 1.0);
        const double shi = std::min(x.rmax * kh, 1.0);
        x.asin_lo = std::asin(slo);
        x.asin_hi = std::asin(shi);
        x.q = (shi > 0.0) ? x.asin_hi / shi : 1.0;
        if (x.layer >= 1 && x.layer <= 16) by_layer[x.layer].push_back(m);
    }
    row_ptr.assign(n + 1, 0);
    col.clear();
    std::vector<int32_t> row;
    for (int a = 0; a < n; ++a) {
        row.clear();
        int nxt[3];
        const int nn = successors(info[a].layer, nxt);
        for (int t = 0; t < nn; ++t) {
            for (int b : by_layer[nxt[t]]) {
                const ModInfo &A = info[a], &B = info[b];
                if (B.rmax <= A.rmin) continue;  // radius must grow along the track
                if (!azimuth_ok(A, B, p)) continue;
                if (!rz_ok(A, B, p)) continue;
                row.push_back(b);
            }
        }
        std::sort(row.begin(), row.end());
        col.insert(col.end(), row.begin(), row.end());
        row_ptr[a + 1] = (int32_t)col.size();
    }
}

}  // namespace lst
