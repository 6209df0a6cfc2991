// Host self-check of the scatterer grid and the DDA walk used on the device
// (same header): for random segments inside the box, the captures found by
// the walk with interval ownership equal the brute-force set, each once.
// With a receive cone (x_lo x_hi alpha_c), scatterers no element can hear are
// left out of the grid and the walk is clipped to a wedge around the cones:
// every capture point of a left-out scatterer must lie outside the acceptance
// cone of every element centre, every capture whose point lies inside some
// cone must be found exactly once, and the walk may report no other pair
// than a real capture of a kept scatterer (each at most once).  With a
// radius, the elements sit on a convex arc (centre of curvature (0, 0, -R),
// end elements at angles phi_lo, phi_hi, each facing along its radius).
// usage: grid_selfcheck <scat.bin> <n> <box.bin> <r_s> <n_segments> <seed>
//                       [x_lo x_hi alpha_c [radius phi_lo phi_hi]]
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <random>
#include <vector>

#include "scatter_grid.h"

using namespace ur;

int main(int argc, char **argv) {
    if (argc < 7) return 2;
    long n = std::atol(argv[2]);
    std::vector<double> S(4 * n), box(6);
    FILE *f = std::fopen(argv[1], "rb");
    if (!f || std::fread(S.data(), 8, S.size(), f) != S.size()) return 2;
    std::fclose(f);
    f = std::fopen(argv[3], "rb");
    if (!f || std::fread(box.data(), 8, 6, f) != 6) return 2;
    std::fclose(f);
    double rs = std::atof(argv[4]);
    long nseg = std::atol(argv[5]);
    const bool cull = argc >= 10;
    RxCone rx{0.0, 0.0, M_PI};
    if (cull) rx = RxCone{std::atof(argv[7]), std::atof(argv[8]), std::atof(argv[9])};
    if (argc >= 13) {
        rx.radius = std::atof(argv[10]);
        rx.phi_lo = std::atof(argv[11]);
        rx.phi_hi = std::atof(argv[12]);
    }
    ScatterGrid g = build_scatter_grid(box.data(), S.data(), n, rs, rs * 1e-5 + 1e-6, cull ? &rx : nullptr);
    std::vector<char> kept(n, 0);
    for (int i : g.items) kept[i] = 1;
    long n_kept = 0;
    for (long i = 0; i < n; ++i) n_kept += kept[i];
    if (n_kept != g.kept) { std::printf("kept count %ld != %ld\n", n_kept, g.kept); return 1; }
    if (!cull && n_kept != n) { std::printf("scatterers missing without a cull\n"); return 1; }
    // structure: every kept scatterer registered in the cell that holds its centre
    for (long i = 0; i < n; ++i) {
        if (!kept[i]) continue;
        int c[3];
        bool inside = true;
        for (int k = 0; k < 3; ++k) {
            c[k] = (int)std::floor((S[4 * i + k] - g.info.lo[k]) * g.info.inv_h);
            if (c[k] < 0 || c[k] >= g.info.n[k]) inside = false;
        }
        if (!inside) continue;
        long cell = ((long)c[2] * g.info.n[1] + c[1]) * g.info.n[0] + c[0];
        bool found = false;
        for (int j = g.cell_start[cell]; j < g.cell_start[cell + 1]; ++j) found |= g.items[j] == i;
        if (!found) { std::printf("scatterer %ld missing from its cell\n", i); return 1; }
    }
    std::mt19937_64 rng(std::atol(argv[6]));
    std::uniform_real_distribution<double> U(0, 1);
    std::normal_distribution<double> N(0, 1);
    long bad = 0, events = 0, cells = 0, tests = 0, culled_events = 0, heard_culled = 0, heard = 0;
    const int n_el = 128;
    auto heard_at = [&](const double *q) {
        for (int e = 0; e < n_el; ++e) {
            double c[3] = {rx.x_lo + (rx.x_hi - rx.x_lo) * e / (n_el - 1), 0.0, 0.0}, n[3] = {0.0, 0.0, 1.0};
            if (rx.radius > 0.0) {
                const double ph = rx.phi_lo + (rx.phi_hi - rx.phi_lo) * e / (n_el - 1);
                c[0] = rx.radius * std::sin(ph);
                c[2] = rx.radius * std::cos(ph) - rx.radius;
                n[0] = std::sin(ph);
                n[2] = std::cos(ph);
            }
            const double v[3] = {q[0] - c[0], q[1] - c[1], q[2] - c[2]};
            const double cosa = (v[0] * n[0] + v[1] * n[1] + v[2] * n[2]) / std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (cosa >= std::cos(rx.alpha_c)) return true;
        }
        return false;
    };
    for (long q = 0; q < nseg; ++q) {
        double o[3], d[3], l = 0;
        for (int k = 0; k < 3; ++k) o[k] = box[k] + (box[3 + k] - box[k]) * U(rng);
        if (q % 5 == 0) o[2] = box[2];
        for (int k = 0; k < 3; ++k) { d[k] = N(rng); l += d[k] * d[k]; }
        l = std::sqrt(l);
        for (int k = 0; k < 3; ++k) d[k] /= l;
        if (q % 11 == 0) { d[0] = 0; d[1] = 0; d[2] = 1; }
        if (q % 13 == 0) { d[0] = 1; d[1] = 0; d[2] = 0; o[2] = box[2] + 7 * g.info.h; }
        double tend = INFINITY;
        for (int k = 0; k < 3; ++k) {
            if (d[k] > 0) tend = std::fmin(tend, (box[3 + k] - o[k]) / d[k]);
            if (d[k] < 0) tend = std::fmin(tend, (box[k] - o[k]) / d[k]);
        }
        tend *= U(rng) < 0.3 ? U(rng) : 1.0;
        std::vector<int> want, must, got;   // kept captures; captures some element hears
        for (long i = 0; i < n; ++i) {
            double p[3] = {S[4 * i] - o[0], S[4 * i + 1] - o[1], S[4 * i + 2] - o[2]};
            double s = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
            if (!(s >= 0 && s < tend)) continue;
            double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
            if (!(pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2] <= rs * rs)) continue;
            const double q[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
            const bool h = cull && heard_at(q);
            heard += h;
            if (kept[i]) {
                want.push_back((int)i);
                if (!cull || h) must.push_back((int)i);
                continue;
            }
            // a left-out capture: its point must be outside every element's cone
            ++culled_events;
            heard_culled += h;
        }
        cells += dda_walk(g.info, o, d, tend, [&](int cell, double ta, double tb) {
            for (int j = g.cell_start[cell]; j < g.cell_start[cell + 1]; ++j) {
                const int i = g.items[j];
                ++tests;
                double p[3] = {S[4 * i] - o[0], S[4 * i + 1] - o[1], S[4 * i + 2] - o[2]};
                double s = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
                if (!(s >= ta && s < tb)) continue;
                double pp[3] = {p[0] - s * d[0], p[1] - s * d[1], p[2] - s * d[2]};
                if (pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2] <= rs * rs) got.push_back(i);
            }
            return true;
        });
        std::sort(want.begin(), want.end());
        std::sort(must.begin(), must.end());
        std::sort(got.begin(), got.end());
        if (std::adjacent_find(got.begin(), got.end()) != got.end()) ++bad;             // twice
        else if (!std::includes(want.begin(), want.end(), got.begin(), got.end())) ++bad;  // not a capture
        else if (!std::includes(got.begin(), got.end(), must.begin(), must.end())) ++bad;  // heard, missed
        else if (!cull && got != want) ++bad;
        events += (long)want.size();
    }
    long occupied = 0;
    for (size_t c = 0; c + 1 < g.cell_start.size(); ++c) occupied += g.cell_start[c + 1] > g.cell_start[c];
    std::printf("grid %dx%dx%d h=%.3g kept=%ld items=%zu occupied=%ld segments=%ld events=%ld culled_events=%ld "
                "heard=%ld cells/seg=%.1f tests/seg=%.1f bad=%ld heard_culled=%ld\n",
                g.info.n[0], g.info.n[1], g.info.n[2], g.info.h, n_kept, g.items.size(), occupied, nseg, events,
                culled_events, heard, (double)cells / nseg, (double)tests / nseg, bad, heard_culled);
    return bad || heard_culled ? 1 : 0;
}
