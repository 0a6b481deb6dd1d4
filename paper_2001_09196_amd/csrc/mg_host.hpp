// Host side of the geometric multigrid hierarchy for the thick-region
// diffusion operator (plain C++, no GPU calls): coarsening of a vertex level
// and the Galerkin stencils of the coarser levels.
//
// A level holds the active vertices of a grid of nvx x nvy x nvz vertices
// (pos: linear vertex index, increasing; slot: grid -> unknown or -1) and a
// 3^dim-point stencil per unknown (offset index o = sum_d (o_d + 1) 3^d).
// Coarsening keeps every other vertex: fine vertex x interpolates from x / 2
// (x even) or from (x - 1) / 2 and (x + 1) / 2 with weight 1/2 (x odd), per
// axis, and the coarse operator is P^T A P.  Sums run in a fixed order, so
// the hierarchy does not depend on anything but its input.
#pragma once
#include <cstddef>
#include <vector>

namespace sn {

struct MgLevelHost {
    int nvx = 1, nvy = 1, nvz = 1;
    std::vector<long> pos;
    std::vector<int> slot;
    std::vector<double> coef;   // [unknown][3^dim]
    std::vector<int> nbr;       // [unknown][3^dim] neighbour unknown or -1
    std::vector<int> chl;       // [unknown][3^dim] fine unknown at 2C + o (coarser levels) or -1
    std::vector<int> par;       // [unknown][2^dim] coarse parents or -1 (all but the last level)
    std::vector<double> pw;     // interpolation weights of the parents
};

inline void mg_coords(long p, int nx, int ny, int out[3]) {
    out[0] = (int)(p % nx);
    out[1] = (int)((p / nx) % ny);
    out[2] = (int)(p / ((long)nx * ny));
}

// stencil neighbours of a level from its slot map
inline void mg_fill_nbr(MgLevelHost& L, int dim) {
    const int ns = dim == 2 ? 9 : 27;
    const int n = (int)L.pos.size();
    L.nbr.assign((size_t)n * ns, -1);
    const int ext[3] = {L.nvx, L.nvy, L.nvz};
    for (int w = 0; w < n; ++w) {
        int cw[3];
        mg_coords(L.pos[w], L.nvx, L.nvy, cw);
        for (int o = 0; o < ns; ++o) {
            int q[3] = {cw[0], cw[1], cw[2]}, t = o;
            bool ok = true;
            for (int d = 0; d < dim; ++d) {
                q[d] += t % 3 - 1;
                t /= 3;
                if (q[d] < 0 || q[d] >= ext[d]) ok = false;
            }
            if (ok) L.nbr[(size_t)w * ns + o] = L.slot[((long)q[2] * L.nvy + q[1]) * L.nvx + q[0]];
        }
    }
}

// lv[1] holds pos, slot and coef of the finest vertex level; appends coarser
// levels until at most nmax unknowns remain (or maxl levels exist) and fills
// nbr of every level, par / pw of all but the last and chl of all but the first.
inline void mg_coarsen(std::vector<MgLevelHost>& lv, int dim, size_t nmax, int maxl) {
    const int ns = dim == 2 ? 9 : 27, nch = 1 << dim;
    mg_fill_nbr(lv[1], dim);
    while (lv.back().pos.size() > nmax && (int)lv.size() < maxl) {
        MgLevelHost cl;
        MgLevelHost& f = lv.back();
        // fine vertex x has parents up to (x + 1) / 2, so the coarse grid
        // holds vertices 0 .. nv / 2
        cl.nvx = f.nvx / 2 + 1;
        cl.nvy = f.nvy / 2 + 1;
        cl.nvz = dim == 3 ? f.nvz / 2 + 1 : 1;
        const int nf = (int)f.pos.size();
        f.par.assign((size_t)nf * nch, -1);
        f.pw.assign((size_t)nf * nch, 0.0);
        std::vector<long> pkey((size_t)nf * nch, -1);
        cl.slot.assign((size_t)cl.nvx * cl.nvy * cl.nvz, -1);
        for (int e = 0; e < nf; ++e) {
            int ce[3];
            mg_coords(f.pos[e], f.nvx, f.nvy, ce);
            int cand[3][2], nc[3];
            double cw[3][2];
            for (int d = 0; d < 3; ++d) {
                if (d >= dim || ce[d] % 2 == 0) {
                    nc[d] = 1;
                    cand[d][0] = ce[d] / 2;
                    cw[d][0] = 1.0;
                } else {
                    nc[d] = 2;
                    cand[d][0] = (ce[d] - 1) / 2;
                    cand[d][1] = (ce[d] + 1) / 2;
                    cw[d][0] = cw[d][1] = 0.5;
                }
            }
            int q = 0;
            for (int a2 = 0; a2 < nc[2]; ++a2)
                for (int a1 = 0; a1 < nc[1]; ++a1)
                    for (int a0 = 0; a0 < nc[0]; ++a0) {
                        const long key = ((long)cand[2][a2] * cl.nvy + cand[1][a1]) * cl.nvx + cand[0][a0];
                        pkey[(size_t)e * nch + q] = key;
                        f.pw[(size_t)e * nch + q] = cw[0][a0] * cw[1][a1] * cw[2][a2];
                        cl.slot[key] = 0;
                        ++q;
                    }
        }
        for (long v = 0; v < (long)cl.slot.size(); ++v)
            if (cl.slot[v] == 0) {
                cl.slot[v] = (int)cl.pos.size();
                cl.pos.push_back(v);
            }
        for (size_t e = 0; e < pkey.size(); ++e)
            if (pkey[e] >= 0) f.par[e] = cl.slot[pkey[e]];
        const int ncn = (int)cl.pos.size();
        // children of every coarse unknown: the fine unknowns at 2C + o
        cl.chl.assign((size_t)ncn * ns, -1);
        const int fext[3] = {f.nvx, f.nvy, f.nvz};
        for (int C = 0; C < ncn; ++C) {
            int cc[3];
            mg_coords(cl.pos[C], cl.nvx, cl.nvy, cc);
            for (int o = 0; o < ns; ++o) {
                int q[3] = {2 * cc[0], 2 * cc[1], 2 * cc[2]}, t = o;
                bool ok = true;
                for (int d = 0; d < dim; ++d) {
                    q[d] += t % 3 - 1;
                    t /= 3;
                    if (q[d] < 0 || q[d] >= fext[d]) ok = false;
                }
                if (ok) cl.chl[(size_t)C * ns + o] = f.slot[((long)q[2] * f.nvy + q[1]) * f.nvx + q[0]];
            }
        }
        // Galerkin stencil: row C = sum over the children f1 (weight w1) of the
        // fine row f1, each fine neighbour interpolated from its parents
        cl.coef.assign((size_t)ncn * ns, 0.0);
        for (int C = 0; C < ncn; ++C) {
            int cc[3];
            mg_coords(cl.pos[C], cl.nvx, cl.nvy, cc);
            for (int o1 = 0; o1 < ns; ++o1) {
                const int f1 = cl.chl[(size_t)C * ns + o1];
                if (f1 < 0) continue;
                double w1 = 1.0;
                for (int d = 0, t = o1; d < dim; ++d, t /= 3)
                    if (t % 3 != 1) w1 *= 0.5;
                for (int o = 0; o < ns; ++o) {
                    const double a = f.coef[(size_t)f1 * ns + o];
                    const int g2 = f.nbr[(size_t)f1 * ns + o];
                    if (g2 < 0 || a == 0.0) continue;
                    for (int q = 0; q < nch; ++q) {
                        const int D = f.par[(size_t)g2 * nch + q];
                        if (D < 0) continue;
                        int cd[3];
                        mg_coords(cl.pos[D], cl.nvx, cl.nvy, cd);
                        int idx = 0, mul = 1;
                        for (int d = 0; d < dim; ++d, mul *= 3) idx += (cd[d] - cc[d] + 1) * mul;
                        cl.coef[(size_t)C * ns + idx] += w1 * a * f.pw[(size_t)g2 * nch + q];
                    }
                }
            }
        }
        mg_fill_nbr(cl, dim);
        lv.push_back(std::move(cl));
    }
}

}  // namespace sn
