// spv_host_repair.hpp -- the host side of the hybrid comparison mode.
//
// The paper's own division of labour for the Voronoi model (Sec. II.C.3-4):
// the device tests every cell's ring each step, the flagged cells go to the
// host, the host rebuilds their rings, and the device re-tests the cells
// those repairs touched, round after round until nothing is flagged.  This
// file is that host repair: for a flagged cell i, every cell of its system
// within a radius R (from a cell list of the step's positions) is a
// candidate, and the ring is traced counter-clockwise by gift-wrapping with
// exact predicates: from the nearest candidate (always a Delaunay
// neighbour; equal distances by tag), the next member after c is the
// left-side candidate p whose circle through (i, c, p) holds no other
// left-side candidate.  The star is accepted when every new circumdisk lies
// inside the search disk (2 max |u_m| <= R, u_m the Voronoi vertices), so
// that each new triangle is empty with respect to all cells; otherwise R
// doubles.  The predicates and the cocircular tie-break are those of the
// device repair (spv_exact.hpp), so both build the same rings.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "spv_common.hpp"
#include "spv_exact.hpp"

namespace spv {

// > 0 iff p lies strictly inside the circle through (0, b, c), (0, b, c)
// counter-clockwise; a double filter, then the exact sign with the tag
// tie-break (ti, tb, tc, tp)
inline int host_incircle(double bx, double by, double cx, double cy, double px, double py, int ti, int tb, int tc,
                         int tp, double scale)
{
    const double nb = bx * bx + by * by, nc = cx * cx + cy * cy, np = px * px + py * py;
    const double t1 = cx * py, t2 = cy * px, t3 = px * by, t4 = py * bx, t5 = bx * cy, t6 = by * cx;
    const double det = nb * (t1 - t2) + nc * (t3 - t4) + np * (t5 - t6);
    const double perm = nb * (std::fabs(t1) + std::fabs(t2)) + nc * (std::fabs(t3) + std::fabs(t4)) +
                        np * (std::fabs(t5) + std::fabs(t6));
    const double bound = 2.0e-15 * perm;
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return incircle_exact_sos(bx, by, cx, cy, px, py, ti, tb, tc, tp, scale);
}

struct HostRepair {
    // cell list of the step's positions: cells[start[b] .. start[b + 1]) in global bin b
    std::vector<int> start, cells, fill;
    // candidates of the cell being repaired
    std::vector<double> dx, dy;
    std::vector<int> id;
    std::vector<int> ring;
    int64_t candidates = 0;  // gathered, over all attempts

    void build(const double* x, const double* y, const int* sys, int N, const std::vector<SysParam>& sp,
               int total_bins)
    {
        start.assign((size_t)total_bins + 1, 0);
        fill.assign((size_t)total_bins, 0);
        cells.resize((size_t)N);
        std::vector<int> bin((size_t)N);
        for (int i = 0; i < N; i++) {
            const SysParam& P = sp[sys[i]];
            const int bx = std::min((int)(x[i] / P.bsx), P.nbx - 1), by = std::min((int)(y[i] / P.bsy), P.nby - 1);
            bin[i] = P.bin_off + by * P.nbx + bx;
            start[bin[i] + 1]++;
        }
        for (int b = 0; b < total_bins; b++) start[b + 1] += start[b];
        for (int i = 0; i < N; i++) cells[start[bin[i]] + fill[bin[i]]++] = i;
    }

    // Rebuild the ring of cell i into `ring` (counter-clockwise, from the
    // smallest tag).  Returns 0, or the error bit (ERR_PRECOND: no certified
    // star below half the box; ERR_CAPACITY: longer than kc).
    unsigned repair(int i, const double* x, const double* y, const int* tag, const int* sys,
                    const std::vector<SysParam>& sp, int kc)
    {
        const SysParam& P = sp[sys[i]];
        const double xi = x[i], yi = y[i];
        const double Rmax = 0.5 * std::min(P.Lx, P.Ly) * (1.0 - 1e-9);
        double R = std::min(P.R0, Rmax);
        for (int attempt = 0; attempt < 64; attempt++) {
            gather(i, xi, yi, R, x, y, P);
            const int n = (int)id.size();
            candidates += n;
            bool closed = trace(i, tag, P.scale);
            const int k = (int)ring.size();
            if (closed && k >= 3) {
                double umax = 0.0;
                for (int m = 0; m < k; m++) {
                    const int p = ring[m], q = ring[(m + 1) % k];
                    const double bx = dx[p], by = dy[p], cx = dx[q], cy = dy[q];
                    const double nb = bx * bx + by * by, nc = cx * cx + cy * cy;
                    const double d = 2.0 * (bx * cy - by * cx);
                    const double ux = (cy * nb - by * nc) / d, uy = (bx * nc - cx * nb) / d;
                    umax = std::max(umax, std::sqrt(ux * ux + uy * uy));
                }
                if (2.0 * umax * (1.0 + 1e-9) <= R) return finish(tag, kc);
            }
            if (R >= Rmax) return ERR_PRECOND;
            R = std::min(2.0 * R, Rmax);
        }
        return ERR_REPAIR;
    }

  private:
    void gather(int i, double xi, double yi, double R, const double* x, const double* y, const SysParam& P)
    {
        dx.clear();
        dy.clear();
        id.clear();
        const int rbx = (int)std::ceil(R / P.bsx), rby = (int)std::ceil(R / P.bsy);
        int wx = 2 * rbx + 1, wy = 2 * rby + 1;
        const int cbx = std::min((int)(xi / P.bsx), P.nbx - 1), cby = std::min((int)(yi / P.bsy), P.nby - 1);
        int bx0 = cbx - rbx, by0 = cby - rby;
        if (wx >= P.nbx) {
            wx = P.nbx;
            bx0 = 0;
        }
        if (wy >= P.nby) {
            wy = P.nby;
            by0 = 0;
        }
        const double R2 = R * R * (1.0 + 1e-12);
        for (int v = 0; v < wy; v++)
            for (int u = 0; u < wx; u++) {
                const int bx = ((bx0 + u) % P.nbx + P.nbx) % P.nbx, by = ((by0 + v) % P.nby + P.nby) % P.nby;
                const int b = P.bin_off + by * P.nbx + bx;
                for (int e = start[b]; e < start[b + 1]; e++) {
                    const int q = cells[e];
                    if (q == i) continue;
                    const double ddx = mimg(x[q] - xi, P.Lx, P.hLx), ddy = mimg(y[q] - yi, P.Ly, P.hLy);
                    if (ddx * ddx + ddy * ddy <= R2) {
                        dx.push_back(ddx);
                        dy.push_back(ddy);
                        id.push_back(q);
                    }
                }
            }
    }

    // gift-wrapping over the candidates (indices into dx, dy, id); true when
    // the ring closes
    bool trace(int i, const int* tag, double scale)
    {
        ring.clear();
        const int n = (int)id.size();
        if (n < 3) return false;
        // nearest candidate: exact squared distance in grid units, ties by tag
        int start_c = -1;
        unsigned __int128 best_d2 = 0;
        for (int q = 0; q < n; q++) {
            const __int128 X = to_units(dx[q], scale), Y = to_units(dy[q], scale);
            const unsigned __int128 d2 = (unsigned __int128)(X * X + Y * Y);
            if (start_c < 0 || d2 < best_d2 || (d2 == best_d2 && tag[id[q]] < tag[id[start_c]])) {
                start_c = q;
                best_d2 = d2;
            }
        }
        ring.push_back(start_c);
        int cur = start_c;
        const int ti = tag[i];
        while ((int)ring.size() <= 64) {
            const double cx = dx[cur], cy = dy[cur];
            int nb = -1;
            for (int q = 0; q < n; q++) {
                if (q == cur) continue;
                const double px = dx[q], py = dy[q];
                if (cross_sign(cx, cy, px, py, cx * py - cy * px, scale) <= 0) continue;
                if (nb < 0 || host_incircle(cx, cy, dx[nb], dy[nb], px, py, ti, tag[id[cur]], tag[id[nb]],
                                            tag[id[q]], scale) > 0)
                    nb = q;
            }
            if (nb < 0) return false;  // open: the disk is too small
            if (nb == start_c) return true;
            ring.push_back(nb);
            cur = nb;
        }
        return false;
    }

    // rotate to start at the smallest tag and map candidates to cells
    unsigned finish(const int* tag, int kc)
    {
        const int k = (int)ring.size();
        if (k > kc) return ERR_CAPACITY;
        int mi = 0;
        for (int m = 1; m < k; m++)
            if (tag[id[ring[m]]] < tag[id[ring[mi]]]) mi = m;
        std::rotate(ring.begin(), ring.begin() + mi, ring.end());
        for (int& r : ring) r = id[r];
        return 0;
    }
};

}  // namespace spv
