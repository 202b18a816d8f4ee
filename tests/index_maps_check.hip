// Host-side check of the AA streaming index maps of the GPU kernels (the
// same header functions the kernels use), for periodic and wall axes, ragged
// and tiny grids and a row stride wider than the grid.  For each step parity:
//   * every load and store slot lies inside the run's block and in a column
//     of the grid (not in row padding);
//   * loads and stores each cover every grid slot exactly once;
//   * each node stores to the same nine slots it loads (AA: in place, no
//     node writes a slot another node reads in the same step);
//   * the value a node writes in direction a is what the next step reads as
//     f_a at x + e_a, or as f_opp(a) at x itself across a wall (Eq. 4 with
//     halfway bounce-back);
//   * the fixed-offset interior form equals the general one on nodes whose
//     neighbours all lie inside the grid, and the upwind node is in the grid;
//   * psi_coord wraps or clamps any coordinate within four grid widths;
//   * the XCD-aware work-list order is a permutation of the work list that
//     gives each of the eight XCDs one contiguous range;
//   * D3Q19 (post-collision state stored at the node, streamed as it is
//     read): the collide pass's tiles cover every node exactly once; each psi
//     neighbour offset lands on the node that psi_coord gives per axis; each
//     node's 19 reads come from the slot a of x - e_a, or from the opposite
//     slot of x across a wall, and together read every slot of the source
//     exactly once;
//   * the fused D3Q19 step's LDS planes, ring and z chunks (check_fused3);
//   * the two-component fused step's tiles, density plane and ring, and its
//     streamed reads: every source slot read exactly once (check_mc).
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include <cstdio>
#include <utility>
#include <vector>

#include "../paper_1306_6445_amd/csrc/lbm_device.hpp"
#include "../paper_1306_6445_amd/csrc/lbm3d_kernels.hpp"
#include "../paper_1306_6445_amd/csrc/lbm_mc_kernels.hpp"

using namespace lbm;

namespace {

struct Grid {
    int nx, ny, bcx, bcy, pitch;
};

int64_t load_slot(int a, int parity, int x, int y, const Nbr &n, int ld, int64_t N);
int64_t store_slot(int a, int parity, int x, int y, const Nbr &n, int ld, int64_t N);

template <int A>
int64_t load_t(int parity, int x, int y, const Nbr &n, int ld, int64_t N)
{
    return parity == 0 ? even_slot<A>(x, y, ld, N) : odd_slot<A>(x, y, n, ld, N);
}

#define DISPATCH(fn, a, ...)                                                                                  \
    switch (a) {                                                                                              \
    case 0: return fn<0>(__VA_ARGS__);                                                                        \
    case 1: return fn<1>(__VA_ARGS__);                                                                        \
    case 2: return fn<2>(__VA_ARGS__);                                                                        \
    case 3: return fn<3>(__VA_ARGS__);                                                                        \
    case 4: return fn<4>(__VA_ARGS__);                                                                        \
    case 5: return fn<5>(__VA_ARGS__);                                                                        \
    case 6: return fn<6>(__VA_ARGS__);                                                                        \
    case 7: return fn<7>(__VA_ARGS__);                                                                        \
    default: return fn<8>(__VA_ARGS__);                                                                       \
    }

int64_t load_slot(int a, int parity, int x, int y, const Nbr &n, int ld, int64_t N)
{
    DISPATCH(load_t, a, parity, x, y, n, ld, N)
}

// the kernels store f*_a where the slot of direction opp(a) is read
int64_t store_slot(int a, int parity, int x, int y, const Nbr &n, int ld, int64_t N)
{
    return load_slot(opp_of(a), parity, x, y, n, ld, N);
}

template <int A>
int64_t inner_t(int64_t idx, int ld, int64_t N)
{
    return odd_slot_inner<A>(idx, ld, N);
}
int64_t inner_slot(int a, int64_t idx, int ld, int64_t N) { DISPATCH(inner_t, a, idx, ld, N) }

template <int A>
int64_t upwind_t(int x, int y, const Nbr &n, int ld)
{
    return upwind_node<A>(x, y, n, ld);
}
int64_t upwind(int a, int x, int y, const Nbr &n, int ld) { DISPATCH(upwind_t, a, x, y, n, ld) }

int fail(const Grid &g, const char *what, int parity, int x, int y, int a)
{
    std::printf("FAIL %s: grid %dx%d bc %d%d pitch %d parity %d node (%d,%d) dir %d\n", what, g.nx, g.ny, g.bcx,
                g.bcy, g.pitch, parity, x, y, a);
    return 1;
}

int check(const Grid &g)
{
    const int ld = g.pitch;
    const int64_t N = (int64_t)ld * g.ny, total = 9 * N;
    auto in_grid = [&](int64_t s) { return s >= 0 && s < total && (s % N) % ld < g.nx; };
    for (int parity = 0; parity < 2; ++parity) {
        std::vector<int> rd(total, 0), wr(total, 0);
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                const Nbr n = neighbours(x, y, g.nx, g.ny, g.bcx, g.bcy);
                std::vector<int64_t> ls, ss;
                for (int a = 0; a < 9; ++a) {
                    const int64_t l = load_slot(a, parity, x, y, n, ld, N);
                    const int64_t s = store_slot(a, parity, x, y, n, ld, N);
                    if (!in_grid(l)) return fail(g, "load slot outside the grid", parity, x, y, a);
                    if (!in_grid(s)) return fail(g, "store slot outside the grid", parity, x, y, a);
                    ++rd[l];
                    ++wr[s];
                    ls.push_back(l);
                    ss.push_back(s);
                    // the reader of this store at the next step
                    const int ex = ex_of(a), ey = ey_of(a);
                    int tx = x + ex, ty = y + ey, ta = a;
                    const bool wall = (g.bcx == BC_WALL && (tx < 0 || tx >= g.nx)) ||
                                      (g.bcy == BC_WALL && (ty < 0 || ty >= g.ny));
                    if (wall) {
                        tx = x;
                        ty = y;
                        ta = opp_of(a);
                    } else {
                        tx = (tx % g.nx + g.nx) % g.nx;
                        ty = (ty % g.ny + g.ny) % g.ny;
                    }
                    const Nbr tn = neighbours(tx, ty, g.nx, g.ny, g.bcx, g.bcy);
                    if (load_slot(ta, parity ^ 1, tx, ty, tn, ld, N) != s)
                        return fail(g, "next step does not read what was written", parity, x, y, a);
                    const int64_t u = upwind(a, x, y, n, ld);
                    if (u < 0 || u >= N || u % ld >= g.nx) return fail(g, "upwind node outside the grid", parity, x, y, a);
                    if (parity == 1 && x >= 1 && x <= g.nx - 2 && y >= 1 && y <= g.ny - 2 &&
                        inner_slot(a, (int64_t)y * ld + x, ld, N) != l)
                        return fail(g, "interior form differs", parity, x, y, a);
                }
                for (int64_t l : ls) {
                    bool found = false;
                    for (int64_t s : ss) found |= s == l;
                    if (!found) return fail(g, "node stores outside the slots it loads", parity, x, y, -1);
                }
            }
        for (int64_t s = 0; s < total; ++s) {
            const int want = in_grid(s) ? 1 : 0;
            if (rd[s] != want || wr[s] != want) {
                const int64_t r = s % N;
                return fail(g, "slot not covered exactly once", parity, (int)(r % ld), (int)(r / ld), (int)(s / N));
            }
        }
    }
    for (int bc = 0; bc < 2; ++bc)
        for (int n : {g.nx, g.ny})
            for (int c = -4 * n; c < 5 * n; ++c) {
                const int v = psi_coord(c, n, bc);
                if (v < 0 || v >= n) return fail(g, "psi_coord out of range", c, n, bc, 0);
                if (bc == BC_PERIODIC && ((v - c) % n) != 0) return fail(g, "psi_coord is not a wrap", c, n, bc, 0);
                if (bc == BC_WALL && c >= 0 && c < n && v != c) return fail(g, "psi_coord moved an inside point", c, n, bc, 0);
            }
    return 0;
}

int check3(int nx, int ny, int nz, int bcx, int bcy, int bcz)
{
    using namespace lbm3;
    const int64_t N = (int64_t)nx * ny * nz, sxy = (int64_t)nx * ny;
    const int txs = collide3_tile_shift(nx);
    const int64_t nb = collide3_blocks(nx, ny, nz);
    std::vector<int> covered(N, 0), slots(19 * N, 0);
    auto fail = [&](const char *what, int x, int y, int z, int a) {
        std::printf("FAIL 3d %s: grid %dx%dx%d bc %d%d%d node (%d,%d,%d) dir %d\n", what, nx, ny, nz, bcx, bcy, bcz, x,
                    y, z, a);
        return 1;
    };
    for (int64_t b = 0; b < nb; ++b)
        for (unsigned t = 0; t < (unsigned)kThreads3; ++t) {
            int x, y, z;
            if (!collide3_node((unsigned)b, t, nx, ny, nz, txs, x, y, z)) continue;
            if (x < 0 || y < 0 || z < 0) return fail("negative coordinate", x, y, z, -1);
            const int64_t n = z * sxy + (int64_t)y * nx + x;
            if (covered[n]++) return fail("node covered twice", x, y, z, -1);
            const AxisNb X = axis_nb(x, nx, bcx, 1), Y = axis_nb(y, ny, bcy, nx), Z = axis_nb(z, nz, bcz, sxy);
            for (int a = 0; a < 19; ++a) {
                const int gx = psi_coord(x + ex3(a), nx, bcx), gy = psi_coord(y + ey3(a), ny, bcy),
                          gz = psi_coord(z + ez3(a), nz, bcz);
                const int64_t want_psi = gz * sxy + (int64_t)gy * nx + gx;
                const int64_t psi = n + nb_off(X, ex3(a)) + nb_off(Y, ey3(a)) + nb_off(Z, ez3(a));
                if (psi != want_psi) return fail("psi neighbour", x, y, z, a);
                // the streamed population f_a(x) comes from the upwind node
                // x - e_a (wrapped), or is the node's own f*_opp(a) across a wall
                const int ux = x - ex3(a), uy = y - ey3(a), uz = z - ez3(a);
                const bool cross = (bcx == BC_WALL && (ux < 0 || ux >= nx)) ||
                                   (bcy == BC_WALL && (uy < 0 || uy >= ny)) ||
                                   (bcz == BC_WALL && (uz < 0 || uz >= nz));
                const int64_t up = (int64_t)((uz + nz) % nz) * sxy + (int64_t)((uy + ny) % ny) * nx + (ux + nx) % nx;
                const int64_t want = cross ? (int64_t)opp3(a) * N + n : (int64_t)a * N + up;
                const int64_t got = pull_slot3(n, X, Y, Z, a, N);
                if (got != want || got < 0 || got >= 19 * N) return fail("pull slot", x, y, z, a);
                if (slots[got]++) return fail("source slot read twice", x, y, z, a);
            }
        }
    for (int64_t n = 0; n < N; ++n)
        if (covered[n] != 1) return fail("node not covered", (int)(n % nx), (int)(n / nx % ny), (int)(n / sxy), -1);
    for (int64_t i = 0; i < 19 * N; ++i)
        if (slots[i] != 1) return fail("source slot not read", (int)(i % N % nx), -1, -1, (int)(i / N));
    return 0;
}

// The fused D3Q19 step: per plane, the interior and ring cells the threads
// write cover the (TX + 2) x (TY + 2) LDS plane exactly once, each cell's
// column is the psi_coord neighbour the cell stands for, every psi an active
// node reads lies in that plane and is the psi_coord neighbour in x and y, and
// the active threads' nodes over all work items and z chunks cover the grid
// exactly once.
int check_fused3(int nx, int ny, int nz, int bcx, int bcy, int bcz, int TX, int TY, int zc)
{
    using namespace lbm3;
    const int PX = TX + 2, PY = TY + 2, PLANE = PX * PY, NT = TX * TY;
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t nb = fused3_blocks(nx, ny, nz, TX, TY, zc);
    std::vector<int> covered(N, 0);
    auto fail = [&](const char *what, int64_t b, int t) {
        std::printf("FAIL fused3 %s: grid %dx%dx%d bc %d%d%d tile %dx%d zc %d block %lld thread %d\n", what, nx, ny,
                    nz, bcx, bcy, bcz, TX, TY, zc, (long long)b, t);
        return 1;
    };
    for (int64_t b = 0; b < nb; ++b) {
        std::vector<int> writes(PLANE, 0);
        std::vector<int64_t> colof(PLANE, -1);
        std::vector<Fused3Thread> th(NT);
        for (int t = 0; t < NT; ++t) {
            const Fused3Thread q = fused3_thread((unsigned)b, t, nx, ny, nz, bcx, bcy, zc, TX, TY);
            th[t] = q;
            if (q.cell < 0 || q.cell >= PLANE) return fail("cell out of the plane", b, t);
            ++writes[q.cell];
            colof[q.cell] = q.col;
            if (q.ring) {
                if (q.rcell < 0 || q.rcell >= PLANE) return fail("ring cell out of the plane", b, t);
                ++writes[q.rcell];
                colof[q.rcell] = q.rcol;
            }
            if (q.col < 0 || q.col >= (int64_t)nx * ny || (q.ring && (q.rcol < 0 || q.rcol >= (int64_t)nx * ny)))
                return fail("column out of the grid", b, t);
            // the gathers use the column's own coordinates for their neighbour offsets
            if (q.cx != psi_coord(q.x, nx, bcx) || q.cy != psi_coord(q.y, ny, bcy) || q.col != (int64_t)q.cy * nx + q.cx)
                return fail("column coordinates", b, t);
            if (q.ring && (q.rcx < 0 || q.rcx >= nx || q.rcy < 0 || q.rcy >= ny || q.rcol != (int64_t)q.rcy * nx + q.rcx))
                return fail("ring column coordinates", b, t);
            if (q.z0 < 0 || q.z1 > nz || q.z0 >= q.z1) return fail("empty or out-of-grid z chunk", b, t);
        }
        for (int c = 0; c < PLANE; ++c)
            if (writes[c] != 1) return fail("LDS cell not written exactly once", b, c);
        for (int t = 0; t < NT; ++t) {
            const Fused3Thread &q = th[t];
            if (!q.active) continue;
            for (int z = q.z0; z < q.z1; ++z) {
                const int64_t n = (int64_t)z * nx * ny + (int64_t)q.y * nx + q.x;
                if (covered[n]++) return fail("node collided twice", b, t);
            }
            if (q.col != (int64_t)q.y * nx + q.x) return fail("active node reads another column", b, t);
            for (int a = 1; a < 19; ++a) {
                const int c = q.cell + ey3(a) * PX + ex3(a);
                if (c < 0 || c >= PLANE) return fail("psi read outside the plane", b, t);
                const int64_t want = (int64_t)psi_coord(q.y + ey3(a), ny, bcy) * nx + psi_coord(q.x + ex3(a), nx, bcx);
                if (colof[c] != want) return fail("psi read from the wrong column", b, t);
            }
        }
        (void)bcz;
    }
    for (int64_t n = 0; n < N; ++n)
        if (covered[n] != 1) return fail("node not collided", -1, (int)n);
    return 0;
}

// The two-component fused step: every tile shape's work items cover the grid
// once; the own cells (rows threads ty apart) and the ring entries write each
// cell of the (tx + 2) x (rows ty + 2) density plane exactly once; every
// neighbour cell an active node reads lies in the plane and holds the
// psi_coord neighbour's column.
int check_mc(int nx, int ny, int bcx, int bcy, int tx, int ty, int rows)
{
    const int LX = tx + 2, LY = rows * ty + 2, nring = 2 * LX + 2 * (LY - 2);
    const int64_t nt = lbmmc::mc_tiles(nx, ny, tx, ty, rows);
    std::vector<int> covered((size_t)nx * ny, 0);
    auto fail = [&](const char *what, int64_t b) {
        std::printf("FAIL mc %s: grid %dx%d bc %d%d tile %dx%d rows %d item %lld\n", what, nx, ny, bcx, bcy, tx, ty,
                    rows, (long long)b);
        return 1;
    };
    for (int64_t b = 0; b < nt; ++b) {
        int x0, y0;
        lbmmc::mc_tile_origin((int)b, nx, tx, ty, rows, x0, y0);
        std::vector<int> writes(LX * LY, 0);
        std::vector<int64_t> colof(LX * LY, -1);
        for (int ly = 0; ly < ty; ++ly)
            for (int lx = 0; lx < tx; ++lx)
                for (int j = 0; j < rows; ++j) {
                    const int x = x0 + lx, y = y0 + ly + j * ty, c = (ly + j * ty + 1) * LX + lx + 1;
                    ++writes[c];
                    colof[c] = (int64_t)psi_coord(y, ny, bcy) * nx + psi_coord(x, nx, bcx);
                }
        for (int k = 0; k < nring; ++k) {
            int lx, ly;
            lbmmc::mc_ring_cell(k, LX, LY, lx, ly);
            if (lx < 0 || lx >= LX || ly < 0 || ly >= LY) return fail("ring cell outside the plane", b);
            ++writes[ly * LX + lx];
            colof[ly * LX + lx] = (int64_t)psi_coord(y0 - 1 + ly, ny, bcy) * nx + psi_coord(x0 - 1 + lx, nx, bcx);
        }
        for (int c = 0; c < LX * LY; ++c)
            if (writes[c] != 1) return fail("plane cell not written exactly once", b);
        for (int ly = 0; ly < ty; ++ly)
            for (int lx = 0; lx < tx; ++lx)
                for (int j = 0; j < rows; ++j) {
                    const int x = x0 + lx, y = y0 + ly + j * ty;
                    if (x >= nx || y >= ny) continue;
                    if (covered[(size_t)y * nx + x]++) return fail("node collided twice", b);
                    const int c = (ly + j * ty + 1) * LX + lx + 1;
                    for (int a = 1; a < 9; ++a) {
                        const int cn = c + ey_of(a) * LX + ex_of(a);
                        const int64_t want =
                            (int64_t)psi_coord(y + ey_of(a), ny, bcy) * nx + psi_coord(x + ex_of(a), nx, bcx);
                        if (cn < 0 || cn >= LX * LY || colof[cn] != want) return fail("neighbour cell", b);
                    }
                }
    }
    for (size_t n = 0; n < covered.size(); ++n)
        if (covered[n] != 1) return fail("node not collided", -1);
    // the streamed read (pull_slot2): f_a(x) from slot a of the upwind node
    // x - e_a (wrapped), or the node's own slot opp(a) across a wall; the
    // nodes' reads take every slot of the source exactly once
    const int64_t N = (int64_t)nx * ny;
    std::vector<int> slots((size_t)(9 * N), 0);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const lbm3::AxisNb X = lbm3::axis_nb(x, nx, bcx, 1), Y = lbm3::axis_nb(y, ny, bcy, nx);
            const int64_t n = (int64_t)y * nx + x;
            for (int a = 0; a < 9; ++a) {
                const int ux = x - ex_of(a), uy = y - ey_of(a);
                const bool cross = (bcx == BC_WALL && (ux < 0 || ux >= nx)) || (bcy == BC_WALL && (uy < 0 || uy >= ny));
                const int64_t up = (int64_t)((uy + ny) % ny) * nx + (ux + nx) % nx;
                const int64_t want = cross ? (int64_t)opp_of(a) * N + n : (int64_t)a * N + up;
                const int64_t got = lbmmc::pull_slot2(n, X, Y, a, N);
                if (got != want || got < 0 || got >= 9 * N) return fail("pull slot", n);
                if (slots[(size_t)got]++) return fail("source slot read twice", n);
            }
        }
    for (size_t i = 0; i < slots.size(); ++i)
        if (slots[i] != 1) return fail("source slot not read", (int64_t)i);
    return 0;
}

}  // namespace

int main()
{
    const int sizes[][2] = {{1, 1}, {1, 5}, {2, 3}, {3, 3}, {5, 1}, {8, 8}, {17, 12}, {64, 4}, {33, 70}, {130, 9}};
    int grids = 0;
    for (const auto &sz : sizes)
        for (int bcx = 0; bcx < 2; ++bcx)
            for (int bcy = 0; bcy < 2; ++bcy)
                for (int pad : {0, 3}) {
                    const Grid g{sz[0], sz[1], bcx, bcy, sz[0] + pad};
                    if (check(g)) return 1;
                    ++grids;
                }
    for (int n = 1; n <= 1000; ++n)
        for (int xcd = 0; xcd < 2; ++xcd) {
            std::vector<int> seen(n, 0), lo(kNumXcd, n), hi(kNumXcd, -1), cnt(kNumXcd, 0);
            for (int b = 0; b < n; ++b) {
                const int t = work_index_of(b, n, xcd);
                if (t < 0 || t >= n || seen[t]++) {
                    std::printf("FAIL work_index_of: n %d xcd %d block %d -> %d\n", n, xcd, b, t);
                    return 1;
                }
                const int k = b % kNumXcd;
                lo[k] = t < lo[k] ? t : lo[k];
                hi[k] = t > hi[k] ? t : hi[k];
                ++cnt[k];
            }
            for (int k = 0; k < kNumXcd && xcd; ++k)
                if (cnt[k] && hi[k] - lo[k] + 1 != cnt[k]) {
                    std::printf("FAIL work_index_of: n %d, XCD %d's range is not contiguous\n", n, k);
                    return 1;
                }
        }
    const int sizes3[][3] = {{1, 1, 1}, {1, 2, 3}, {3, 3, 3}, {5, 4, 3}, {17, 6, 5}, {16, 16, 2},
                             {33, 7, 3}, {64, 3, 2}, {130, 5, 3}, {256, 2, 2}, {300, 3, 2}};
    int grids3 = 0;
    for (const auto &sz : sizes3)
        for (int bc = 0; bc < 8; ++bc) {
            if (check3(sz[0], sz[1], sz[2], bc & 1, (bc >> 1) & 1, (bc >> 2) & 1)) return 1;
            ++grids3;
        }
    int fused3 = 0;
    for (const auto &sz : sizes3)
        for (int bc = 0; bc < 8; ++bc)
            for (const auto &tile : {std::pair<int, int>(32, 8), {32, 16}, {64, 4}, {64, 8}, {64, 16}})
                for (int zc : {1, 3, 32}) {
                    if (!lbm3::fused3_shape_ok(tile.first, tile.second)) return 1;
                    if (check_fused3(sz[0], sz[1], sz[2], bc & 1, (bc >> 1) & 1, (bc >> 2) & 1, tile.first,
                                     tile.second, zc))
                        return 1;
                    ++fused3;
                }
    int mc = 0;
    const int sizes_mc[][2] = {{1, 1}, {1, 5}, {3, 3}, {7, 2}, {33, 9}, {64, 8}, {65, 17}, {130, 9}, {300, 5}};
    for (const auto &sz : sizes_mc)
        for (int bc = 0; bc < 4; ++bc)
            for (int tx : {32, 64, 128, 256})
                for (int ty : {1, 2, 4, 8})
                    for (int rows : {1, 2, 4}) {
                        if (!lbmmc::mc_shape_ok(tx, ty, rows)) continue;
                        if (check_mc(sz[0], sz[1], bc & 1, bc >> 1, tx, ty, rows)) return 1;
                        ++mc;
                    }
    std::printf("ok: %d grids, %d 3d grids, %d fused 3d layouts, %d two-component layouts\n", grids, grids3, fused3,
                mc);
    return 0;
}
