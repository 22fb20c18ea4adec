// gf_kernels.hip -- region bodies, the persistent program kernel, the
// per-region kernel with in-kernel reduction finalize, gf_reduce and the
// bandwidth probe. gfx950 only; built with -ffp-contract=off so every
// elementwise value is rounded exactly as the legacy loop writes it.
#include <type_traits>
#include "gf_device.h"

namespace gf {

constexpr int kMaxWg = 256;         // workgroup size limit of the region kernels
constexpr int kMaxWgHist = 1024;    // histogram kernels (one 128 KiB workgroup per CU)
constexpr int kLdsRed = kMaxWgHist / kWave;
constexpr int kHistPart = 65536;    // bins counted per workgroup pass (16-bit counters, 128 KiB of LDS)

// ---------------------------------------------------------------------------
// Work decomposition shared by host and device.
// ---------------------------------------------------------------------------

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct StencilGeom {
    int64_t nxc, nyt, nzs;  // x chunks, y tiles, z segments
};

__host__ __device__ inline StencilGeom j3_geom(int64_t n, const Tiling &t)
{
    StencilGeom g;
    const int64_t interior = n > 2 ? n - 2 : 0;
    g.nxc = cdiv(n, t.wg_size);
    g.nyt = cdiv(interior, t.tile_y);
    g.nzs = cdiv(interior, t.tile_z);
    return g;
}

typedef double gf_d2 __attribute__((ext_vector_type(2)));

__host__ __device__ inline StencilGeom j3v2_geom(int64_t n, const Tiling &t)
{
    StencilGeom g = j3_geom(n, t);
    g.nxc = cdiv(n, 2 * (int64_t)t.wg_size);
    return g;
}

// 2D: a work item is a chunk of columns (two per thread for even n, one for
// odd n) times a segment of tile_y rows that the workgroup marches through.
__host__ __device__ inline StencilGeom j2_geom(int64_t n, const Tiling &t)
{
    StencilGeom g;
    const int64_t interior = n > 2 ? n - 2 : 0;
    g.nxc = cdiv(n, 2 * (int64_t)t.wg_size);  // two columns per thread
    g.nyt = cdiv(interior, t.tile_y);
    g.nzs = 1;
    return g;
}

__host__ __device__ inline int64_t chunk_elems(const Tiling &t) { return (int64_t)t.wg_size * t.items; }

// SpMV rows per work item: half the workgroup, so a block of a stencil-like
// matrix (<= 30 nonzeros per row) fits the LDS product tile.
__host__ __device__ inline int64_t spmv_rows(const Tiling &t) { return t.wg_size / 2; }

// Histogram work: chunks of wg_size * items * 4 keys (each thread reads
// `items` 16-byte groups of four keys); every chunk is counted once per part
// of kHistPart bins, and item = chunk * parts + part.
struct HistGeom {
    int64_t nbins, parts, chunk_keys, nchunks, nitems;
};

__host__ __device__ inline HistGeom hist_geom(int64_t n, uint32_t mask, const Tiling &t)
{
    HistGeom g;
    g.nbins = (int64_t)mask + 1;
    g.parts = cdiv(g.nbins, kHistPart);
    g.chunk_keys = (int64_t)t.wg_size * t.items * 4;
    g.nchunks = cdiv(n, g.chunk_keys);
    g.nitems = g.nchunks * g.parts;
    return g;
}

int64_t region_items(const DStep &st, int64_t n, const Tiling &t)
{
    switch (st.kind) {
    case GF_R_JACOBI3D: {
        StencilGeom g = (n & 1) ? j3_geom(n, t) : j3v2_geom(n, t);
        return g.nxc * g.nyt * g.nzs;
    }
    case GF_R_JACOBI2D: {
        StencilGeom g = j2_geom(n, t);
        return g.nxc * g.nyt;
    }
    case GF_R_SPMV:
        return cdiv(n, spmv_rows(t));
    case GF_R_DOT:
    case GF_R_AXPBY:
        return cdiv(n, chunk_elems(t));
    case GF_R_HIST:
        return hist_geom(n, st.mask, t).nitems;
    case GF_R_OWNER:
        return 0;  // thread-level static schedule, no tiles
    default:
        return 0;
    }
}

__device__ inline int64_t region_items_dev(const DStep &st, int64_t n, const Tiling &t)
{
    switch (st.kind) {
    case GF_R_JACOBI3D: {
        StencilGeom g = (n & 1) ? j3_geom(n, t) : j3v2_geom(n, t);
        return g.nxc * g.nyt * g.nzs;
    }
    case GF_R_JACOBI2D: {
        StencilGeom g = j2_geom(n, t);
        return g.nxc * g.nyt;
    }
    case GF_R_SPMV:
        return cdiv(n, spmv_rows(t));
    case GF_R_DOT:
    case GF_R_AXPBY:
        return cdiv(n, chunk_elems(t));
    case GF_R_HIST:
        return hist_geom(n, st.mask, t).nitems;
    default:
        return 0;
    }
}

// ---------------------------------------------------------------------------
// Region bodies. Each processes one work item with the whole workgroup and
// returns the thread's private reduction value (identity if none).
// ---------------------------------------------------------------------------

// 3D 7-point Jacobi, 2.5-D blocking: the workgroup owns a (row chunk of
// wg_size x) x (TY rows) column of the grid and marches along z over one
// segment. Each thread keeps its column of planes z-1, z, z+1 in registers,
// so every value of u is fetched from memory once per tile plus the two
// y-halo rows and two z-halo planes; x neighbours are re-read from L1.
template <int TY>
__device__ __forceinline__ double j3_item(const double *u_, double *w_, int64_t n, int64_t item, const Tiling &t,
                                          bool want_red)
{
    GF_GLOBAL const double *__restrict__ u = gptr(u_);
    GF_GLOBAL double *__restrict__ w = gptr(w_);
    const StencilGeom g = j3_geom(n, t);
    const int64_t xc = item % g.nxc;
    const int64_t rest = item / g.nxc;
    const int64_t yt = rest % g.nyt;
    const int64_t zs = rest / g.nyt;
    const int64_t x = xc * blockDim.x + threadIdx.x;
    const int64_t y0 = 1 + yt * TY;
    const int ny = (int)(n - 1 - y0 < TY ? n - 1 - y0 : TY);
    const int64_t z0 = 1 + zs * t.tile_z;
    const int64_t z1 = (z0 + t.tile_z < n - 1) ? z0 + t.tile_z : n - 1;
    const bool xload = x < n;
    const bool xin = x >= 1 && x <= n - 2;
    const int64_t SY = n, SZ = n * n;
    const double c6 = 1.0 / 6.0;
    double mx = -INFINITY;
    double pm[TY], pc[TY + 2], pn[TY + 2];
#pragma unroll
    for (int r = 0; r < TY; ++r)
        pm[r] = 0.0;
#pragma unroll
    for (int r = 0; r < TY + 2; ++r)
        pc[r] = pn[r] = 0.0;
    if (xload) {
        GF_GLOBAL const double *b = u + (z0 - 1) * SZ + y0 * SY + x;
#pragma unroll
        for (int r = 0; r < TY; ++r)
            if (r < ny)
                pm[r] = b[r * SY];
        b = u + z0 * SZ + (y0 - 1) * SY + x;
#pragma unroll
        for (int r = 0; r < TY + 2; ++r)
            if (r < ny + 2)
                pc[r] = b[r * SY];
    }
    for (int64_t z = z0; z < z1; ++z) {
        if (xload) {
            GF_GLOBAL const double *b = u + (z + 1) * SZ + (y0 - 1) * SY + x;
#pragma unroll
            for (int r = 0; r < TY + 2; ++r)
                if (r < ny + 2)
                    pn[r] = b[r * SY];
        }
        if (xin) {
            GF_GLOBAL const double *row = u + z * SZ + y0 * SY + x;
            GF_GLOBAL double *out = w + z * SZ + y0 * SY + x;
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (r < ny) {
                    const double xl = row[r * SY - 1];
                    const double xr = row[r * SY + 1];
                    const double v = (((xl + xr) + (pc[r] + pc[r + 2])) + (pm[r] + pn[r + 1])) * c6;
                    __builtin_nontemporal_store(v, out + r * SY);
                    if (want_red) {
                        const double d = fabs(v - pc[r + 1]);
                        mx = d > mx ? d : mx;
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < TY; ++r)
            pm[r] = pc[r + 1];
#pragma unroll
        for (int r = 0; r < TY + 2; ++r)
            pc[r] = pn[r];
    }
    return mx;
}

// Lane shifts across the whole wavefront (DPP wave_shr:1 / wave_shl:1):
// lane i receives lane i-1's (shr) or lane i+1's (shl) value; the lane at
// the wavefront edge receives 0 and is fixed up by the caller.
__device__ __forceinline__ double wave_shr1(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_shl1(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// 3D 7-point Jacobi for even n: each thread owns an x-pair (one 16-byte load
// per row), a column of TY rows, and marches z. x-neighbours come from the
// adjacent lanes by DPP shifts; the edge lanes of each wavefront swap their
// values through LDS once per plane (which also keeps the workgroup's
// wavefronts in step), and only the workgroup's outermost lanes re-read a
// neighbour from cache when the row spans several workgroups. y-neighbours
// come from the thread's own rows plus two halo rows, z-neighbours from the
// register planes. Plane z+2 is requested before plane z is computed.
// Rows that no neighbouring tile reads again (the tile's inner rows) are
// loaded with the streaming hint so they do not evict the halo rows that the
// adjacent tile is about to read. FULL tiles (all TY rows present) run
// without per-row guards; lanes past the row end load a clamped in-bounds
// address and store nothing.
template <int TY>
__device__ __forceinline__ gf_d2 ld_row(GF_GLOBAL const double *p, int r)
{
    // r indexes rows y0-1 .. y0+TY; rows y0-1, y0, y0+TY-1, y0+TY are shared
    if (r >= 2 && r <= TY - 1)
        return __builtin_nontemporal_load((GF_GLOBAL const gf_d2 *)p);
    return *(GF_GLOBAL const gf_d2 *)p;
}

// One tile of planes [z0, z1). PF (1 or 2) planes ahead of the computed
// plane z are in flight: registers hold planes z-1 (own rows), z, z+1 and,
// for PF = 2, z+2, while the next plane is requested at the top of the step.
// The two depths are written out separately: folding them into one ring
// array cost a fifth of the bandwidth at depth 1 (measured).
template <int TY, int PF, bool FULL>
__device__ __forceinline__ double j3v2_tile(GF_GLOBAL const double *__restrict__ u, GF_GLOBAL double *__restrict__ w,
                                            int64_t n, int64_t x, int64_t y0, int ny, int64_t z0, int64_t z1,
                                            bool want_red)
{
    static_assert(PF == 1 || PF == 2, "prefetch depth 1 or 2");
    __shared__ double s_edge[2][kMaxWg / kWave][TY][2];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const bool xload = x < n;
    const int64_t xs = xload ? x : n - 2;          // clamped load column (even, in bounds)
    const bool in0 = xload && x >= 1;              // column x is interior (x <= n-2 as x is even)
    const bool in1 = xload && x + 1 <= n - 2;      // column x+1 is interior
    const bool gather_l = wv == 0 && lane == 0 && xs >= 1;
    const bool gather_r = wv == nw - 1 && lane == kWave - 1 && xs + 2 <= n - 1;
    const int64_t SY = n, SZ = n * n;
    const double c6 = 1.0 / 6.0;
    double mx = -INFINITY;
    // pm: plane z-1 (own rows); pc: plane z; pn: plane z+1; pa: z+2 (PF = 2);
    // pf: the plane being requested (z+1+PF)
    gf_d2 pm[TY], pc[TY + 2], pn[TY + 2], pa[PF == 2 ? TY + 2 : 1], pf[TY + 2];
    const gf_d2 zero2 = {0.0, 0.0};
    GF_GLOBAL const double *col = u + (y0 - 1) * SY + xs;  // row y0-1 of plane 0
#pragma unroll
    for (int r = 0; r < TY; ++r)
        pm[r] = (FULL || r < ny) ? ld_row<TY>(col + (z0 - 1) * SZ + (r + 1) * SY, r + 1) : zero2;
    // planes z0 and z0+1 exist (z0+1 <= z1 <= n-1); z0+2 may be past the grid
#pragma unroll
    for (int r = 0; r < TY + 2; ++r) {
        pc[r] = (FULL || r < ny + 2) ? ld_row<TY>(col + z0 * SZ + r * SY, r) : zero2;
        pn[r] = (FULL || r < ny + 2) ? ld_row<TY>(col + (z0 + 1) * SZ + r * SY, r) : zero2;
        pf[r] = zero2;
    }
    if constexpr (PF == 2) {
        const bool have = z0 + 2 <= z1;
#pragma unroll
        for (int r = 0; r < TY + 2; ++r)
            pa[r] = (have && (FULL || r < ny + 2)) ? ld_row<TY>(col + (z0 + 2) * SZ + r * SY, r) : zero2;
    }
    for (int64_t z = z0; z < z1; ++z) {
        if (z + 1 + PF <= z1) {
#pragma unroll
            for (int r = 0; r < TY + 2; ++r)
                if (FULL || r < ny + 2)
                    pf[r] = ld_row<TY>(col + (z + 1 + PF) * SZ + r * SY, r);
        }
        const int par = (int)(z & 1);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                s_edge[par][wv][r][0] = pc[r + 1].x;
        }
        if (lane == kWave - 1) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                s_edge[par][wv][r][1] = pc[r + 1].y;
        }
        GF_GLOBAL const double *frow = u + z * SZ + y0 * SY + xs;
        double gl[TY], gr[TY];
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            gl[r] = 0.0;
            gr[r] = 0.0;
        }
        if (gather_l || gather_r) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                if (FULL || r < ny) {
                    const double g = frow[r * SY + (gather_l ? -1 : 2)];
                    gl[r] = g;
                    gr[r] = g;
                }
        }
        __syncthreads();
        GF_GLOBAL double *out = w + z * SZ + y0 * SY + xs;
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            if (FULL || r < ny) {
                const gf_d2 c = pc[r + 1];
                const double sl = wave_shr1(c.y);
                const double sr = wave_shl1(c.x);
                const double el = wv > 0 ? s_edge[par][wv - 1][r][1] : gl[r];
                const double er = wv < nw - 1 ? s_edge[par][wv + 1][r][0] : gr[r];
                const double xl = lane == 0 ? el : sl;
                const double xr = lane == kWave - 1 ? er : sr;
                gf_d2 v;
                v.x = (((xl + c.y) + (pc[r].x + pc[r + 2].x)) + (pm[r].x + pn[r + 1].x)) * c6;
                v.y = (((c.x + xr) + (pc[r].y + pc[r + 2].y)) + (pm[r].y + pn[r + 1].y)) * c6;
                if (in0 && in1) {
                    __builtin_nontemporal_store(v, (GF_GLOBAL gf_d2 *)(out + r * SY));
                } else if (in0) {
                    out[r * SY] = v.x;
                } else if (in1) {
                    out[r * SY + 1] = v.y;
                }
                if (want_red) {
                    const double d0 = in0 ? fabs(v.x - c.x) : -INFINITY;
                    const double d1 = in1 ? fabs(v.y - c.y) : -INFINITY;
                    const double d = d0 > d1 ? d0 : d1;
                    mx = d > mx ? d : mx;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < TY; ++r)
            pm[r] = pc[r + 1];
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
            pc[r] = pn[r];
            if constexpr (PF == 2) {
                pn[r] = pa[r];
                pa[r] = pf[r];
            } else {
                pn[r] = pf[r];
            }
        }
    }
    return mx;
}

template <int TY, int PF>
__device__ __forceinline__ double j3v2_item(const double *u_, double *w_, int64_t n, int64_t item, const Tiling &t,
                                            bool want_red)
{
    const StencilGeom g = j3v2_geom(n, t);
    const int64_t xc = item % g.nxc;
    const int64_t rest = item / g.nxc;
    const int64_t yt = rest % g.nyt;
    const int64_t zs = rest / g.nyt;
    const int64_t x = (xc * blockDim.x + threadIdx.x) * 2;
    const int64_t y0 = 1 + yt * TY;
    const int ny = (int)(n - 1 - y0 < TY ? n - 1 - y0 : TY);
    const int64_t z0 = 1 + zs * t.tile_z;
    const int64_t z1 = (z0 + t.tile_z < n - 1) ? z0 + t.tile_z : n - 1;
    if (ny == TY)
        return j3v2_tile<TY, PF, true>(gptr(u_), gptr(w_), n, x, y0, ny, z0, z1, want_red);
    return j3v2_tile<TY, PF, false>(gptr(u_), gptr(w_), n, x, y0, ny, z0, z1, want_red);
}

// 2D 5-point Jacobi. The workgroup owns a chunk of columns and marches down
// a segment of rows [y0, y1): each thread owns two adjacent columns (one
// 16-byte access per row) and keeps rows y-1, y and y+1 in registers while
// the next kJ2Ahead rows are in flight, so every value of u is fetched once
// per segment plus two halo rows. x-neighbours come from the adjacent lanes
// by DPP shifts; the first and last lane of each wavefront also load their
// outer neighbour with every row (a cache hit: the adjacent wavefront reads
// that line), so wavefronts never wait for each other. The ring of rows is
// indexed with compile-time slots (the step loop is unrolled by the ring
// size). For odd n the rows start on 8-byte boundaries, so the 16-byte
// accesses are only 8-byte aligned (ODD), and the row's last column n-1
// falls to a thread of its own: that thread loads the pair (n-2, n-1) and
// passes column n-1 on as its left value. Lanes past the row end load an
// in-bounds pair and store nothing.
constexpr int kJ2Ahead = 4;
constexpr int kJ2Ring = kJ2Ahead + 3;
typedef double gf_d2u __attribute__((ext_vector_type(2), aligned(8)));

template <bool ODD>
__device__ __forceinline__ double j2m_seg(GF_GLOBAL const double *__restrict__ u, GF_GLOBAL double *__restrict__ w,
                                          int64_t n, int64_t x, int64_t y0, int64_t y1, bool want_red)
{
    typedef typename std::conditional<ODD, gf_d2u, gf_d2>::type A;  // access type
    const int lane = threadIdx.x & (kWave - 1);
    // x is even; for even n x <= n-2 whenever x < n, for odd n x may be n-1
    const int64_t xs = x <= n - 2 ? x : n - 2;  // first column of the loaded pair
    const bool in0 = x >= 1 && x <= n - 2;      // column x is interior
    const bool in1 = x + 1 <= n - 2;            // column x+1 is interior
    const bool last = ODD && x == n - 1;        // holds column n-1 alone
    // the wavefront's edge lanes read the neighbour column beyond the
    // wavefront: lane 0 the one on its left, the last lane the one on its right
    const int64_t eoff = lane == 0 ? -1 : 2;
    const bool edge = (lane == 0 && xs >= 1) || (lane == kWave - 1 && xs + 2 <= n - 1);
    const int64_t L = y1 - y0;  // rows computed; rows y0-1 .. y1 are read
    GF_GLOBAL const double *base = u + (y0 - 1) * n + xs;
    auto ld = [&](int64_t j) -> gf_d2 { return *(GF_GLOBAL const A *)(base + j * n); };
    gf_d2 ring[kJ2Ring];
    double eg[kJ2Ring];
#pragma unroll
    for (int j = 0; j < kJ2Ring; ++j) {
        ring[j] = gf_d2{0.0, 0.0};
        eg[j] = 0.0;
    }
    // rows y0-1 and y0 are only needed as the rows above; the edge value of
    // a row is needed when that row is computed (rows 1 .. L)
#pragma unroll
    for (int j = 0; j < kJ2Ahead + 2; ++j)
        if (j <= L + 1) {
            ring[j] = ld(j);
            if (edge && j >= 1 && j <= L)
                eg[j] = base[j * n + eoff];
        }
    double acc = 0.0;
    for (int64_t b0 = 0; b0 < L; b0 += kJ2Ring) {
#pragma unroll
        for (int k = 0; k < kJ2Ring; ++k) {
            const int64_t i = b0 + k;  // computing row y0 + i from ring slots k, k+1, k+2
            if (i < L) {
                const int64_t jl = i + kJ2Ahead + 2;
                if (jl <= L + 1) {
                    ring[(k + kJ2Ahead + 2) % kJ2Ring] = ld(jl);
                    if (edge && jl <= L)
                        eg[(k + kJ2Ahead + 2) % kJ2Ring] = base[jl * n + eoff];
                }
                const gf_d2 up = ring[k];
                const gf_d2 c = ring[(k + 1) % kJ2Ring];
                const gf_d2 dn = ring[(k + 2) % kJ2Ring];
                const double g = eg[(k + 1) % kJ2Ring];
                // this thread's first and last column of the row
                const double lo = last ? c.y : c.x;
                const double hi = c.y;
                const double sl = wave_shr1(hi);
                const double sr = wave_shl1(lo);
                const double xl = lane == 0 ? g : sl;
                const double xr = lane == kWave - 1 ? g : sr;
                GF_GLOBAL double *out = w + (y0 + i) * n + xs;
                gf_d2 v;
                v.x = ((xl + c.y) + (up.x + dn.x)) * 0.25;
                v.y = ((c.x + xr) + (up.y + dn.y)) * 0.25;
                // w is read again only in the next sweep: streaming stores
                // (measured 2 % faster on the batched instances)
                if (in0 && in1)
                    __builtin_nontemporal_store(v, (GF_GLOBAL A *)out);
                else if (in0)
                    __builtin_nontemporal_store(v.x, out);
                else if (in1)
                    __builtin_nontemporal_store(v.y, out + 1);
                if (want_red) {
                    if (in0) {
                        const double d = v.x - c.x;
                        acc = acc + d * d;
                    }
                    if (in1) {
                        const double d = v.y - c.y;
                        acc = acc + d * d;
                    }
                }
            }
        }
    }
    return acc;
}

__device__ __forceinline__ double j2_item(const double *u_, double *w_, int64_t n, int64_t item, const Tiling &t,
                                          bool want_red)
{
    const StencilGeom g = j2_geom(n, t);
    const int64_t xc = item % g.nxc;
    const int64_t ys = item / g.nxc;
    const int64_t y0 = 1 + ys * t.tile_y;
    const int64_t y1 = (y0 + t.tile_y < n - 1) ? y0 + t.tile_y : n - 1;
    const int64_t x = (xc * blockDim.x + threadIdx.x) * 2;
    if (n & 1)
        return j2m_seg<true>(gptr(u_), gptr(w_), n, x, y0, y1, want_red);
    return j2m_seg<false>(gptr(u_), gptr(w_), n, x, y0, y1, want_red);
}

// CSR SpMV over a block of wg_size/2 rows (CSR-stream): the block's products
// val[k] * x[col[k]] are formed by a coalesced pass over its nonzeros into
// LDS (eight gathers in flight per thread), then each of the first R threads
// sums its own row serially in stored column order, exactly as the legacy
// loop does (same products, same order, no contraction). Blocks with more
// nonzeros than the LDS tile fall back to one thread per row.
// 30 KiB of products per workgroup (960 per wavefront: 32 rows of up to 30
// nonzeros): with the kernel's other LDS a workgroup stays under 32 KiB in
// whole allocation granules, so five 256-thread workgroups fit a CU's 160 KiB.
// At 32 KiB only four fit, and the latency-bound SpMV ran 5 % slower.
constexpr int kSpmvLds = 3840;
constexpr int kSpmvWaveRows = 32;     // rows per wavefront
constexpr int kSpmvWaveLds = kSpmvLds / (kMaxWg / kWave);  // product slots per wavefront
constexpr int kSpmvUnroll = 8;

// CSR SpMV, one work item = wg_size / 2 consecutive rows, split into
// 32-row slices, one per wavefront. A wavefront streams its slice's
// nonzeros (coalesced col/val loads, eight in flight per lane, then the x
// gathers) into its own LDS slice as products val * x[col]; then lane r sums
// row r's products serially in column order (the serial loop's order, so y
// is bit-exact). Wavefronts share no LDS and never wait for each other. A
// slice whose nonzeros exceed its LDS share takes the direct row loop (same
// order).
__device__ __forceinline__ void spmv_item(const int32_t *rowptr_, const int32_t *col_, const double *val_,
                                          const double *x_, double *y_, int64_t n, int64_t item, int64_t R)
{
    __shared__ double s_prod[kSpmvLds];
    GF_GLOBAL const int32_t *__restrict__ rowptr = gptr(rowptr_);
    GF_GLOBAL const int32_t *__restrict__ col = gptr(col_);
    GF_GLOBAL const double *__restrict__ val = gptr(val_);
    GF_GLOBAL const double *__restrict__ x = gptr(x_);
    GF_GLOBAL double *__restrict__ y = gptr(y_);
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    double *slot = s_prod + wv * kSpmvWaveLds;
    const int64_t blk = item * R;
    const int64_t blk_end = blk + R < n ? blk + R : n;
    const int64_t a = blk + (int64_t)wv * kSpmvWaveRows;
    if (a >= blk_end)
        return;
    const int64_t b = a + kSpmvWaveRows < blk_end ? a + kSpmvWaveRows : blk_end;
    const int64_t row = a + lane;
    const bool mine = row < b;
    // the slice's extent and this lane's row extent, requested together
    const int32_t k0 = rowptr[a];
    const int32_t nnz = rowptr[b] - k0;
    const int32_t rb = mine ? rowptr[row] : 0;
    const int32_t re = mine ? rowptr[row + 1] : 0;
    if (nnz <= kSpmvWaveLds) {
        for (int32_t base = lane; base < nnz; base += kSpmvUnroll * kWave) {
            int32_t c[kSpmvUnroll];
            double v[kSpmvUnroll], xv[kSpmvUnroll];
#pragma unroll
            for (int j = 0; j < kSpmvUnroll; ++j) {
                const int32_t kk = base + j * kWave;
                c[j] = kk < nnz ? col[k0 + kk] : 0;
                v[j] = kk < nnz ? val[k0 + kk] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kSpmvUnroll; ++j)
                xv[j] = base + j * kWave < nnz ? x[c[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < kSpmvUnroll; ++j)
                if (base + j * kWave < nnz)
                    slot[base + j * kWave] = v[j] * xv[j];
        }
        // the wavefront's LDS writes complete before its lanes read them
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        if (mine) {
            const int32_t e = re - k0;
            double acc = 0.0;
            int32_t k = rb - k0;
            for (; k + 8 <= e; k += 8) {
                double p[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    p[j] = slot[k + j];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc = acc + p[j];
            }
            for (; k < e; ++k)
                acc = acc + slot[k];
            y[row] = acc;
        }
        // the next item's writes to this slice wait for these reads
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __builtin_amdgcn_wave_barrier();
    } else if (mine) {
        double acc = 0.0;
        for (int32_t k = rb; k < re; ++k)
            acc = acc + val[k] * x[col[k]];
        y[row] = acc;
    }
}

// dot and axpby: a work item is `items` rows of blockDim.x consecutive
// elements; each thread requests all of its elements before using them.
template <int ITEMS>
__device__ __forceinline__ double dot_item_t(GF_GLOBAL const double *__restrict__ a,
                                             GF_GLOBAL const double *__restrict__ b, int64_t n, int64_t base)
{
    double av[ITEMS], bv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x + threadIdx.x;
        av[k] = i < n ? a[i] : 0.0;
        bv[k] = i < n ? b[i] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (base + (int64_t)k * blockDim.x + threadIdx.x < n)
            acc = acc + av[k] * bv[k];
    return acc;
}

__device__ __forceinline__ double dot_item(const double *a_, const double *b_, int64_t n, int64_t item,
                                           const Tiling &t)
{
    GF_GLOBAL const double *__restrict__ a = gptr(a_);
    GF_GLOBAL const double *__restrict__ b = gptr(b_);
    const int64_t base = item * chunk_elems(t);
    switch (t.items) {
    case 1: return dot_item_t<1>(a, b, n, base);
    case 2: return dot_item_t<2>(a, b, n, base);
    case 4: return dot_item_t<4>(a, b, n, base);
    case 8: return dot_item_t<8>(a, b, n, base);
    default: break;
    }
    double acc = 0.0;
    for (int k = 0; k < t.items; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x + threadIdx.x;
        if (i < n)
            acc = acc + a[i] * b[i];
    }
    return acc;
}

template <int ITEMS>
__device__ __forceinline__ void axpby_item_t(GF_GLOBAL double *out, GF_GLOBAL const double *x, double s,
                                             GF_GLOBAL const double *y, int64_t n, int64_t base)
{
    double xv[ITEMS], yv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x + threadIdx.x;
        xv[k] = i < n ? x[i] : 0.0;
        yv[k] = i < n ? y[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x + threadIdx.x;
        if (i < n)
            out[i] = xv[k] + s * yv[k];
    }
}

// out may alias x or y: every element is read before it is written, by the
// same thread.
__device__ __forceinline__ void axpby_item(double *out_, const double *x_, double s, const double *y_, int64_t n,
                                           int64_t item, const Tiling &t)
{
    GF_GLOBAL double *out = gptr(out_);
    GF_GLOBAL const double *x = gptr(x_);
    GF_GLOBAL const double *y = gptr(y_);
    const int64_t base = item * chunk_elems(t);
    switch (t.items) {
    case 1: axpby_item_t<1>(out, x, s, y, n, base); return;
    case 2: axpby_item_t<2>(out, x, s, y, n, base); return;
    case 4: axpby_item_t<4>(out, x, s, y, n, base); return;
    case 8: axpby_item_t<8>(out, x, s, y, n, base); return;
    default: break;
    }
    for (int k = 0; k < t.items; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x + threadIdx.x;
        if (i < n)
            out[i] = x[i] + s * y[i];
    }
}

// Histogram, phase 1: this worker counts the keys of its chunks whose bin
// falls in its part (all of a worker's items share one part because the
// worker stride is a multiple of the part count) into 16-bit counters packed
// two per 32-bit LDS word, with non-returning LDS atomics, then writes them
// as its partial row of 16-bit counts. Once per 32768 keys at most (every
// chunk, or every few when chunks are smaller; a chunk is at most 32768
// keys, checked on the host) the workgroup moves 0x8000 of every counter
// that reached 0x8000 into the global bin: a counter is below 0x8000 after a
// scan and grows by at most 32768 before the next one, so it never wraps and
// no carry crosses into the neighbouring counter; the final counters fit in
// 16 bits. Integer counts are exact in any order.
__device__ __forceinline__ void hist_count(uint32_t *s_h, uint32_t key, uint32_t mask, uint32_t lo, uint32_t span)
{
    const uint32_t b = (key & mask) - lo;
    if (b < span)
        __hip_atomic_fetch_add(&s_h[b >> 1], 1u << ((b & 1u) * 16u), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void hist_escape(uint32_t *s_h, GF_GLOBAL uint32_t *bins, uint32_t lo, uint32_t span)
{
    __syncthreads();
    for (uint32_t wd = threadIdx.x; wd < (span + 1) / 2; wd += blockDim.x) {
        uint32_t v = s_h[wd];
        if (v & 0x80008000u) {
            if (v & 0x8000u) {
                __hip_atomic_fetch_add(&bins[lo + 2 * wd], 0x8000u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v -= 0x8000u;
            }
            if (v & 0x80000000u) {
                __hip_atomic_fetch_add(&bins[lo + 2 * wd + 1], 0x8000u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v -= 0x80000000u;
            }
            s_h[wd] = v;
        }
    }
    __syncthreads();
}

typedef uint32_t gf_u4 __attribute__((ext_vector_type(4)));

// The keys of one chunk for this thread: ITEMS groups of four consecutive
// keys, group k at base + (k * blockDim.x + threadIdx.x) * 4. Every chunk
// but the one holding the end of the array is whole (no guards); in that
// one, missing keys are left out of the count.
template <int ITEMS>
__device__ __forceinline__ void hist_load(GF_GLOBAL const uint32_t *keys, int64_t n, int64_t base, gf_u4 (&v)[ITEMS])
{
    const uint32_t B4 = blockDim.x * 4u;
    GF_GLOBAL const uint32_t *p = keys + base + threadIdx.x * 4u;
    if (base + (int64_t)ITEMS * B4 <= n) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            v[k] = *(GF_GLOBAL const gf_u4 *)(p + k * B4);
        return;
    }
    const int64_t left0 = n - base - threadIdx.x * 4;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t left = left0 - (int64_t)k * B4;
        v[k] = gf_u4{0u, 0u, 0u, 0u};
        if (left >= 4)
            v[k] = *(GF_GLOBAL const gf_u4 *)(p + k * B4);
        else
            for (int j = 0; j < left; ++j)
                v[k][j] = p[k * B4 + j];
    }
}

template <int ITEMS>
__device__ __forceinline__ void hist_count_all(uint32_t *s_h, const gf_u4 (&v)[ITEMS], int64_t n, int64_t base,
                                               uint32_t mask, uint32_t lo, uint32_t span)
{
    const uint32_t B4 = blockDim.x * 4u;
    if (base + (int64_t)ITEMS * B4 <= n) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            hist_count(s_h, v[k].x, mask, lo, span);
            hist_count(s_h, v[k].y, mask, lo, span);
            hist_count(s_h, v[k].z, mask, lo, span);
            hist_count(s_h, v[k].w, mask, lo, span);
        }
        return;
    }
    const int64_t left0 = n - base - threadIdx.x * 4;
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t left = left0 - (int64_t)k * B4;
        for (int j = 0; j < 4 && j < left; ++j)
            hist_count(s_h, v[k][j], mask, lo, span);
    }
}

// Up to four groups per thread, the next chunk's keys are requested before
// this chunk is counted, so their latency hides behind the LDS atomics and
// the escape scan (eight groups double-buffered would not fit the 128
// registers of a 1024-thread workgroup). s_h: the workgroup's
// kHistPart / 2 LDS words.
template <int ITEMS>
__device__ __forceinline__ void hist_phase1_t(uint32_t *s_h, const uint32_t *keys_, uint32_t *bins_,
                                              uint32_t *rows_, uint32_t mask, int64_t n, int64_t worker, int64_t G,
                                              const Tiling &t)
{
    GF_GLOBAL const uint32_t *__restrict__ keys = gptr(keys_);
    GF_GLOBAL uint32_t *bins = gptr(bins_);
    const HistGeom g = hist_geom(n, mask, t);
    const int64_t part = worker % g.parts;
    const uint32_t lo = (uint32_t)(part * kHistPart);
    const int64_t span64 = g.nbins - (int64_t)lo < kHistPart ? g.nbins - (int64_t)lo : kHistPart;
    const uint32_t span = (uint32_t)span64;
    for (int i = threadIdx.x; i < kHistPart / 2; i += blockDim.x)
        s_h[i] = 0u;
    __syncthreads();
    constexpr bool kAhead = ITEMS <= 4;
    // A chunk adds at most chunk_keys to a counter, so escaping after every
    // `every` chunks, every * chunk_keys <= 0x8000, keeps each counter (below
    // 0x8000 after an escape) within 16 bits; small chunks share one scan.
    const int64_t every = g.chunk_keys >= 0x8000 ? 1 : 0x8000 / g.chunk_keys;
    int64_t since = 0;
    gf_u4 cur[ITEMS], nxt[kAhead ? ITEMS : 1];
    if (kAhead && worker < g.nitems)
        hist_load<ITEMS>(keys, n, (worker / g.parts) * g.chunk_keys, cur);
    for (int64_t it = worker; it < g.nitems; it += G) {
        const int64_t base = (it / g.parts) * g.chunk_keys;
        const bool scan = ++since == every;
        if (scan)
            since = 0;
        if constexpr (kAhead) {
            const bool more = it + G < g.nitems;
            if (more)
                hist_load<ITEMS>(keys, n, ((it + G) / g.parts) * g.chunk_keys, nxt);
            hist_count_all<ITEMS>(s_h, cur, n, base, mask, lo, span);
            if (scan)
                hist_escape(s_h, bins, lo, span);
            if (more) {
#pragma unroll
                for (int k = 0; k < ITEMS; ++k)
                    cur[k] = nxt[k];
            }
        } else {
            hist_load<ITEMS>(keys, n, base, cur);
            hist_count_all<ITEMS>(s_h, cur, n, base, mask, lo, span);
            if (scan)
                hist_escape(s_h, bins, lo, span);
        }
    }
    // the rows below hold the counters as 16-bit entries: every counter is
    // at most 0x7FFF plus the keys of the chunks since the last escape; the
    // workgroup's counting is complete before they are read
    __syncthreads();
    // the packed LDS word holds bins 2w (low half) and 2w+1 (high half): as
    // a 32-bit store it lays down the two 16-bit row entries in order
    GF_GLOBAL uint32_t *row = gptr(rows_) + worker * (kHistPart / 2);
    for (uint32_t wd = threadIdx.x; wd < (span + 1) / 2; wd += blockDim.x)
        row[wd] = s_h[wd];
}

__device__ __forceinline__ void hist_phase1(const uint32_t *keys, uint32_t *bins, uint32_t *rows, uint32_t mask,
                                            int64_t n, int64_t worker, int64_t G, const Tiling &t)
{
    __shared__ uint32_t s_h[kHistPart / 2];
    switch (t.items) {
    case 1: hist_phase1_t<1>(s_h, keys, bins, rows, mask, n, worker, G, t); break;
    case 2: hist_phase1_t<2>(s_h, keys, bins, rows, mask, n, worker, G, t); break;
    case 4: hist_phase1_t<4>(s_h, keys, bins, rows, mask, n, worker, G, t); break;
    default: hist_phase1_t<8>(s_h, keys, bins, rows, mask, n, worker, G, t); break;
    }
}

// Histogram, phase 2: bins[b] += the sum of b's entries over the `rows_used`
// partial rows (row w holds part w % parts). A work unit is four adjacent
// bins times one slice of the rows (every S-th row of the part, S chosen so
// the units cover the threads); its four sums go to the bins with integer
// atomics, exact in any order. Threads [first, first + stride) share the
// units.
__device__ __forceinline__ void hist_merge(uint32_t *bins_, const uint32_t *rows_, uint32_t mask, int64_t rows_used,
                                           int64_t first, int64_t stride)
{
    GF_GLOBAL uint32_t *bins = gptr(bins_);
    GF_GLOBAL const uint16_t *rows = (GF_GLOBAL const uint16_t *)gptr(rows_);
    const int64_t nbins = (int64_t)mask + 1;
    const int64_t parts = cdiv(nbins, kHistPart);
    const int64_t quads = cdiv(nbins, 4);
    const int64_t per_part = rows_used / parts;  // rows of each part
    int64_t S = stride / quads;
    S = S < 1 ? 1 : (S > per_part ? per_part : S);
    for (int64_t u = first; u < quads * S; u += stride) {
        const int64_t q = u % quads;
        const int64_t sl = u / quads;
        const int64_t b0 = q * 4;
        const int64_t part = b0 / kHistPart;
        const int64_t off = b0 - part * kHistPart;
        uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        // unrolled so that several row loads are in flight per thread (the
        // persistent kernel runs this with one workgroup per CU)
#pragma unroll 8
        for (int64_t j = sl; j < per_part; j += S) {
            const int64_t w = part + j * parts;
            typedef uint16_t gf_h4 __attribute__((ext_vector_type(4)));
            const gf_h4 r = *(GF_GLOBAL const gf_h4 *)(rows + w * kHistPart + off);
            s0 += r.x;
            s1 += r.y;
            s2 += r.z;
            s3 += r.w;
        }
        if (s0)
            __hip_atomic_fetch_add(&bins[b0], s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s1 && b0 + 1 < nbins)
            __hip_atomic_fetch_add(&bins[b0 + 1], s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s2 && b0 + 2 < nbins)
            __hip_atomic_fetch_add(&bins[b0 + 2], s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s3 && b0 + 3 < nbins)
            __hip_atomic_fetch_add(&bins[b0 + 3], s3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// GF_R_OWNER: the static schedule executed literally over all T threads.
__device__ __forceinline__ void owner_region(int32_t *owner, int64_t n, int64_t chunk, int64_t T, int64_t tid)
{
    if (chunk <= 0) {
        int64_t lo, hi;
        static_range(n, T, tid, &lo, &hi);
        for (int64_t i = lo; i < hi; ++i)
            owner[i] = (int32_t)tid;
    } else {
        for (int64_t c0 = tid * chunk; c0 < n; c0 += T * chunk)
            for (int64_t i = c0; i < c0 + chunk && i < n; ++i)
                owner[i] = (int32_t)tid;
    }
}

// GF_R_PHASES: a `parallel` region with manual worksharing (Section 3.3):
// thread t of T owns a balanced contiguous block of [0, n) and runs P
// producer/consumer phases, each reading what other threads (and
// workgroups) wrote in the previous one; `bar` is the `omp barrier` across
// all workgroups between phases (the region's own end barrier follows the
// last one). Returns false if a barrier failed.
template <typename Bar>
__device__ bool phases_region(GF_GLOBAL double *a, GF_GLOBAL double *b, GF_GLOBAL int32_t *owner, int64_t n,
                              int64_t P, int64_t shift, int64_t t, int64_t T, Bar bar)
{
    int64_t lo, hi;
    static_range(n, T, t, &lo, &hi);
    if (owner)
        for (int64_t i = lo; i < hi; ++i)
            owner[i] = (int32_t)t;
    GF_GLOBAL const double *src = a;
    GF_GLOBAL double *dst = b;
    for (int64_t p = 0; p < P; ++p) {
        if (p > 0 && !bar())
            return false;
        for (int64_t i = lo; i < hi; ++i) {
            int64_t k = i + shift;
            if (k >= n)
                k -= n;
            dst[i] = src[i] + src[k];
        }
        GF_GLOBAL double *nsrc = dst;
        dst = (GF_GLOBAL double *)src;
        src = nsrc;
    }
    return true;
}

// Executes one work item of a region; returns the thread's reduction value.
// op[i] is the region's i-th array operand (slot st.arr[i] resolved by the
// caller); s is the AXPBY coefficient scal[st.sc[1]] * st.c.
template <unsigned KMASK, int TY, int PF>
__device__ __forceinline__ double region_item(const DStep &st, void *const *op, double s, int64_t n, int64_t item,
                                              const Tiling &t)
{
    const bool red = st.red_op != GF_OP_NONE;
    switch (st.kind) {
    case GF_R_JACOBI3D:
        if constexpr ((KMASK >> GF_R_JACOBI3D) & 1u) {
            if ((n & 1) == 0)
                return j3v2_item<TY, PF>((const double *)op[0], (double *)op[1], n, item, t, red);
            return j3_item<TY>((const double *)op[0], (double *)op[1], n, item, t, red);
        }
        break;
    case GF_R_JACOBI2D:
        if constexpr ((KMASK >> GF_R_JACOBI2D) & 1u)
            return j2_item((const double *)op[0], (double *)op[1], n, item, t, red);
        break;
    case GF_R_SPMV:
        if constexpr ((KMASK >> GF_R_SPMV) & 1u) {
            spmv_item((const int32_t *)op[0], (const int32_t *)op[1], (const double *)op[2], (const double *)op[3],
                      (double *)op[4], n, item, spmv_rows(t));
            return 0.0;
        }
        break;
    case GF_R_DOT:
        if constexpr ((KMASK >> GF_R_DOT) & 1u)
            return dot_item((const double *)op[0], (const double *)op[1], n, item, t);
        break;
    case GF_R_AXPBY:
        if constexpr ((KMASK >> GF_R_AXPBY) & 1u) {
            axpby_item((double *)op[0], (const double *)op[1], s, (const double *)op[2], n, item, t);
            return 0.0;
        }
        break;
    default:
        break;
    }
    return red_identity(st.red_op);
}

// ---------------------------------------------------------------------------
// Serial steps of the initial thread (called by one thread).
// ---------------------------------------------------------------------------

__device__ inline void serial_scalar(int kind, const int32_t *sc, double c, double *scal)
{
    switch (kind) {
    case GF_S_SET:
        scal[sc[0]] = c;
        break;
    case GF_S_COPY:
        scal[sc[0]] = scal[sc[1]];
        break;
    case GF_S_DIV:
        scal[sc[0]] = scal[sc[1]] / scal[sc[2]];
        break;
    case GF_S_SQRT:
        scal[sc[0]] = sqrt(scal[sc[1]]);
        break;
    default:
        break;
    }
}

__device__ inline void serial_printf(const RpcRing &rpc, int32_t fmt_id, int32_t nargs, uint32_t flags,
                                     const int32_t *sc, int32_t iter, const double *scal, int32_t *err)
{
    uint64_t args[8];
    args[0] = (uint64_t)(int64_t)(iter + 1);
    for (int k = 1; k < nargs && k < 4; ++k)
        args[k] = __double_as_longlong(scal[sc[k - 1]]);
    rpc_call(rpc, kCalleePrintf, (uint32_t)fmt_id, (uint32_t)nargs, args, flags, nullptr, err);
}

// ---------------------------------------------------------------------------
// General host call (Section 3.2), made by one whole wavefront. Lane 0 takes
// the ticket, waits until the slot is free and fills the header with the
// value words; the 64 lanes copy the objects of read and read-write
// references into the slot's payload (16-byte pieces, or bytes for objects
// that are not 16-byte aligned); lane 0 publishes the request. A blocking
// call then waits for completion, the lanes copy the objects of write and
// read-write references back, and lane 0 frees the slot. base(a) gives the
// array that holds the object of reference argument a under the caller's
// current slot bindings. Returns the host's return value (0 when posted, -1
// after a timeout, which also sets the error word).
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool call_fires(int32_t iter, int32_t every)
{
    return iter < 0 || (every > 0 && (iter + 1) % every == 0);
}

__device__ __forceinline__ void wave_copy(char *dst, const char *src, int64_t n, int lane)
{
    if ((((uintptr_t)dst | (uintptr_t)src | (uint64_t)n) & 15u) == 0) {
        for (int64_t i = (int64_t)lane * 16; i < n; i += kWave * 16)
            *(uint4 *)(dst + i) = *(const uint4 *)(src + i);
    } else {
        for (int64_t i = lane; i < n; i += kWave)
            dst[i] = src[i];
    }
}

__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename Base>
__device__ int64_t serial_call(const RpcRing &rpc, int32_t call_id, uint32_t flags, Base base, const double *scal,
                               int32_t iter, int32_t *err)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const DCall &cs = rpc.calls[call_id];
    const bool timed = (flags & GF_STEP_TIMED) != 0;
    const bool blocking = (flags & GF_STEP_BLOCKING) != 0;
    const uint64_t c0 = timed ? now_ticks() : 0;
    const uint64_t nslots = (uint64_t)rpc.mask + 1;
    uint64_t t = 0;
    int ok = 1;
    if (lane == 0) {
        t = __hip_atomic_fetch_add(rpc.ticket, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t >= nslots && !rpc_wait_word(&rpc.slots[t & rpc.mask].freed, t - nslots + 1, rpc, err))
            ok = 0;
    }
    t = first_lane_u64(t);
    if (!__builtin_amdgcn_readfirstlane(ok))
        return -1;
    RpcSlot *slot = rpc.slots + (t & rpc.mask);
    char *pl = rpc.payloads + (size_t)(t & rpc.mask) * rpc.payload;
    bool copy_out = false;
    if (lane == 0) {
        for (int k = 0; k < cs.nargs; ++k) {
            const DCallArg &a = cs.a[k];
            uint64_t w = 0;
            if (a.kind == GF_ARG_CONST) {
                w = (uint64_t)a.value;
            } else if (a.kind == GF_ARG_SCALAR) {
                const double v = scal[a.slot];
                w = a.type == 'i' ? (uint64_t)(int64_t)v : (uint64_t)__double_as_longlong(v);
            } else if (a.kind == GF_ARG_ITER) {
                w = (uint64_t)(int64_t)(iter + 1);
            }
            slot->args[k] = w;
        }
        slot->callee = kCalleeCall;
        slot->fmt_id = (uint32_t)call_id;
        slot->nargs = (uint32_t)cs.nargs;
        slot->flags = flags;
    }
    const uint64_t c1 = timed ? now_ticks() : 0;
    // objects that lane 0 may have written just before (history records)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    // heap references not found in the heap travel as values
    uint32_t hflags = 0;
    for (int k = 0; k < cs.nargs; ++k) {
        const DCallArg &a = cs.a[k];
        if (a.kind == GF_ARG_REF) {
            if (a.mode & GF_REF_READ)
                wave_copy(pl + a.pos, (const char *)base(a) + a.start, a.size, lane);
            copy_out |= (a.mode & GF_REF_WRITE) != 0;
        } else if (a.kind == GF_ARG_HEAPREF) {
            // lane 0 looks the pointer up in the heap's record of live objects
            uint64_t st = 0, by = 0;
            if (lane == 0) {
                const uint64_t p = ((const uint64_t *)base(a))[a.start];
                if (!rpc.heap.base || !heapdev::heap_find(rpc.heap, (const void *)p, &st, &by) ||
                    by > (uint64_t)a.size)
                    by = 0;
                slot->args[k] = by ? (by << 32) | (p - ((uint64_t)(uintptr_t)rpc.heap.base + st)) : p;
            }
            st = first_lane_u64(st);
            by = first_lane_u64(by);
            if (by == 0)
                hflags |= kHeapValueFlag0 << k;
            else if (a.mode & GF_REF_READ)
                wave_copy(pl + a.pos, rpc.heap.base + st, (int64_t)by, lane);
            // the slot is freed by the device whenever the call site copies back
            copy_out |= (a.mode & GF_REF_WRITE) != 0;
        }
    }
    // rewritten only when a heap pointer travels as a value (a late store to
    // host memory would add a PCIe write to the publication's wait)
    if (hflags && lane == 0)
        slot->flags = flags | hflags;
    // every lane's payload stores before lane 0's publication
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (lane == 0)
        __hip_atomic_store(&slot->seq, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint64_t c2 = timed ? now_ticks() : 0;
    uint64_t c3 = c2, c4 = c2;
    int64_t ret = 0;
    if (blocking) {
        if (lane == 0) {
            ok = rpc_wait_word(&slot->done, t + 1, rpc, err) ? 1 : 0;
            ret = ok ? __hip_atomic_load(&slot->ret, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : -1;
        }
        ok = __builtin_amdgcn_readfirstlane(ok);
        ret = (int64_t)first_lane_u64((uint64_t)ret);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        c3 = timed ? now_ticks() : 0;
        if (copy_out) {
            if (ok)
                for (int k = 0; k < cs.nargs; ++k) {
                    const DCallArg &a = cs.a[k];
                    if (!(a.mode & GF_REF_WRITE))
                        continue;
                    if (a.kind == GF_ARG_REF) {
                        wave_copy((char *)base(a) + a.start, pl + a.pos, a.size, lane);
                    } else if (a.kind == GF_ARG_HEAPREF) {
                        // the caller's object is the one found at the start of the call
                        // (it cannot be freed meanwhile); look it up again rather than
                        // keep it in registers across the wait
                        uint64_t st = 0, by = 0;
                        if (lane == 0) {
                            const uint64_t p = ((const uint64_t *)base(a))[a.start];
                            if (!rpc.heap.base || !heapdev::heap_find(rpc.heap, (const void *)p, &st, &by) ||
                                by > (uint64_t)a.size)
                                by = 0;
                        }
                        st = first_lane_u64(st);
                        by = first_lane_u64(by);
                        if (by)
                            wave_copy(rpc.heap.base + st, pl + a.pos, (int64_t)by, lane);
                    }
                }
            // the payload reads are complete before the slot is handed back
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            if (lane == 0)
                __hip_atomic_store(&slot->freed, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        c4 = timed ? now_ticks() : 0;
    }
    if (timed && lane == 0) {
        unsigned long long *st = rpc.call_stats + (int64_t)call_id * kCallStatWords;
        __hip_atomic_fetch_add(st + 0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(st + 1, (unsigned long long)(c1 - c0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(st + 2, (unsigned long long)(c2 - c1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(st + 3, (unsigned long long)(c3 - c2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(st + 4, (unsigned long long)(c4 - c3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return ret;
}

// ---------------------------------------------------------------------------
// Persistent program kernel (the whole main loop in one cooperative launch;
// Section 3.3 with the kernel split replaced by in-kernel grid barriers).
// Every workgroup walks the step list. Region work items are dealt
// round-robin over workers; after each region a grid barrier stands for the
// implicit barrier of `parallel for`. Serial steps are executed redundantly by
// every workgroup on its own LDS copy of the scalar variables, which stay
// identical because every workgroup reduces the same partials in the same
// order; only workgroup 0 performs side effects (records, RPC, write-back).
// ---------------------------------------------------------------------------

constexpr unsigned kFamHist = (1u << GF_R_HIST) | (1u << GF_R_OWNER);

template <unsigned KMASK>
constexpr int family_max_threads()
{
    return KMASK == kFamHist ? kMaxWgHist : kMaxWg;
}

// Waves per SIMD the persistent kernel is compiled to fit (168 VGPRs for
// three). The 3D stencil with tiles of one or two rows and one plane in
// flight: three 256-thread workgroups per CU (its register need sits just
// above that; the compiler fits it without spilling). The 2D stencil: left
// alone the compiler gives the persistent kernel 187 VGPRs (two waves per
// SIMD) although the marching tile itself needs about 86 (the per-region
// kernel's count); at three waves it spills a few words outside the march,
// and batched runs, whose large instances are bound by rows in flight per
// wavefront, go 8-14 % faster. Four waves spill inside the march and are slower.
template <unsigned KMASK, int TY, int PF>
constexpr int persistent_min_waves()
{
    if (KMASK == ((1u << GF_R_JACOBI3D) | (1u << GF_R_OWNER)) && TY <= 2 && PF == 1)
        return 3;
    if (KMASK == ((1u << GF_R_JACOBI2D) | (1u << GF_R_OWNER)))
        return 3;
    return 1;
}

template <unsigned KMASK, int TY, int PF>
__global__ void __launch_bounds__(family_max_threads<KMASK>())
    __attribute__((amdgpu_waves_per_eu(persistent_min_waves<KMASK, TY, PF>())))
    k_persistent(DProg prog, DInst inst_arg, Tiling t_arg, Scratch scr, RpcRing rpc, BatchTable batch)
{
    __shared__ double s_scal[GF_MAX_SCALARS];
    __shared__ void *s_arr[GF_MAX_ARRAYS];
    __shared__ double s_red[kLdsRed];
    __shared__ BarrierState s_bar;
    __shared__ XcdState s_xcd;
    __shared__ int32_t s_local;

    // Single instance: the whole grid, tree or XCD barrier. Batched: this
    // workgroup's group of its instance, flat group barrier (the same-XCD
    // form when the table keeps every group on one XCD).
    const bool batched = batch.wg != nullptr;
    BatchEntry be;
    if (batched) {
        be = batch.wg[blockIdx.x];
    } else {
        be.inst = 0;
        be.member = (int32_t)blockIdx.x;
        be.gsize = (int32_t)gridDim.x;
        be.tile_y = 0;
        be.part_off = 0;
    }
    if (batched && batch.aligned) {
        // The table puts every group in one residue class of blockIdx.x mod
        // the XCD count. The dispatcher deals workgroups to XCDs round-robin,
        // but the XCD that takes workgroup 0 varies from launch to launch, so
        // a class lands on some one XCD, not necessarily the one its number
        // names. Every workgroup checks that it shares an XCD with the first
        // workgroup of its class to arrive (word 1 + class of the placement
        // line, tagged with the launch's epoch) and counts itself in word 0
        // if not; a tree barrier over the whole grid makes the count final.
        __shared__ BarrierState s_gbar;
        uint64_t *place = (uint64_t *)(scr.lines + (int64_t)kBatchPlaceLine * kLineWords);
        if (threadIdx.x == 0) {
            s_gbar.gen = __hip_atomic_load(scr.lines + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_gbar.ok = 1;
            const uint32_t xcc = hw_xcc_id();
            uint64_t *cls = place + 1 + blockIdx.x % kNumXcd;
            const uint64_t mine = ((uint64_t)scr.epoch << 32) | (xcc + 1u);
            uint64_t seen = __hip_atomic_load(cls, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while ((uint32_t)(seen >> 32) != scr.epoch) {
                if (__hip_atomic_compare_exchange_strong(cls, &seen, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                    seen = mine;
                    break;
                }
            }
            const uint32_t bad = (xcc >= (uint32_t)kNumXcd || seen != mine) ? 1u : 0u;
            uint64_t old = __hip_atomic_load(place, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                const uint64_t nw = ((uint32_t)(old >> 32) == scr.epoch) ? old + bad
                                                                           : (((uint64_t)scr.epoch << 32) | bad);
                if (__hip_atomic_compare_exchange_strong(place, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        __syncthreads();
        if (!tree_barrier(scr.lines + 1, scr.lines + kTreeLine0 * kLineWords, blockIdx.x, gridDim.x, &s_gbar,
                          scr.error, scr.barrier_timeout_ticks))
            return;
        if (threadIdx.x == 0) {
            const uint64_t v = __hip_atomic_load(place, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_local = ((uint32_t)(v >> 32) == scr.epoch && (uint32_t)v == 0u) ? 1 : 0;
        }
        __syncthreads();
        if (be.inst < 0)
            return;  // an idle entry of the table
    } else if (threadIdx.x == 0) {
        s_local = 0;
    }
    // rows per tile: this instance's own when the table gives one
    Tiling t = t_arg;
    if (batched && be.tile_y > 0)
        t.tile_y = be.tile_y;
    const DInst &inst = batched ? batch.inst[be.inst] : inst_arg;
    // workgroup-uniform: kept in scalar registers
    const int64_t G = uniform_i64(be.gsize);
    const int64_t member = uniform_i64(be.member);
    const int64_t worker = uniform_i64(batched ? member : worker_id(blockIdx.x, G, t.xcd_remap));
    uint32_t *gline = scr.lines + (int64_t)(kGroupLine0 + be.inst) * kLineWords;
    uint32_t *genw = batched ? gline + 1 : scr.lines + 1;  // generation word
    uint32_t *tree = scr.lines + kTreeLine0 * kLineWords;
    const bool xmode = !batched && scr.barrier_kind == kBarrierXcd && G >= kXcdBarrierMinWg;
    // MAX reductions under the XCD barrier fold into two 64-bit slots (one
    // atomic max per workgroup instead of a partial per work item that every
    // workgroup reads back after the barrier)
    uint64_t *max_slot = (uint64_t *)(scr.lines + (int64_t)kMaxSlotLine0 * kLineWords);
    auto barrier = [&](uint64_t *reset = nullptr) -> bool {
        if (G == 1) {
            // a group of one workgroup: a workgroup-scope barrier suffices
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
            return true;
        }
        if (batched)
            return s_local ? local_group_barrier(gline, (uint32_t)G, &s_bar, scr.error, scr.barrier_timeout_ticks)
                           : flat_barrier(gline, (uint32_t)G, &s_bar, scr.error, scr.barrier_timeout_ticks);
        if (xmode && s_xcd.use)
            return xcd_barrier(scr.lines, s_xcd, &s_bar, scr.error, scr.barrier_timeout_ticks, reset);
        return tree_barrier(genw, tree, (uint32_t)member, (uint32_t)G, &s_bar, scr.error, scr.barrier_timeout_ticks);
    };
    if (threadIdx.x < GF_MAX_SCALARS)
        s_scal[threadIdx.x] = inst.scal[threadIdx.x];
    if (threadIdx.x < GF_MAX_ARRAYS)
        s_arr[threadIdx.x] = inst.arr[threadIdx.x];
    const int n_pro = prog.n_pro, n_steps = prog.n_steps;
    const int64_t last_region = prog.last_region;
    if (threadIdx.x == 0) {
        s_bar.gen = __hip_atomic_load(genw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_bar.ok = 1;
        s_xcd.use = 0;
        if (xmode)
            xcd_register(scr.lines, scr.epoch, &s_xcd);
    }
    __syncthreads();
    if (xmode) {
        if (member == 0 && threadIdx.x == 0) {
            __hip_atomic_store(max_slot, kMaxKeyIdentity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(max_slot + kLineWords / 2, kMaxKeyIdentity, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!tree_barrier(genw, tree, (uint32_t)member, (uint32_t)G, &s_bar, scr.error, scr.barrier_timeout_ticks))
            return;
        if (threadIdx.x == 0)
            xcd_finalize(scr.lines, scr.epoch, &s_xcd);
        __syncthreads();
    }

    int parity = 0;   // partials half of the next reduction
    int mparity = 0;  // max slot of the next folded MAX reduction
    const int64_t total = (int64_t)n_pro + (int64_t)prog.iters * prog.n_body;
    // (sidx, iter): the step and the body iteration of flattened step si,
    // advanced incrementally
    int sidx = 0;
    int32_t iter = n_pro > 0 ? -1 : 0;
    for (int64_t si = 0; si < total; ++si) {
        if (si > 0) {
            ++sidx;
            if (sidx == n_steps) {
                sidx = n_pro;
                ++iter;
            } else if (sidx == n_pro) {
                iter = 0;
            }
        }
        const DStep &st = prog.steps[sidx];
        if (st.kind < 32) {
            const int64_t n = inst.ip[st.np];
            const bool red = st.red_op != GF_OP_NONE;
            // after the last region, a region without a reduction needs no
            // barrier: the serial steps that may follow touch no region data;
            // nor does a nowait region (the caller vouches for what follows)
            const bool need_bar = red || (si != last_region && !(st.flags & GF_STEP_NOWAIT));
            double *part = scr.partials + (parity ? scr.partials_cap : 0) + be.part_off;
            void *op[5];
#pragma unroll
            for (int k = 0; k < 5; ++k)
                op[k] = uniform_ptr(st.arr[k] >= 0 ? s_arr[st.arr[k]] : nullptr);
            const double coef = uniform_f64((st.kind == GF_R_AXPBY) ? s_scal[st.sc[1]] * st.c : 0.0);
            if (st.kind == GF_R_OWNER) {
                owner_region((int32_t *)op[0], n, st.chunk, G * blockDim.x, member * blockDim.x + threadIdx.x);
            } else if (st.kind == GF_R_PHASES) {
                if constexpr ((KMASK >> GF_R_PHASES) & 1u) {
                    if (!phases_region(gptr((double *)op[0]), gptr((double *)op[1]), gptr((int32_t *)op[2]), n,
                                       st.chunk, (int64_t)st.mask, member * blockDim.x + threadIdx.x,
                                       G * blockDim.x, barrier))
                        return;
                }
            } else if (st.kind == GF_R_HIST) {
                if constexpr ((KMASK >> GF_R_HIST) & 1u) {
                    hist_phase1((const uint32_t *)op[0], (uint32_t *)op[1], scr.hist_rows, st.mask, n, worker, G, t);
                    if (!barrier())
                        return;
                    hist_merge((uint32_t *)op[1], scr.hist_rows, st.mask, G, worker * blockDim.x + threadIdx.x,
                               G * blockDim.x);
                }
            } else {
                const int64_t nitems = region_items_dev(st, n, t);
                // fold: this workgroup's max over its items, then one atomic
                const bool fold = red && st.red_op == GF_OP_MAX && xmode && s_xcd.use;
                uint64_t *slot = max_slot + (mparity ? kLineWords / 2 : 0);
                double wmax = -INFINITY;
                for (int64_t it = worker; it < nitems; it += G) {
                    double v = region_item<KMASK, TY, PF>(st, op, coef, n, it, t);
                    if (red) {
                        v = block_reduce_rt(st.red_op, v, s_red);
                        if (fold)
                            wmax = v > wmax ? v : wmax;
                        else if (threadIdx.x == 0)
                            part[it] = v;
                    }
                }
                if (fold && threadIdx.x == 0 && worker < nitems)
                    __hip_atomic_fetch_max(slot, max_key(wmax), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (red && !fold && xmode && s_xcd.use && G > 1) {
                    // Other reductions under the XCD barrier: the last
                    // workgroup to arrive reduces the partials once (the same
                    // fixed order as below) and publishes the value; the
                    // others read one word instead of every partial.
                    uint64_t *sum_slot = (uint64_t *)(scr.lines + (int64_t)kRedSlotLine * kLineWords);
                    if (!xcd_barrier_fin(scr.lines, s_xcd, &s_bar, scr.error, scr.barrier_timeout_ticks, [&]() {
                            const double v = reduce_partials(st.red_op, part, nitems, s_red);
                            if (threadIdx.x == 0)
                                __hip_atomic_store(sum_slot, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        }))
                        return;
                    if (threadIdx.x == 0)
                        s_scal[st.sc[0]] = red_apply(
                            st.red_op, s_scal[st.sc[0]],
                            __longlong_as_double(
                                (long long)__hip_atomic_load(sum_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                    parity ^= 1;
                    __syncthreads();
                    continue;
                }
                // the last arrival resets the other slot, which the previous
                // folded region used and every workgroup has read by now
                if (need_bar && !barrier(fold ? max_slot + (mparity ? 0 : kLineWords / 2) : nullptr))
                    return;
                if (red) {
                    if (fold) {
                        if (threadIdx.x == 0)
                            s_scal[st.sc[0]] = red_apply(
                                st.red_op, s_scal[st.sc[0]],
                                max_unkey(__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                        mparity ^= 1;
                    } else {
                        const double v = reduce_partials(st.red_op, part, nitems, s_red);
                        if (threadIdx.x == 0)
                            s_scal[st.sc[0]] = red_apply(st.red_op, s_scal[st.sc[0]], v);
                    }
                    parity ^= 1;
                }
                __syncthreads();
                continue;
            }
            if (need_bar && !barrier())
                return;
        } else if (st.kind == GF_S_CALL) {
            // the first workgroup's first wavefront makes the call; the
            // barrier publishes the objects it copied back and the return
            // value to every workgroup
            if (call_fires(iter, st.every)) {
                int64_t *retw = (int64_t *)(gline + 4);
                if (member == 0 && threadIdx.x < kWave) {
                    const int64_t r = serial_call(
                        rpc, st.fmt_id, st.flags, [&](const DCallArg &a) { return (char *)s_arr[a.slot]; }, s_scal,
                        iter, scr.error);
                    if (threadIdx.x == 0)
                        __hip_atomic_store(retw, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (!barrier())
                    return;
                if (threadIdx.x == 0 && st.sc[0] >= 0)
                    s_scal[st.sc[0]] = (double)__hip_atomic_load(retw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else if (threadIdx.x == 0) {
            if (st.kind == GF_S_SWAP) {
                void *tmp = s_arr[st.arr[0]];
                s_arr[st.arr[0]] = s_arr[st.arr[1]];
                s_arr[st.arr[1]] = tmp;
            } else if (st.kind == GF_S_RECORD) {
                if (member == 0 && iter >= 0)
                    ((double *)s_arr[st.arr[0]])[iter] = s_scal[st.sc[0]];
            } else if (st.kind == GF_S_PRINTF) {
                if (member == 0 && iter >= 0 && st.every > 0 && (iter + 1) % st.every == 0)
                    serial_printf(rpc, st.fmt_id, st.nargs, st.flags, st.sc, iter, s_scal, scr.error);
            } else {
                serial_scalar(st.kind, st.sc, st.c, s_scal);
            }
        }
        // consecutive serial steps run back to back on thread 0; the
        // workgroup synchronises before the next region reads their results
        if (st.kind < 32 || si + 1 == total || prog.steps[sidx + 1 == n_steps ? n_pro : sidx + 1].kind < 32)
            __syncthreads();
    }
    if (member == 0 && threadIdx.x < GF_MAX_SCALARS)
        inst.scal[threadIdx.x] = s_scal[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Per-region kernel: one launch per region. Work items are dealt over the
// grid; with a reduction clause each item writes its partial and the last
// workgroup to finish (arrival counter) reduces all partials in a fixed
// order, combines the result into the scalar variable and runs the serial
// glue that follows the region in the program.
// ---------------------------------------------------------------------------

// Called by the first wavefront of the finishing workgroup: a GF_S_CALL
// uses all of its lanes, the other serial steps lane 0 alone.
__device__ inline void run_glue(const RegionLaunch &rl, const RpcRing &rpc, int32_t *err)
{
    const bool lane0 = threadIdx.x == 0;
    for (int g = 0; g < rl.n_glue; ++g) {
        const Glue &gl = rl.glue[g];
        if (gl.kind == GF_S_CALL) {
            if (call_fires(gl.iter, gl.every)) {
                const int64_t r = serial_call(
                    rpc, gl.fmt_id, gl.flags, [&](const DCallArg &a) { return (char *)gl.obj[a.ref]; }, rl.scal,
                    gl.iter, err);
                if (lane0 && gl.sc[0] >= 0)
                    rl.scal[gl.sc[0]] = (double)r;
            }
        } else if (!lane0) {
            continue;
        } else if (gl.kind == GF_S_RECORD) {
            if (gl.iter >= 0)
                gl.rec[gl.iter] = rl.scal[gl.sc[0]];
        } else if (gl.kind == GF_S_PRINTF) {
            if (gl.iter >= 0 && gl.every > 0 && (gl.iter + 1) % gl.every == 0)
                serial_printf(rpc, gl.fmt_id, gl.nargs, gl.flags, gl.sc, gl.iter, rl.scal, err);
        } else {
            serial_scalar(gl.kind, gl.sc, gl.c, rl.scal);
        }
    }
}

template <unsigned KMASK, int TY, int PF>
__global__ void __launch_bounds__(family_max_threads<KMASK>()) k_region(RegionLaunch rl, Tiling t, Scratch scr,
                                                                         RpcRing rpc)
{
    __shared__ double s_red[kLdsRed];
    __shared__ int s_last;
    const DStep &st = rl.step;
    const int64_t G = gridDim.x;
    const bool red = st.red_op != GF_OP_NONE;
    double *part = scr.partials;
    if (st.kind == GF_R_OWNER) {
        owner_region((int32_t *)rl.arr[0], rl.n, st.chunk, G * blockDim.x,
                     (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    } else if (st.kind == GF_R_HIST) {
        // phase 1 only; k_hist_merge finishes the region and runs the glue
        if constexpr ((KMASK >> GF_R_HIST) & 1u)
            hist_phase1((const uint32_t *)rl.arr[0], (uint32_t *)rl.arr[1], scr.hist_rows, st.mask, rl.n,
                        worker_id(blockIdx.x, G, t.xcd_remap), G, t);
        return;
    } else if (st.kind < 32) {
        const double coef = (st.kind == GF_R_AXPBY) ? rl.scal[st.sc[1]] * st.c : 0.0;
        const int64_t worker = worker_id(blockIdx.x, G, t.xcd_remap);
        for (int64_t it = worker; it < rl.n_items; it += G) {
            double v = region_item<KMASK, TY, PF>(st, rl.arr, coef, rl.n, it, t);
            if (red) {
                v = block_reduce_rt(st.red_op, v, s_red);
                if (threadIdx.x == 0)
                    __hip_atomic_store(part + it, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (!red && rl.n_glue == 0)
        return;
    // Last-workgroup finalize. The finishing workgroup reads the partials
    // (stored at agent scope above, so they are in memory once acknowledged)
    // and the scalars, which this region does not write. Only glue that
    // reads the region's arrays (a host call with references) needs every
    // workgroup's L2 written back first; otherwise settling suffices: each
    // workgroup's loads have returned and its partials are acknowledged
    // before it counts itself done. The per-workgroup L2 write-back is most
    // of the finalize's cost (a 16 MiB axpby takes 10 us alone, 34 us with
    // it).
    // Counting is two-level: workgroup b arrives on sub-counter b mod 8 (its
    // own 128-byte line), and the last arrival of each sub-counter on the
    // top counter. One word taking every workgroup's atomic serialised them
    // (about 10 us for 1,024 workgroups).
    uint32_t *cnt = scr.lines + (int64_t)(kFinalizeLine0 + rl.inst) * kLineWords;
    if (rl.publish)
        wg_publish();
    else
        wg_settle();
    if (threadIdx.x == 0) {
        const uint32_t ug = (uint32_t)G, g = blockIdx.x % kNumXcd;
        const uint32_t nsub = ug < (uint32_t)kNumXcd ? ug : (uint32_t)kNumXcd;
        const uint32_t members = ug / kNumXcd + (g < ug % kNumXcd ? 1u : 0u);
        uint32_t *sub = scr.lines + ((int64_t)kFinalizeSubLine0 + (int64_t)rl.inst * kNumXcd + g) * kLineWords;
        int last = 0;
        if (__hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
            // every member of this sub-counter has arrived: reset it for the
            // next launch (the launch boundary orders the two)
            __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nsub - 1;
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last)
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (red) {
        const double v = reduce_partials<true>(st.red_op, part, rl.n_items, s_red);
        if (threadIdx.x == 0)
            rl.scal[st.sc[0]] = red_apply(st.red_op, rl.scal[st.sc[0]], v);
    }
    if (threadIdx.x < kWave)
        run_glue(rl, rpc, scr.error);
    if (threadIdx.x == 0)
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Kernel split (paper, Section 3.3): the main program runs on one thread of
// a one-wavefront kernel; a region is a blocking RPC asking the host to
// launch the region kernel and wait for it. Serial steps act directly on the
// instance's scalar variables in device memory; SWAPs permute a table of the
// array slots (4 bits per slot) that travels with each request. The RPC's
// system-scope release and acquire order the main thread's scalar writes
// before the region and the region's results before the next serial step.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kWave) k_main(DProg prog, DInst inst, RpcRing rpc, Scratch scr)
{
    // the whole wavefront walks the program (a GF_S_CALL uses every lane);
    // lane 0 alone performs the other side effects
    const bool lane0 = threadIdx.x == 0;
    uint64_t perm = 0;
    for (int k = 0; k < GF_MAX_ARRAYS; ++k)
        perm |= (uint64_t)k << (4 * k);
    auto slot_of = [&](int a) -> int { return (int)((perm >> (4 * a)) & 15u); };
    double *scal = inst.scal;
    const int64_t total = (int64_t)prog.n_pro + (int64_t)prog.iters * prog.n_body;
    int sidx = 0;
    int32_t iter = prog.n_pro > 0 ? -1 : 0;
    for (int64_t si = 0; si < total; ++si) {
        if (si > 0) {
            ++sidx;
            if (sidx == prog.n_steps) {
                sidx = prog.n_pro;
                ++iter;
            } else if (sidx == prog.n_pro) {
                iter = 0;
            }
        }
        const DStep &st = prog.steps[sidx];
        if (st.kind < 32) {
            int ok = 1;
            if (lane0) {
                uint64_t args[3] = {(uint64_t)sidx, (uint64_t)(int64_t)iter, perm};
                int64_t ret = -1;
                if (!rpc_call(rpc, kCalleeRegion, 0, 3, args, GF_STEP_BLOCKING, &ret, scr.error)) {
                    ok = 0;
                } else if (ret != 0) {
                    set_error(scr.error, kErrRegionLaunch);
                    ok = 0;
                }
            }
            if (!__builtin_amdgcn_readfirstlane(ok))
                return;
            // every lane sees the region's results
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        } else if (st.kind == GF_S_SWAP) {
            const int a = st.arr[0], b = st.arr[1];
            const uint64_t va = (perm >> (4 * a)) & 15u, vb = (perm >> (4 * b)) & 15u;
            perm &= ~((uint64_t)15 << (4 * a)) & ~((uint64_t)15 << (4 * b));
            perm |= (vb << (4 * a)) | (va << (4 * b));
        } else if (st.kind == GF_S_CALL) {
            if (call_fires(iter, st.every)) {
                const int64_t r = serial_call(
                    rpc, st.fmt_id, st.flags,
                    [&](const DCallArg &a) { return (char *)inst.arr[slot_of(a.slot)]; }, scal, iter, scr.error);
                if (lane0 && st.sc[0] >= 0)
                    scal[st.sc[0]] = (double)r;
            }
        } else if (!lane0) {
            continue;
        } else if (st.kind == GF_S_RECORD) {
            if (iter >= 0)
                ((double *)inst.arr[slot_of(st.arr[0])])[iter] = scal[st.sc[0]];
        } else if (st.kind == GF_S_PRINTF) {
            if (iter >= 0 && st.every > 0 && (iter + 1) % st.every == 0)
                serial_printf(rpc, st.fmt_id, st.nargs, st.flags, st.sc, iter, scal, scr.error);
        } else {
            serial_scalar(st.kind, st.sc, st.c, scal);
        }
    }
    // the region kernels and the host read the scalars after the kernel ends
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
}

hipError_t launch_main(const DProg &prog, const DInst &inst, const RpcRing &rpc, const Scratch &scr, hipStream_t s)
{
    hipLaunchKernelGGL(k_main, dim3(1), dim3(kWave), 0, s, prog, inst, rpc, scr);
    return hipGetLastError();
}

// Histogram phase 2 of the per-region mode: merge the `rows_used` partial
// rows of phase 1 into the bins; the last workgroup runs the glue.
__global__ void __launch_bounds__(kMaxWg) k_hist_merge(RegionLaunch rl, int64_t rows_used, Scratch scr, RpcRing rpc)
{
    __shared__ int s_last;
    const int64_t G = gridDim.x;
    hist_merge((uint32_t *)rl.arr[1], scr.hist_rows, rl.step.mask, rows_used,
               (int64_t)blockIdx.x * blockDim.x + threadIdx.x, G * blockDim.x);
    if (rl.n_glue == 0)
        return;
    uint32_t *cnt = scr.lines + (int64_t)(kFinalizeLine0 + rl.inst) * kLineWords;
    wg_publish();
    if (threadIdx.x == 0) {
        const uint32_t a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (a == (uint32_t)G - 1);
    }
    __syncthreads();
    if (!s_last)
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x < kWave)
        run_glue(rl, rpc, scr.error);
    if (threadIdx.x == 0)
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Per-region launch of GF_R_PHASES: the in-region barrier is a grid barrier
// inside the kernel (the persistent kernel's counters, free while no
// persistent launch of this context runs), so the host launches at most one
// co-resident wave of workgroups. The last workgroup runs the glue.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kMaxWg) k_phases(RegionLaunch rl, Scratch scr, RpcRing rpc)
{
    __shared__ BarrierState s_bar;
    __shared__ int s_last;
    const int64_t G = gridDim.x;
    uint32_t *genw = scr.lines + 1;
    uint32_t *tree = scr.lines + kTreeLine0 * kLineWords;
    if (threadIdx.x == 0) {
        s_bar.gen = __hip_atomic_load(genw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_bar.ok = 1;
    }
    __syncthreads();
    auto bar = [&]() -> bool {
        if (G == 1) {
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
            return true;
        }
        return tree_barrier(genw, tree, blockIdx.x, (uint32_t)G, &s_bar, scr.error, scr.barrier_timeout_ticks);
    };
    if (!phases_region(gptr((double *)rl.arr[0]), gptr((double *)rl.arr[1]), gptr((int32_t *)rl.arr[2]), rl.n,
                       rl.step.chunk, (int64_t)rl.step.mask, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                       G * blockDim.x, bar))
        return;
    if (rl.n_glue == 0)
        return;
    uint32_t *cnt = scr.lines + (int64_t)(kFinalizeLine0 + rl.inst) * kLineWords;
    wg_publish();
    if (threadIdx.x == 0) {
        const uint32_t a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (a == (uint32_t)G - 1);
    }
    __syncthreads();
    if (!s_last)
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x < kWave)
        run_glue(rl, rpc, scr.error);
    if (threadIdx.x == 0)
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_phases(const RegionLaunch &rl, int wg_size, int num_wg, const Scratch &scr, const RpcRing &rpc,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_phases, dim3(num_wg), dim3(wg_size), 0, s, rl, scr, rpc);
    return hipGetLastError();
}

int phases_capacity(int wg_size, int num_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_phases), wg_size, 0) !=
        hipSuccess)
        return 0;
    // one slot per CU is left free (the kernel split's main kernel may hold one)
    return (per_cu > 1 ? per_cu - 1 : per_cu) * num_cu;
}

// ---------------------------------------------------------------------------
// Kernel selection. Families: the bodies a program uses decide which
// instantiation runs, so a program only pays the registers of its own bodies.
// ---------------------------------------------------------------------------

constexpr unsigned kFamJ3 = (1u << GF_R_JACOBI3D) | (1u << GF_R_OWNER);
static_assert(persistent_min_waves<kFamJ3, 2, 1>() == 3, "3D stencil family mask");
constexpr unsigned kFamJ2 = (1u << GF_R_JACOBI2D) | (1u << GF_R_OWNER);
static_assert(persistent_min_waves<kFamJ2, 1, 1>() == 3, "2D stencil family mask");
constexpr unsigned kFamVec =
    (1u << GF_R_SPMV) | (1u << GF_R_DOT) | (1u << GF_R_AXPBY) | (1u << GF_R_OWNER) | (1u << GF_R_PHASES);
constexpr unsigned kFamAll = kFamJ3 | kFamJ2 | kFamVec;  // the histogram runs only in its own family

static unsigned program_kinds(const DProg &p)
{
    unsigned m = 0;
    for (int i = 0; i < p.n_steps; ++i)
        if (p.steps[i].kind < 32)
            m |= 1u << p.steps[i].kind;
    return m;
}

static unsigned pick_family(unsigned kinds)
{
    if ((kinds & ~kFamHist) == 0 && (kinds & (1u << GF_R_HIST)))
        return kFamHist;
    if ((kinds & ~kFamJ3) == 0)
        return kFamJ3;
    if ((kinds & ~kFamJ2) == 0)
        return kFamJ2;
    if ((kinds & ~kFamVec) == 0)
        return kFamVec;
    return kFamAll;
}

typedef void (*PersistentFn)(DProg, DInst, Tiling, Scratch, RpcRing, BatchTable);
typedef void (*RegionFn)(RegionLaunch, Tiling, Scratch, RpcRing);

// The prefetch depth is a kernel template parameter so each kernel carries
// one plane ring; depth 2 exists only for the 3D stencil family at the tile
// heights the tuner explores.
template <unsigned F>
static PersistentFn persistent_for_ty(int ty, int pf)
{
    if constexpr (F == kFamVec || F == kFamHist || F == kFamJ2) {
        return ty >= 1 && pf == 1 ? k_persistent<F, 1, 1> : nullptr;
    } else {
        if constexpr (F == kFamJ3) {
            if (pf == 2) {
                switch (ty) {
                case 1: return k_persistent<F, 1, 2>;
                case 2: return k_persistent<F, 2, 2>;
                case 4: return k_persistent<F, 4, 2>;
                case 8: return k_persistent<F, 8, 2>;
                default: return nullptr;
                }
            }
        }
        if (pf != 1)
            return nullptr;
        switch (ty) {
        case 1: return k_persistent<F, 1, 1>;
        case 2: return k_persistent<F, 2, 1>;
        case 4: return k_persistent<F, 4, 1>;
        case 8: return k_persistent<F, 8, 1>;
        case 16: return k_persistent<F, 16, 1>;
        default: return nullptr;
        }
    }
}

template <unsigned F>
static RegionFn region_for_ty(int ty, int pf)
{
    if constexpr (F == kFamVec || F == kFamHist || F == kFamJ2) {
        return ty >= 1 && pf == 1 ? k_region<F, 1, 1> : nullptr;
    } else {
        if constexpr (F == kFamJ3) {
            if (pf == 2) {
                switch (ty) {
                case 1: return k_region<F, 1, 2>;
                case 2: return k_region<F, 2, 2>;
                case 4: return k_region<F, 4, 2>;
                case 8: return k_region<F, 8, 2>;
                default: return nullptr;
                }
            }
        }
        if (pf != 1)
            return nullptr;
        switch (ty) {
        case 1: return k_region<F, 1, 1>;
        case 2: return k_region<F, 2, 1>;
        case 4: return k_region<F, 4, 1>;
        case 8: return k_region<F, 8, 1>;
        case 16: return k_region<F, 16, 1>;
        default: return nullptr;
        }
    }
}

// Families other than the 3D stencil have no plane ring: their prefetch
// depth is ignored.
static PersistentFn persistent_fn(unsigned fam, int ty, int pf)
{
    switch (fam) {
    case kFamJ3: return persistent_for_ty<kFamJ3>(ty, pf);
    case kFamJ2: return persistent_for_ty<kFamJ2>(1, 1);
    case kFamVec: return persistent_for_ty<kFamVec>(1, 1);
    case kFamHist: return persistent_for_ty<kFamHist>(1, 1);
    default: return persistent_for_ty<kFamAll>(ty, 1);
    }
}

static RegionFn region_fn(int kind, int ty, int pf)
{
    switch (kind) {
    case GF_R_JACOBI3D: return region_for_ty<kFamJ3>(ty, pf);
    case GF_R_JACOBI2D: return region_for_ty<kFamJ2>(1, 1);
    case GF_R_HIST: return region_for_ty<kFamHist>(1, 1);
    default: return region_for_ty<kFamVec>(1, 1);
    }
}

bool program_is_hist_family(const DProg &prog) { return pick_family(program_kinds(prog)) == kFamHist; }

bool program_mixes_hist(const DProg &prog)
{
    const unsigned k = program_kinds(prog);
    return (k & (1u << GF_R_HIST)) && (k & ~kFamHist);
}

int64_t hist_row_words() { return kHistPart; }

int64_t hist_parts(uint32_t mask) { return cdiv((int64_t)mask + 1, kHistPart); }

hipError_t launch_hist_merge(const RegionLaunch &rl, int64_t rows_used, const Scratch &scr, const RpcRing &rpc,
                             int num_cu, hipStream_t s)
{
    // one thread per (four bins, slice of up to 16 rows of the part)
    const int64_t nbins = (int64_t)rl.step.mask + 1;
    const int64_t per_part = rows_used / cdiv(nbins, kHistPart);
    const int64_t slices = per_part < 16 ? (per_part < 1 ? 1 : per_part) : 16;
    int64_t g = cdiv(cdiv(nbins, 4) * slices, kMaxWg);
    if (g > (int64_t)num_cu * 16)
        g = (int64_t)num_cu * 16;
    hipLaunchKernelGGL(k_hist_merge, dim3((unsigned)g), dim3(kMaxWg), 0, s, rl, rows_used, scr, rpc);
    return hipGetLastError();
}

int region_capacity(int kind, const Tiling &t, int num_cu)
{
    RegionFn fn = region_fn(kind, t.tile_y, t.prefetch);
    if (!fn)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), t.wg_size, 0) !=
        hipSuccess)
        return 0;
    return per_cu * num_cu;
}

int persistent_capacity(const DProg &prog, const Tiling &t, int num_cu)
{
    PersistentFn fn = persistent_fn(pick_family(program_kinds(prog)), t.tile_y, t.prefetch);
    if (!fn)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), t.wg_size, 0) !=
        hipSuccess)
        return 0;
    return per_cu * num_cu;
}

hipError_t launch_persistent(const DProg &prog, const DInst &inst, const Tiling &t, int num_wg, const Scratch &scr,
                             const RpcRing &rpc, hipStream_t s, const BatchTable *batch)
{
    PersistentFn fn = persistent_fn(pick_family(program_kinds(prog)), t.tile_y, t.prefetch);
    if (!fn)
        return hipErrorInvalidValue;
    DProg p = prog;
    DInst i = inst;
    Tiling tt = t;
    Scratch sc = scr;
    RpcRing r = rpc;
    BatchTable bt{nullptr, nullptr, 0};
    if (batch)
        bt = *batch;
    void *args[] = {&p, &i, &tt, &sc, &r, &bt};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(num_wg), dim3(t.wg_size), args, 0, s);
}

hipError_t launch_region(const RegionLaunch &rl, const Tiling &t, int num_wg, const Scratch &scr,
                         const RpcRing &rpc, hipStream_t s)
{
    RegionFn fn = region_fn(rl.step.kind, t.tile_y, t.prefetch);
    if (!fn)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(num_wg), dim3(t.wg_size), 0, s, rl, t, scr, rpc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gf_reduce: a stand-alone reduction region over a device array. Fixed
// two-level tree: each workgroup reduces a contiguous block (strided per
// thread), the last workgroup reduces the per-block partials in order.
// ---------------------------------------------------------------------------

template <typename T, int OP>
struct TRed;
template <typename T>
struct TRed<T, GF_OP_SUM> {
    static __device__ T id() { return (T)0; }
    static __device__ T ap(T a, T b) { return a + b; }
};
template <typename T>
struct TRed<T, GF_OP_MAX> {
    static __device__ T id();
    static __device__ T ap(T a, T b) { return a > b ? a : b; }
};
template <>
__device__ double TRed<double, GF_OP_MAX>::id() { return -INFINITY; }
template <>
__device__ uint64_t TRed<uint64_t, GF_OP_MAX>::id() { return 0; }
template <>
__device__ int64_t TRed<int64_t, GF_OP_MAX>::id() { return INT64_MIN; }

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int off)
{
    if constexpr (sizeof(T) == 8) {
        int64_t b;
        __builtin_memcpy(&b, &v, 8);
        b = __shfl_xor((long long)b, off, kWave);
        __builtin_memcpy(&v, &b, 8);
        return v;
    } else {
        return __shfl_xor(v, off, kWave);
    }
}

template <typename T, int OP>
__device__ __forceinline__ T block_reduce_t(T v, T *lds)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = TRed<T, OP>::ap(v, shfl_xor_t(v, off));
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane == 0)
        lds[wid] = v;
    __syncthreads();
    if (wid == 0) {
        v = lane < nw ? lds[lane] : TRed<T, OP>::id();
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1)
            v = TRed<T, OP>::ap(v, shfl_xor_t(v, off));
    }
    __syncthreads();
    return v;
}

// In: element type TI; accumulation/output type T (u32 sums widen to u64).
template <typename TI, typename T, int OP>
__global__ void __launch_bounds__(kMaxWg) k_reduce(const TI *__restrict__ in, int64_t n, T *out, T *partials,
                                                    uint32_t *cnt)
{
    __shared__ T s_red[kLdsRed];
    __shared__ int s_last;
    const int64_t G = gridDim.x;
    const int64_t per = cdiv(n, G);
    const int64_t lo = blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    T acc = TRed<T, OP>::id();
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
        acc = TRed<T, OP>::ap(acc, (T)in[i]);
    acc = block_reduce_t<T, OP>(acc, s_red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = acc;
    wg_publish();
    if (threadIdx.x == 0) {
        const uint32_t a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (a == (uint32_t)G - 1);
    }
    __syncthreads();
    if (!s_last)
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    T v = TRed<T, OP>::id();
    for (int64_t i = threadIdx.x; i < G; i += blockDim.x)
        v = TRed<T, OP>::ap(v, partials[i]);
    v = block_reduce_t<T, OP>(v, s_red);
    if (threadIdx.x == 0) {
        out[0] = v;
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

int64_t reduce_grid(int64_t n, int num_cu, int64_t max_wg)
{
    // Enough workgroups to stream at full bandwidth, each with >= 4K elements.
    int64_t g = cdiv(n, 4096);
    int64_t gmax = (int64_t)num_cu * 4;
    if (gmax > max_wg)
        gmax = max_wg;
    if (g > gmax)
        g = gmax;
    if (g < 1)
        g = 1;
    return g;
}

hipError_t launch_reduce(int op, int dt, const void *in, int64_t n, void *out, const Scratch &scr, int num_cu,
                         hipStream_t s)
{
    uint32_t *cnt = scr.lines + (int64_t)(kFinalizeLine0 + GF_MAX_INSTANCES - 1) * kLineWords;
    return launch_reduce_into(op, dt, in, n, out, scr.partials, cnt, reduce_grid(n, num_cu, INT32_MAX), s);
}

__global__ void __launch_bounds__(kWave) k_clear_u32(uint32_t *p, int32_t n)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0u;
}

hipError_t launch_clear_u32(uint32_t *p, int32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(kWave), 0, s, p, n);
    return hipGetLastError();
}

// The reduction kernels on caller-given scratch: `part` holds g partials of
// the accumulation type (8 bytes each), `cnt` one counter word that is zero
// on entry and is left zero.
hipError_t launch_reduce_into(int op, int dt, const void *in, int64_t n, void *out, void *part, uint32_t *cnt,
                              int64_t g, hipStream_t s)
{
    const dim3 grid((unsigned)g), blk(kMaxWg);
#define GF_RED(TI, T, OP) \
    hipLaunchKernelGGL((k_reduce<TI, T, OP>), grid, blk, 0, s, (const TI *)in, n, (T *)out, (T *)part, cnt)
    if (op == GF_OP_SUM) {
        switch (dt) {
        case GF_F64: GF_RED(double, double, GF_OP_SUM); break;
        case GF_U32: GF_RED(uint32_t, uint64_t, GF_OP_SUM); break;
        case GF_U64: GF_RED(uint64_t, uint64_t, GF_OP_SUM); break;
        case GF_I64: GF_RED(int64_t, int64_t, GF_OP_SUM); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (dt) {
        case GF_F64: GF_RED(double, double, GF_OP_MAX); break;
        case GF_U32: GF_RED(uint32_t, uint64_t, GF_OP_MAX); break;
        case GF_U64: GF_RED(uint64_t, uint64_t, GF_OP_MAX); break;
        case GF_I64: GF_RED(int64_t, int64_t, GF_OP_MAX); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef GF_RED
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Copy kernel: the achievable HBM ceiling (16-byte loads and nontemporal
// stores, grid-stride).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kMaxWg) k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, int64_t n)
{
    // four 16-byte loads in flight per thread per trip
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        double2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            __builtin_nontemporal_store(v[k].x, &dst[i + k * stride].x);
            __builtin_nontemporal_store(v[k].y, &dst[i + k * stride].y);
        }
    }
    for (; i < n; i += stride) {
        const double2 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
    }
}

// One tile of 4 x 16 bytes per thread, no grid-stride loop: the whole array
// is covered by the grid (STREAM-style).
__global__ void __launch_bounds__(kMaxWg) k_copy_tiles(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                      int64_t n)
{
    // 16-byte accesses with streaming hints on both sides: measured the
    // fastest copy form (1 GiB)
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x;
    GF_GLOBAL const gf_d2 *s2 = (GF_GLOBAL const gf_d2 *)src;
    GF_GLOBAL gf_d2 *d2 = (GF_GLOBAL gf_d2 *)dst;
    gf_d2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * blockDim.x < n)
            v[k] = __builtin_nontemporal_load(s2 + base + k * blockDim.x);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * blockDim.x < n)
            __builtin_nontemporal_store(v[k], d2 + base + k * blockDim.x);
}

hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, int num_wg, hipStream_t s)
{
    const int64_t n = nbytes / 16;
    if (num_wg <= 0) {
        const int64_t g = cdiv(n, (int64_t)kMaxWg * 4);
        if (g > 0)
            hipLaunchKernelGGL(k_copy_tiles, dim3((unsigned)g), dim3(kMaxWg), 0, s, (const double2 *)src,
                               (double2 *)dst, n);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_copy, dim3(num_wg), dim3(kMaxWg), 0, s, (const double2 *)src, (double2 *)dst, n);
    return hipGetLastError();
}

}  // namespace gf
