// Device functions shared by the gfx950 kernels of the polyenergetic
// cone-beam projector: ray set-up, the two-level voxel walk and the plain
// spectral group sum.
//
// One lane follows one ray (one detector pixel of one angle); one wavefront
// covers a compact tile of detector pixels of one angle (8 x 8, or 16 x 4
// where the phantom covers few detector rows), so its rays are neighbours in
// space: they cross the same bricks at nearly the same steps (little
// divergence), share voxel cache lines and write their results as short
// coalesced row segments.
//
// Ray traversal (Sec. II.F: a projection is the line integral of the
// attenuation along the ray; Sec. II.C: the phantom holds material labels,
// so the integral is sum_m mu_m(E) L_m): entry and exit are found in FP64 by
// the slab method, the ray is re-based at its entry point and then walked
// in FP32 distance from there (incremental form of Siddon's exact method),
// over bricks of voxels first and over single voxels only inside bricks
// whose labels differ.  Each plane crossing is t0 + k dt evaluated with one
// rounding, so the error does not grow with the number of planes.  Path
// length is charged to a material only when the label changes, with
// compensated (Kahan) summation, so its error scales with the number of
// material transitions rather than with the number of voxels.
#pragma once

#include "fcat_internal.h"

#include <cmath>

namespace fcat {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// BF16 bits of x, round to nearest, ties to even.
__device__ __forceinline__ uint32_t bf16_rne(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to packed BF16 (a in the low half), round to nearest, ties to
// even: one v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    const bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// hi = bf16(v), lo = bf16(v - hi) for a pair of floats (v - hi is exact in FP32).
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t &hi, uint32_t &lo)
{
    hi = pack_bf16x2(a, b);
    lo = pack_bf16x2(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Orders the LDS accesses of one wavefront around this point (a compiler and
// memory fence at wavefront scope): needed where a wavefront reuses its own
// LDS block under another type or layout.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hardware hands consecutive workgroups to the 8 XCDs in turn.  Remap so that
// each XCD (and its L2) works through one contiguous range of rays.  The
// grid is padded to a multiple of kXcds so the map is a bijection.
__device__ __forceinline__ int xcd_block(int nblk_padded)
{
    const int b = blockIdx.x;
    const int per = nblk_padded / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Pixel of lane `lane` of wavefront gw (see TraceGeom::tile_log2u): tiles of
// an angle in row-major order, lanes row-major inside a tile.
struct PixelOf {
    int al, iv, iu;
    bool valid;
};

__device__ __forceinline__ int tiles_per_angle(const TraceGeom &G)
{
    const int tu = 1 << G.tile_log2u, tv = kWave >> G.tile_log2u;
    return ((G.nu + tu - 1) / tu) * ((G.nv + tv - 1) / tv);
}

__device__ __forceinline__ PixelOf pixel_of(const TraceGeom &G, int gw, int lane)
{
    const int tu = 1 << G.tile_log2u;
    const int tu_n = (G.nu + tu - 1) >> G.tile_log2u;
    const int per = tiles_per_angle(G);
    PixelOf p;
    p.al = gw / per;
    const int rem = gw - p.al * per;
    const int tv_i = rem / tu_n, tu_i = rem - tv_i * tu_n;
    p.iv = (tv_i << (6 - G.tile_log2u)) + (lane >> G.tile_log2u);
    p.iu = (tu_i << G.tile_log2u) + (lane & (tu - 1));
    p.valid = p.iv < G.nv && p.iu < G.nu;
    return p;
}

// A read-only table seen through the constant address space.  The compiler
// then loads its wave-uniform entries once per wavefront (scalar loads)
// even after an LDS fence, a wave barrier, an asm statement or a store it
// cannot prove disjoint from the table, any of which otherwise turns them
// into one load per lane.  Only for data that no kernel of the launch
// writes (the spectral tables and the network's terms).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *const_table(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Per-ray constants of the two-level walk.  Distances t are measured in mm
// from the point where the ray enters the grid.
struct Ray {
    float t_end;        // exit distance
    float t0[3];        // first voxel-plane crossing per axis (inf if parallel)
    float dt[3];        // distance between voxel-plane crossings (0 if parallel)
    float inv_dt[3];    // 1 / dt (0 if parallel)
    float tc0[3];       // first brick-plane crossing per axis (inf if parallel)
    float dtc[3];       // distance between brick-plane crossings (0 if parallel, so that
                        // k * dtc + tc0 stays inf without a test)
    int i0[3];          // entry voxel
    int sgn[3];         // direction of travel per axis: +1, -1, or 0 if parallel
    float t_bg;         // length outside the background box (TraceGeom::clip), all of it background
    bool walk;          // the ray meets the background box: the walk runs over [0, t_end)
};

// FP64 set-up of the ray from the source to the centre of pixel (iv, iu):
// entry and exit by the slab method, then everything re-based at the entry
// point and rounded once to FP32.
__device__ __forceinline__ bool setup_ray(const TraceGeom &G, double ct, double st, int iv, int iu, Ray &r)
{
    const double pu = ((double)iu - G.cu) * G.du + G.off_u;
    const double pv = ((double)iv - G.cv) * G.dv + G.off_v;
    const double s[3] = {G.sid * ct, G.sid * st, 0.0};
    const double p[3] = {-G.back * ct - pu * st, -G.back * st + pu * ct, pv};
    double d[3], inv[3];
    double amin = 0.0, amax = 1.0;
    bool inside = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        d[ax] = p[ax] - s[ax];
        const double lo = G.lo[ax];
        const double hi = G.lo[ax] + G.n[ax] * G.h[ax];
        if (d[ax] == 0.0) {
            inv[ax] = 0.0;
            inside = inside && s[ax] >= lo && s[ax] < hi;
        } else {
            inv[ax] = 1.0 / d[ax];
            const double a0 = (lo - s[ax]) * inv[ax];
            const double a1 = (hi - s[ax]) * inv[ax];
            amin = fmax(amin, fmin(a0, a1));
            amax = fmin(amax, fmax(a0, a1));
        }
    }
    if (!inside || !(amax > amin)) return false;
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    // the walk covers the background box only; the rest of the ray is
    // background and is charged in one sum
    int clo[3] = {0, 0, 0}, chi[3] = {G.n[0], G.n[1], G.n[2]};
    r.t_bg = 0.0f;
    r.walk = true;
    const auto *c = const_table(G.clip);
    // (wave-uniform: a box that is the whole grid clips nothing)
    if (G.clip && !(c[7] != 0 && c[1] == 0 && c[2] == 0 && c[3] == 0 && c[4] == G.n[0] && c[5] == G.n[1] &&
                    c[6] == G.n[2])) {
        double bmin = amin, bmax = amax;
        bool meets = c[7] != 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            clo[ax] = c[1 + ax];
            chi[ax] = c[4 + ax];
            const double lo = G.lo[ax] + clo[ax] * G.h[ax];
            const double hi = G.lo[ax] + chi[ax] * G.h[ax];
            if (d[ax] == 0.0) {
                meets = meets && s[ax] >= lo && s[ax] < hi;
            } else {
                const double a0 = (lo - s[ax]) * inv[ax];
                const double a1 = (hi - s[ax]) * inv[ax];
                bmin = fmax(bmin, fmin(a0, a1));
                bmax = fmin(bmax, fmax(a0, a1));
            }
        }
        if (!meets || !(bmax > bmin)) {
            r.t_bg = (float)((amax - amin) * len);
            r.t_end = 0.0f;
            r.walk = false;
            return true;
        }
        r.t_bg = (float)(((bmin - amin) + (amax - bmax)) * len);
        amin = bmin;
        amax = bmax;
    }
    r.t_end = (float)((amax - amin) * len);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double q = (s[ax] + amin * d[ax] - G.lo[ax]) * G.inv_h[ax];
        // entering through a plane: the voxel beyond it in the direction of travel
        int i = d[ax] < 0.0 ? (int)ceil(q) - 1 : (int)floor(q);
        i = min(max(i, clo[ax]), chi[ax] - 1);
        r.i0[ax] = i;
        if (d[ax] != 0.0) {
            const int plane = d[ax] > 0.0 ? i + 1 : i;
            const double ap = (G.lo[ax] + plane * G.h[ax] - s[ax]) * inv[ax];
            const double step = G.h[ax] * len * fabs(inv[ax]);
            r.t0[ax] = (float)fmax((ap - amin) * len, 0.0);
            r.dt[ax] = (float)step;
            // only the first estimate of a crossing count uses it (the count
            // is then corrected by up to one), so a reciprocal of about one
            // ulp suffices
            r.inv_dt[ax] = __builtin_amdgcn_rcpf(r.dt[ax]);
            const int b = i / kBrickEdge;
            const int bplane = (d[ax] > 0.0 ? b + 1 : b) * kBrickEdge;
            const double bp = (G.lo[ax] + bplane * G.h[ax] - s[ax]) * inv[ax];
            r.tc0[ax] = (float)fmax((bp - amin) * len, 0.0);
            r.dtc[ax] = (float)(step * kBrickEdge);
            r.sgn[ax] = d[ax] > 0.0 ? 1 : -1;
        } else {
            r.t0[ax] = INFINITY;
            r.dt[ax] = 0.0f;
            r.inv_dt[ax] = 0.0f;
            r.tc0[ax] = INFINITY;
            r.dtc[ax] = 0.0f;
            r.sgn[ax] = 0;
        }
    }
    return true;
}

// Per-lane material accumulators in LDS.  A run of path length is charged
// to its material only when the label changes, but the lanes of a wavefront
// change label at different steps, so a register file indexed by
// compare-select (two selects per material and value) would cost the whole
// wavefront tens of instructions on almost every step.  LDS takes the
// material as an index instead.  Layout per wavefront: FP32 sums [MP+1][64],
// then the Kahan compensations [MP+1][64] held as BF16 (a compensation is
// below half an ulp of its sum; BF16 keeps it to 0.4%, which leaves the
// compensated sum's error far below one FP32 ulp and keeps the block small
// enough for full occupancy).  Lane-contiguous, free of bank conflicts.
template <int MP>
struct MatAcc {
    float *sum;          // this lane's slot of the sums
    uint16_t *comp;      // this lane's slot of the compensations

    __device__ __forceinline__ MatAcc(float *wave_block, int lane)
        : sum(wave_block + lane), comp(reinterpret_cast<uint16_t *>(wave_block + (MP + 1) * kWave) + lane)
    {
    }
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int m = 0; m < MP + 1; ++m) {
            sum[m * kWave] = 0.0f;
            comp[m * kWave] = 0;
        }
    }
    // Compensated add of x to material m.  Labels outside 0..MP-1 go to a
    // spare slot (index MP) that is never read, so no test is needed.
    __device__ __forceinline__ void add(unsigned m, float x)
    {
        const unsigned k = min(m, static_cast<unsigned>(MP));
        const float l = sum[k * kWave];
        const float c = bf16_value(comp[k * kWave]);
        const float y = x - c;
        const float t = l + y;
        comp[k * kWave] = static_cast<uint16_t>(pack_bf16x2((t - l) - y, 0.0f));
        sum[k * kWave] = t;
    }
    __device__ __forceinline__ void read(float (&L)[MP]) const
    {
#pragma unroll
        for (int m = 0; m < MP; ++m) L[m] = sum[m * kWave];
    }
};

// LDS floats per wavefront of MatAcc<MP> (sums plus half-size compensations).
template <int MP>
constexpr int mat_acc_floats() { return (MP + 1) * kWave + ((MP + 1) * kWave + 1) / 2; }

// Number of crossings of one axis at or before distance T: the k with
// t0 + (k-1) dt <= T < t0 + k dt, evaluated with the same rounded formula
// the walk uses, so that a walk resumed at T stays consistent with one that
// had stepped through every plane.
__device__ __forceinline__ float crossings_before(float T, float t0, float dt, float inv_dt)
{
    // Branch-free.  A parallel axis (t0 = inf, dt = inv_dt = 0) gives 0, as
    // does T < t0: the first estimate is then 1 and the first test takes it
    // back to 0.
    float k = floorf(fmaxf(T - t0, 0.0f) * inv_dt) + 1.0f;
    k -= (fmaf(k - 1.0f, dt, t0) > T) ? 1.0f : 0.0f;
    k += (fmaf(k, dt, t0) <= T) ? 1.0f : 0.0f;
    return k;
}

// Step counters of the walk.  The projector uses NoCount (every call
// compiles away); fcat_walk_stats uses StepCount to measure the work the walk
// actually does: per lane, brick steps, mixed bricks entered and voxel steps
// inside them, and per wavefront the iterations of the voxel loop (each one
// issues for all 64 lanes, so their count times 64 is the lane slots the
// voxel loop occupies).
struct NoCount {
    __device__ __forceinline__ void brick() {}
    __device__ __forceinline__ void mixed() {}
    __device__ __forceinline__ void voxel() {}
};
struct StepCount {
    uint32_t bricks = 0, mixed_bricks = 0, voxels = 0, wave_voxel_iters = 0;
    __device__ __forceinline__ void brick() { ++bricks; }
    __device__ __forceinline__ void mixed() { ++mixed_bricks; }
    __device__ __forceinline__ void voxel()
    {
        ++voxels;
        // the lowest active lane counts the wavefront's iteration
        const uint64_t active = __ballot(1);
        if ((threadIdx.x & (kWave - 1)) == (unsigned)(__ffsll((unsigned long long)active) - 1)) ++wave_voxel_iters;
    }
};

// Voxel-level stepping inside one mixed brick: the next crossing time and
// the crossings taken per axis, and the voxel's offset in the brick.  Each
// step moves to the nearest crossing (x if t0 is the nearest, else y if t1
// is, else z), updates that axis's counter and recomputes all three
// crossings as t0 + k dt with one rounding each.  It is written with scalar
// members and selects of values only: an array indexed by a select, or a
// select between captured variables, is turned by the compiler into a
// select of addresses and a load from scratch memory.
struct VoxelStepper {
    float t0, t1, t2;
    float k0, k1, k2;
    int loc;
    __device__ __forceinline__ float step(const Ray &r, int dl0, int dl1, int dl2)
    {
        const float tn = fminf(t0, fminf(t1, t2));
        const bool cx = (t0 == tn);
        const bool cy = (t1 == tn);
        const bool ey = cy && !cx;            // exclusive: the axis that steps
        const bool ez = !cx && !cy;
        const int dyz = cy ? dl1 : dl2;
        loc += cx ? dl0 : dyz;
        k0 += cx ? 1.0f : 0.0f;
        k1 += ey ? 1.0f : 0.0f;
        k2 += ez ? 1.0f : 0.0f;
        t0 = fmaf(k0, r.dt[0], r.t0[0]);      // parallel axis: 0 * 0 + inf
        t1 = fmaf(k1, r.dt[1], r.t0[1]);
        t2 = fmaf(k2, r.dt[2], r.t0[2]);
        return tn;
    }
};

// Two-level exact walk (Siddon's path lengths, found hierarchically).
//
// The grid is tiled into B x B x B bricks; bricks[] holds the label of a
// brick whose voxels all share one label, or -1.  The coarse walk crosses
// brick planes; a uniform brick contributes its whole segment to its label
// in one step, and only inside mixed bricks does the fine walk cross the
// individual voxel planes.  Crossing k + 1 of an axis lies at t0 + k dt (one
// rounding from its exact value) for both levels; path length is charged to
// a material only when the label changes, with compensated summation.
//
// acc_wave is this wavefront's MatAcc block in LDS; L receives the sums.
template <int MP, typename Count = NoCount>
__device__ __forceinline__ void trace_bricks(const Ray &r, bool hit, const TraceGeom &G,
                                             const int8_t *__restrict__ labels_bm,
                                             const int8_t *__restrict__ bricks, float *acc_wave, float (&L)[MP],
                                             Count &&count = Count())
{
    MatAcc<MP> acc(acc_wave, threadIdx.x & (kWave - 1));
    acc.clear();
    const int bg = G.clip ? const_table(G.clip)[0] : 0;
    if (!hit || !r.walk) {
        // a ray that misses the background box is background all along
#pragma unroll
        for (int m = 0; m < MP; ++m) L[m] = (hit && m == bg) ? r.t_bg : 0.0f;
        return;
    }
    const float t_end = r.t_end;
    const uint8_t *lbase = reinterpret_cast<const uint8_t *>(labels_bm) - kLabelPad;
    const int nbx = G.nb[0], nby = G.nb[1];
    const int last_brick = G.nb[0] * G.nb[1] * G.nb[2] - 1;
    const int lstride[3] = {1, kBrickEdge, kBrickEdge * kBrickEdge};
    const int bstride[3] = {1, nbx, nbx * nby};

    float kc[3] = {0.0f, 0.0f, 0.0f};
    float tc[3] = {r.tc0[0], r.tc0[1], r.tc0[2]};
    const int db0 = r.sgn[0] * bstride[0], db1 = r.sgn[1] * bstride[1], db2 = r.sgn[2] * bstride[2];
    // voxel-index steps per axis, as separate values: an array indexed by a
    // select would be kept in scratch memory
    const int dl0 = r.sgn[0] * lstride[0], dl1 = r.sgn[1] * lstride[1], dl2 = r.sgn[2] * lstride[2];
    int bc[3] = {r.i0[0] / kBrickEdge, r.i0[1] / kBrickEdge, r.i0[2] / kBrickEdge};
    int blin = (bc[2] * nby + bc[1]) * nbx + bc[0];
    int bl = bricks[blin];
    unsigned cur = MP;       // the spare slot: nothing charged before the first cell
    float run = 0.0f;
    float T_in = 0.0f;
    int budget = G.nb[0] + G.nb[1] + G.nb[2] + 4;
    bool active = true;
    while (active) {
        count.brick();
        const float tco = fminf(tc[0], fminf(tc[1], tc[2]));
        const bool last = !(tco < t_end) || --budget < 0;
        const float T_out = last ? t_end : tco;
        // the next brick and its map entry, loaded here so that the load's
        // latency passes under this brick's work (after the last brick the
        // clamped index reads an entry that is not used)
        const bool bx = (tc[0] == tco);
        const bool ty = (tc[1] == tco);
        const int dbyz = ty ? db1 : db2;
        const int blin_next = blin + (bx ? db0 : dbyz);
        const int bl_next = bricks[min(max(blin_next, 0), last_brick)];
        if (bl >= 0) {
            if (static_cast<unsigned>(bl) != cur) {
                acc.add(cur, T_in - run);
                cur = bl;
                run = T_in;
            }
        } else {
            count.mixed();
            // fine walk over [T_in, T_out) inside brick `blin`, whose
            // kBrickVox labels are contiguous in the brick-major copy: resume the
            // voxel counters at T_in, then step plane by plane
            // The voxel is kept inside the brick: where rounding of the two
            // levels disagrees about a plane at T_in, the brick decides.
            float k[3], t[3];
            int loc = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int b0 = bc[a] * kBrickEdge;
                // a parallel axis counts no crossings and stays in its voxel
                const float kk = crossings_before(T_in, r.t0[a], r.dt[a], r.inv_dt[a]);
                const int ia = min(max(r.i0[a] + r.sgn[a] * (int)kk, b0), b0 + kBrickEdge - 1);
                k[a] = (float)(r.sgn[a] * (ia - r.i0[a]));
                t[a] = fmaf(k[a], r.dt[a], r.t0[a]);
                loc += (ia - b0) * lstride[a];
            }
            // offsets from the start of the padding: unsigned 32-bit, so each
            // label load takes the wave-uniform base plus one vector offset
            const uint32_t boff = kLabelPad + (uint32_t)min(max(blin, 0), last_brick) * kBrickVox;
            VoxelStepper w{t[0], t[1], t[2], k[0], k[1], k[2], (int)(boff + loc)};
            unsigned lab = lbase[boff + loc];
            // the walk runs one crossing ahead of the label comparison, so
            // each label load has a step's worth of work to arrive
            float tn = w.step(r, dl0, dl1, dl2);
            unsigned labn = lbase[(uint32_t)w.loc];
            if (lab != cur) {
                acc.add(cur, T_in - run);
                cur = lab;
                run = T_in;
            }
            for (int f = 0; f < 3 * kBrickEdge + 3; ++f) {
                if (!(tn < T_out)) break;
                count.voxel();
                const float tn2 = w.step(r, dl0, dl1, dl2);
                const unsigned lab2 = lbase[(uint32_t)w.loc];
                if (labn != cur) {
                    acc.add(cur, tn - run);
                    cur = labn;
                    run = tn;
                }
                tn = tn2;
                labn = lab2;
            }
        }
        if (last) {
            active = false;
        } else {
            const bool by = !bx && ty;
            const bool bz = !bx && !ty;
            blin = blin_next;
            bc[0] += bx ? r.sgn[0] : 0;
            bc[1] += by ? r.sgn[1] : 0;
            bc[2] += bz ? r.sgn[2] : 0;
            kc[0] += bx ? 1.0f : 0.0f;
            kc[1] += by ? 1.0f : 0.0f;
            kc[2] += bz ? 1.0f : 0.0f;
            tc[0] = fmaf(kc[0], r.dtc[0], r.tc0[0]);
            tc[1] = fmaf(kc[1], r.dtc[1], r.tc0[1]);
            tc[2] = fmaf(kc[2], r.dtc[2], r.tc0[2]);
            T_in = tco;
            bl = bl_next;
        }
    }
    acc.add(cur, t_end - run);
    if (r.t_bg > 0.0f) acc.add(static_cast<unsigned>(bg), r.t_bg);
    acc.read(L);
}


// sum over the bins of one group of w_e exp(-sum_m mu[e][m] L_m)   (Eq. 3),
// evaluated as w_e 2^-x with x = sum_m (mu[e][m] log2 e) L_m from the
// base-2 table.  Scaling the table instead of each optical depth costs one
// more rounding per table entry (a relative 2^-24 of each mu, as if the
// input had been rounded once more) and leaves x with the rounding error of
// its own FMA chain, the same as that of the base-e sum it replaces; 2^-x is
// the hardware base-2 exponential (about one ulp).
template <int MP>
__device__ __forceinline__ float group_sum(const float (&L)[MP], const SpecTables &T, int e0, int e1)
{
    const auto *mu2 = const_table(T.mu2T);
    const auto *w = const_table(T.w);
    float acc = 0.0f;
    // two bins per iteration: their table loads issue together and their
    // chains of FMAs interleave
#pragma unroll 2
    for (int e = e0; e < e1; ++e) {
        const auto *mrow = mu2 + e * MP;
        float x = 0.0f;
#pragma unroll
        for (int m = 0; m < MP; ++m) x = fmaf(mrow[m], L[m], x);
        acc = fmaf(w[e], __builtin_amdgcn_exp2f(-x), acc);
    }
    return acc;
}

// Reports a non-finite flood or scatter value read for this ray
// (bad[1] |= 1).  Only the error case pays for the atomic.  Call it after
// the last read of the spectral tables: the compiler cannot tell that the
// flag word is not part of a table, and a store before those reads would
// turn their wave-uniform scalar loads into per-lane vector loads.
__device__ __forceinline__ void flag_nonfinite(int *bad, float i0, float sc)
{
    if (bad && !(isfinite(i0) && isfinite(sc))) atomicOr(bad + 1, 1);
}

__device__ __forceinline__ double angle_of(const TraceGeom &G, int a)
{
    return G.angles ? G.angles[a] : (2.0 * M_PI) * (double)a / (double)G.n_angles;
}

// Sine and cosine of angle a (wave-uniform): from the table when the caller
// prepared one (scalar loads), else evaluated here.
__device__ __forceinline__ void angle_trig(const TraceGeom &G, int a, double &st, double &ct)
{
    if (G.trig) {
        const auto *t = const_table(G.trig);
        ct = t[2 * a];
        st = t[2 * a + 1];
    } else {
        sincos(angle_of(G, a), &st, &ct);
    }
}

}  // namespace fcat
