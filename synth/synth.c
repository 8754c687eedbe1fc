/*
 * Seeded synthetic segmentation volumes.
 *
 * These generators stand in for the connectomics, cell and material datasets
 * the paper evaluates on (Results, dataset table), which are not available
 * here.  They hold none of the compression method's arithmetic: they only
 * produce raw label volumes, which both the CPU oracle and the GPU path then
 * consume byte-for-byte.
 *
 * Random numbers: PCG32 (O'Neill 2014, "PCG: A Family of Simple Fast
 * Space-Efficient Statistically Good Algorithms for Random Number
 * Generation", the pcg32 XSH-RR 64/32 generator), written from its published
 * definition.  Label scrambling uses the 32-bit MurmurHash3 finaliser, a
 * bijection on u32.
 *
 * Volumes are linear x-fastest: v[(z*ny + y)*nx + x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- PCG32 */
typedef struct { uint64_t state, inc; } pcg32;

static uint32_t pcg32_next(pcg32* r) {
    uint64_t old = r->state;
    r->state = old * 6364136223846793005ULL + r->inc;
    uint32_t xorshifted = (uint32_t)(((old >> 18u) ^ old) >> 27u);
    uint32_t rot = (uint32_t)(old >> 59u);
    return (xorshifted >> rot) | (xorshifted << ((-rot) & 31));
}

static void pcg32_seed(pcg32* r, uint64_t seed, uint64_t stream) {
    r->state = 0u;
    r->inc = (stream << 1u) | 1u;
    pcg32_next(r);
    r->state += seed;
    pcg32_next(r);
}

/* uniform double in [0,1) with 53 random bits */
static double pcg32_double(pcg32* r) {
    uint64_t hi = pcg32_next(r) >> 5, lo = pcg32_next(r) >> 6;
    return (double)(hi * 67108864ULL + lo) * (1.0 / 9007199254740992.0);
}

/* uniform integer in [0, n) by rejection (n >= 1) */
static uint32_t pcg32_below(pcg32* r, uint32_t n) {
    uint32_t threshold = (uint32_t)(-n) % n;
    for (;;) {
        uint32_t v = pcg32_next(r);
        if (v >= threshold) return v % n;
    }
}

static uint64_t pcg32_u64(pcg32* r) {
    uint64_t hi = pcg32_next(r);
    return (hi << 32) | pcg32_next(r);
}

static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85ebca6bu;
    h ^= h >> 13; h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t synth_pcg32_first(uint64_t seed, uint64_t stream) {
    pcg32 r; pcg32_seed(&r, seed, stream); return pcg32_next(&r);
}

/* ------------------------------------------------------------- Voronoi */
/*
 * Nearest-seed labelling.  Voxel (x,y,z) is measured at its centre
 * (x+.5, y+.5, z+.5); the nearest seed in squared float64 distance wins and
 * exact ties go to the lower seed index.  Work is organised in 8^3 voxel
 * blocks: for a block with centre c and half-diagonal h, the nearest seed of
 * any voxel lies within d0 + 2h of c, where d0 is the distance from c to its
 * own nearest seed, so only those candidates are scanned per voxel.
 */
typedef struct {
    const double* pts;   /* n x 3 */
    int n;
    double cell;         /* grid cell edge */
    int gx, gy, gz;
    int* cell_start;     /* gx*gy*gz + 1 */
    int* cell_items;     /* n */
} seed_grid;

static void grid_build(seed_grid* g, const double* pts, int n, double ex, double ey, double ez) {
    double vol = ex * ey * ez;
    double cell = cbrt(vol / (n > 0 ? n : 1) * 2.0);
    if (cell < 1.0) cell = 1.0;
    g->pts = pts; g->n = n; g->cell = cell;
    g->gx = (int)ceil(ex / cell); g->gy = (int)ceil(ey / cell); g->gz = (int)ceil(ez / cell);
    if (g->gx < 1) g->gx = 1;
    if (g->gy < 1) g->gy = 1;
    if (g->gz < 1) g->gz = 1;
    size_t nc = (size_t)g->gx * g->gy * g->gz;
    g->cell_start = (int*)calloc(nc + 1, sizeof(int));
    g->cell_items = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int* cid = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) {
        int cx = (int)(pts[3 * i] / cell), cy = (int)(pts[3 * i + 1] / cell), cz = (int)(pts[3 * i + 2] / cell);
        if (cx >= g->gx) cx = g->gx - 1;
        if (cy >= g->gy) cy = g->gy - 1;
        if (cz >= g->gz) cz = g->gz - 1;
        if (cx < 0) cx = 0;
        if (cy < 0) cy = 0;
        if (cz < 0) cz = 0;
        cid[i] = (cz * g->gy + cy) * g->gx + cx;
        g->cell_start[cid[i] + 1]++;
    }
    for (size_t c = 0; c < nc; c++) g->cell_start[c + 1] += g->cell_start[c];
    int* fill = (int*)malloc(sizeof(int) * (nc + 1));
    memcpy(fill, g->cell_start, sizeof(int) * (nc + 1));
    for (int i = 0; i < n; i++) g->cell_items[fill[cid[i]]++] = i; /* ascending index per cell */
    free(fill);
    free(cid);
}

static void grid_free(seed_grid* g) { free(g->cell_start); free(g->cell_items); }

static double d2(const double* p, double x, double y, double z) {
    double dx = p[0] - x, dy = p[1] - y, dz = p[2] - z;
    return dx * dx + dy * dy + dz * dz;
}

/* all seeds with distance to (x,y,z) <= r appended to out (sorted ascending) */
static int cmp_int(const void* a, const void* b) { return (*(const int*)a > *(const int*)b) - (*(const int*)a < *(const int*)b); }

static int grid_within(const seed_grid* g, double x, double y, double z, double r, int* out, int cap) {
    int n = 0;
    double r2 = r * r;
    int x0 = (int)floor((x - r) / g->cell), x1 = (int)floor((x + r) / g->cell);
    int y0 = (int)floor((y - r) / g->cell), y1 = (int)floor((y + r) / g->cell);
    int z0 = (int)floor((z - r) / g->cell), z1 = (int)floor((z + r) / g->cell);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (z0 < 0) z0 = 0;
    if (x1 >= g->gx) x1 = g->gx - 1;
    if (y1 >= g->gy) y1 = g->gy - 1;
    if (z1 >= g->gz) z1 = g->gz - 1;
    for (int cz = z0; cz <= z1; cz++)
        for (int cy = y0; cy <= y1; cy++)
            for (int cx = x0; cx <= x1; cx++) {
                int c = (cz * g->gy + cy) * g->gx + cx;
                for (int k = g->cell_start[c]; k < g->cell_start[c + 1]; k++) {
                    int i = g->cell_items[k];
                    if (d2(g->pts + 3 * i, x, y, z) <= r2 && n < cap) out[n++] = i;
                }
            }
    qsort(out, (size_t)n, sizeof(int), cmp_int);
    return n;
}

/* nearest seed distance to (x,y,z), exact over all seeds via ring growth */
static double grid_nearest_dist(const seed_grid* g, double x, double y, double z, int* scratch, int cap) {
    double r = g->cell;
    for (;;) {
        int n = grid_within(g, x, y, z, r, scratch, cap);
        if (n > 0) {
            double best = INFINITY;
            for (int k = 0; k < n; k++) {
                double d = d2(g->pts + 3 * scratch[k], x, y, z);
                if (d < best) best = d;
            }
            return sqrt(best);
        }
        r *= 2.0;
        if (r > 1e9) return INFINITY;
    }
}

/*
 * Label the sub-box [ox,ox+sx) x [oy,oy+sy) x [oz,oz+sz) of a volume whose
 * seeds are given in its own voxel frame.  out is sx*sy*sz, x fastest; the
 * label of seed i is labels[i] (u64).  Seeds must be non-empty.
 */
static void voronoi_box(const seed_grid* g, const uint64_t* labels, int ox, int oy, int oz, int sx, int sy, int sz,
                        uint64_t* out64, uint32_t* out32) {
    const int B = 8;
    int cap = g->n;
    int* cand = (int*)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
    for (int bz = 0; bz < sz; bz += B)
        for (int by = 0; by < sy; by += B)
            for (int bx = 0; bx < sx; bx += B) {
                int ex = bx + B < sx ? B : sx - bx, ey = by + B < sy ? B : sy - by, ez = bz + B < sz ? B : sz - bz;
                double cx = ox + bx + ex * 0.5, cy = oy + by + ey * 0.5, cz = oz + bz + ez * 0.5;
                double h = 0.5 * sqrt((double)(ex * ex + ey * ey + ez * ez));
                double d0 = grid_nearest_dist(g, cx, cy, cz, cand, cap);
                int nc = grid_within(g, cx, cy, cz, d0 + 2.0 * h + 1e-6, cand, cap);
                for (int z = 0; z < ez; z++)
                    for (int y = 0; y < ey; y++)
                        for (int x = 0; x < ex; x++) {
                            double px = ox + bx + x + 0.5, py = oy + by + y + 0.5, pz = oz + bz + z + 0.5;
                            double best = INFINITY;
                            int bi = -1;
                            for (int k = 0; k < nc; k++) {
                                double d = d2(g->pts + 3 * cand[k], px, py, pz);
                                if (d < best) { best = d; bi = cand[k]; } /* cand ascending: ties keep lower */
                            }
                            size_t o = ((size_t)(bz + z) * sy + (by + y)) * sx + (bx + x);
                            if (out64) out64[o] = labels[bi];
                            else out32[o] = (uint32_t)labels[bi];
                        }
            }
    free(cand);
}

/*
 * Voronoi volume: n_seeds seeds uniform in [0,nx)x[0,ny)x[0,nz) (float64),
 * label of seed i = i + 1.  Seeds drawn from PCG32(seed, stream 1).
 */
int synth_voronoi_u32(uint32_t* out, int nx, int ny, int nz, int n_seeds, uint64_t seed, int nthreads) {
    if (n_seeds < 1) return -1;
    double* pts = (double*)malloc(sizeof(double) * 3 * (size_t)n_seeds);
    uint64_t* labels = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_seeds);
    pcg32 r; pcg32_seed(&r, seed, 1);
    for (int i = 0; i < n_seeds; i++) {
        pts[3 * i] = pcg32_double(&r) * nx;
        pts[3 * i + 1] = pcg32_double(&r) * ny;
        pts[3 * i + 2] = pcg32_double(&r) * nz;
        labels[i] = (uint64_t)(i + 1);
    }
    seed_grid g; grid_build(&g, pts, n_seeds, nx, ny, nz);
    /* one slab of 8 z-planes per work item; slabs are independent */
    int nslab = (nz + 7) / 8;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int s = 0; s < nslab; s++) {
        int z0 = s * 8, sz = z0 + 8 <= nz ? 8 : nz - z0;
        voronoi_box(&g, labels, 0, 0, z0, nx, ny, sz, NULL, out + (size_t)z0 * ny * nx);
    }
    grid_free(&g);
    free(pts); free(labels);
    return 0;
}

/*
 * Background voids: spheres of label 0, centre uniform in the volume, radius
 * uniform in [rmin, rmax), stamped one after another (PCG32 stream 2) until at
 * least frac of all voxels are 0.  A voxel is inside when its centre lies
 * within the radius.  Returns the number of spheres used.
 */
long synth_voids_u32(uint32_t* vol, int nx, int ny, int nz, double frac, double rmin, double rmax, uint64_t seed) {
    size_t total = (size_t)nx * ny * nz, zeros = 0;
    for (size_t i = 0; i < total; i++) zeros += vol[i] == 0;
    pcg32 r; pcg32_seed(&r, seed, 2);
    long used = 0;
    while ((double)zeros < frac * (double)total) {
        double cx = pcg32_double(&r) * nx, cy = pcg32_double(&r) * ny, cz = pcg32_double(&r) * nz;
        double rad = rmin + pcg32_double(&r) * (rmax - rmin);
        int x0 = (int)floor(cx - rad), x1 = (int)ceil(cx + rad);
        int y0 = (int)floor(cy - rad), y1 = (int)ceil(cy + rad);
        int z0 = (int)floor(cz - rad), z1 = (int)ceil(cz + rad);
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (z0 < 0) z0 = 0;
        if (x1 > nx) x1 = nx;
        if (y1 > ny) y1 = ny;
        if (z1 > nz) z1 = nz;
        double r2 = rad * rad;
        for (int z = z0; z < z1; z++)
            for (int y = y0; y < y1; y++)
                for (int x = x0; x < x1; x++) {
                    double dx = x + 0.5 - cx, dy = y + 0.5 - cy, dz = z + 0.5 - cz;
                    if (dx * dx + dy * dy + dz * dz <= r2) {
                        uint32_t* v = vol + ((size_t)z * ny + y) * nx + x;
                        if (*v) { *v = 0; zeros++; }
                    }
                }
        used++;
    }
    return used;
}

/* ------------------------------------------------------------- neurites */
/*
 * Tube t (0-based, in order) is drawn from PCG32(seed, stream 1000 + t):
 *   K ~ U{4..8} control points; P0 uniform in the isotropic frame
 *   [0,nx) x [0,ny) x [0,nz*za); each next point = previous + step * u, with
 *   u uniform on the unit sphere;
 *   radius r ~ U[3, 20); label = fmix32((t+1) * key), key odd and drawn from
 *   PCG32(seed, stream 999), so labels are distinct and nonzero.
 * The centre line is the uniform Catmull-Rom spline through the control
 * points (end points repeated), sampled at 4 points per span; the tube is the
 * union of capsules of radius r around consecutive samples.  Voxels are
 * anisotropic: voxel (x,y,z) sits at the isotropic point
 * (x+.5, y+.5, (z+.5)*za), so with za = 4 structures appear squashed 4x
 * along z, as in serial-section EM stacks.  Later tubes overwrite earlier
 * ones.  Rasterisation is exact per voxel centre up to float rounding:
 * for every (y, z) row the x-interval inside each capsule is solved in
 * closed form.
 */
typedef struct {
    int nseg;
    double* a;   /* nseg x 3 segment start */
    double* b;   /* nseg x 3 segment end */
    double r;
    uint32_t label;
    double zlo, zhi; /* isotropic z extent incl. radius */
} tube;

static void catmull_rom(const double* p0, const double* p1, const double* p2, const double* p3, double t, double* o) {
    double t2 = t * t, t3 = t2 * t;
    for (int k = 0; k < 3; k++)
        o[k] = 0.5 * ((2.0 * p1[k]) + (-p0[k] + p2[k]) * t + (2.0 * p0[k] - 5.0 * p1[k] + 4.0 * p2[k] - p3[k]) * t2 +
                      (-p0[k] + 3.0 * p1[k] - 3.0 * p2[k] + p3[k]) * t3);
}

#define TUBE_SAMPLES 4

static void make_tube(tube* tb, uint64_t seed, int t, uint32_t key, int nx, int ny, double niso_z, double step_len) {
    pcg32 r; pcg32_seed(&r, seed, 1000ULL + (uint64_t)t);
    int K = 4 + (int)pcg32_below(&r, 5);
    double P[10][3];
    P[1][0] = pcg32_double(&r) * nx; P[1][1] = pcg32_double(&r) * ny; P[1][2] = pcg32_double(&r) * niso_z;
    for (int k = 1; k < K; k++) {
        double uz = 2.0 * pcg32_double(&r) - 1.0, phi = 2.0 * M_PI * pcg32_double(&r);
        double s = sqrt(1.0 - uz * uz);
        P[k + 1][0] = P[k][0] + step_len * s * cos(phi);
        P[k + 1][1] = P[k][1] + step_len * s * sin(phi);
        P[k + 1][2] = P[k][2] + step_len * uz;
    }
    tb->r = 3.0 + 17.0 * pcg32_double(&r);
    tb->label = fmix32((uint32_t)(t + 1) * key);
    memcpy(P[0], P[1], sizeof(P[0]));
    memcpy(P[K + 1], P[K], sizeof(P[0]));
    int nspan = K - 1;
    tb->nseg = nspan * TUBE_SAMPLES;
    tb->a = (double*)malloc(sizeof(double) * 3 * (size_t)tb->nseg);
    tb->b = (double*)malloc(sizeof(double) * 3 * (size_t)tb->nseg);
    double prev[3];
    memcpy(prev, P[1], sizeof(prev));
    int si = 0;
    for (int sp = 0; sp < nspan; sp++)
        for (int s = 1; s <= TUBE_SAMPLES; s++) {
            double q[3];
            catmull_rom(P[sp], P[sp + 1], P[sp + 2], P[sp + 3], (double)s / TUBE_SAMPLES, q);
            for (int k = 0; k < 3; k++) { tb->a[3 * si + k] = prev[k]; tb->b[3 * si + k] = q[k]; }
            memcpy(prev, q, sizeof(prev));
            si++;
        }
    tb->zlo = 1e300; tb->zhi = -1e300;
    for (int i = 0; i < tb->nseg; i++) {
        double lo = fmin(tb->a[3 * i + 2], tb->b[3 * i + 2]) - tb->r, hi = fmax(tb->a[3 * i + 2], tb->b[3 * i + 2]) + tb->r;
        if (lo < tb->zlo) tb->zlo = lo;
        if (hi > tb->zhi) tb->zhi = hi;
    }
}

/* x-interval [lo, hi] of the ball (c, r) on the row (py, pz); returns 0 if empty */
static int ball_row(const double* c, double r, double py, double pz, double* lo, double* hi) {
    double e = r * r - (py - c[1]) * (py - c[1]) - (pz - c[2]) * (pz - c[2]);
    if (e < 0) return 0;
    double s = sqrt(e);
    *lo = c[0] - s; *hi = c[0] + s;
    return 1;
}

/* x-interval of the finite cylinder (a, b, r) on the row (py, pz) */
static int cyl_row(const double* a, const double* b, double r, double py, double pz, double* lo, double* hi) {
    double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    double dd = dx * dx + dy * dy + dz * dz;
    if (dd <= 1e-12) return 0;
    double qy = py - a[1], qz = pz - a[2];
    double c0 = -a[0] * dx + qy * dy + qz * dz; /* q.d = dx*x + c0 */
    /* parameter range 0 <= (dx*x + c0)/dd <= 1 */
    double tlo = -INFINITY, thi = INFINITY;
    if (dx > 1e-12) { tlo = -c0 / dx; thi = (dd - c0) / dx; }
    else if (dx < -1e-12) { tlo = (dd - c0) / dx; thi = -c0 / dx; }
    else if (c0 < 0 || c0 > dd) return 0;
    /* distance to the line: A x^2 + B x + C <= 0 */
    double A = (dy * dy + dz * dz) / dd;
    double B = -2.0 * a[0] - 2.0 * dx * c0 / dd;
    double C = a[0] * a[0] + qy * qy + qz * qz - c0 * c0 / dd - r * r;
    double xlo, xhi;
    if (A < 1e-12) {
        if (C > 0) return 0;
        xlo = -INFINITY; xhi = INFINITY;
    } else {
        double disc = B * B - 4.0 * A * C;
        if (disc < 0) return 0;
        double s = sqrt(disc);
        xlo = (-B - s) / (2.0 * A); xhi = (-B + s) / (2.0 * A);
    }
    if (tlo > xlo) xlo = tlo;
    if (thi < xhi) xhi = thi;
    if (xlo > xhi) return 0;
    *lo = xlo; *hi = xhi;
    return 1;
}

static void stamp_capsule(uint32_t* slab, int nx, int ny, int z0, int z1, double za, const double* a, const double* b,
                          double r, uint32_t label) {
    double ylo = fmin(a[1], b[1]) - r, yhi = fmax(a[1], b[1]) + r;
    double zlo = fmin(a[2], b[2]) - r, zhi = fmax(a[2], b[2]) + r;
    int ya = (int)ceil(ylo - 0.5), yb = (int)floor(yhi - 0.5);
    int zA = (int)ceil(zlo / za - 0.5), zB = (int)floor(zhi / za - 0.5);
    if (ya < 0) ya = 0;
    if (yb > ny - 1) yb = ny - 1;
    if (zA < z0) zA = z0;
    if (zB > z1 - 1) zB = z1 - 1;
    for (int z = zA; z <= zB; z++) {
        double pz = (z + 0.5) * za;
        for (int y = ya; y <= yb; y++) {
            double py = y + 0.5, lo = INFINITY, hi = -INFINITY, l, h;
            if (ball_row(a, r, py, pz, &l, &h)) { lo = fmin(lo, l); hi = fmax(hi, h); }
            if (ball_row(b, r, py, pz, &l, &h)) { lo = fmin(lo, l); hi = fmax(hi, h); }
            if (cyl_row(a, b, r, py, pz, &l, &h)) { lo = fmin(lo, l); hi = fmax(hi, h); }
            if (lo > hi) continue;
            double fa = ceil(lo - 0.5), fb = floor(hi - 0.5);
            if (fa < 0) fa = 0;
            if (fb > nx - 1) fb = nx - 1;
            uint32_t* row = slab + ((size_t)(z - z0) * ny + y) * nx;
            for (int x = (int)fa; x <= (int)fb; x++) row[x] = label;
        }
    }
}

/*
 * Write z-planes [z0, z1) of the neurite volume into out ((z1-z0)*ny*nx,
 * background 0).  Any slab decomposition yields the same voxels as one call
 * over the full range, so large volumes can be produced slab by slab.
 */
int synth_neurite_u32(uint32_t* out, int nx, int ny, int nz, int z0, int z1, int n_tubes, double step_len, double za,
                      uint64_t seed, int nthreads) {
    if (z0 < 0 || z1 > nz || z0 >= z1 || za <= 0) return -1;
    memset(out, 0, sizeof(uint32_t) * (size_t)(z1 - z0) * ny * nx);
    pcg32 kr; pcg32_seed(&kr, seed, 999);
    uint32_t key = pcg32_next(&kr) | 1u;
    double niso_z = nz * za;
    tube* tubes = (tube*)malloc(sizeof(tube) * (size_t)n_tubes);
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int t = 0; t < n_tubes; t++) make_tube(&tubes[t], seed, t, key, nx, ny, niso_z, step_len);
    /* z sub-slabs of 4 planes processed in parallel; each applies all tubes in order */
    const int SUB = 4;
    int nsub = (z1 - z0 + SUB - 1) / SUB;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int s = 0; s < nsub; s++) {
        int sa = z0 + s * SUB, sb = sa + SUB < z1 ? sa + SUB : z1;
        double isa = (sa - 0.5) * za, isb = (sb + 0.5) * za;
        uint32_t* slab = out + (size_t)(sa - z0) * ny * nx;
        for (int t = 0; t < n_tubes; t++) {
            const tube* tb = &tubes[t];
            if (tb->zhi < isa || tb->zlo > isb) continue;
            for (int i = 0; i < tb->nseg; i++) {
                const double* a = tb->a + 3 * i;
                const double* b = tb->b + 3 * i;
                double zl = fmin(a[2], b[2]) - tb->r, zh = fmax(a[2], b[2]) + tb->r;
                if (zh < isa || zl > isb) continue;
                stamp_capsule(slab, nx, ny, sa, sb, za, a, b, tb->r, tb->label);
            }
        }
    }
    for (int t = 0; t < n_tubes; t++) { free(tubes[t].a); free(tubes[t].b); }
    free(tubes);
    return 0;
}

/* ------------------------------------------------------- uneven bricks */
/*
 * One brick of the uneven-content u64 batch.  Brick `id` draws from
 * PCG32(seed, stream 5000000 + id): kind u in [0,1): u < 0.4 constant (one
 * random u64), u < 0.8 Voronoi (k ~ U{2..64} seeds uniform in [0,b)^3,
 * random u64 labels, nearest seed with ties to the lower index), else noise
 * (i.i.d. random u64 per voxel).  out is b^3, x fastest.  Returns the kind
 * (0 constant, 1 Voronoi, 2 noise).
 */
int synth_uneven_brick_u64(uint64_t* out, int b, uint64_t seed, uint64_t id) {
    pcg32 r; pcg32_seed(&r, seed, 5000000ULL + id);
    double u = pcg32_double(&r);
    size_t n = (size_t)b * b * b;
    if (u < 0.4) {
        uint64_t v = pcg32_u64(&r);
        for (size_t i = 0; i < n; i++) out[i] = v;
        return 0;
    }
    if (u < 0.8) {
        int k = 2 + (int)pcg32_below(&r, 63);
        double pts[64 * 3];
        uint64_t labels[64];
        for (int i = 0; i < k; i++) {
            pts[3 * i] = pcg32_double(&r) * b;
            pts[3 * i + 1] = pcg32_double(&r) * b;
            pts[3 * i + 2] = pcg32_double(&r) * b;
            labels[i] = pcg32_u64(&r);
        }
        seed_grid g; grid_build(&g, pts, k, b, b, b);
        voronoi_box(&g, labels, 0, 0, 0, b, b, b, out, NULL);
        grid_free(&g);
        return 1;
    }
    for (size_t i = 0; i < n; i++) out[i] = pcg32_u64(&r);
    return 2;
}

/*
 * Tile layout of the uneven batch: tile `t` is one 64^3 brick or eight 32^3
 * bricks, a fair coin from PCG32(seed, stream 4000000 + t).  Returns 1 when
 * split.
 */
int synth_uneven_tile_split(uint64_t seed, uint64_t t) {
    pcg32 r; pcg32_seed(&r, seed, 4000000ULL + t);
    return pcg32_double(&r) < 0.5;
}

/* ----------------------------------------------------- small test bricks */
/*
 * A b^3 brick (u64 labels) for tests: `kind` 0 = i.i.d. labels drawn from
 * {base, ..., base + nlab - 1}; 1 = Voronoi with nlab seeds, labels base+i;
 * 2 = axis-aligned slabs along a random axis with nlab labels.
 */
void synth_test_brick_u64(uint64_t* out, int b, int kind, int nlab, uint64_t base, uint64_t seed) {
    pcg32 r; pcg32_seed(&r, seed, 77);
    size_t n = (size_t)b * b * b;
    if (nlab < 1) nlab = 1;
    if (kind == 0) {
        for (size_t i = 0; i < n; i++) out[i] = base + pcg32_below(&r, (uint32_t)nlab);
    } else if (kind == 1) {
        double pts[256 * 3];
        uint64_t labels[256];
        if (nlab > 256) nlab = 256;
        for (int i = 0; i < nlab; i++) {
            pts[3 * i] = pcg32_double(&r) * b;
            pts[3 * i + 1] = pcg32_double(&r) * b;
            pts[3 * i + 2] = pcg32_double(&r) * b;
            labels[i] = base + (uint64_t)i;
        }
        seed_grid g; grid_build(&g, pts, nlab, b, b, b);
        voronoi_box(&g, labels, 0, 0, 0, b, b, b, out, NULL);
        grid_free(&g);
    } else {
        int axis = (int)pcg32_below(&r, 3);
        for (int z = 0; z < b; z++)
            for (int y = 0; y < b; y++)
                for (int x = 0; x < b; x++) {
                    int c = axis == 0 ? x : axis == 1 ? y : z;
                    out[((size_t)z * b + y) * b + x] = base + (uint64_t)((c * nlab) / b);
                }
    }
}

/* ------------------------------------------------- uneven batch (parallel) */
/*
 * Bricks 0..n-1 of the uneven-content batch into one flat array: brick k is
 * synth_uneven_brick_u64(seed, k) of side 1 << log2b[k], stored from element
 * elem_off[k].  kinds[k] receives its kind.  Same bytes as brick-by-brick
 * generation; OpenMP over bricks.
 */
void synth_uneven_batch_u64(uint64_t* out, const uint64_t* elem_off, const uint8_t* log2b, uint64_t n, uint64_t seed,
                            int32_t* kinds, int nthreads) {
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads > 0 ? nthreads : 1)
    for (long k = 0; k < (long)n; k++)
        kinds[k] = synth_uneven_brick_u64(out + elem_off[k], 1 << log2b[k], seed, (uint64_t)k);
}
