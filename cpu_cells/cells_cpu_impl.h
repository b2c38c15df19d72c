/*
 * Cell-list Lennard-Jones molecular dynamics on the host, in the precision
 * REAL (float or double); included once per precision by cells_cpu.c with
 * NAME(x) giving each function its suffix.
 *
 * The same algorithm as the GPU path, written the plain CPU way: cells of
 * side >= r_c, n_c = int(L / r_c) per dimension (section 3.2), rebuilt every
 * step by a counting sort; forces over the 27 neighbour cells (section 3),
 * each pair from both sides (full shell, so threads never write the same
 * atom); the force-shifted LJ force of section 2; velocity Verlet. OpenMP
 * over cells and atoms.
 */

typedef struct NAME(state) {
    int64_t n, nc, ncells;
    REAL box, inv_s;
    int64_t* cell;   /* cell of each atom */
    int64_t* start;  /* ncells + 1 CSR offsets */
    int64_t* order;  /* atoms in cell order */
    REAL* xs;        /* positions in cell order (3 per atom) */
    REAL* fs;        /* forces in cell order */
} NAME(state);

static REAL NAME(wrap)(REAL x, REAL L) {
    x -= L * FLOOR(x / L);
    if (x >= L) x -= L;
    if (x < (REAL)0 || x >= L) x = (REAL)0;
    return x;
}

static void NAME(rebuild)(NAME(state)* S, REAL* pos) {
    const int64_t n = S->n, nc = S->nc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            pos[3 * i + d] = NAME(wrap)(pos[3 * i + d], S->box);
            int64_t k = (int64_t)(pos[3 * i + d] * S->inv_s);
            c[d] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
        }
        S->cell[i] = c[0] + nc * (c[1] + nc * c[2]);
    }
    for (int64_t c = 0; c <= S->ncells; ++c) S->start[c] = 0;
    for (int64_t i = 0; i < n; ++i) S->start[S->cell[i] + 1]++;
    for (int64_t c = 0; c < S->ncells; ++c) S->start[c + 1] += S->start[c];
    /* stable scatter: atoms of a cell keep their index order */
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)S->ncells);
    for (int64_t c = 0; c < S->ncells; ++c) fill[c] = S->start[c];
    for (int64_t i = 0; i < n; ++i) S->order[fill[S->cell[i]]++] = i;
    free(fill);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) S->xs[3 * k + d] = pos[3 * S->order[k] + d];
}

/* Forces in user order into force (3 per atom). */
static void NAME(forces)(NAME(state)* S, const cc_params* p, REAL* force) {
    const int64_t nc = S->nc;
    const REAL L = S->box;
    const REAL rc = (REAL)p->rc, rc2 = rc * rc;
    const REAL s2 = (REAL)(p->sigma * p->sigma), e24 = (REAL)(24.0 * p->epsilon);
    /* f_LJ(r_c) = (24 eps / r_c) [2 (s/r_c)^12 - (s/r_c)^6] */
    const REAL q = s2 / rc2, q6 = q * q * q;
    const REAL fc = e24 / rc * ((REAL)2 * q6 * q6 - q6);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < S->ncells; ++c) {
        const int64_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        for (int64_t a = S->start[c]; a < S->start[c + 1]; ++a) {
            const REAL xi = S->xs[3 * a], yi = S->xs[3 * a + 1], zi = S->xs[3 * a + 2];
            REAL fx = 0, fy = 0, fz = 0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t jx = cx + dx, jy = cy + dy, jz = cz + dz;
                        /* the periodic image of the neighbour cell */
                        REAL sx = 0, sy = 0, sz = 0;
                        if (jx < 0) { jx += nc; sx = -L; } else if (jx >= nc) { jx -= nc; sx = L; }
                        if (jy < 0) { jy += nc; sy = -L; } else if (jy >= nc) { jy -= nc; sy = L; }
                        if (jz < 0) { jz += nc; sz = -L; } else if (jz >= nc) { jz -= nc; sz = L; }
                        const int64_t cj = jx + nc * (jy + nc * jz);
                        for (int64_t b = S->start[cj]; b < S->start[cj + 1]; ++b) {
                            if (b == a) continue;
                            const REAL ddx = xi - (S->xs[3 * b] + sx);
                            const REAL ddy = yi - (S->xs[3 * b + 1] + sy);
                            const REAL ddz = zi - (S->xs[3 * b + 2] + sz);
                            const REAL r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                            if (r2 < rc2) {
                                const REAL ir2 = (REAL)1 / r2, r = SQRT(r2);
                                const REAL t = s2 * ir2, t6 = t * t * t;
                                /* (f_LJ(r) - f_LJ(r_c)) / r */
                                const REAL g = e24 * ir2 * ((REAL)2 * t6 * t6 - t6) - fc / r;
                                fx += g * ddx;
                                fy += g * ddy;
                                fz += g * ddz;
                            }
                        }
                    }
            S->fs[3 * a] = fx;
            S->fs[3 * a + 1] = fy;
            S->fs[3 * a + 2] = fz;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < S->n; ++k)
        for (int d = 0; d < 3; ++d) force[3 * S->order[k] + d] = S->fs[3 * k + d];
}

/* nsteps velocity-Verlet steps of pos/vel (3 per atom, updated in place);
 * force receives the forces of the final state. Returns 0, or -1 when the
 * box holds fewer than 3 cells per dimension or memory runs out. */
int NAME(run)(const cc_params* p, int64_t n, REAL* pos, REAL* vel, REAL* force, int32_t nsteps) {
    NAME(state) S;
    S.n = n;
    S.box = (REAL)p->box;
    S.nc = (int64_t)(p->box / p->rc);
    if (S.nc < 3) return -1;
    S.ncells = S.nc * S.nc * S.nc;
    S.inv_s = (REAL)((double)S.nc / p->box);
    S.cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    S.start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S.ncells + 1));
    S.order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    S.xs = (REAL*)malloc(sizeof(REAL) * 3 * (size_t)n);
    S.fs = (REAL*)malloc(sizeof(REAL) * 3 * (size_t)n);
    if (!S.cell || !S.start || !S.order || !S.xs || !S.fs) {
        free(S.cell); free(S.start); free(S.order); free(S.xs); free(S.fs);
        return -1;
    }
    const REAL dt = (REAL)p->dt, h = (REAL)(0.5 * p->dt / p->mass);
    NAME(rebuild)(&S, pos);
    NAME(forces)(&S, p, force);
    for (int32_t k = 0; k < nsteps; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < 3 * n; ++i) {
            vel[i] += h * force[i];
            pos[i] += dt * vel[i];
        }
        NAME(rebuild)(&S, pos);
        NAME(forces)(&S, p, force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += h * force[i];
    }
    free(S.cell); free(S.start); free(S.order); free(S.xs); free(S.fs);
    return 0;
}
