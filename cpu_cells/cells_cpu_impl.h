/*
 * Cell-list Lennard-Jones molecular dynamics on the host, in the precision
 * REAL (float or double); included once per precision by cells_cpu.c with
 * NAME(x) giving each function its suffix.
 *
 * The same algorithm as the GPU path, written the way a CPU runs it well:
 * cells of side >= r_c, n_c = int(L / r_c) per dimension (section 3.2),
 * rebuilt every step by a counting sort; forces over the 27 neighbour cells
 * (section 3), each pair from both sides (full shell, as on the GPU, so
 * threads never write the same atom); the force-shifted LJ force of section
 * 2; velocity Verlet. OpenMP over cells and atoms. Positions are kept in cell
 * order as three arrays (x, y, z), and the pair loop runs in SIMD lanes: every
 * candidate is evaluated, and the cutoff and the atom itself are masked out by
 * selects instead of branches.
 */

typedef struct NAME(state) {
    int64_t n, nc, ncells;
    int nthreads;
    REAL box, inv_s;
    int64_t* cell;   /* cell of each atom */
    int64_t* start;  /* ncells + 1 CSR offsets */
    int64_t* order;  /* atoms in cell order */
    int64_t* tcount; /* per-thread counts, nthreads x ncells (the counting sort) */
    REAL* xs;        /* positions in cell order, x then y then z (n each) */
    REAL* fs;        /* forces in cell order (3 per atom) */
} NAME(state);

static REAL NAME(wrap)(REAL x, REAL L) {
    x -= L * FLOOR(x / L);
    if (x >= L) x -= L;
    if (x < (REAL)0 || x >= L) x = (REAL)0;
    return x;
}

/* Contiguous share [lo, hi) of n items for thread t of nt. */
static void NAME(share)(int64_t n, int t, int nt, int64_t* lo, int64_t* hi) {
    *lo = n * t / nt;
    *hi = n * (t + 1) / nt;
}

/* Stable counting sort of the atoms by cell: thread t counts its contiguous
 * share of the atoms per cell, the counts are scanned cell-major and thread-
 * minor, and each thread scatters its share in index order, so within a cell
 * the atoms keep their index order whatever the thread count. */
static void NAME(rebuild)(NAME(state)* S, REAL* pos) {
    const int64_t n = S->n, nc = S->nc, ncells = S->ncells;
    const int nt = S->nthreads;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num();
#else
        const int t = 0;
#endif
        int64_t lo, hi;
        NAME(share)(n, t, nt, &lo, &hi);
        int64_t* cnt = S->tcount + (size_t)t * (size_t)ncells;
        for (int64_t c = 0; c < ncells; ++c) cnt[c] = 0;
        for (int64_t i = lo; i < hi; ++i) {
            int64_t c[3];
            for (int d = 0; d < 3; ++d) {
                pos[3 * i + d] = NAME(wrap)(pos[3 * i + d], S->box);
                int64_t k = (int64_t)(pos[3 * i + d] * S->inv_s);
                c[d] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
            }
            const int64_t ci = c[0] + nc * (c[1] + nc * c[2]);
            S->cell[i] = ci;
            cnt[ci]++;
        }
#pragma omp barrier
#pragma omp single
        {
            int64_t run = 0;
            for (int64_t c = 0; c < ncells; ++c) {
                S->start[c] = run;
                for (int u = 0; u < nt; ++u) {
                    int64_t* q = S->tcount + (size_t)u * (size_t)ncells + c;
                    const int64_t v = *q;
                    *q = run;  /* thread u's first slot in cell c */
                    run += v;
                }
            }
            S->start[ncells] = run;
        }
        for (int64_t i = lo; i < hi; ++i) S->order[cnt[S->cell[i]]++] = i;
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            const int64_t i = S->order[k];
            S->xs[k] = pos[3 * i];
            S->xs[n + k] = pos[3 * i + 1];
            S->xs[2 * n + k] = pos[3 * i + 2];
        }
    }
}

/* Forces in user order into force (3 per atom). Each home cell gathers its
 * 27-cell neighbourhood, image shifts applied, into the thread's contiguous
 * buffers once; every home atom then runs one SIMD loop over all of it (as the
 * GPU kernel stages the neighbourhood in LDS). */
static void NAME(forces)(NAME(state)* S, const cc_params* p, REAL* force) {
    const int64_t nc = S->nc, n = S->n;
    const REAL L = S->box;
    const REAL rc = (REAL)p->rc, rc2 = rc * rc;
    const REAL s2 = (REAL)(p->sigma * p->sigma), e24 = (REAL)(24.0 * p->epsilon);
    /* f_LJ(r_c) = (24 eps / r_c) [2 (s/r_c)^12 - (s/r_c)^6] */
    const REAL q = s2 / rc2, q6 = q * q * q;
    const REAL fc = e24 / rc * ((REAL)2 * q6 * q6 - q6);
    const REAL* X = S->xs;
    const REAL* Y = S->xs + n;
    const REAL* Z = S->xs + 2 * n;
    int64_t most = 0;
    for (int64_t c = 0; c < S->ncells; ++c)
        if (S->start[c + 1] - S->start[c] > most) most = S->start[c + 1] - S->start[c];
    const int64_t cap = 27 * most + 1;
#pragma omp parallel num_threads(S->nthreads)
    {
        REAL* hx = (REAL*)malloc(sizeof(REAL) * 3 * (size_t)cap);
        REAL* hy = hx + cap;
        REAL* hz = hy + cap;
#pragma omp for schedule(dynamic, 16)
        for (int64_t c = 0; c < S->ncells; ++c) {
            const int64_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
            int64_t m = 0, self0 = 0;
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
                        if (dx == 0 && dy == 0 && dz == 0) self0 = m;
                        for (int64_t b = S->start[cj]; b < S->start[cj + 1]; ++b, ++m) {
                            hx[m] = X[b] + sx;
                            hy[m] = Y[b] + sy;
                            hz[m] = Z[b] + sz;
                        }
                    }
            for (int64_t a = S->start[c]; a < S->start[c + 1]; ++a) {
                const REAL xi = X[a], yi = Y[a], zi = Z[a];
                const int64_t self = self0 + (a - S->start[c]);
                REAL fx = 0, fy = 0, fz = 0;
#pragma omp simd reduction(+ : fx, fy, fz)
                for (int64_t k = 0; k < m; ++k) {
                    const REAL ddx = xi - hx[k];
                    const REAL ddy = yi - hy[k];
                    const REAL ddz = zi - hz[k];
                    const REAL r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    const int in = (r2 < rc2) & (k != self);
                    const REAL rs = in ? r2 : rc2;  /* no division by zero for the atom itself */
                    const REAL ir2 = (REAL)1 / rs, rinv = SQRT(ir2);
                    const REAL t = s2 * ir2, t6 = t * t * t;
                    /* (f_LJ(r) - f_LJ(r_c)) / r */
                    const REAL g = in ? e24 * ir2 * ((REAL)2 * t6 * t6 - t6) - fc * rinv : (REAL)0;
                    fx += g * ddx;
                    fy += g * ddy;
                    fz += g * ddz;
                }
                S->fs[3 * a] = fx;
                S->fs[3 * a + 1] = fy;
                S->fs[3 * a + 2] = fz;
            }
        }
        free(hx);
    }
#pragma omp parallel for schedule(static) num_threads(S->nthreads)
    for (int64_t k = 0; k < n; ++k)
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
#ifdef _OPENMP
    S.nthreads = omp_get_max_threads();
#else
    S.nthreads = 1;
#endif
    S.cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    S.start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S.ncells + 1));
    S.order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    S.tcount = (int64_t*)malloc(sizeof(int64_t) * (size_t)S.nthreads * (size_t)S.ncells);
    S.xs = (REAL*)malloc(sizeof(REAL) * 3 * (size_t)n);
    S.fs = (REAL*)malloc(sizeof(REAL) * 3 * (size_t)n);
    if (!S.cell || !S.start || !S.order || !S.tcount || !S.xs || !S.fs) {
        free(S.cell); free(S.start); free(S.order); free(S.tcount); free(S.xs); free(S.fs);
        return -1;
    }
    const REAL dt = (REAL)p->dt, h = (REAL)(0.5 * p->dt / p->mass);
    NAME(rebuild)(&S, pos);
    NAME(forces)(&S, p, force);
    for (int32_t k = 0; k < nsteps; ++k) {
#pragma omp parallel for schedule(static) num_threads(S.nthreads)
        for (int64_t i = 0; i < 3 * n; ++i) {
            vel[i] += h * force[i];
            pos[i] += dt * vel[i];
        }
        NAME(rebuild)(&S, pos);
        NAME(forces)(&S, p, force);
#pragma omp parallel for schedule(static) num_threads(S.nthreads)
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += h * force[i];
    }
    free(S.cell); free(S.start); free(S.order); free(S.tcount); free(S.xs); free(S.fs);
    return 0;
}
