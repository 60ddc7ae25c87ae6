/*
 * Serial CPU oracle for the parallel cellular Potts model sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation written from the paper (Sultan,
 * Devi, Mueller, Textor 2023, "A parallelized cellular Potts model that
 * enables simulations at tissue scale").  It shares no code, header, table
 * generator or helper with the GPU library.
 *
 * What is computed (paper references by section / equation):
 *   - Hamiltonian: adhesion + volume constraint (Methods, eq. 1), perimeter /
 *     surface constraint (Methods, eq. 3), with a Moore neighbourhood
 *     (Methods, text after eq. 1).
 *   - Acceptance: Boltzmann / Metropolis rule (Methods, eq. 2), realised as an
 *     integer test of a uniform 32-bit draw against a threshold
 *     floor(2^32 exp(-dH/T)) composed from three FP64-built tables.
 *   - Act extension: per-site activity, geometric mean over the site's own
 *     cell within its Moore neighbourhood, dH_act term (Methods, eq. 7-8),
 *     decay by one per MCS.
 *   - Parallel scheme: checkerboard of thread areas with 2^d colours that
 *     take turns (Results, "Designing a parallel execution scheme", Fig. 2A),
 *     one barrier per copy attempt (Results, "Aligning the lattice update
 *     statistics", Fig. 3A), per-cell volume / surface updated by summing all
 *     deltas of an activation (Fig. 2B, atomics), and copy attempts that read
 *     per-cell counters as they stood when the activation began (the
 *     stale-read tolerance of the same section) plus the attempting thread's
 *     own earlier deltas.
 *   - Persistence extension (Methods, eq. 5-6): a direction per cell,
 *     updated after every MCS from the displacement of the cell's centroid
 *     over the last dt MCS, mixed with the previous direction by mu and
 *     renormalised; a copy into a site favoured in proportion to how well the
 *     copy direction (source -> target) aligns with the copying cell's
 *     direction.  Kept in integer fixed point (see persistence_update).
 *   - Chemotaxis extension (Methods, eq. 4): a fixed vector field C; a copy
 *     from source i into a target is favoured in proportion to how well its
 *     direction aligns with C at i (same sign reading and fixed point as the
 *     persistence term).
 *   - Serial CPM (Methods, first paragraph) and a symmetric-proposal variant
 *     used only to pin the Hamiltonian + acceptance against Boltzmann
 *     weights.
 *
 * The random numbers of every copy attempt come from Philox4x32-10 (Salmon,
 * Moraes, Dror, Shaw, SC'11), keyed by the seed and counted by (thread area,
 * MCS, activation/attempt, lattice id).  The paper's own GPU generator is a
 * different one; a counter-based generator is what makes runs reproducible
 * independent of thread scheduling.
 *
 * Integer conventions: energies are int64 in units of 2^-16; parameters are
 * quantised with llround(x * 65536).  Lattice values: -1 obstacle (never
 * copied, never overwritten), 0 medium, 1..C cells.  Site index
 * i = x + Lx*(y + Ly*z), x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

/* ------------------------------------------------------------------ model */

typedef struct orc_model {
    int32_t ndim;          /* 2 or 3 */
    int32_t L[3];          /* Lx, Ly, Lz; Lz = 1 in 2D */
    int32_t s;             /* sub-area edge; thread area edge is 2s */
    int32_t k;             /* copy attempts per thread per activation */
    int32_t n_types;       /* type 0 is medium */
    int32_t obstacle_type; /* type used for J lookups against obstacle sites, -1 if none */
    double T;              /* temperature */
    uint64_t seed;
    uint32_t lattice_id;
    int32_t act_enabled;   /* 1 to include the Act term and Act bookkeeping */
    const double *J;           /* n_types x n_types, row-major */
    const double *lambda_V;    /* per type */
    const int32_t *V_target;   /* per type */
    const double *lambda_S;    /* per type */
    const int32_t *S_target;   /* per type */
    const double *lambda_act;  /* per type (used when act_enabled) */
    const int32_t *max_act;    /* per type; a type is motile iff max_act > 0 */
    const double *lambda_P;    /* per type, persistence strength (NULL: no persistence term) */
    const double *mu_P;        /* per type, weight of the previous direction, 0..1 */
    int32_t dt_P;              /* MCS looked back for the displacement, >= 1 */
    const double *lambda_C;    /* per type, chemotaxis strength (NULL: no chemotaxis term) */
    const int16_t *C_field;    /* the vector field C: components x, y (, z) of each site, sites in
                                * lattice order, in units of 2^-14 */
} orc_model;

/* Quantised energy parameters and acceptance tables. */
typedef struct orc_q {
    int64_t J[16][16];
    int64_t lV[16], lS[16], R[16];
    int64_t Vt[16], St[16];
    int32_t maxact[16];
    int32_t nnb;
    int32_t nb[26][3]; /* (dx, dy, dz) */
    uint64_t TI[8192];
    int32_t nTI;
    uint64_t TM[256], TL[256];
    int64_t LG[256];
    uint64_t EH[2048], EM[256], EL[256];
    int64_t lP[16];        /* persistence strength, 2^-16 */
    int64_t muP[16];       /* previous-direction weight, 2^-14 */
    int64_t lC[16];        /* chemotaxis strength, 2^-16 */
    int32_t U[27][3];      /* unit vector of offset (dx,dy,dz), index (dx+1)+3(dy+1)+9(dz+1), 2^-14 */
} orc_q;

static int64_t quantise(double x) { return (int64_t)llround(x * 65536.0); }

/* floor(2^32 * exp(x)) for x <= 0, built in FP64. */
static uint64_t fix32_exp(double x) { return (uint64_t)floor(exp(x) * 4294967296.0); }

/* Moore neighbourhood offsets in lexicographic order, z slowest, x fastest,
 * the zero offset left out. */
static void build_neighbours(int ndim, orc_q *q)
{
    int n = 0;
    int zr = ndim == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                q->nb[n][0] = dx; q->nb[n][1] = dy; q->nb[n][2] = dz;
                n++;
            }
    q->nnb = n;
}

/*
 * Acceptance tables (Methods, eq. 2).  For dH = q * 2^-16 > 0 with
 * q = h*2^16 + m*2^8 + l, the threshold is
 *     THR(q) = floor(TI[h] * TM[m] * TL[l] / 2^64)
 * with TI[h] = floor(2^32 e^{-h/T}), TM[m] = floor(2^32 e^{-m/(256 T)}),
 * TL[l] = floor(2^32 e^{-l/(65536 T)}).  TI runs until its first zero entry;
 * beyond it THR is 0.
 */
static int build_tables(double T, orc_q *q)
{
    int h = 0;
    for (;;) {
        uint64_t v = fix32_exp(-(double)h / T);
        if (v == 0) break;
        if (h >= 8192) return ORC_EINVAL;
        q->TI[h] = v;
        h++;
    }
    q->nTI = h;
    for (int m = 0; m < 256; m++) q->TM[m] = fix32_exp(-(double)m / (256.0 * T));
    for (int l = 0; l < 256; l++) q->TL[l] = fix32_exp(-(double)l / (65536.0 * T));
    /* Act geometric mean in the log domain: LG[a] = round(ln(a) * 2^24). */
    q->LG[0] = 0;
    for (int a = 1; a < 256; a++) q->LG[a] = (int64_t)llround(log((double)a) * 16777216.0);
    /* exp(l * 2^-24) split as exp(hi/2^8) * exp(mid/2^16) * exp(lo/2^24). */
    for (int i = 0; i < 2048; i++) q->EH[i] = (uint64_t)floor(exp((double)i / 256.0) * 16777216.0);
    for (int i = 0; i < 256; i++) q->EM[i] = (uint64_t)floor(exp((double)i / 65536.0) * 2147483648.0);
    for (int i = 0; i < 256; i++) q->EL[i] = (uint64_t)floor(exp((double)i / 16777216.0) * 1073741824.0);
    return ORC_OK;
}

static uint64_t threshold(const orc_q *q, int64_t dh)
{
    uint64_t u = (uint64_t)dh;
    uint64_t hh = u >> 16;
    if (hh >= (uint64_t)q->nTI) return 0;
    unsigned __int128 p = (unsigned __int128)q->TI[hh] * q->TM[(u >> 8) & 255];
    p = p * q->TL[u & 255];
    return (uint64_t)(p >> 64);
}

static int model_prepare(const orc_model *m, orc_q *q)
{
    if (!m || (m->ndim != 2 && m->ndim != 3)) return ORC_EINVAL;
    if (m->n_types < 1 || m->n_types > 16) return ORC_EINVAL;
    if (!(m->T > 0.0)) return ORC_EINVAL;
    memset(q, 0, sizeof(*q));
    for (int a = 0; a < m->n_types; a++) {
        for (int b = 0; b < m->n_types; b++) q->J[a][b] = quantise(m->J[a * m->n_types + b]);
        q->lV[a] = quantise(m->lambda_V[a]);
        q->lS[a] = quantise(m->lambda_S[a]);
        q->Vt[a] = m->V_target[a];
        q->St[a] = m->S_target[a];
        q->maxact[a] = m->act_enabled ? m->max_act[a] : 0;
        q->R[a] = (m->act_enabled && m->max_act[a] > 0)
                      ? quantise(m->lambda_act[a] / (double)m->max_act[a]) : 0;
    }
    build_neighbours(m->ndim, q);
    if (m->lambda_P) {
        if (!m->mu_P || m->dt_P < 1) return ORC_EINVAL;
        for (int a = 0; a < m->n_types; a++) {
            if (!(m->mu_P[a] >= 0.0 && m->mu_P[a] <= 1.0)) return ORC_EINVAL;
            q->lP[a] = quantise(m->lambda_P[a]);
            q->muP[a] = (int64_t)llround(m->mu_P[a] * 16384.0);
        }
    }
    if (m->lambda_C) {
        if (!m->C_field) return ORC_EINVAL;
        for (int a = 0; a < m->n_types; a++) q->lC[a] = quantise(m->lambda_C[a]);
    }
    /* unit vectors of the Moore offsets, rounded to 2^-14 in FP64 */
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int i = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                double len = sqrt((double)(dx * dx + dy * dy + dz * dz));
                int o[3] = {dx, dy, dz};
                for (int d = 0; d < 3; d++) q->U[i][d] = len > 0 ? (int32_t)llround(o[d] / len * 16384.0) : 0;
            }
    return build_tables(m->T, q);
}

/* ------------------------------------------------------------------ philox */

/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
 * multiplications, with the key bumped by the Weyl constants between rounds. */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

int oracle_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    philox4x32_10(ctr, key, out);
    return ORC_OK;
}

/* ------------------------------------------------------------------ lattice helpers */

typedef struct orc_state {
    const orc_model *m;
    const orc_q *q;
    int32_t *lat;
    const int32_t *type; /* per label 0..C */
    int32_t C;
    uint8_t *act;        /* may be NULL when act is disabled */
    int64_t *V, *S;      /* per label 0..C, entries for 0 unused */
    const int32_t *P;    /* per label 0..C, 3 components (2^-14); NULL without persistence */
} orc_state;

static int wrapc(int v, int L) { v %= L; return v < 0 ? v + L : v; }

static int64_t site_of(const orc_model *m, int x, int y, int z)
{
    x = wrapc(x, m->L[0]); y = wrapc(y, m->L[1]); z = wrapc(z, m->L[2]);
    return (int64_t)x + (int64_t)m->L[0] * ((int64_t)y + (int64_t)m->L[1] * z);
}

static void coords_of(const orc_model *m, int64_t i, int *x, int *y, int *z)
{
    *x = (int)(i % m->L[0]);
    *y = (int)((i / m->L[0]) % m->L[1]);
    *z = (int)(i / ((int64_t)m->L[0] * m->L[1]));
}

static int type_of_label(const orc_state *st, int32_t label)
{
    if (label < 0) return st->m->obstacle_type;
    return st->type[label];
}

/* ------------------------------------------------------------------ act */

/* Geometric-mean activity at site x (Methods, eq. 8), over x and those of its
 * Moore neighbours that belong to the same cell as x, in the fixed-point
 * log domain: GM = exp(floor(sum LG[Act]/|M|) * 2^-24), returned as
 * floor-composed 2^16 fixed point.  Zero for medium, obstacle, non-motile
 * cells, or when any activity in the set is zero. */
static int64_t gm_act(const orc_state *st, int64_t x)
{
    const orc_model *m = st->m;
    const orc_q *q = st->q;
    int32_t cell = st->lat[x];
    if (cell <= 0) return 0;
    if (q->maxact[st->type[cell]] <= 0) return 0;
    int cx, cy, cz;
    coords_of(m, x, &cx, &cy, &cz);
    int64_t sum = 0;
    int64_t count = 0;
    if (st->act[x] == 0) return 0;
    sum += q->LG[st->act[x]];
    count++;
    for (int n = 0; n < q->nnb; n++) {
        int64_t y = site_of(m, cx + q->nb[n][0], cy + q->nb[n][1], cz + q->nb[n][2]);
        if (st->lat[y] != cell) continue;
        if (st->act[y] == 0) return 0;
        sum += q->LG[st->act[y]];
        count++;
    }
    int64_t ell = sum / count; /* both non-negative: floor */
    uint64_t hi = (uint64_t)ell >> 16, mid = ((uint64_t)ell >> 8) & 255, lo = (uint64_t)ell & 255;
    uint64_t p1 = (q->EH[hi] * q->EM[mid]) >> 31;
    uint64_t p2 = (p1 * q->EL[lo]) >> 30;
    return (int64_t)(p2 >> 8);
}

int oracle_gm_act(const orc_model *m, const int32_t *lat, const int32_t *type, int32_t C,
                  const uint8_t *act, int64_t site, int64_t *gm_out)
{
    orc_q *q = (orc_q *)malloc(sizeof(orc_q));
    if (!q) return ORC_ENOMEM;
    if (model_prepare(m, q) != ORC_OK) { free(q); return ORC_EINVAL; }
    orc_state st = {m, q, (int32_t *)lat, type, C, (uint8_t *)act, NULL, NULL, NULL};
    *gm_out = gm_act(&st, site);
    free(q);
    return ORC_OK;
}

/* ------------------------------------------------------------------ energy */

/*
 * Local energy change of setting site t from its label to `nl`
 * (Methods, eq. 1 and eq. 3; act term eq. 7).  V and S are the per-cell
 * counters the attempt reads.  Also returns the surface deltas of the losing
 * and the gaining cell.
 */
static int64_t delta_h(const orc_state *st, int64_t t, int64_t src, int32_t nl,
                       const int64_t *V, const int64_t *S, int64_t *dS_old, int64_t *dS_new)
{
    const orc_model *m = st->m;
    const orc_q *q = st->q;
    int32_t ol = st->lat[t];
    int to = type_of_label(st, ol), tn = type_of_label(st, nl);
    int x, y, z;
    coords_of(m, t, &x, &y, &z);
    int64_t adh = 0;
    int64_t k_old = 0, k_new = 0;
    for (int n = 0; n < q->nnb; n++) {
        int64_t u = site_of(m, x + q->nb[n][0], y + q->nb[n][1], z + q->nb[n][2]);
        int32_t lu = st->lat[u];
        int tu = type_of_label(st, lu);
        if (lu != nl) adh += q->J[tn][tu];
        if (lu != ol) adh -= q->J[to][tu];
        if (lu == ol) k_old++;
        if (lu == nl) k_new++;
    }
    int64_t nnb = q->nnb;
    int64_t dso = 2 * k_old - nnb;
    int64_t dsn = nnb - 2 * k_new;
    int64_t vol = 0, surf = 0;
    if (ol >= 1) {
        vol += q->lV[to] * (1 - 2 * (V[ol] - q->Vt[to]));
        surf += q->lS[to] * (2 * dso * (S[ol] - q->St[to]) + dso * dso);
    }
    if (nl >= 1) {
        vol += q->lV[tn] * (2 * (V[nl] - q->Vt[tn]) + 1);
        surf += q->lS[tn] * (2 * dsn * (S[nl] - q->St[tn]) + dsn * dsn);
    }
    int64_t actterm = 0;
    if (m->act_enabled && src >= 0) {
        int64_t gt = gm_act(st, t), gs = gm_act(st, src);
        int64_t rt = ol >= 1 ? q->R[to] : 0, rs = nl >= 1 ? q->R[tn] : 0;
        actterm = (rt * gt - rs * gs) >> 16; /* arithmetic shift: floor */
    }
    /* persistence (eq. 5): the copying cell nl extends from src into t; the
     * term is -lambda_P * (unit copy direction . its direction), so copies
     * along the direction are favoured */
    int64_t pers = 0;
    if (m->lambda_P && st->P && nl >= 1 && src >= 0) {
        int sx, sy, sz;
        coords_of(m, src, &sx, &sy, &sz);
        int o[3] = {x - sx, y - sy, z - sz};
        for (int d = 0; d < 3; d++) {
            /* undo the periodic wrap: source and target are Moore neighbours */
            if (o[d] > 1) o[d] -= m->L[d];
            if (o[d] < -1) o[d] += m->L[d];
        }
        const int32_t *u = q->U[(o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
        const int32_t *p = st->P + 3 * (int64_t)nl;
        int64_t dot = (int64_t)u[0] * p[0] + (int64_t)u[1] * p[1] + (int64_t)u[2] * p[2];
        pers = -((q->lP[tn] * dot) >> 28); /* arithmetic shift: floor, then negated */
    }
    /* chemotaxis (eq. 4): the field at the source i, dotted with the unit
     * vector of the copy from i into the target; read like persistence, the
     * copying cell nl is favoured when it extends along the field */
    int64_t chem = 0;
    if (m->lambda_C && nl >= 1 && src >= 0) {
        int sx, sy, sz;
        coords_of(m, src, &sx, &sy, &sz);
        int o[3] = {x - sx, y - sy, z - sz};
        for (int d = 0; d < 3; d++) {
            if (o[d] > 1) o[d] -= m->L[d];
            if (o[d] < -1) o[d] += m->L[d];
        }
        const int32_t *u = q->U[(o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
        const int16_t *c = m->C_field + (int64_t)m->ndim * src;
        int64_t dot = 0;
        for (int d = 0; d < m->ndim; d++) dot += (int64_t)u[d] * c[d];
        chem = -((q->lC[tn] * dot) >> 28);
    }
    *dS_old = dso;
    *dS_new = dsn;
    return adh + vol + surf + actterm + pers + chem;
}

int oracle_delta_h(const orc_model *m, const int32_t *lat, const int32_t *type, int32_t C,
                   const uint8_t *act, const int64_t *V, const int64_t *S, int64_t t,
                   int64_t src, int32_t new_label, int64_t *dh_out, const int32_t *P)
{
    orc_q *q = (orc_q *)malloc(sizeof(orc_q));
    if (!q) return ORC_ENOMEM;
    if (model_prepare(m, q) != ORC_OK) { free(q); return ORC_EINVAL; }
    orc_state st = {m, q, (int32_t *)lat, type, C, (uint8_t *)act, NULL, NULL, P};
    int64_t a, b;
    *dh_out = delta_h(&st, t, src, new_label, V, S, &a, &b);
    free(q);
    return ORC_OK;
}

static int accept(const orc_q *q, int64_t dh, uint32_t u)
{
    if (dh <= 0) return 1;
    return (uint64_t)u < threshold(q, dh);
}

int oracle_threshold(double T, const int64_t *dh, int64_t n, uint64_t *thr_out)
{
    if (!(T > 0.0)) return ORC_EINVAL;
    orc_q *q = (orc_q *)malloc(sizeof(orc_q));
    if (!q) return ORC_ENOMEM;
    if (build_tables(T, q) != ORC_OK) { free(q); return ORC_EINVAL; }
    for (int64_t i = 0; i < n; i++) thr_out[i] = dh[i] <= 0 ? ((uint64_t)1 << 32) : threshold(q, dh[i]);
    free(q);
    return ORC_OK;
}

int oracle_tables(double T, uint64_t *TI, int32_t max_ti, int32_t *n_ti, uint64_t *TM, uint64_t *TL)
{
    if (!(T > 0.0)) return ORC_EINVAL;
    orc_q *q = (orc_q *)malloc(sizeof(orc_q));
    if (!q) return ORC_ENOMEM;
    if (build_tables(T, q) != ORC_OK) { free(q); return ORC_EINVAL; }
    *n_ti = q->nTI;
    for (int i = 0; i < q->nTI && i < max_ti; i++) TI[i] = q->TI[i];
    memcpy(TM, q->TM, sizeof q->TM);
    memcpy(TL, q->TL, sizeof q->TL);
    free(q);
    return ORC_OK;
}

/* ------------------------------------------------------------------ counters */

/* V(c) = number of sites of c; S(c) = number of ordered (site of c,
 * Moore neighbour not of c) pairs (Methods, text after eq. 3). */
int oracle_recount(const orc_model *m, const int32_t *lat, int32_t C, int64_t *V, int64_t *S)
{
    orc_q q;
    if (!m || (m->ndim != 2 && m->ndim != 3)) return ORC_EINVAL;
    memset(&q, 0, sizeof q);
    build_neighbours(m->ndim, &q);
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    for (int32_t c = 0; c <= C; c++) { V[c] = 0; S[c] = 0; }
    for (int64_t i = 0; i < N; i++) {
        int32_t c = lat[i];
        if (c < 0) continue;
        if (c > C) return ORC_EINVAL;
        V[c]++;
        int x, y, z;
        coords_of(m, i, &x, &y, &z);
        for (int n = 0; n < q.nnb; n++) {
            int64_t u = site_of(m, x + q.nb[n][0], y + q.nb[n][1], z + q.nb[n][2]);
            if (lat[u] != c) S[c]++;
        }
    }
    return ORC_OK;
}

/* Per-cell volume, surface and centroid sums.  The centroid sum of a cell is
 * taken over its sites, each expressed as the periodic image nearest to the
 * cell's first site in index order (minimum image per axis), so that a cell
 * straddling the boundary is not torn in two. */
int oracle_cell_stats(const orc_model *m, const int32_t *lat, int32_t C, int64_t *V, int64_t *S,
                      int64_t *centroid_sum /* (C+1) x ndim */)
{
    int rc = oracle_recount(m, lat, C, V, S);
    if (rc != ORC_OK || !centroid_sum) return rc;
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    int64_t *ref = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    if (!ref) return ORC_ENOMEM;
    for (int32_t c = 0; c <= C; c++) ref[c] = -1;
    for (int64_t i = 0; i < (int64_t)(C + 1) * m->ndim; i++) centroid_sum[i] = 0;
    for (int64_t i = 0; i < N; i++) {
        int32_t c = lat[i];
        if (c <= 0) continue;
        if (ref[c] < 0) ref[c] = i;
        int p[3], r[3];
        coords_of(m, i, &p[0], &p[1], &p[2]);
        coords_of(m, ref[c], &r[0], &r[1], &r[2]);
        for (int d = 0; d < m->ndim; d++) {
            int L = m->L[d];
            int diff = p[d] - r[d];
            if (diff > L / 2) diff -= L;
            if (diff < -(L - 1) / 2) diff += L;
            centroid_sum[(int64_t)c * m->ndim + d] += r[d] + diff;
        }
    }
    free(ref);
    return ORC_OK;
}

/* ------------------------------------------------------------------ sweeps */

static void commit(orc_state *st, int64_t t, int32_t nl)
{
    st->lat[t] = nl;
    if (st->m->act_enabled && st->act) {
        int tn = nl >= 1 ? st->type[nl] : -1;
        st->act[t] = (nl >= 1 && st->q->maxact[tn] > 0) ? (uint8_t)st->q->maxact[tn] : 0;
    }
}

static void act_decay(orc_state *st)
{
    if (!st->m->act_enabled || !st->act) return;
    const orc_model *m = st->m;
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    for (int64_t i = 0; i < N; i++)
        if (st->act[i] > 0) st->act[i]--;
}

static int check_state(const orc_model *m, const int32_t *lat, int32_t C)
{
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    for (int64_t i = 0; i < N; i++)
        if (lat[i] < -1 || lat[i] > C) return ORC_EINVAL;
    return ORC_OK;
}

/* Persistence state of a run: per cell the direction P (3 components,
 * 2^-14), the centroid history hist ((dt+1) slots of 3 components, 2^-16)
 * and the number t of direction updates done. */
typedef struct orc_pers {
    int32_t *P;
    int64_t *hist;
    int64_t *t;
} orc_pers;

static int sweep_dcs(const orc_model *m, const orc_q *qp, int32_t *lat, const int32_t *type, int32_t C,
                     uint8_t *act, int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs,
                     int64_t *stats, int32_t *target_log, orc_pers *pers);
static int sweep_serial(const orc_model *m, const orc_q *qp, int32_t *lat, const int32_t *type, int32_t C,
                        uint8_t *act, int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs,
                        int32_t symmetric, int64_t *stats, int32_t *target_log, orc_pers *pers);

/* floor(sqrt(n)), exact for 0 <= n < 2^62 (the FP64 root is only a first guess) */
static int64_t isqrt64(int64_t n)
{
    if (n <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)n);
    while (r > 0 && r * r > n) r--;
    while ((r + 1) * (r + 1) <= n) r++;
    return r;
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if (a % b != 0 && a < 0) q--;
    return q;
}

/* Centroids of every cell in 2^-16 fixed point: floor(centroid sum * 2^16 / V),
 * the sum taken as in oracle_cell_stats. */
static int centroids_fixed(const orc_model *m, const int32_t *lat, int32_t C, int64_t *X, int64_t *V)
{
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *cs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1) * 3);
    if (!S || !cs) { free(S); free(cs); return ORC_ENOMEM; }
    int rc = oracle_cell_stats(m, lat, C, V, S, cs);
    for (int32_t c = 0; c <= C && rc == ORC_OK; c++)
        for (int d = 0; d < 3; d++)
            X[3 * (int64_t)c + d] = (d < m->ndim && V[c] > 0) ? floor_div(cs[(int64_t)c * m->ndim + d] * 65536, V[c]) : 0;
    free(S); free(cs);
    return rc;
}

/*
 * Direction update after an MCS (eq. 6), in integers.  For every cell alive:
 * X = its centroid (2^-16); D = X - X(dt updates ago), each component brought
 * to the minimum image [-L/2, L/2) * 2^16; u = trunc(D * 2^14 / |D|) (0 if D
 * is 0), |.| = floor of the Euclidean norm; p = (2^14 - mu) * u + mu * P;
 * P = trunc(p * 2^14 / |p|) (0 if p is 0).  Dead cells get P = 0.  The
 * history holds dt + 1 centroids per cell: update t writes slot t mod (dt+1)
 * and reads slot (t + 1) mod (dt+1), which holds the centroid of update
 * t - dt, or the initial one.
 */
static int persistence_update(const orc_model *m, const orc_q *q, const int32_t *lat, const int32_t *type,
                              int32_t C, orc_pers *pers)
{
    int64_t *X = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1) * 3);
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    if (!X || !V) { free(X); free(V); return ORC_ENOMEM; }
    int rc = centroids_fixed(m, lat, C, X, V);
    const int64_t slots = m->dt_P + 1;
    const int64_t t = *pers->t + 1;
    for (int32_t c = 1; c <= C && rc == ORC_OK; c++) {
        int32_t *P = pers->P + 3 * (int64_t)c;
        int64_t *h = pers->hist + 3 * slots * (int64_t)c;
        if (V[c] == 0) { P[0] = P[1] = P[2] = 0; continue; }
        int64_t D[3];
        for (int d = 0; d < 3; d++) {
            D[d] = X[3 * (int64_t)c + d] - h[3 * ((t + 1) % slots) + d];
            int64_t W = (int64_t)m->L[d] * 65536;
            int64_t w = D[d] % W;
            if (w < 0) w += W;
            if (w >= W / 2) w -= W;
            D[d] = d < m->ndim ? w : 0;
        }
        for (int d = 0; d < 3; d++) h[3 * (t % slots) + d] = X[3 * (int64_t)c + d];
        int64_t nd = isqrt64(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        int64_t mu = q->muP[type[c]];
        int64_t pv[3];
        for (int d = 0; d < 3; d++) {
            int64_t u = nd > 0 ? (D[d] * 16384) / nd : 0;
            pv[d] = (16384 - mu) * u + mu * P[d];
        }
        int64_t np = isqrt64(pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2]);
        for (int d = 0; d < 3; d++) P[d] = np > 0 ? (int32_t)((pv[d] * 16384) / np) : 0;
    }
    *pers->t = t;
    free(X); free(V);
    return rc;
}

/* Start of a run with persistence: P = 0 and every history slot = the
 * current centroid. */
int oracle_persist_init(const orc_model *m, const int32_t *lat, int32_t C, int32_t *P, int64_t *hist,
                        int64_t *t)
{
    if (!m || m->dt_P < 1) return ORC_EINVAL;
    int64_t *X = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1) * 3);
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    if (!X || !V) { free(X); free(V); return ORC_ENOMEM; }
    int rc = centroids_fixed(m, lat, C, X, V);
    const int64_t slots = m->dt_P + 1;
    for (int32_t c = 0; c <= C && rc == ORC_OK; c++) {
        for (int d = 0; d < 3; d++) P[3 * (int64_t)c + d] = 0;
        for (int64_t k = 0; k < slots; k++)
            for (int d = 0; d < 3; d++) hist[3 * (slots * c + k) + d] = X[3 * (int64_t)c + d];
    }
    *t = 0;
    free(X); free(V);
    return rc;
}

/* One direction update (for tests): as after an MCS. */
int oracle_persist_update(const orc_model *m, const int32_t *lat, const int32_t *type, int32_t C, int32_t *P,
                          int64_t *hist, int64_t *t)
{
    if (!m || !m->lambda_P) return ORC_EINVAL;
    orc_q *q = (orc_q *)malloc(sizeof(orc_q));
    if (!q) return ORC_ENOMEM;
    int rc = model_prepare(m, q);
    orc_pers pers = {P, hist, t};
    if (rc == ORC_OK) rc = persistence_update(m, q, lat, type, C, &pers);
    free(q);
    return rc;
}

/* The per-MCS end of a sweep: Act decays, then the persistence directions
 * are updated. */
static int end_of_mcs(orc_state *st, orc_pers *pers)
{
    act_decay(st);
    if (st->m->lambda_P && pers) return persistence_update(st->m, st->q, st->lat, st->type, st->C, pers);
    return ORC_OK;
}

/*
 * The deterministic parallel scheme.  One MCS is (2s)^d / k activations.
 * Activation a has colour a mod 2^d; in it every thread area makes k copy
 * attempts inside the sub-area of edge s at offset s*colour within the area.
 * Attempts of one activation read the per-cell counters of the activation
 * start, plus their own thread's earlier deltas; all deltas are summed into
 * the counters when the activation ends.  Act decays at the end of each MCS.
 *
 * stats (nullable, 3 entries): attempts, attempts past the early rejection,
 * accepted copies.  target_log (nullable): target site of every attempt in
 * the order (mcs, activation, area, attempt).
 */
int oracle_sweep(const orc_model *m, int32_t *lat, const int32_t *type, int32_t C, uint8_t *act,
                 int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs, int64_t *stats,
                 int32_t *target_log)
{
    orc_q *qp = (orc_q *)malloc(sizeof(orc_q));
    if (!qp) return ORC_ENOMEM;
    int rc = model_prepare(m, qp);
    if (rc == ORC_OK) rc = sweep_dcs(m, qp, lat, type, C, act, V, S, mcs0, n_mcs, stats, target_log, NULL);
    free(qp);
    return rc;
}

/* oracle_sweep with the persistence term: P, hist, t as set up by
 * oracle_persist_init and carried from call to call. */
int oracle_sweep_p(const orc_model *m, int32_t *lat, const int32_t *type, int32_t C, uint8_t *act,
                   int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs, int64_t *stats,
                   int32_t *P, int64_t *hist, int64_t *t)
{
    if (!m->lambda_P || !P || !hist || !t) return ORC_EINVAL;
    orc_q *qp = (orc_q *)malloc(sizeof(orc_q));
    if (!qp) return ORC_ENOMEM;
    orc_pers pers = {P, hist, t};
    int rc = model_prepare(m, qp);
    if (rc == ORC_OK) rc = sweep_dcs(m, qp, lat, type, C, act, V, S, mcs0, n_mcs, stats, NULL, &pers);
    free(qp);
    return rc;
}

static int sweep_dcs(const orc_model *m, const orc_q *qp, int32_t *lat, const int32_t *type, int32_t C,
                     uint8_t *act, int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs,
                     int64_t *stats, int32_t *target_log, orc_pers *pers)
{
    const orc_q *q = qp;
    int d = m->ndim;
    int s = m->s, k = m->k;
    if (s < 1 || k < 1) return ORC_EINVAL;
    int sd = 1;
    for (int i = 0; i < d; i++) sd *= s;
    if (sd % k != 0) return ORC_EINVAL;
    for (int i = 0; i < d; i++)
        if (m->L[i] % (2 * s) != 0) return ORC_EINVAL;
    if (d == 2 && m->L[2] != 1) return ORC_EINVAL;
    if (m->act_enabled && (s < 2 || !act)) return ORC_EINVAL;
    if (check_state(m, lat, C) != ORC_OK) return ORC_EINVAL;

    int na[3] = {m->L[0] / (2 * s), m->L[1] / (2 * s), d == 3 ? m->L[2] / (2 * s) : 1};
    int64_t n_areas = (int64_t)na[0] * na[1] * na[2];
    int colours = 1 << d;
    int n_act = colours * sd / k; /* (2s)^d / k */
    uint32_t key[2] = {(uint32_t)m->seed, (uint32_t)(m->seed >> 32)};

    orc_state st = {m, q, lat, type, C, act, V, S, pers ? pers->P : NULL};
    int64_t *Vr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *Sr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *dV = (int64_t *)calloc((size_t)(C + 1), sizeof(int64_t));
    int64_t *dS = (int64_t *)calloc((size_t)(C + 1), sizeof(int64_t));
    /* own deltas of the current thread: at most 2k distinct cells */
    int32_t *own_c = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * k));
    int64_t *own_v = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * k));
    int64_t *own_s = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * k));
    if (!Vr || !Sr || !dV || !dS || !own_c || !own_v || !own_s) {
        free(Vr); free(Sr); free(dV); free(dS); free(own_c); free(own_v); free(own_s);
        return ORC_ENOMEM;
    }
    int64_t log_pos = 0;

    for (int32_t mi = 0; mi < n_mcs; mi++) {
        uint32_t mcs = (uint32_t)(mcs0 + (uint64_t)mi);
        for (int alpha = 0; alpha < n_act; alpha++) {
            int phi = alpha % colours;
            int col[3] = {phi & 1, (phi >> 1) & 1, (phi >> 2) & 1};
            memcpy(Vr, V, sizeof(int64_t) * (size_t)(C + 1));
            memcpy(Sr, S, sizeof(int64_t) * (size_t)(C + 1));
            for (int64_t a = 0; a < n_areas; a++) {
                int ax = (int)(a % na[0]);
                int ay = (int)((a / na[0]) % na[1]);
                int az = (int)(a / ((int64_t)na[0] * na[1]));
                int own_n = 0;
                for (int j = 0; j < k; j++) {
                    uint32_t ctr[4] = {(uint32_t)a, mcs, ((uint32_t)alpha << 8) | (uint32_t)j,
                                       m->lattice_id};
                    uint32_t u[4];
                    philox4x32_10(ctr, key, u);
                    uint32_t o = (uint32_t)(((uint64_t)u[0] * (uint64_t)sd) >> 32);
                    int ox = (int)(o % (uint32_t)s);
                    int oy = (int)((o / (uint32_t)s) % (uint32_t)s);
                    int oz = (int)(o / (uint32_t)(s * s));
                    int tx = 2 * s * ax + s * col[0] + ox;
                    int ty = 2 * s * ay + s * col[1] + oy;
                    int tz = d == 3 ? 2 * s * az + s * col[2] + oz : 0;
                    int64_t t = site_of(m, tx, ty, tz);
                    if (target_log) target_log[log_pos++] = (int32_t)t;
                    if (stats) stats[0]++;
                    int n = (int)(((uint64_t)u[1] * (uint64_t)q->nnb) >> 32);
                    int64_t src = site_of(m, tx + q->nb[n][0], ty + q->nb[n][1], tz + q->nb[n][2]);
                    int32_t lt = lat[t], ls = lat[src];
                    if (lt == ls || lt < 0 || ls < 0) continue;
                    if (stats) stats[1]++;
                    /* counters this attempt sees: snapshot + own deltas */
                    int64_t vo = 0, so = 0, vn = 0, sn = 0;
                    for (int i = 0; i < own_n; i++) {
                        if (own_c[i] == lt) { vo += own_v[i]; so += own_s[i]; }
                        if (own_c[i] == ls) { vn += own_v[i]; sn += own_s[i]; }
                    }
                    /* delta_h reads V[label], S[label]; hand it patched copies for the two cells */
                    int64_t sv_ot = Vr[lt], ss_ot = Sr[lt], sv_nt = Vr[ls], ss_nt = Sr[ls];
                    Vr[lt] += vo; Sr[lt] += so;
                    Vr[ls] += vn; Sr[ls] += sn;
                    int64_t dso, dsn;
                    int64_t dh = delta_h(&st, t, src, ls, Vr, Sr, &dso, &dsn);
                    Vr[lt] = sv_ot; Sr[lt] = ss_ot; Vr[ls] = sv_nt; Sr[ls] = ss_nt;
                    if (!accept(q, dh, u[2])) continue;
                    if (stats) stats[2]++;
                    commit(&st, t, ls);
                    if (lt >= 1) { dV[lt] -= 1; dS[lt] += dso; }
                    if (ls >= 1) { dV[ls] += 1; dS[ls] += dsn; }
                    if (k > 1) {
                        int32_t cells[2] = {lt, ls};
                        int64_t vv[2] = {-1, 1}, ss[2] = {dso, dsn};
                        for (int e = 0; e < 2; e++) {
                            if (cells[e] < 1) continue;
                            int i;
                            for (i = 0; i < own_n; i++)
                                if (own_c[i] == cells[e]) break;
                            if (i == own_n) { own_c[i] = cells[e]; own_v[i] = 0; own_s[i] = 0; own_n++; }
                            own_v[i] += vv[e];
                            own_s[i] += ss[e];
                        }
                    }
                }
            }
            for (int32_t c = 1; c <= C; c++) {
                V[c] += dV[c]; S[c] += dS[c];
                dV[c] = 0; dS[c] = 0;
            }
        }
        if (end_of_mcs(&st, pers) != ORC_OK) {
            free(Vr); free(Sr); free(dV); free(dS); free(own_c); free(own_v); free(own_s);
            return ORC_ENOMEM;
        }
    }
    free(Vr); free(Sr); free(dV); free(dS); free(own_c); free(own_v); free(own_s);
    return ORC_OK;
}

/*
 * The serial CPM (Methods, first paragraph): N = |lattice| copy attempts per
 * MCS, each at a uniformly drawn site, copying from a uniformly drawn Moore
 * neighbour; counters always exact.  When `symmetric` is set the proposal is
 * instead a uniformly drawn new label among all labels other than the
 * target's (0..C, obstacles excluded); that chain satisfies detailed balance
 * with respect to exp(-H/T) and is used only to pin H and the acceptance.
 * Random numbers: Philox with counter (attempt, mcs, 0xFFFFFF00, lattice id).
 */
int oracle_serial_sweep(const orc_model *m, int32_t *lat, const int32_t *type, int32_t C, uint8_t *act,
                        int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs, int32_t symmetric,
                        int64_t *stats, int32_t *target_log)
{
    orc_q *qp = (orc_q *)malloc(sizeof(orc_q));
    if (!qp) return ORC_ENOMEM;
    int rc = model_prepare(m, qp);
    if (rc == ORC_OK)
        rc = sweep_serial(m, qp, lat, type, C, act, V, S, mcs0, n_mcs, symmetric, stats, target_log, NULL);
    free(qp);
    return rc;
}

static int sweep_serial(const orc_model *m, const orc_q *qp, int32_t *lat, const int32_t *type, int32_t C,
                        uint8_t *act, int64_t *V, int64_t *S, uint64_t mcs0, int32_t n_mcs,
                        int32_t symmetric, int64_t *stats, int32_t *target_log, orc_pers *pers)
{
    const orc_q *q = qp;
    if (m->act_enabled && !act) return ORC_EINVAL;
    if (check_state(m, lat, C) != ORC_OK) return ORC_EINVAL;
    if (symmetric && C < 1) return ORC_EINVAL;
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    if (N >= ((int64_t)1 << 32)) return ORC_EINVAL;
    uint32_t key[2] = {(uint32_t)m->seed, (uint32_t)(m->seed >> 32)};
    orc_state st = {m, q, lat, type, C, act, V, S, pers ? pers->P : NULL};
    int64_t log_pos = 0;
    for (int32_t mi = 0; mi < n_mcs; mi++) {
        uint32_t mcs = (uint32_t)(mcs0 + (uint64_t)mi);
        for (int64_t i = 0; i < N; i++) {
            uint32_t ctr[4] = {(uint32_t)i, mcs, 0xFFFFFF00u, m->lattice_id};
            uint32_t u[4];
            philox4x32_10(ctr, key, u);
            int64_t t = (int64_t)(((uint64_t)u[0] * (uint64_t)N) >> 32);
            if (target_log) target_log[log_pos++] = (int32_t)t;
            if (stats) stats[0]++;
            int32_t lt = lat[t];
            int32_t ls;
            int64_t src = -1;
            if (symmetric) {
                if (lt < 0) continue;
                uint32_t l = (uint32_t)(((uint64_t)u[1] * (uint64_t)C) >> 32);
                ls = (int32_t)l < lt ? (int32_t)l : (int32_t)l + 1;
            } else {
                int x, y, z;
                coords_of(m, t, &x, &y, &z);
                int n = (int)(((uint64_t)u[1] * (uint64_t)q->nnb) >> 32);
                src = site_of(m, x + q->nb[n][0], y + q->nb[n][1], z + q->nb[n][2]);
                ls = lat[src];
                if (lt == ls || lt < 0 || ls < 0) continue;
            }
            if (stats) stats[1]++;
            int64_t dso, dsn;
            int64_t dh = delta_h(&st, t, src, ls, V, S, &dso, &dsn);
            if (!accept(q, dh, u[2])) continue;
            if (stats) stats[2]++;
            commit(&st, t, ls);
            if (lt >= 1) { V[lt] -= 1; S[lt] += dso; }
            if (ls >= 1) { V[ls] += 1; S[ls] += dsn; }
        }
        if (end_of_mcs(&st, pers) != ORC_OK) return ORC_ENOMEM;
    }
    return ORC_OK;
}

/*
 * Independent replicate runs for distribution tests: replicate r starts from
 * the same initial lattice and uses lattice id (model lattice id + r), which
 * gives it its own Philox stream.  mode 0 = parallel scheme, 1 = serial CPM,
 * 2 = serial symmetric proposal.  Writes the final lattices (n_rep x N).
 */
/* Replicates of an Act model under the parallel scheme: replicate r starts
 * from lat0 and act0 with lattice id m->lattice_id + r and runs n_mcs MCS;
 * its final labels and activities go to final_lat and final_act. */
int oracle_replicates_act(const orc_model *m, const int32_t *lat0, const uint8_t *act0, const int32_t *type,
                          int32_t C, int32_t n_mcs, int32_t n_rep, int32_t *final_lat, uint8_t *final_act)
{
    if (!m->act_enabled) return ORC_EINVAL;
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    orc_q *qp = (orc_q *)malloc(sizeof(orc_q));
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int rc = (qp && V && S) ? ORC_OK : ORC_ENOMEM;
    if (rc == ORC_OK) rc = model_prepare(m, qp);
    orc_model mr = *m;
    for (int32_t r = 0; r < n_rep && rc == ORC_OK; r++) {
        int32_t *lat = final_lat + (int64_t)r * N;
        uint8_t *act = final_act + (int64_t)r * N;
        memcpy(lat, lat0, sizeof(int32_t) * (size_t)N);
        memcpy(act, act0, (size_t)N);
        rc = oracle_recount(m, lat, C, V, S);
        if (rc != ORC_OK) break;
        mr.lattice_id = m->lattice_id + (uint32_t)r;
        rc = sweep_dcs(&mr, qp, lat, type, C, act, V, S, 0, n_mcs, NULL, NULL, NULL);
    }
    free(qp); free(V); free(S);
    return rc;
}

int oracle_replicates(const orc_model *m, const int32_t *lat0, const int32_t *type, int32_t C,
                      int32_t n_mcs, int32_t n_rep, int32_t mode, int32_t *final_lat)
{
    if (m->act_enabled) return ORC_EINVAL;
    int64_t N = (int64_t)m->L[0] * m->L[1] * m->L[2];
    orc_q *qp = (orc_q *)malloc(sizeof(orc_q));
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int rc = (qp && V && S) ? ORC_OK : ORC_ENOMEM;
    if (rc == ORC_OK) rc = model_prepare(m, qp);
    orc_model mr = *m;
    for (int32_t r = 0; r < n_rep && rc == ORC_OK; r++) {
        int32_t *lat = final_lat + (int64_t)r * N;
        memcpy(lat, lat0, sizeof(int32_t) * (size_t)N);
        rc = oracle_recount(m, lat, C, V, S);
        if (rc != ORC_OK) break;
        mr.lattice_id = m->lattice_id + (uint32_t)r;
        if (mode == 0)
            rc = sweep_dcs(&mr, qp, lat, type, C, NULL, V, S, 0, n_mcs, NULL, NULL, NULL);
        else
            rc = sweep_serial(&mr, qp, lat, type, C, NULL, V, S, 0, n_mcs, mode == 2, NULL, NULL, NULL);
    }
    free(qp); free(V); free(S);
    return rc;
}
