/*
 * fillgen.c -- seeded synthetic waveform-digitizer fills.
 *
 * Stands in for the paper's data simulator and test-beam data (Section 3,
 * final paragraphs), which are not available: 12-bit ADC samples of one
 * calorimeter (a 6 x 9 grid of crystals) sampled at 800 MSPS (Section 3,
 * detector description), with negative positron pulses whose rate decays
 * with the muon lifetime.
 *
 * This file holds none of the island-chopping arithmetic: it only writes raw
 * samples (and a truth list of pulses). Both the HIP library and the CPU
 * oracle read the buffers it fills.
 *
 * Recipe (per fill, all draws from a counter-based hash of the seed so that
 * the result does not depend on the thread count):
 *   pedestal of channel c   ~ U(ped_lo, ped_hi)            (real valued)
 *   noise per sample        ~ N(0, noise_sigma)            (table inverse CDF)
 *   pulse times             inhomogeneous Poisson process with intensity
 *                           rate_mult * lambda0 * exp(-t / tau) per sample,
 *                           drawn as time-transformed unit-rate arrivals
 *   amplitude               ~ U(amp_lo, amp_hi) ADC counts
 *   template (negative)     exp(-d^2 / (2 rise_sigma^2)) for d < 0,
 *                           exp(-d / fall_tau) for d >= 0, d = t - t0,
 *                           truncated to [t0 - 12, t0 + 60]
 *   crystal split           1..max_crystals crystals (uniform count), a
 *                           4-neighbour connected cluster grown from a uniform
 *                           seed crystal, fractions ~ Dirichlet(1, ..., 1)
 *   sample value            clip(floor(ped_c + noise - sum A frac shape + 0.5),
 *                           0, 4095), padding columns [N, stride) set to 0.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t grid_rows;      /* crystal grid rows (6)                      */
    int32_t grid_cols;      /* crystal grid columns (9); C = rows * cols   */
    int64_t n_samples;      /* N                                          */
    int64_t row_stride;     /* elements between channel rows, >= N        */
    double rate_mult;       /* m: multiplies the initial pulse rate        */
    double lambda0;         /* initial pulses per sample at m = 1          */
    double tau_samples;     /* rate decay constant in samples              */
    double amp_lo, amp_hi;  /* pulse amplitude range, ADC                  */
    double ped_lo, ped_hi;  /* pedestal range, ADC                         */
    double noise_sigma;     /* ADC                                         */
    double rise_sigma;      /* samples                                     */
    double fall_tau;        /* samples                                     */
    int32_t max_crystals;   /* 1..4                                        */
    int32_t adc_max;        /* 4095 for 12 bits                            */
} synth_params;

typedef struct {
    double t0;              /* peak time, samples                          */
    double amp;             /* ADC counts                                  */
    int32_t n_cry;
    int32_t cry[4];
    double frac[4];
} synth_pulse;

/* ---- counter-based random numbers (SplitMix64 finaliser) ---------------- */

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

enum { DOM_PED = 1, DOM_NOISE = 2, DOM_ARRIVAL = 3, DOM_PULSE = 4 };

static uint64_t draw(uint64_t seed, uint64_t domain, uint64_t index)
{
    return mix64(mix64(seed ^ (domain * 0xD6E8FEB86659FD93ull)) + index);
}

static double unit(uint64_t h) /* uniform in (0, 1) */
{
    return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* ---- inverse normal CDF table ------------------------------------------- */

#define QBITS 12
#define QN (1 << QBITS)
static double g_qtab[QN + 1];
static pthread_once_t g_qonce = PTHREAD_ONCE_INIT;

static double norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

static void build_qtab(void)
{
    for (int i = 0; i <= QN; i++) {
        double p = ((double)i + 0.5) / (double)(QN + 1);
        double lo = -10.0, hi = 10.0;
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (lo + hi);
            if (norm_cdf(mid) < p)
                lo = mid;
            else
                hi = mid;
        }
        g_qtab[i] = 0.5 * (lo + hi);
    }
}

static double gauss(uint64_t h)
{
    uint32_t u = (uint32_t)(h >> 32);
    uint32_t i = u >> (32 - QBITS);
    double f = (double)(u & ((1u << (32 - QBITS)) - 1)) * (1.0 / (double)(1u << (32 - QBITS)));
    return g_qtab[i] + f * (g_qtab[i + 1] - g_qtab[i]);
}

/* ---- pulse list ---------------------------------------------------------- */

static int64_t make_pulses(uint64_t seed, const synth_params *p, synth_pulse **out)
{
    const int C = p->grid_rows * p->grid_cols;
    const double N = (double)p->n_samples;
    const double a = p->rate_mult * p->lambda0 * p->tau_samples; /* Lambda(inf) */
    const double total = a * (1.0 - exp(-N / p->tau_samples));   /* Lambda(N)   */
    int64_t cap = 1024, n = 0;
    synth_pulse *v = (synth_pulse *)malloc((size_t)cap * sizeof *v);
    if (!v)
        return -1;
    double E = 0.0;
    for (int64_t k = 0;; k++) {
        E += -log(unit(draw(seed, DOM_ARRIVAL, (uint64_t)k)));
        if (!(E < total) || a <= 0.0)
            break;
        if (n == cap) {
            cap *= 2;
            synth_pulse *nv = (synth_pulse *)realloc(v, (size_t)cap * sizeof *v);
            if (!nv) {
                free(v);
                return -1;
            }
            v = nv;
        }
        synth_pulse *q = &v[n];
        uint64_t base = (uint64_t)n * 64;
        q->t0 = -p->tau_samples * log(1.0 - E / a);
        q->amp = p->amp_lo + (p->amp_hi - p->amp_lo) * unit(draw(seed, DOM_PULSE, base + 0));
        int want = 1 + (int)(unit(draw(seed, DOM_PULSE, base + 1)) * p->max_crystals);
        if (want > p->max_crystals)
            want = p->max_crystals;
        if (want > C)
            want = C;
        int seedc = (int)(unit(draw(seed, DOM_PULSE, base + 2)) * C);
        if (seedc >= C)
            seedc = C - 1;
        q->n_cry = 1;
        q->cry[0] = seedc;
        uint64_t ctr = base + 3;
        for (int tries = 0; q->n_cry < want && tries < 50; tries++) {
            int from = q->cry[(int)(unit(draw(seed, DOM_PULSE, ctr++)) * q->n_cry) % q->n_cry];
            int dir = (int)(unit(draw(seed, DOM_PULSE, ctr++)) * 4) & 3;
            int r = from / p->grid_cols, c = from % p->grid_cols;
            if (dir == 0) r -= 1;
            if (dir == 1) r += 1;
            if (dir == 2) c -= 1;
            if (dir == 3) c += 1;
            if (r < 0 || r >= p->grid_rows || c < 0 || c >= p->grid_cols)
                continue;
            int cand = r * p->grid_cols + c, dup = 0;
            for (int j = 0; j < q->n_cry; j++)
                dup |= (q->cry[j] == cand);
            if (!dup)
                q->cry[q->n_cry++] = cand;
        }
        double s = 0.0;
        for (int j = 0; j < q->n_cry; j++) {
            q->frac[j] = -log(unit(draw(seed, DOM_PULSE, base + 40 + (uint64_t)j)));
            s += q->frac[j];
        }
        for (int j = 0; j < q->n_cry; j++)
            q->frac[j] /= s;
        n++;
    }
    *out = v;
    return n;
}

/* ---- rendering ------------------------------------------------------------ */

typedef struct {
    uint64_t seed;
    const synth_params *p;
    int16_t *out;
    const synth_pulse *pulses;
    const int64_t *chan_start; /* per channel, into chan_list */
    const int64_t *chan_list;  /* pulse indices grouped by channel */
    const double *chan_frac;
    int next;                  /* shared work counter */
    pthread_mutex_t lock;
} render_job;

static void render_channel(render_job *J, int c, double *acc)
{
    const synth_params *p = J->p;
    const int64_t N = p->n_samples;
    memset(acc, 0, (size_t)(N > 0 ? N : 1) * sizeof(double));
    const double inv2s2 = 1.0 / (2.0 * p->rise_sigma * p->rise_sigma);
    for (int64_t j = J->chan_start[c]; j < J->chan_start[c + 1]; j++) {
        const synth_pulse *q = &J->pulses[J->chan_list[j]];
        double a = q->amp * J->chan_frac[j];
        int64_t lo = (int64_t)ceil(q->t0 - 12.0), hi = (int64_t)floor(q->t0 + 60.0);
        if (lo < 0) lo = 0;
        if (hi > N - 1) hi = N - 1;
        for (int64_t t = lo; t <= hi; t++) {
            double d = (double)t - q->t0;
            double shape = d < 0.0 ? exp(-d * d * inv2s2) : exp(-d / p->fall_tau);
            acc[t] -= a * shape;
        }
    }
    double ped = p->ped_lo + (p->ped_hi - p->ped_lo) * unit(draw(J->seed, DOM_PED, (uint64_t)c));
    int16_t *row = J->out + (int64_t)c * p->row_stride;
    uint64_t nkey = mix64(J->seed ^ (DOM_NOISE * 0xD6E8FEB86659FD93ull)) + ((uint64_t)c << 40);
    for (int64_t t = 0; t < N; t++) {
        double v = ped + p->noise_sigma * gauss(mix64(nkey + (uint64_t)t)) + acc[t];
        double r = floor(v + 0.5);
        if (r < 0.0) r = 0.0;
        if (r > (double)p->adc_max) r = (double)p->adc_max;
        row[t] = (int16_t)r;
    }
    for (int64_t t = N; t < p->row_stride; t++)
        row[t] = 0;
}

static void *render_worker(void *arg)
{
    render_job *J = (render_job *)arg;
    const int C = J->p->grid_rows * J->p->grid_cols;
    double *acc = (double *)malloc((size_t)(J->p->n_samples > 0 ? J->p->n_samples : 1) * sizeof(double));
    if (!acc)
        return (void *)1;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int c = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (c >= C)
            break;
        render_channel(J, c, acc);
    }
    free(acc);
    return NULL;
}

/* Fills out[C * row_stride] (C = grid_rows * grid_cols) for one calorimeter
 * fill. Writes up to truth_cap pulses to truth (may be NULL). Returns the
 * number of pulses drawn, or a negative value on bad parameters or memory
 * failure. */
int64_t synth_fill(uint64_t seed, const synth_params *p, int16_t *out,
                   synth_pulse *truth, int64_t truth_cap, int32_t nthreads)
{
    if (!p || !out || p->grid_rows <= 0 || p->grid_cols <= 0 || p->n_samples < 0 ||
        p->row_stride < p->n_samples || p->max_crystals < 1 || p->max_crystals > 4)
        return -2;
    pthread_once(&g_qonce, build_qtab);
    const int C = p->grid_rows * p->grid_cols;
    synth_pulse *pulses = NULL;
    int64_t np = make_pulses(seed, p, &pulses);
    if (np < 0)
        return -1;
    int64_t *chan_start = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
    int64_t nrefs = 0;
    for (int64_t k = 0; k < np; k++)
        nrefs += pulses[k].n_cry;
    int64_t *chan_list = (int64_t *)malloc((size_t)(nrefs + 1) * sizeof(int64_t));
    double *chan_frac = (double *)malloc((size_t)(nrefs + 1) * sizeof(double));
    int64_t *fillpos = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    if (!chan_start || !chan_list || !chan_frac || !fillpos) {
        free(pulses); free(chan_start); free(chan_list); free(chan_frac); free(fillpos);
        return -1;
    }
    for (int64_t k = 0; k < np; k++)
        for (int j = 0; j < pulses[k].n_cry; j++)
            chan_start[pulses[k].cry[j] + 1]++;
    for (int c = 0; c < C; c++)
        chan_start[c + 1] += chan_start[c];
    for (int64_t k = 0; k < np; k++)
        for (int j = 0; j < pulses[k].n_cry; j++) {
            int c = pulses[k].cry[j];
            int64_t at = chan_start[c] + fillpos[c]++;
            chan_list[at] = k;
            chan_frac[at] = pulses[k].frac[j];
        }
    render_job J;
    J.seed = seed;
    J.p = p;
    J.out = out;
    J.pulses = pulses;
    J.chan_start = chan_start;
    J.chan_list = chan_list;
    J.chan_frac = chan_frac;
    J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    if (nt > C)
        nt = C;
    pthread_t th[256];
    int bad = 0;
    for (int i = 1; i < nt; i++)
        if (pthread_create(&th[i], NULL, render_worker, &J) != 0) {
            nt = i;
            break;
        }
    bad |= render_worker(&J) != NULL;
    for (int i = 1; i < nt; i++) {
        void *r = NULL;
        pthread_join(th[i], &r);
        bad |= r != NULL;
    }
    pthread_mutex_destroy(&J.lock);
    if (truth)
        for (int64_t k = 0; k < np && k < truth_cap; k++)
            truth[k] = pulses[k];
    free(pulses); free(chan_start); free(chan_list); free(chan_frac); free(fillpos);
    return bad ? -1 : np;
}
