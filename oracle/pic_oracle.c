/* CPU oracle for the spin-dependent hot-electron particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY -- loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Plain FP64 C, particle-major:
 * every primary tree is followed particle by particle through all of its steps, with a
 * LIFO of the secondaries it spawns.  No blocking, no fusion; the steps appear in the
 * order of the Strang splitting of arXiv:1807.04733 Eq. (15):
 *     Source(dt/2) Transport(dt/2) Scattering(dt) Transport(dt/2) Source(dt/2)
 * followed by the moments of Eq. (16) (density) and Eq. (23) (spin current).
 *
 * Readings of the paper that the text leaves open (the same list is kept with the
 * design notes): the scattering probability in one step is p = 1 - exp(-dt/tau_eff)
 * (Sec. III.A: the chance that some event occurs during the step) with at most one
 * event per step evaluated at the mid-step state; an inelastic event splits E into
 * uE (kept by the scattering carrier, Eq. 7: uniform final energy) and (1-u)E (the
 * secondary, energy conservation); both products below E_min are removed at once;
 * newborn secondaries receive only the second transport half step in their birth
 * step; deposits are taken after the full step (time slot n <-> t = (n+1) dt).
 *
 * Random numbers: Philox4x32-10 keyed by the seed, counter = (uid_lo, uid_hi, step, tag)
 * with one fixed tag per purpose, so every draw is a pure function of
 * (seed, particle, step, purpose) and independent of processing order.  The event
 * decisions of the two steps 2m and 2m+1 share one counter (step field 2m, tag DECIDE):
 * word 0 decides step 2m, word 1 step 2m+1.
 *
 * Compile with -ffp-contract=off: every decision is taken on IEEE binary64 results of
 * the operations written here, in this order.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TAG_SCAT   0x000u
#define TAG_SPAWN  0x100u
#define TAG_HALF1  0x200u
#define TAG_HALF2  0x300u
#define TAG_INJECT 0x400u
#define TAG_DECIDE 0x500u
#define MAX_HITS   8
#define MAX_LAYERS 16

/* ------------------------------------------------------------------ Philox4x32-10 */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
 * each round multiplies counter words 0 and 2 by two fixed odd constants, takes the
 * 64-bit products apart, and mixes the high halves with the other two words and the
 * round key; the key advances by two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod_b;
    uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod_a;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(const orc_problem* P, uint32_t uid_lo, uint32_t uid_hi, uint32_t step,
                 uint32_t tag, uint32_t w[4]) {
  uint32_t ctr[4] = {uid_lo, uid_hi, step, tag};
  for (int64_t i = 0; i < P->n_script; ++i) {   /* scripted words, if this counter is listed */
    const uint32_t* e = P->script + 8 * i;
    if (e[0] == ctr[0] && e[1] == ctr[1] && e[2] == ctr[2] && e[3] == ctr[3]) {
      memcpy(w, e + 4, 4 * sizeof(uint32_t));
      return;
    }
  }
  uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* uniform on (0,1), exact in binary64 */
static double unif(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
/* uniform direction cosine on (-1,1), exact and never 0 */
static double cosine(uint32_t w) { return ((double)w + 0.5) * 0x1p-31 - 1.0; }

static double stored(const orc_problem* P, double x) {
  return P->state_fp64 ? x : (double)(float)x;
}

/* ------------------------------------------------------------------ particles */
typedef struct {
  double z, mu;            /* z: working value inside a step; mu: at storage precision */
  uint32_t E;
  uint32_t root, lin;
  int layer, spin, gen;
  uint32_t w;              /* superparticle weight, 2^-16 units (Eq. 10) */
  int ev[4];               /* events, transmissions, reflections, spawns */
  int dead;                /* absorption step or -1 */
  int n_next;              /* first step still to run */
  int newborn;             /* 1: born mid-step n_next, only the second half step remains */
  double* S;               /* causal score (gradient mode) */
} particle;

typedef struct {
  particle* items;
  int n, cap;
} pstack;

static int push(pstack* s, const particle* p) {
  if (s->n == s->cap) {
    int nc = s->cap ? 2 * s->cap : 64;
    particle* ni = (particle*)realloc(s->items, sizeof(particle) * (size_t)nc);
    if (!ni) return -1;
    s->items = ni;
    s->cap = nc;
  }
  s->items[s->n++] = *p;
  return 0;
}

typedef struct {
  const orc_problem* P;
  orc_output* O;
  int inst_id;
  const orc_instance* I;
  int64_t dens_off, cur_off, gen_off;
  int K;                    /* gradient length, 0 if off */
  double* grad;             /* thread-local accumulator */
  double* tree_score;       /* per-tree mode: sum of scores of the current tree */
  double tree_return;       /* per-tree mode: sum of g * deposit of the current tree */
  pstack* stack;
  int error;
} worker;

static void count(worker* W, int n, int which, int64_t by) {
#pragma omp atomic
  W->O->counters[(int64_t)n * ORC_NCOUNTERS + which] += by;
}

static void add_score(worker* W, particle* p, int k, double s) {
  if (!W->K) return;
  if (W->O->grad_per_tree) W->tree_score[k] += s;
  else p->S[k] += s;
}

/* Transmission probability of table t at energy E: a constant, or linear interpolation
 * on TE equidistant nodes (clamped beyond the last node).  The weights of the two nodes
 * are returned for the gradient. */
static double transmission(const orc_instance* I, int t, uint32_t E, int* k0, double* w0,
                           double* w1) {
  const double* tab = I->T + (int64_t)t * I->t_entries;
  if (I->t_entries == 1) {
    *k0 = 0; *w0 = 1.0; *w1 = 0.0;
    return tab[0];
  }
  double x = ((double)E * 0x1p-30) * I->T_scale;
  int k = (int)floor(x);
  if (k >= I->t_entries - 1) {
    *k0 = I->t_entries - 1; *w0 = 1.0; *w1 = 0.0;
    return tab[I->t_entries - 1];
  }
  double f = x - (double)k;
  *k0 = k; *w0 = 1.0 - f; *w1 = f;
  return tab[k] + (tab[k + 1] - tab[k]) * f;
}

/* Linear interpolation on n equidistant nodes at E = k / scale eV, clamped beyond the last
 * (the same rule as the transmission tables). */
static double node_interp(const double* tab, int n, double scale, uint32_t E) {
  const double x = ((double)E * 0x1p-30) * scale;
  const int k = (int)floor(x);
  if (k >= n - 1) return tab[n - 1];
  const double f = x - (double)k;
  return tab[k] + (tab[k + 1] - tab[k]) * f;
}

/* Speed of the carrier's channel in `layer` at energy E (Fig. 1(a)). */
static double speed(const orc_instance* I, int layer, int spin, uint32_t E) {
  const int c = I->ch_of[layer * 2 + spin];
  if (I->e_nodes > 0) return node_interp(I->v_node + (int64_t)c * I->e_nodes, I->e_nodes, I->e_scale, E);
  return I->v[c];
}

/* Energy dependence of the inelastic rate, 1/tau(E) = inv_tau0 * Ek (Fig. 1(b), Eq. 2). */
static double rate_shape(const orc_problem* P, const orc_instance* I, int c, uint32_t E) {
  if (I->e_nodes > 0) return node_interp(I->r_node + (int64_t)c * I->e_nodes, I->e_nodes, I->e_scale, E);
  const double E_ev = (double)E * 0x1p-30;
  return P->tau_exp == 2 ? E_ev * E_ev : 1.0;
}

/* Transport over half a step, Eq. (18): straight flight at v cos(theta); full reflection
 * at the vacuum surfaces; at an interface the carrier is transmitted with probability T
 * (one uniform draw per hit) or reflected.  A transmitted carrier keeps its direction and
 * covers the rest of the half step at the new layer's speed. */
static void half_step(worker* W, particle* p, int n, uint32_t tag) {
  const orc_problem* P = W->P;
  const orc_instance* I = W->I;
  const double h = 0.5 * P->dt;
  const int L = I->n_layers;
  uint32_t uid_lo = p->root, uid_hi = p->lin;
  double z_end = p->z + (speed(I, p->layer, p->spin, p->E) * p->mu) * h;
  int draws = 0, hits = 0;
  for (;;) {
    const int l = p->layer;
    const double lo = I->z_bound[l], hi = I->z_bound[l + 1];
    int dir;
    double b;
    if (z_end > hi) { dir = 0; b = hi; }
    else if (z_end < lo) { dir = 1; b = lo; }
    else break;
    if (++hits > MAX_HITS) { W->error = 2; break; }
    const int outer = dir == 0 ? (l == L - 1) : (l == 0);
    if (outer) {
      z_end = b - (z_end - b);
      p->mu = -p->mu;
      p->ev[2]++;
      count(W, n, ORC_C_REFL_SURF, 1);
      continue;
    }
    const int iface = dir == 0 ? l : l - 1;
    const int nl = dir == 0 ? l + 1 : l - 1;
    const int t = I->tt_of[(iface * 2 + dir) * 2 + p->spin];
    int k0;
    double w0, w1;
    const double T = transmission(I, t, p->E, &k0, &w0, &w1);
    uint32_t w[4];
    draw(P, uid_lo, uid_hi, (uint32_t)n, tag + (uint32_t)draws, w);
    draws++;
    const int base = I->n_channels + t * I->t_entries + k0;
    if (unif(w[0]) < T) {
      const double r = speed(I, nl, p->spin, p->E) / speed(I, l, p->spin, p->E);
      z_end = b + (z_end - b) * r;
      p->layer = nl;
      p->ev[1]++;
      count(W, n, ORC_C_TRANSMIT, 1);
      add_score(W, p, base, w0 / T);
      if (w1 != 0.0) add_score(W, p, base + 1, w1 / T);
    } else {
      z_end = b - (z_end - b);
      p->mu = -p->mu;
      p->ev[2]++;
      count(W, n, ORC_C_REFL_IF, 1);
      add_score(W, p, base, -w0 / (1.0 - T));
      if (w1 != 0.0) add_score(W, p, base + 1, -w1 / (1.0 - T));
    }
  }
  p->z = z_end;
}

/* Monte-Carlo scattering over the full step (Eq. 14, Sec. III.A).  Returns 1 if a
 * secondary was created (written to *child). */
static int scatter(worker* W, particle* p, int n, particle* child) {
  const orc_problem* P = W->P;
  const orc_instance* I = W->I;
  const int l = p->layer, c = I->ch_of[l * 2 + p->spin];
  uint32_t d[4], w[4];
  /* the event decision of step n: word n mod 2 of the pair counter (step field n - n mod 2) */
  draw(P, p->root, p->lin, (uint32_t)n & ~1u, TAG_DECIDE, d);
  /* Eq. (2): 1/tau_eff = 1/tau_el + 1/tau(E); 1/tau(E) = inv_tau0 * Ek with Ek = (E/1 eV)^
   * tau_exp, or the channel's rate table */
  const double Ek = rate_shape(P, I, c, p->E);
  const double rate = Ek * I->inv_tau0[c] + I->inv_tau_el[l];
  const double x = P->dt * rate;
  const double prob = -expm1(-x);
  const double x_in = P->dt * (Ek * I->inv_tau0[c]);
  if (!(unif(d[n & 1]) < prob)) {
    add_score(W, p, c, x_in);            /* d/d ln tau0 of log(1 - p) */
    return 0;
  }
  add_score(W, p, c, -x_in * exp(-x) / prob);
  /* the event's own words: 1 channel, 2 new direction, 3 energy split (word 0 unused) */
  draw(P, p->root, p->lin, (uint32_t)n, TAG_SCAT, w);
  p->ev[0]++;
  if (P->absorb_next && p->E < P->e_min_fx) {
    /* Sec. III.A: a carrier of the lowest energy bin leaves the hot population at its
     * next scattering event (quasi-thermalised) */
    p->dead = n;
    count(W, n, ORC_C_ABSORBED, 1);
    count(W, n, ORC_C_E_ABSORBED, (int64_t)p->E);
    return 0;
  }
  const int elastic = I->inv_tau_el[l] > 0.0 && unif(w[1]) < I->inv_tau_el[l] / rate;
  if (I->inv_tau_el[l] > 0.0) add_score(W, p, c, elastic ? x_in / x : -1.0 + x_in / x);
  /* random-k approximation: the outgoing direction is isotropic (Eq. 4) */
  p->mu = stored(P, cosine(w[2]));
  if (elastic) {                        /* Eq. (8): energy and spin kept */
    count(W, n, ORC_C_EV_EL, 1);
    return 0;
  }
  count(W, n, ORC_C_EV_EE, 1);
  /* Eq. (7): uniform final energy uE; the lifted carrier takes (1-u)E (energy conserved) */
  const uint32_t E = p->E;
  const uint32_t E1 = (uint32_t)(((uint64_t)w[3] * (uint64_t)E) >> 32);
  const uint32_t E2 = E - E1;
  p->E = E1;
  int made = 0;
  if (P->secondaries) {
    if (E2 >= P->e_min_fx || P->absorb_next) {
      uint32_t s[4];
      draw(P, p->root, p->lin, (uint32_t)n, TAG_SPAWN, s);
      *child = *p;
      child->E = E2;
      child->mu = stored(P, cosine(s[0]));
      /* Eq. (19): secondaries carry the equilibrium polarisation of the layer */
      child->spin = unif(s[1]) < 0.5 * (1.0 + I->P0[l]) ? 0 : 1;
      child->gen = p->gen < 255 ? p->gen + 1 : 255;
      uint32_t lin = s[2];
      if (lin == 0 || lin == p->lin) {
        lin = s[3] | 1u;
        if (lin == p->lin) lin ^= 2u;
      }
      child->lin = lin;
      memset(child->ev, 0, sizeof(child->ev));
      child->dead = -1;
      child->n_next = n;
      child->newborn = 1;
      child->S = NULL;
      p->ev[3]++;
      count(W, n, ORC_C_SPAWNED, 1);
      made = 1;
    } else {
      count(W, n, ORC_C_SEC_ABSORBED, 1);
      count(W, n, ORC_C_E_ABSORBED, (int64_t)E2);
    }
  }
  if (E1 < P->e_min_fx && !P->absorb_next) {
    p->dead = n;
    count(W, n, ORC_C_ABSORBED, 1);
    count(W, n, ORC_C_E_ABSORBED, (int64_t)E1);
  }
  return made;
}

static int energy_bin(const orc_problem* P, uint32_t E) {
  int b = 0;
  for (int k = 0; k < P->n_ebins; ++k)
    if (P->e_edges[k] <= E) b = k;
  return b;
}

/* Moments after the full step (Eqs. 16, 23): particle count per (depth, energy, spin)
 * and the sum of v cos(theta) per (depth, spin), in 2^-32 nm/fs fixed point.  Weighted
 * superparticles (Eq. 10) add their weight instead of 1: w 2^16 to the density and
 * rint(v cos(theta) w 2^32) to the current. */
static void deposit(worker* W, particle* p, int n) {
  const orc_problem* P = W->P;
  const orc_instance* I = W->I;
  int zb = (int)floor(p->z * I->inv_dz);
  if (zb < 0) zb = 0;
  if (zb > I->nz - 1) zb = I->nz - 1;
  double g = 0.0;
  if (n % P->dens_stride == 0) {
    const int eb = energy_bin(P, p->E);
    const int64_t idx = W->dens_off +
        (((int64_t)(n / P->dens_stride) * I->nz + zb) * P->n_ebins + eb) * 2 + p->spin;
    const uint64_t add = P->weighted ? (uint64_t)p->w : 1u;
#pragma omp atomic
    W->O->dens[idx] += add;
    if (W->K && W->O->g_dens)
      g += P->weighted ? W->O->g_dens[idx] * ((double)p->w * 0x1p-16) : W->O->g_dens[idx];
    if (W->O->gen) {
      /* mean generation map of Sec. V (Figs. 5, 7): the sum of the labels per cell, to be
       * divided by the cell's count */
      const int64_t gi = W->gen_off + ((int64_t)(n / P->dens_stride) * I->nz + zb) * 2 + p->spin;
#pragma omp atomic
      W->O->gen[gi] += (uint64_t)p->gen * add;
    }
  }
  if (n % P->cur_stride == 0) {
    const double vm = speed(I, p->layer, p->spin, p->E) * p->mu;
    const int64_t val =
        P->weighted ? llrint((vm * (double)p->w) * 65536.0) : llrint(vm * 4294967296.0);
    const int64_t idx = W->cur_off + ((int64_t)(n / P->cur_stride) * I->nz + zb) * 2 + p->spin;
#pragma omp atomic
    W->O->cur[idx] += val;
    if (W->K && W->O->g_cur) g += W->O->g_cur[idx] * ((double)val * 0x1p-32);
  }
  if (W->K && g != 0.0) {
    if (W->O->grad_per_tree) W->tree_return += g;
    else
      for (int k = 0; k < W->K; ++k) W->grad[k] += g * p->S[k];
  }
}

static void record(worker* W, const particle* p) {
  orc_output* O = W->O;
  if (!O->rec_uid) return;
  int64_t i;
#pragma omp atomic capture
  i = O->n_rec++;
  if (i >= O->rec_cap) { W->error = 3; return; }
  O->rec_uid[i] = (uint64_t)p->root | ((uint64_t)p->lin << 32);
  O->rec_z[i] = p->z;
  O->rec_mu[i] = p->mu;
  O->rec_E[i] = p->E;
  O->rec_layer[i] = p->layer;
  O->rec_spin[i] = p->spin;
  O->rec_gen[i] = p->gen;
  O->rec_dead[i] = p->dead;
  O->rec_inst[i] = W->inst_id;
  if (O->rec_w) O->rec_w[i] = p->w;
  for (int k = 0; k < 4; ++k) O->rec_ev[i * 4 + k] = p->ev[k];
}

static void run_particle(worker* W, particle* p) {
  const orc_problem* P = W->P;
  for (int n = p->n_next; n < P->n_steps; ++n) {
    const int only_second_half = p->newborn && n == p->n_next;
    if (!only_second_half) {
      half_step(W, p, n, TAG_HALF1);
      particle child;
      if (scatter(W, p, n, &child)) {
        if (W->K && !W->O->grad_per_tree) {
          child.S = (double*)malloc(sizeof(double) * (size_t)W->K);
          memcpy(child.S, p->S, sizeof(double) * (size_t)W->K);
        }
        if (push(W->stack, &child)) { W->error = 4; return; }
      }
      if (p->dead >= 0) {       /* an absorbed carrier keeps its mid-step state */
        p->z = stored(P, p->z);
        break;
      }
    }
    half_step(W, p, n, TAG_HALF2);
    p->z = stored(P, p->z);
    deposit(W, p, n);
    count(W, n, ORC_C_ALIVE, 1);
  }
  record(W, p);
}

/* Weight of a primary of spin s and initial energy E0 (Eq. 10), 2^-16 units. */
static uint32_t primary_weight(const orc_instance* I, int s, uint32_t E0) {
  if (I->w_nodes <= 0) return 1u << 16;
  const double w = node_interp(I->w_node + (int64_t)s * I->w_nodes, I->w_nodes, I->w_scale, E0);
  return (uint32_t)llrint(w * 65536.0);
}

/* Source term, Eq. (17): one primary per root, created at the start of its step with a
 * depth from the pump profile, an isotropic direction, a spin and an energy. */
static void run_root(worker* W, int64_t j, int n0) {
  const orc_problem* P = W->P;
  const orc_instance* I = W->I;
  const uint64_t root = I->root_offset + (uint64_t)j;
  uint32_t w[4];
  draw(P, (uint32_t)root, 0u, 0xFFFFFFFFu, TAG_INJECT, w);
  double z0;
  if (I->src_lambda > 0.0)   /* exp(-z/lambda) truncated to the excited layer */
    z0 = I->src_z_lo - I->src_lambda * log1p(-unif(w[0]) * I->src_cd);
  else                       /* homogeneous excitation */
    z0 = I->src_z_lo + unif(w[0]) * (I->src_z_hi - I->src_z_lo);
  particle p;
  memset(&p, 0, sizeof(p));
  p.z = stored(P, z0);
  p.mu = stored(P, cosine(w[1]));
  p.spin = unif(w[2]) < I->src_up_frac ? 0 : 1;
  p.E = I->src_e_lo[p.spin] + (uint32_t)(((uint64_t)w[3] * (uint64_t)I->src_e_span[p.spin]) >> 32);
  p.w = primary_weight(I, p.spin, p.E);
  p.layer = 0;
  for (int l = 0; l < I->n_layers; ++l)
    if (I->z_bound[l] <= p.z) p.layer = l;
  p.root = (uint32_t)root;
  p.lin = 0;
  p.gen = 1;
  p.dead = -1;
  p.n_next = n0;
  p.newborn = 0;
  if (W->K && !W->O->grad_per_tree) p.S = (double*)calloc((size_t)W->K, sizeof(double));
  count(W, n0, ORC_C_INJECTED, 1);
  count(W, n0, ORC_C_W_INJECTED, (int64_t)p.w);
  if (W->K && W->O->grad_per_tree) {
    memset(W->tree_score, 0, sizeof(double) * (size_t)W->K);
    W->tree_return = 0.0;
  }
  W->stack->n = 0;
  if (push(W->stack, &p)) { W->error = 4; return; }
  while (W->stack->n > 0) {
    particle q = W->stack->items[--W->stack->n];
    run_particle(W, &q);
    free(q.S);
  }
  if (W->K && W->O->grad_per_tree && W->tree_return != 0.0)
    for (int k = 0; k < W->K; ++k) W->grad[k] += W->tree_return * W->tree_score[k];
}

static int validate(const orc_problem* P) {
  if (P->n_instances < 1 || P->n_steps < 1 || !(P->dt > 0.0)) return 1;
  if (P->tau_exp != 0 && P->tau_exp != 2) return 1;
  if (P->n_ebins < 1 || P->dens_stride < 1 || P->cur_stride < 1) return 1;
  for (int i = 0; i < P->n_instances; ++i) {
    const orc_instance* I = &P->inst[i];
    if (I->n_layers < 1 || I->n_layers > MAX_LAYERS || I->nz < 1) return 1;
    for (int l = 0; l < I->n_layers; ++l)
      if (!(I->z_bound[l + 1] > I->z_bound[l])) return 1;
    int64_t tot = 0;
    for (int n = 0; n < P->n_steps; ++n) tot += I->sched[n];
    if (I->root_offset + (uint64_t)tot > 0xFFFFFFFFull) return 1;
    if (P->inst[0].n_channels != I->n_channels || P->inst[0].n_ttables != I->n_ttables ||
        P->inst[0].t_entries != I->t_entries) return 1;
    if (I->w_nodes < 0 || I->w_nodes > 64) return 1;
    if (I->w_nodes > 0 && !(I->w_scale >= 0.0 && I->w_scale <= 1e8)) return 1;
    for (int k = 0; k < 2 * I->w_nodes; ++k)
      if (!(I->w_node[k] >= 0x1p-16 && I->w_node[k] <= 0x1p15)) return 1;
  }
  return 0;
}

int orc_run(const orc_problem* P, orc_output* O) {
  if (validate(P)) return 1;
  const int NI = P->n_instances;
  int64_t* dens_off = (int64_t*)calloc((size_t)NI, sizeof(int64_t));
  int64_t* cur_off = (int64_t*)calloc((size_t)NI, sizeof(int64_t));
  int64_t* gen_off = (int64_t*)calloc((size_t)NI, sizeof(int64_t));
  int64_t* job_start = (int64_t*)calloc((size_t)NI + 1, sizeof(int64_t));
  const int nds = (P->n_steps + P->dens_stride - 1) / P->dens_stride;
  const int ncs = (P->n_steps + P->cur_stride - 1) / P->cur_stride;
  int64_t d = 0, c = 0, gsum = 0;
  for (int i = 0; i < NI; ++i) {
    const orc_instance* I = &P->inst[i];
    dens_off[i] = d;
    cur_off[i] = c;
    gen_off[i] = gsum;
    d += (int64_t)nds * I->nz * P->n_ebins * 2;
    c += (int64_t)ncs * I->nz * 2;
    gsum += (int64_t)nds * I->nz * 2;
    int64_t tot = 0;
    for (int n = 0; n < P->n_steps; ++n) tot += I->sched[n];
    int64_t lo = P->root_lo > 0 ? P->root_lo : 0;
    int64_t hi = P->root_hi >= 0 && P->root_hi < tot ? P->root_hi : tot;
    job_start[i + 1] = job_start[i] + (hi > lo ? hi - lo : 0);
  }
  const int K = O->grad ? P->inst[0].n_channels + P->inst[0].n_ttables * P->inst[0].t_entries : 0;
  if (O->grad) memset(O->grad, 0, sizeof(double) * (size_t)K);
  O->n_rec = 0;
  int error = 0;
  const int64_t n_jobs = job_start[NI];
  if (P->n_threads > 0) {
#ifdef _OPENMP
    omp_set_num_threads(P->n_threads);
#endif
  }
#pragma omp parallel
  {
    pstack stack = {0};
    worker W;
    memset(&W, 0, sizeof(W));
    W.P = P;
    W.O = O;
    W.K = K;
    W.stack = &stack;
    if (K) {
      W.grad = (double*)calloc((size_t)K, sizeof(double));
      W.tree_score = (double*)calloc((size_t)K, sizeof(double));
    }
    int inst_cached = -1;
    int64_t* cum = NULL;
#pragma omp for schedule(dynamic, 64)
    for (int64_t job = 0; job < n_jobs; ++job) {
      int i = 0;
      while (job_start[i + 1] <= job) ++i;
      const orc_instance* I = &P->inst[i];
      if (i != inst_cached) {
        free(cum);
        cum = (int64_t*)malloc(sizeof(int64_t) * ((size_t)P->n_steps + 1));
        cum[0] = 0;
        for (int n = 0; n < P->n_steps; ++n) cum[n + 1] = cum[n] + I->sched[n];
        inst_cached = i;
        W.inst_id = i;
        W.I = I;
        W.dens_off = dens_off[i];
        W.cur_off = cur_off[i];
        W.gen_off = gen_off[i];
      }
      const int64_t lo = P->root_lo > 0 ? P->root_lo : 0;
      const int64_t j = lo + (job - job_start[i]);
      int n0 = 0;
      while (cum[n0 + 1] <= j) ++n0;
      run_root(&W, j, n0);
    }
    free(cum);
    if (K) {
#pragma omp critical
      for (int k = 0; k < K; ++k) O->grad[k] += W.grad[k];
      free(W.grad);
      free(W.tree_score);
    }
    if (W.error) {
#pragma omp critical
      error = W.error;
    }
    free(stack.items);
  }
  free(dens_off);
  free(cur_off);
  free(gen_off);
  free(job_start);
  return error;
}
