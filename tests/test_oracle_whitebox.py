"""White-box pins of the CPU oracle with scripted random words.

The oracle can replace the Philox words of listed counters by given ones.  Each test
below forces a short history -- which events happen, which way an interface decision
goes -- and compares the oracle's final state with positions, directions and energies
worked out by hand from the transport rule (Eq. 18), the Strang order of Eq. (15), the
inelastic split (Eq. 7), the secondary's spin (Eq. 19) and the interface rule of
Sec. III.A.  The maps from a 32-bit word w to a uniform u = (w + 1/2) 2^-32 and to a
direction cosine mu = (w + 1/2) 2^-31 - 1 are the random-number format of both
implementations; every other number is derived in the comments.  All values used are
exact in binary64, so the comparisons are exact.
"""
import numpy as np

import workloads as W

INF = float("inf")
TAG_SCAT, TAG_SPAWN, TAG_HALF1, TAG_HALF2, TAG_INJECT, TAG_DECIDE = (
    0x000, 0x100, 0x200, 0x300, 0x400, 0x500)
NEVER = 0xFFFFFFFF            # u = 1 - 2^-33: no event, reflect at any T < 1
ALWAYS = 0                    # u = 2^-33: event, transmit at any T > 2^-33


def mu_of(w):
    return (w + 0.5) * 2.0 ** -31 - 1.0


def row(ctr, words):
    return list(ctr) + list(words)


def _by_uid(rec):
    return {int(u): i for i, u in enumerate(rec["uid"])}


def test_scripted_split_absorption_and_newborn_half_step(oracle_lib):
    """One primary in a 100 nm Au slab (v = 1 nm/fs, dt = 1 fs, h = 1/2), constant
    tau0 = 40 fs, E_min = 0.1 eV, injected at z0 = 50 nm, mu0 = 1/2 + 2^-32, spin down
    (injection word 2 ~ 1 against the pump's spin-up fraction 1/2), E0 = 1.5 eV.

    The event decisions of steps 0 and 1 are the words 0 and 1 of one counter (step
    field 0, tag 0x500), that of step 2 word 0 of the counter with step field 2; an
    event's own words (channel, direction, split) are words 1-3 of its step's counter
    with tag 0.
    Step 0: half step to z_mid = 50.25 + 2^-33; forced inelastic event (decision word 0);
      new direction from word 2 = 2^30: mu1 = -1/2 + 2^-32; kept energy from word 3 = 2^31:
      E1 = E0/2 (Eq. 7, uniform fraction 1/2), the secondary gets E0/2 (>= E_min).  The
      spawn words give the secondary mu_c = 3/4 + 2^-32 (word 0 = 0xE0000000), spin up
      (word 1 = 0 against (1 + P0)/2 = 1/2 in Au, Eq. 19) and lineage 0x1234 (word 2).
      Second half steps from z_mid: parent 50 + 2^-32, secondary 50.625 + 2^-32.
    Step 1: parent to z_mid = 49.75 + 3 2^-33; forced event, mu = 1 - 2^-32 (word 2 =
      0xFFFFFFFF), kept fraction 1/16 (word 3 = 2^28): E = E0/32 = 0.046875 eV < E_min, so
      the parent is removed with its mid-step state; its secondary (E0/2 - E0/32 =
      0.703125 eV) gets mu = -1 + 2^-32 (word 0 = 0), spin down (word 1 ~ 1), lineage
      0x5678 and half a step: 49.25 + 2^-31.  The first secondary flies on, no event:
      51.375 + 2^-31.
    Step 2: no events; the secondaries fly a whole step: 52.125 + 3 2^-32 and
      48.25 + 3 2^-32."""
    E0 = W.e_fx(1.5)
    prob = W.homogeneous(thickness=100.0, n_primaries=1, n_steps=3, tau0=40.0, tau_exp=0,
                         dt=1.0, src=(50.0, 50.0), e0_ev=1.5, e_min_ev=0.1, up_frac=0.5,
                         state_fp64=True)
    c1, c2 = 0x1234, 0x5678
    script = [
        row((0, 0, NEVER, TAG_INJECT), (0, 0xC0000000, NEVER, 0)),
        row((0, 0, 0, TAG_DECIDE), (ALWAYS, ALWAYS, 0, 0)),
        row((0, 0, 0, TAG_SCAT), (0, 0, 0x40000000, 0x80000000)),
        row((0, 0, 0, TAG_SPAWN), (0xE0000000, 0, c1, 0)),
        row((0, 0, 1, TAG_SCAT), (0, 0, 0xFFFFFFFF, 0x10000000)),
        row((0, 0, 1, TAG_SPAWN), (0, NEVER, c2, 0)),
        row((0, c1, 0, TAG_DECIDE), (0, NEVER, 0, 0)),
        row((0, c1, 2, TAG_DECIDE), (NEVER, 0, 0, 0)),
        row((0, c2, 2, TAG_DECIDE), (NEVER, 0, 0, 0)),
    ]
    res = oracle_lib.run(prob, records=True, script=script)
    rec = res.records
    ix = _by_uid(rec)
    p, a, b = ix[0], ix[c1 << 32], ix[c2 << 32]
    assert len(rec["uid"]) == 3
    # the parent: removed at step 1 with its mid-step state
    assert rec["dead"][p] == 1
    assert rec["z"][p] == 49.75 + 3 * 2.0 ** -33
    assert rec["mu"][p] == 1.0 - 2.0 ** -32 == mu_of(0xFFFFFFFF)
    assert rec["E"][p] == E0 // 32
    assert (rec["spin"][p], rec["gen"][p]) == (1, 1)
    assert list(rec["ev"][p]) == [2, 0, 0, 2]
    # the first secondary
    assert rec["dead"][a] == -1
    assert rec["z"][a] == 52.125 + 3 * 2.0 ** -32
    assert rec["mu"][a] == 0.75 + 2.0 ** -32 == mu_of(0xE0000000)
    assert rec["E"][a] == E0 // 2
    assert (rec["spin"][a], rec["gen"][a]) == (0, 2)
    # the second secondary
    assert rec["dead"][b] == -1
    assert rec["z"][b] == 48.25 + 3 * 2.0 ** -32
    assert rec["mu"][b] == -1.0 + 2.0 ** -32
    assert rec["E"][b] == E0 // 2 - E0 // 32
    assert (rec["spin"][b], rec["gen"][b]) == (1, 2)
    # counters per step
    names = oracle_lib.COUNTER_NAMES
    col = lambda k: list(res.counters[:, names.index(k)])
    assert col("injected") == [1, 0, 0]
    assert col("ev_ee") == [1, 1, 0] and col("spawned") == [1, 1, 0]
    assert col("absorbed") == [0, 1, 0] and col("e_absorbed") == [0, E0 // 32, 0]
    assert col("alive") == [2, 2, 2]
    # moments after step 0: both carriers in depth bin 50, parent down, secondary up;
    # current rint(v mu 2^32): parent -2^31 + 1, secondary 3 2^30 + 1
    d0 = res.dens[0][0]
    assert d0[50, 0, 0] == 1 and d0[50, 0, 1] == 1 and d0.sum() == 2
    c0 = res.cur[0][0]
    assert c0[50, 1] == -(2 ** 31) + 1 and c0[50, 0] == 3 * 2 ** 30 + 1
    assert np.count_nonzero(c0) == 2


def test_scripted_interface_decisions(oracle_lib):
    """Fe(15)/Au(100) with v = 1/2 nm/fs for the Fe majority channel and 1 nm/fs in Au,
    tau -> infinity, dt = 1 fs, distinct transmissions per table: Fe->Au 0.8 (majority),
    Au->Fe 0.7 (majority).  Three spin-up carriers (one instance each):

    A: z0 = 14.75, mu = 1/2 + 2^-32.  First half step ends at 14.875 + 2^-34 (inside Fe,
       no draw).  Second half step would end at 15 + 2^-33: a +z hit of the interface,
       decided by the first draw of the second half step (tag 0x300) against the Fe->Au
       majority table: u just below 0.8 transmits; the rest of the flight, 2^-33, is
       rescaled by v_Au/v_Fe = 2: z = 15 + 2^-32, layer Au, direction kept.
    B: z0 = 15.125 (in Au), mu = -1/2 + 2^-32.  First half step ends at 14.875 + 2^-33: a
       -z hit decided by the first draw of the first half step (tag 0x200) against the
       Au->Fe majority table 0.7: u just above 0.7 reflects: z = 15.125 - 2^-33, mu =
       1/2 - 2^-32; the second half step ends at 15.375 - 2^-32 in Au.
    C: z0 = 0.125 (in Fe), mu = -1/2 + 2^-32.  The second half step would end at
       -0.125 + 2^-33: the vacuum surface reflects it to 0.125 - 2^-33 with mu = 1/2 - 2^-32,
       using no draw (a scripted draw for it would be ignored)."""
    v = (0.5, 0.25, 1.0, 1.0)
    T = (0.8, 0.4, 0.7, 0.3)
    insts = []
    for z0 in (14.75, 15.125, 0.125):
        it = W.make_instance(W.bilayer(15.0, 100.0), n_primaries=1, n_steps=1, v=v,
                             T_values=T, tau0=(INF,) * 4, src_lambda=0.0)
        it.src_z_lo = it.src_z_hi = z0
        insts.append(it)
    insts = W.with_root_offsets(insts)
    prob = W.Problem(insts, seed=0, dt=1.0, n_steps=1, state_fp64=True)
    below_08 = 3435973836           # u(w) < 0.8 < u(w + 1): the last word that transmits
    above_07 = 3006477107           # u(w - 1) < 0.7 < u(w): the first word that reflects
    assert (below_08 + 0.5) / 2 ** 32 < 0.8 < (below_08 + 1.5) / 2 ** 32
    assert (above_07 - 0.5) / 2 ** 32 < 0.7 < (above_07 + 0.5) / 2 ** 32
    up, down = 0xC0000000, 0x40000000
    script = [
        row((0, 0, NEVER, TAG_INJECT), (0, up, 0, 0)),
        row((1, 0, NEVER, TAG_INJECT), (0, down, 0, 0)),
        row((2, 0, NEVER, TAG_INJECT), (0, down, 0, 0)),
        row((0, 0, 0, TAG_HALF2), (below_08, 0, 0, 0)),
        row((1, 0, 0, TAG_HALF1), (above_07, 0, 0, 0)),
        row((2, 0, 0, TAG_HALF2), (ALWAYS, 0, 0, 0)),
    ]
    res = oracle_lib.run(prob, records=True, script=script)
    rec = res.records
    ix = _by_uid(rec)
    a, b, c = ix[0], ix[1], ix[2]
    assert (rec["z"][a], rec["layer"][a], rec["mu"][a]) == (15.0 + 2.0 ** -32, 1, 0.5 + 2.0 ** -32)
    assert (rec["z"][b], rec["layer"][b], rec["mu"][b]) == (15.375 - 2.0 ** -32, 1, 0.5 - 2.0 ** -32)
    assert (rec["z"][c], rec["layer"][c], rec["mu"][c]) == (0.125 - 2.0 ** -33, 0, 0.5 - 2.0 ** -32)
    assert list(rec["ev"][a]) == [0, 1, 0, 0]
    assert list(rec["ev"][b]) == [0, 0, 1, 0]
    assert list(rec["ev"][c]) == [0, 0, 1, 0]
    names = oracle_lib.COUNTER_NAMES
    assert res.counters[0, names.index("transmit")] == 1
    assert res.counters[0, names.index("refl_if")] == 1
    assert res.counters[0, names.index("refl_surf")] == 1
    # the same decisions flipped by one unit of the word: A reflects, B transmits
    script[3] = row((0, 0, 0, TAG_HALF2), (below_08 + 1, 0, 0, 0))
    script[4] = row((1, 0, 0, TAG_HALF1), (above_07 - 1, 0, 0, 0))
    rec = oracle_lib.run(prob, records=True, script=script).records
    ix = _by_uid(rec)
    a, b = ix[0], ix[1]
    # A: mirrored about 15 from 15 + 2^-33, then the step is over
    assert (rec["z"][a], rec["layer"][a], rec["mu"][a]) == (15.0 - 2.0 ** -33, 0, -0.5 - 2.0 ** -32)
    # B: 2^-33 - 1/8 past the interface, rescaled by v_Fe/v_Au = 1/2: 14.9375 + 2^-34,
    # then the second half step in Fe at 1/2 nm/fs: 14.8125 + 2^-33
    assert (rec["z"][b], rec["layer"][b], rec["mu"][b]) == (14.8125 + 2.0 ** -33, 0, -0.5 + 2.0 ** -32)


def test_scripted_transmission_tie_reflects(oracle_lib):
    """A draw exactly equal to T does not transmit (the decision is u < T): with
    T = 1/2 + 2^-33 = u(2^31), carrier A of the previous test reflects on the word 2^31 and
    transmits on 2^31 - 1."""
    t = 0.5 + 2.0 ** -33
    assert (2 ** 31 + 0.5) / 2 ** 32 == t
    it = W.make_instance(W.bilayer(15.0, 100.0), n_primaries=1, n_steps=1,
                         v=(0.5, 0.25, 1.0, 1.0), T_values=(t, t, t, t), tau0=(INF,) * 4,
                         src_lambda=0.0)
    it.src_z_lo = it.src_z_hi = 14.75
    prob = W.Problem([it], seed=0, dt=1.0, n_steps=1, state_fp64=True)
    inject = row((0, 0, NEVER, TAG_INJECT), (0, 0xC0000000, 0, 0))
    for word, layer, z in ((2 ** 31, 0, 15.0 - 2.0 ** -33), (2 ** 31 - 1, 1, 15.0 + 2.0 ** -32)):
        rec = oracle_lib.run(prob, records=True,
                             script=[inject, row((0, 0, 0, TAG_HALF2), (word, 0, 0, 0))]).records
        assert (rec["layer"][0], rec["z"][0]) == (layer, z)
