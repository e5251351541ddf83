"""Shared certification and reporting for the GPU-against-oracle parity tests
(not a test module).

A row is certified when nudging every parameter by 1, 4, 16, 64 and 256 ulps
either way leaves the oracle's cost and tier unchanged: its outcome does not
hang on rounding.  Where the goal predicate psi_g decides the tier (every action
succeeded), the row's tier is certified only when the oracle's final object
position also lies farther from the boundary of the goal region than 0.8 of
the object's smallest half extent: an object whose centre is nearer than its
own half size can be resting across the boundary - a block that comes to rest
straddling a thin container wall (the vertex-face contact model lets a 0.1 m
block settle across a 2 cm wall) has its inside / outside decided by the
rounding of a chaotic landing, which parameter nudges do not probe.  Likewise
psi_g's rest condition must be decided: the object at rest for the last
REST_STEPS control steps (the early stop's settling window), or moving at
least twice the rest speed at T; an object that slides to a stop just before
T reaches rest at a step the FP32 rounding of the slide decides.  On certified rows the GPU's tier must equal the oracle's;
every disagreement is printed with its row, both tiers and both costs,
together with how many rows the certification kept."""
import numpy as np

GOAL_MARGIN = 0.8    # of the object's smallest half extent
REST_STEPS = 100     # control steps at rest before T


def goal_margin(w, pos):
    """Distance of each final object position (n x 3) from the boundary of the
    scene's goal region (inside or outside): the goal table's top-face slab
    (pick-and-place), or the goal box (move-and-push)."""
    sc = w["scene"]
    pos = np.asarray(pos, np.float64)[:, :3]
    if sc.get("goal_static", -1) >= 0:
        b = sc["static_boxes"][sc["goal_static"]]
        c, h = np.array(b["center"], np.float64), np.array(b["half"], np.float64)
        top = c[2] + h[2]
        lo = np.array([c[0] - h[0], c[1] - h[1], top])
        hi = np.array([c[0] + h[0], c[1] + h[1], top + 2.0 * sc["object"]["half"][2]])
    else:
        gb = sc["goal_box"]
        c, h = np.array(gb["center"], np.float64), np.array(gb["half"], np.float64)
        lo, hi = c - h, c + h
    inside = np.all((pos >= lo) & (pos <= hi), axis=1)
    depth = np.min(np.minimum(pos - lo, hi - pos), axis=1)                         # inside: to the nearest face
    gap = np.linalg.norm(np.maximum(np.maximum(lo - pos, pos - hi), 0.0), axis=1)  # outside: to the region
    return np.where(inside, depth, gap)


def goal_decided(w, tier_ref, pose_ref, speed_ref, rest_ref):
    """Rows whose tier does not hang on where or when the object came to rest:
    an action failed (tier 2, 3); or the final position is farther than
    GOAL_MARGIN of the object's smallest half extent from the goal region's
    boundary and the object was at rest for the last REST_STEPS control steps
    or still moved at twice the rest speed (oracle's speed_ref, rest_ref:
    final speed, consecutive final steps at rest)."""
    sc = w["scene"]
    m = GOAL_MARGIN * min(sc["object"]["half"])
    rest_ok = (np.asarray(rest_ref) >= REST_STEPS) | (np.asarray(speed_ref) >= 2.0 * sc["rest_speed"])
    return (np.asarray(tier_ref) >= 2) | ((goal_margin(w, pose_ref) > m) & rest_ok)


WIDE = (16, 64, 256)  # ulps: the further nudges every row must withstand


def nudged(Z, ulps, sign):
    """Every parameter moved by `ulps` FP32 ulps toward +inf (sign 1) or -inf (-1)."""
    for _ in range(ulps):
        Z = np.nextafter(Z, np.float32(sign * np.inf)).astype(np.float32)
    return Z


def certify(oracle, w, seed, Z, inst=0):
    """The oracle's outcome of rows Z and which rows are certified.

    A row is certified when nudging every parameter by 1, 4, 16, 64 and 256
    FP32 ulps either way leaves the oracle's tier and cost unchanged.  The FP32
    rollout's rounding perturbs the state throughout the horizon, not once at
    the start, so an outcome that moves under nudges of the inputs this small
    (an action decided on the step a threshold is crossed, a grasp that barely
    closes, an object knocked over or landing) is not decided by the method at
    FP32 precision, and two FP32 evaluations of it that round differently may
    both be right.  Where psi_g decides the tier, goal_decided is required too.
    Returns dict(cost, tier, pose, steps, spread (the final object position's
    largest move under the 1- and 4-ulp nudges), ok (cost and tier), okt (tier))."""
    c0, t0, p0, _, s0, sp0, rs0 = oracle.rollout(w, seed, Z, inst=inst, with_steps=True, with_rest=True)
    tol = 1e-6 if w["scene"]["kind"] == "push" else 1e-9
    ok = np.ones(len(Z), bool)
    spread = np.zeros(len(Z))
    for ulps in (1, 4):
        for sign in (1, -1):
            c, t, p, _ = oracle.rollout(w, seed, nudged(Z, ulps, sign), inst=inst)
            ok &= (t == t0) & (np.abs(c - c0) < tol)
            spread = np.maximum(spread, np.max(np.abs(p[:, :3] - p0[:, :3]), axis=1))
    wide = np.nonzero(ok)[0]
    if wide.size:
        for ulps in WIDE:
            for sign in (1, -1):
                c, t, _, _ = oracle.rollout(w, seed, nudged(Z[wide], ulps, sign), inst=inst)
                ok[wide] &= (t == t0[wide]) & (np.abs(c - c0[wide]) < tol)
    okt = ok & goal_decided(w, t0, p0, sp0, rs0) if w["scene"]["kind"] != "push" else ok.copy()
    return dict(cost=c0, tier=t0, pose=p0, steps=s0, spread=spread, ok=ok, okt=okt)


def tier_mismatches(tag, ok, tier_gpu, tier_ref, cost_gpu, cost_ref, rows=None):
    """Print the certification count and every certified row whose tiers differ; return those rows."""
    ok = np.asarray(ok, bool)
    rows = np.arange(len(ok)) if rows is None else np.asarray(rows)
    bad = np.nonzero(ok & (np.asarray(tier_gpu) != np.asarray(tier_ref)))[0]
    print("%s: %d of %d rows certified (%d dropped); %d tier mismatches on certified rows"
          % (tag, ok.sum(), len(ok), len(ok) - ok.sum(), len(bad)))
    out = []
    for i in bad:
        print("  row %d: gpu tier %d cost %.4f, oracle tier %d cost %.4f"
              % (rows[i], tier_gpu[i], cost_gpu[i], tier_ref[i], cost_ref[i]))
        out.append(int(rows[i]))
    return out


def median_agreement(tag, gpu, ref, rel=1e-2):
    """Paired seeds of Alg. 1 (the GPU's best cost and the oracle's, same seed):
    at least half of the seeds agree within `rel`, and the medians agree within
    `rel` or two standard errors of the median, whichever is larger.

    The FP32 and FP64 runs share iteration 0's samples, so most seeds end at
    the same plan; a seed whose elites part ways ends wherever CE takes it.
    At small populations the seeds' best costs spread so widely that the
    sampling error of a 32-seed median (1.2533 sd / sqrt(n), from the
    oracle's spread) exceeds 1 % of the median, and a 1 % bound on the medians
    alone would fail by chance; the paired count has no such noise."""
    g, r = np.asarray(gpu, np.float64), np.asarray(ref, np.float64)
    relgap = np.abs(g - r) / np.abs(r)
    se = 1.2533 * np.std(r) / np.sqrt(len(r))
    mg, mr = np.median(g), np.median(r)
    print("%s: median best cost GPU %.4f oracle %.4f (standard error of the median %.4f); seeds within %.0e: %d of %d"
          % (tag, mg, mr, se, rel, int(np.sum(relgap <= rel)), len(r)))
    assert np.median(relgap) <= rel
    assert abs(mg - mr) <= max(rel * abs(mr), 2.0 * se)
