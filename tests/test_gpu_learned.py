"""The trained proposal network (paper_2310_10023_amd/proposal_weights.npz) on
the held-out benchmark city (seed 1000; the network saw cities 0-49 only).

  * What the network gains over no network: the true yaw bin of a fresh scan
    is among its four best yaw bins far more often than chance (4 of 64).
  * Learned-order localization (prior-ordered initial set plus seed beam, the
    prior coming from the network on the device) equals the oracle run with
    the same logits and beam width, bit for bit, on full-size city queries.
Node savings against the plain search are measured by bench.py, not asserted
here (on held-out maps the translation head is weak; see the design notes)."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2310_10023_amd as bbs
from paper_2310_10023_amd import proposal
import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(bbs.__file__), "proposal_weights.npz")
RESULT_KEYS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
               "initial_size", "initial_kept", "seeded", "seed_score")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def city_net():
    c = synth.city_scene(1000)
    say("city map points", len(c.points))
    net = proposal.Net(max_batch=16, params=np.load(WEIGHTS)["params"])
    return c, bbs.Map(c.points, 1.0, 6), net, oracle.Map(c.points, 1.0, 6)


def scan(c, seed):
    return synth.scan_scene(c, seed, 10000, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.5)


def test_trained_yaw_head_beats_chance_on_held_out_city(city_net):
    say("held-out yaw accuracy")
    c, _, net, _ = city_net
    scans = [scan(c, 100 + s) for s in range(16)]
    logits = net.forward(np.stack([proposal.bev_image(s.points) for s in scans]))
    hits = sum(proposal.yaw_bin(s.pose[5]) in np.argsort(-lg[:64])[:4] for s, lg in zip(scans, logits))
    say("top-4 yaw hits", hits, "of", len(scans))
    assert hits >= 8          # chance: 16 * 4 / 64 = 1


@pytest.mark.parametrize("seed", [0, 14])
def test_learned_order_localization_equals_oracle(city_net, seed):
    say("learned localize seed", seed)
    c, g, net, o = city_net
    sc = scan(c, seed)
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(10000)
    prior = net.forward(proposal.bev_image(sc.points)[None])[0]
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=10000, prior=prior, seed_beam=16)
    assert got["prior_used"] == 1 and got["seed_beam_used"] == 16
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=10000, threads=16, prior=prior, seed_beam=16)
    for k in RESULT_KEYS:
        assert got[k] == want[k], (k, got[k], want[k])


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_prior_falls_back_to_plain(city_net, bad):
    """A prior with a non-finite logit is not used: the search runs plain
    (no prior ordering, no seed beam) and gives the plain result."""
    say("non-finite prior", bad)
    c, g, net, _ = city_net
    sc = scan(c, 0)
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(10000)
    prior = net.forward(proposal.bev_image(sc.points)[None])[0].astype(np.float32).copy()
    prior[70] = bad
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=10000, prior=prior, seed_beam=16)
    plain = bbs.localize(g, sc.points, lo, hi, T, batch_size=10000)
    assert got["prior_used"] == 0 and got["seed_beam_used"] == 0 and got["seeded"] == 0
    for k in RESULT_KEYS:
        assert got[k] == plain[k], (k, got[k], plain[k])
