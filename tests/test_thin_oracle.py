"""Pins of the candidate-thinning variant of the oracle (occl_ref_detect_ex
flag 2), on the CPU.  The variant follows the future work named in the
paper's summary (Sec. 6, a thinner candidate list): a candidate whose
scanline pixel at g = -1 is a candidate is not scanned, every other candidate
scans g = -h .. h + m over the run of m <= h candidates that follows it."""
import json
import os

import numpy as np
import pytest

from tests.test_oracle_pins import _layered_integer_scene, _small_c1, zbuffer_occlusion

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thin_hand.json")


def _cases():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_thin_hand_worked(ref, case):
    """Hand-derived masks of both the method and the variant on one-row
    frames: one where the merged window gains a hit and one where the capped
    run loses one (catches a missing extension, an uncapped run and followers
    that are still scanned)."""
    D = np.float32(case["D"])[None, :]
    M, _, nc = ref.detect(D, [0], [1.0], [case["L"]])
    Mt, _, nt = ref.detect(D, [0], [1.0], [case["L"]], thin=True)
    assert np.nonzero(M[0, 0])[0].tolist() == case["exact"]
    assert np.nonzero(Mt[0, 0])[0].tolist() == case["thin"]
    # thinning changes which candidates are scanned, not Eq. (2)'s candidates
    assert nc[0] == nt[0] == len(case["candidates"])


def _candidates(D, alpha):
    """Eq. (1)-(2) on an axis direction (written out for the test's precondition)."""
    ex = np.zeros_like(D)
    ey = np.zeros_like(D)
    ex[:, :-1] = D[:, 1:] - D[:, :-1]
    ey[:-1, :] = D[1:, :] - D[:-1, :]
    c, s = {0: (1, 0), 90: (0, 1), 180: (-1, 0), 270: (0, -1)}[alpha]
    E = np.sqrt(ex * ex + ey * ey)
    return (E > 1.0) & (ex * c + ey * s > 0), (c, s)


@pytest.mark.parametrize("seed", range(6))
def test_thin_equals_method_without_collinear_candidates(ref, seed):
    """With no two candidates next to each other along the scanline there is
    no follower and no run, so the variant is the method itself."""
    rng = np.random.default_rng(seed)
    H, W, L = 96, 128, 24
    D = np.full((H, W), np.float32(rng.uniform(0.5, 3)), np.float32)
    for (ya, xa) in ((L + 2, L + 2), (H // 2 + 8, W // 2 + 8)):
        h, w = int(rng.integers(8, 24)), int(rng.integers(8, 24))
        D[ya:ya + h, xa:xa + w] = np.float32(D[0, 0] + rng.uniform(1.5, 8.0))
    for alpha in (0, 90, 180, 270):
        cand, (c, s) = _candidates(D, alpha)
        ys, xs = np.nonzero(cand)
        nb = (ys - s >= 0) & (ys - s < H) & (xs - c >= 0) & (xs - c < W)
        assert not cand[(ys - s)[nb], (xs - c)[nb]].any()  # precondition: no follower
        M, _, _ = ref.detect(D, [alpha], [1.0], [L])
        Mt, _, _ = ref.detect(D, [alpha], [1.0], [L], thin=True)
        np.testing.assert_array_equal(Mt[0], M[0], err_msg=f"alpha={alpha}")


def _stair_scene(rng, H, W, n):
    """Integer fronto-parallel layers stepped up one pixel at a time on one
    side, so neighbouring pixels along the axes are both candidates."""
    D = np.full((H, W), float(rng.integers(0, 3) * 2), np.float32)
    for _ in range(n):
        base = float(D.max())
        h, w = int(rng.integers(3, H // 2)), int(rng.integers(4, W // 2))
        y0, x0 = int(rng.integers(0, H - h)), int(rng.integers(0, W - w))
        side = int(rng.integers(0, 4))
        for j in range(int(rng.integers(2, 4))):
            ya, yb, xa, xb = y0, y0 + h, x0, x0 + w
            if side == 0:
                xa += j
            elif side == 1:
                xb -= j
            elif side == 2:
                ya += j
            else:
                yb -= j
            D[ya:yb, xa:xb] = base + 2 * (j + 1)
    return D


@pytest.mark.parametrize("seed", range(12))
def test_thin_equals_zbuffer_on_equality_class(ref, seed):
    """Integer fronto-parallel scenes with a reach covering every strip: on
    axis directions a head's merged window is the union of its followers'
    windows, and the variant's mask is the brute-force z-buffer's, like the
    method's.  Half the scenes are staircases, so followers occur."""
    rng = np.random.default_rng(900 + seed)
    H, W = int(rng.integers(10, 40)), int(rng.integers(10, 48))
    D = (_stair_scene(rng, H, W, int(rng.integers(1, 4))) if seed % 2 == 0
         else _layered_integer_scene(rng, H, W, int(rng.integers(1, 6))))
    L = int(2 * (D.max() - D.min()) + 4)
    followers = 0
    for alpha in (0, 90, 180, 270):
        cand, (c, s) = _candidates(D, alpha)
        ys, xs = np.nonzero(cand)
        nb = (ys - s >= 0) & (ys - s < H) & (xs - c >= 0) & (xs - c < W)
        followers += int(cand[(ys - s)[nb], (xs - c)[nb]].sum())
        Mt, _, _ = ref.detect(D, [alpha], [1.0], [L], thin=True)
        np.testing.assert_array_equal(Mt[0], zbuffer_occlusion(D, alpha, 0.5), err_msg=f"alpha={alpha}")
    if seed % 2 == 0:
        assert followers > 0


@pytest.mark.parametrize("seed", range(4))
def test_thin_transpose_symmetry(ref, seed):
    """M(D^T, 90 - alpha) = M(D, alpha)^T holds for the variant too: the
    follower and run tests read scanline pixels, which transpose exactly
    with the direction."""
    D = _small_c1(seed)
    angles = [0, 45, 90, 135, 180, 225, 270, 315, 26.56505117707799, 10, 77]
    ratios = np.float32([1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 1, 1.4142135, 2.236068, 1.7, 0.8])
    L = [20, 28, 20, 28, 20, 28, 20, 28, 40, 30, 16]
    M, _, _ = ref.detect(D, angles, ratios, L, thin=True)
    Mt, _, _ = ref.detect(np.ascontiguousarray(D.T), [90.0 - a for a in angles], ratios, L, thin=True)
    for v in range(len(angles)):
        np.testing.assert_array_equal(Mt[v], M[v].T, err_msg=f"view {v}")


def test_thin_rejects_tight_map(ref):
    D = np.zeros((4, 4), np.float32)
    with pytest.raises(ValueError):
        ref.detect(D, [0], [1.0], [5], want_tight=True, thin=True)
