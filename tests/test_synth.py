"""The seeded input generator: determinism and the documented recipe."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "synth_crc.json")


def test_generator_crc_frozen(synth):
    want = json.load(open(GOLD))
    for i in range(3):
        assert synth.crc32(synth.plain_640(i)) == want[f"plain_640/{i}"]
        assert synth.crc32(synth.plain_1080(i)) == want[f"plain_1080/{i}"]
    for i in (0, 17, 40, 63):
        sc, _ = synth.mixed_batch_scene(i)
        assert [sc.W, sc.H, sc.n_lanes, synth.crc32(synth.mixed_batch(i))] == want[f"mixed_batch/{i}"]
    c, s = synth.trig_q14(360)
    assert [synth.crc32(c), synth.crc32(s)] == want["trig_q14/360"]


def test_same_seed_same_bytes_and_pitch(synth):
    sc = synth.scene_road(97, 61)
    a = synth.gen_frame(sc, 1234)
    b = synth.gen_frame(sc, 1234, pitch=128)
    assert (a == b[:, :97]).all() and (b[:, 97:] == 0).all()
    assert not (a == synth.gen_frame(sc, 1235)).all()


def test_background_statistics(synth):
    img = synth.gen_frame(synth.Scene(640, 480, n_lanes=0), 7).astype(np.float64)
    assert abs(img.mean() - 90.0) < 0.2 and abs(img.std() - 12.0) < 0.2


def test_salt_fraction(synth):
    img = synth.gen_frame(synth.Scene(640, 480, n_lanes=0, salt_p=0.02), 3)
    frac = (img == 255).mean()
    assert 0.018 < frac < 0.022


def test_mixed_batch_sizes(synth):
    sizes = [synth.mixed_batch_scene(i)[0] for i in range(64)]
    for q, (W, H) in enumerate(synth.MIXED_SIZES):
        assert all((s.W, s.H) == (W, H) for s in sizes[16 * q:16 * q + 16])
    assert all(2 <= s.n_lanes <= 6 for s in sizes)


def test_lanes_are_bright_bands(synth):
    sc = synth.scene_plain_640()
    seed = synth.frame_seed(0, 0, 0)
    img = synth.gen_frame(sc, seed)
    seg = synth.lane_segments(sc, seed)
    for x0, y0, x1, y1 in seg:
        # the pixel on the segment a quarter of the way up is lane-bright
        x, y = x0 + 0.25 * (x1 - x0), y0 + 0.25 * (y1 - y0)
        xi, yi = int(round(x)), int(round(y))
        if 0 <= xi < 640 and 0 <= yi < 480:
            assert img[yi, xi] >= 200
