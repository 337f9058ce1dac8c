"""Write synth_crc.json: CRC32 of seeded generator frames.

These are regression values of the INPUT generator only (no lane-detection
arithmetic is involved), so that a change to the frame recipe is noticed.
Run:  python tests/golden/make_synth_crc.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_2212_09460_amd import synth  # noqa: E402

out = {}
for i in range(3):
    out[f"plain_640/{i}"] = synth.crc32(synth.plain_640(i))
    out[f"plain_1080/{i}"] = synth.crc32(synth.plain_1080(i))
for i in (0, 17, 40, 63):
    sc, seed = synth.mixed_batch_scene(i)
    out[f"mixed_batch/{i}"] = [sc.W, sc.H, sc.n_lanes, synth.crc32(synth.mixed_batch(i))]
c, s = synth.trig_q14(360)
out["trig_q14/360"] = [synth.crc32(c), synth.crc32(s)]
c, s = synth.trig_q14(180)
out["trig_q14/180"] = [synth.crc32(c), synth.crc32(s)]
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_crc.json"), "w") as f:
    json.dump(out, f, indent=1, sort_keys=True)
print(out)
