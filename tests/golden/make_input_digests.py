"""Writes tests/golden/input_digests.txt: SHA-256 of every array the seeded
generators produce for the workloads (no method arithmetic).  Run by hand
after a deliberate generator change:
    python tests/golden/make_input_digests.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1609_03986_amd import synth  # noqa: E402


def digests():
    out = {}
    for name, w in (("small", synth.workload_small()), ("hd", synth.workload_hd())):
        for key in sorted(w):
            if hasattr(w[key], "tobytes"):
                out["%s.%s" % (name, key)] = hashlib.sha256(w[key].tobytes()).hexdigest()
    out["triplets"] = hashlib.sha256(synth.triplet_table().tobytes()).hexdigest()
    out["triplets_64x8"] = hashlib.sha256(synth.triplet_table_geom(64, 8).tobytes()).hexdigest()
    out["gaussian_weights_8_2_128"] = hashlib.sha256(synth.gaussian_weights(8, 2.0, 128).tobytes()).hexdigest()
    return out


def main():
    with open(os.path.join(HERE, "input_digests.txt"), "w") as fh:
        fh.write("# SHA-256 of the seeded synthetic inputs (written by make_input_digests.py).\n")
        for k, v in digests().items():
            fh.write("%s = %s\n" % (k, v))


if __name__ == "__main__":
    main()
