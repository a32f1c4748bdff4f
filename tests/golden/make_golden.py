"""Writes tests/golden/small_descriptors.txt.  Calls only the oracle and the
seeded input generators; run it by hand after a justified oracle change:
    python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1609_03986_amd import synth  # noqa: E402


def main():
    trip = synth.triplet_table()
    w = synth.workload_small()
    d, f = oracle.extract(w["query_image"], w["query_kps"][:256], trip)
    assert f == 0
    with open(os.path.join(HERE, "small_descriptors.txt"), "w") as fh:
        fh.write("# Oracle descriptors (uint32[256][16], little-endian) of the first 256\n")
        fh.write("# keypoints of the 640x480 upright workload, seeded triplet table.\n")
        fh.write("# Written by tests/golden/make_golden.py (oracle only).\n")
        fh.write("sha256_first256 = %s\n" % hashlib.sha256(d.tobytes()).hexdigest())
        fh.write("sha256_triplets = %s\n" % hashlib.sha256(trip.tobytes()).hexdigest())
        fh.write("popcount_first256 = %d\n" % int(sum(bin(int(x)).count("1") for x in d.ravel())))


if __name__ == "__main__":
    main()
