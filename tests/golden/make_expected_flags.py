"""Writes the oracle's flags for the full-size batching workload (50,000
candidate pairs from a pool of 4,096 meshes, face counts log-uniform in
[500, 100,000]) to tests/golden/c3_flags.txt, so that the GPU parity test
need not rerun the exact oracle for several minutes.

Calls only the generators (seeded inputs) and oracle/ (the expected values);
nothing here touches the HIP library.  The file records the SHA-256 of the
exact input bytes; the test refuses the stored flags if they differ.

    python tests/golden/make_expected_flags.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "c3_flags.txt")


def input_digest(A, B, pairs) -> str:
    h = hashlib.sha256()
    for S in (A, B):
        for a in (S.verts, S.faces, S.vert_off, S.face_off):
            h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.ascontiguousarray(np.asarray(pairs, np.int32)).tobytes())
    return h.hexdigest()


def load(path=OUT):
    """(digest, flags u8[P]) from a stored file."""
    digest, n, hexbits = None, None, []
    for line in open(path):
        line = line.strip()
        if line.startswith("# sha256 "):
            digest = line.split()[2]
        elif line.startswith("# pairs "):
            n = int(line.split()[2])
        elif line and not line.startswith("#"):
            hexbits.append(line)
    bits = np.frombuffer(bytes.fromhex("".join(hexbits)), np.uint8)
    return digest, np.unpackbits(bits)[:n].astype(np.uint8)


def main():
    import oracle
    from paper_2609_24513_amd import synth
    A, B, pairs = synth.make_c3()
    flags = oracle.join(A, B, pairs, mode=1)
    hexs = np.packbits(flags).tobytes().hex()
    with open(OUT, "w") as fh:
        fh.write("# Exact oracle flags (1 = the closed surfaces share a point) of the batching workload:\n")
        fh.write("# synth.make_c3() with its defaults (seed 3, 50,000 pairs, pool 4,096, faces 500..100,000).\n")
        fh.write("# Written by tests/golden/make_expected_flags.py from oracle.join (exact SAT, mode 1).\n")
        fh.write("# sha256 %s\n" % input_digest(A, B, pairs))
        fh.write("# pairs %d\n" % flags.shape[0])
        fh.write("# true %d\n" % int(flags.sum()))
        for k in range(0, len(hexs), 100):
            fh.write(hexs[k:k + 100] + "\n")
    print("wrote", OUT, int(flags.sum()), "of", flags.shape[0])


if __name__ == "__main__":
    main()
