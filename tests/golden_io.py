"""Reader for the hand-worked text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] in ("rows", "cols"):
                sections[parts[0]] = int(parts[1])
            elif len(parts) == 1 and parts[0].isalpha():
                cur = parts[0]
                sections[cur] = []
            else:
                sections[cur].append([float(x) for x in parts])
    H, W = sections["rows"], sections["cols"]
    dem = np.array(sections["dem"], dtype=np.float32).reshape(H, W)
    dirs = np.array(sections["dirs"], dtype=np.float64).astype(np.uint8).reshape(H, W)
    area = np.array(sections["area"], dtype=np.float64).astype(np.uint32).reshape(H, W)
    return dem, dirs, area
