"""Reader for the small text fixtures in this folder (sections in [brackets])."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read(name):
    sections = {}
    cur = None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                sections[cur] = []
                continue
            sections[cur].append(line.split())
    return sections
