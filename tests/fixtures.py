"""Reader for the text fixtures under tests/golden/ (values printed in the
paper, each file citing its passage): one "name value" pair per line, '#'
starts a comment."""
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, value = line.split()
                vals[key] = float(value)
    return vals
