"""Numbers printed in the paper, stored as text fixtures (paper_values.json);
each entry carries the passage it comes from."""
import json
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_values.json")


def paper_value(key):
    with open(_PATH) as fh:
        return json.load(fh)[key]
