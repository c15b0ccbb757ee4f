"""CPU oracle of the ASE-DF method -- test infrastructure only (see oracle.py)."""
