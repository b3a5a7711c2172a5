"""Oracle package -- test infrastructure only (see amg.py)."""
