"""Stored expected values.

The paper prints no worked example with values (its tables give campaign
runtimes of designs that are not published), so no fixture here comes from
the paper itself.  Expected values of the full-size workloads are computed by
the oracle when the tests run (tests/full_size_ref.py) rather than stored.
"""
