"""Test package (lets tests import shared helpers such as tests.parity)."""
