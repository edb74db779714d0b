"""MI355X-native conservative implicit scheme for steady diatomic (Rykov) flow.

Importing the package is cheap: the HIP library is loaded by
``paper_2303_10846_amd.binding`` on first use.
"""
__version__ = "0.1.0"
