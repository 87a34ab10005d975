"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Nothing here is part of the encoder: these modules only draw the target fields
and random primitive sets that stand in for the paper's datasets (which are not
available).  They hold none of the encoder's arithmetic.
"""
